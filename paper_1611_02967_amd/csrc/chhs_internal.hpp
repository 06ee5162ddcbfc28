// Internal declarations shared by the host driver and the kernels of libchhs.
//
// Grid conventions (App. A of arXiv 1611.02967): cell-centred fields over an
// nx x ny (x nz) box of one spacing h, interior cells only, x fastest.
// Homogeneous Neumann data (eqn:nbc1-3) are applied by leaving boundary faces
// out of every stencil sum: a missing neighbour contributes no flux.
//
// Every launch covers a batch of independent instances: a block finds its
// instance and cells through a task table (one entry per block) and the level
// through a table of descriptors in device memory.  A single grid is a batch
// of one.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace chhs {

constexpr int kMaxLevels = 16;       // levels per instance
constexpr int kBlock = 256;          // threads per block of the cell kernels
constexpr int kMaxTailLevels = 8;    // levels handled by the single-workgroup tail
constexpr size_t kTailLdsBudget = 150 * 1024;   // LDS bytes the tail may stage
constexpr int kPartialStride = 16;   // doubles per block in the partial buffer
constexpr int kResStride = 16;       // doubles per instance in the result area

// Working view of one multigrid level of one instance.
//   u = (phi, mu, p)      the current iterate; (phi_alt, mu_alt, p_alt) the other
//                         copy, written by out-of-place kernels
//   ub                    u as restricted from the finer level (FAS)
//   f                     right-hand side of the three rows of (2.5)-(2.7)
//   fr                    coarse levels: the restricted residual R(f - N(u)) of
//                         the finer level, from which the FAS right-hand side
//                         f = fr + N(u) is formed (out of place, so that a
//                         kernel forming f never races a neighbour's read)
//   pstar, psi            phi_* (2.4) and phi^m (second argument of chi), cell
//                         averages of the finer level's on coarse levels
//   b                     base state of the correction form (mixed precision
//                         inner solve); null in the plain form
// lam = s/h^2, kap = 3/4 eps^2 / h^2, gamma as in (1.3).  order = 2: chi of
// (2.4); order = 1 (the first-order bootstrap step): chi(phi) = phi^3 and
// kap = eps^2 / h^2.
template <typename T>
struct Level {
    T* phi;
    T* mu;
    T* p;
    T* ub0;
    T* ub1;
    T* ub2;
    T* f0;
    T* f1;
    T* f2;
    T* fr0;
    T* fr1;
    T* fr2;
    T* pstar;
    T* psi;
    T* b;
    T* phi_alt;
    T* mu_alt;
    T* p_alt;
    int nx, ny, nz, n;
    int order;
    T lam, kap, gamma, h;
};

// Descriptor of one level of one instance, written once at init.  u[c] is copy
// c of (phi, mu, p); levels without a second copy repeat the first.
template <typename T>
struct LevelDesc {
    T* u[2][3];
    T* ub[3];
    T* f[3];
    T* fr[3];
    T* pstar;
    T* psi;
    T* b;
    int nx, ny, nz, n;
    int order;
    T lam, kap, gamma, h;
};

template <typename T>
__host__ __device__ inline Level<T> make_view(const LevelDesc<T>& d, int cur) {
    Level<T> v;
    v.phi = d.u[cur][0];
    v.mu = d.u[cur][1];
    v.p = d.u[cur][2];
    v.phi_alt = d.u[cur ^ 1][0];
    v.mu_alt = d.u[cur ^ 1][1];
    v.p_alt = d.u[cur ^ 1][2];
    v.ub0 = d.ub[0];
    v.ub1 = d.ub[1];
    v.ub2 = d.ub[2];
    v.f0 = d.f[0];
    v.f1 = d.f[1];
    v.f2 = d.f[2];
    v.fr0 = d.fr[0];
    v.fr1 = d.fr[1];
    v.fr2 = d.fr[2];
    v.pstar = d.pstar;
    v.psi = d.psi;
    v.b = d.b;
    v.nx = d.nx;
    v.ny = d.ny;
    v.nz = d.nz;
    v.n = d.n;
    v.order = d.order;
    v.lam = d.lam;
    v.kap = d.kap;
    v.gamma = d.gamma;
    v.h = d.h;
    return v;
}

// Per-instance constants in device memory.
struct InstInfo {
    int dim, nlev, tail;   // levels; first level of the one-workgroup tail
    int off;               // offset of the instance in packed caller arrays
    int n0;                // cells of the finest level
    int fused;             // the finest-level post launch yields the norm partials
    int order;             // 2: the scheme (2.4)-(2.7); 1: the first-order step
    double h, eps, gamma, dt;
};

struct CellTask { int inst; int cell0; };      // kBlock consecutive cells of one level
struct TileTask { int inst; int bx; int by; }; // one tile of a 2D level
struct StripTask { int inst; int sx; int y0; int y1; };   // rows [y0, y1) of strip sx
struct Range { int begin; int end; };          // an instance's blocks in a partial buffer
struct FoldTask { int inst; int begin; int end; };   // partials [begin, end) of one instance
struct Step3Task { int inst; int bx; int by; int z0; int z1; };   // tile (bx, by), planes [z0, z1)

// Arguments common to every batched launch.
template <typename T>
struct Batch {
    const LevelDesc<T>* desc;   // [inst * kMaxLevels + level]
    const int* active;          // instance takes part in this cycle (nullptr: all)
    int level;                  // level of the launch (the finer one for transfers)
    int cur;                    // current copy of u on `level`
    int cur_c;                  // current copy of u on level + 1
    // Deferred p shift: the finest level's p is stored before subtracting its
    // mean pshift[inst * kResStride + 4]; a launch given pshift subtracts it
    // where it reads that p (nullptr: nothing pending).
    const double* pshift;
};

// ---- per-cell kernels (chhs_kernels.hip); dim is 2 or 3 ----------------------------
// With partial: also the norm partials of the initial guess's residual, as
// launch_residual_partials gives them (one per task).  With frozen32 (mixed
// precision): also phi_* and phi^m rounded to FP32 on the finest level of that
// hierarchy, and with partial the residual rounded to FP32 as that level's
// right-hand side and b = phi^m.
void launch_setup(int dim, const Batch<double>& b, const CellTask* t, int nt, const InstInfo* info,
                  const double* phi_prev, const double* phi_cur, const double* mu,
                  const double* p, double* partial, const Batch<float>* frozen32, hipStream_t st);
// FP64 overloads act on the plain form, FP32 overloads on the correction form
// of the mixed-precision inner solve (restriction then also averages b).
void launch_restrict_frozen(int dim, const Batch<double>& b, const CellTask* t, int nt,
                            hipStream_t st);
void launch_restrict_frozen(int dim, const Batch<float>& b, const CellTask* t, int nt,
                            hipStream_t st);
// The same restriction from level `from` down to each instance's coarsest
// level, one workgroup per instance (levels below a few thousand cells).
void launch_restrict_frozen_chain(int dim, const LevelDesc<double>* desc, const InstInfo* info,
                                  int n_inst, int from, hipStream_t st);
void launch_restrict_frozen_chain(int dim, const LevelDesc<float>* desc, const InstInfo* info,
                                  int n_inst, int from, hipStream_t st);
void launch_smooth(int dim, const Batch<double>& b, const CellTask* t, int nt, int color,
                   hipStream_t st);
void launch_smooth(int dim, const Batch<float>& b, const CellTask* t, int nt, int color,
                   hipStream_t st);
// One color of one step with one thread per cell of the color (even nx; task
// cell0 counts cells of the color).
void launch_smooth_color(int dim, const Batch<double>& b, const CellTask* t, int nt, int color,
                         hipStream_t st);
void launch_smooth_color(int dim, const Batch<float>& b, const CellTask* t, int nt, int color,
                         hipStream_t st);
void launch_restrict_residual(int dim, const Batch<double>& b, const CellTask* t, int nt,
                              hipStream_t st);
void launch_restrict_residual(int dim, const Batch<float>& b, const CellTask* t, int nt,
                              hipStream_t st);
void launch_coarse_rhs(int dim, const Batch<double>& b, const CellTask* t, int nt, hipStream_t st);
void launch_coarse_rhs(int dim, const Batch<float>& b, const CellTask* t, int nt, hipStream_t st);
// u += P(u_c - ub_c) in place on the current copy of level b.level; bilinear:
// cell-centred bi/trilinear interpolation, else piecewise-constant injection.
void launch_prolong(int dim, const Batch<double>& b, const CellTask* t, int nt, bool bilinear,
                    hipStream_t st);
void launch_prolong(int dim, const Batch<float>& b, const CellTask* t, int nt, bool bilinear,
                    hipStream_t st);
// Mixed precision (finest level): a zero FP32 correction; the FP64 outer step
// u' = u (+ e), R = f - N(u') written as u' (other FP64 copy), R and b = phi'
// in FP32, and norm partials (as launch_residual_partials); an instance
// inactive now but flagged in was_active (its flags of the previous
// refinement; nullptr: every inactive instance) copies its iterate into the
// other copy.
void launch_zero_correction(const Batch<float>& b32, const CellTask* t, int nt, hipStream_t st);
// The same outer step on 2D finest levels, by row marching: task = window of
// kMarchCols columns (StripTask::sx) x rows [y0, y1); partial[task] gets the
// task's sums.
constexpr int kMarchCols = 128;
void launch_mixed_residual_rows(const Batch<double>& b64, const Batch<float>& b32,
                                const StripTask* t, int nt, int add, const int* was_active,
                                double* partial, hipStream_t st);
void launch_mixed_residual(int dim, const Batch<double>& b64, const Batch<float>& b32,
                           const CellTask* t, int nt, int add, const int* was_active,
                           double* partial, hipStream_t st);
// partial[block][0..3] = sum R_phi^2, R_mu^2, R_p^2, p over the block's cells
void launch_residual_partials(int dim, const Batch<double>& b, const CellTask* t, int nt,
                              double* partial, hipStream_t st);
// Per instance i (one block each), if active[i] (or active == nullptr): sums
// its partials in a fixed order -- partial_t[ranges_t[i]] when use_fused and
// info[i].fused, else partial[ranges[i]]; res[i*kResStride + 0..3] = ||R_phi||,
// ||R_mu||, ||R_p||, combined norm; 4 = mean(p); 5 = 1 if the norm is not
// finite; count != 0: cycles[i] += 1; act_next[i] = norm > tol, finite and
// cycles[i] < max_cycles.  Inactive instances keep their results.
// dst[q] = the sum of src[t[q].begin .. t[q].end) (4 doubles per partial, in
// index order within each thread's stride, then over the block), for the
// tasks of active instances.
void launch_fold_partials(const double* src, const FoldTask* t, int nt, const int* active,
                          double* dst, hipStream_t st);
// The same for the energy partials (eight sums and a maximum each).
void launch_fold_energy(const double* src, const FoldTask* t, int nt, double* dst, hipStream_t st);
void launch_inst_reduce(const double* partial, const Range* ranges, const double* partial_t,
                        const Range* ranges_t, int use_fused, const InstInfo* info,
                        const int* active, int* act_next, int* cycles, double* res, int n_inst,
                        double tol, int max_cycles, int count, hipStream_t st);
// p -= mean(p) (res slot 4) on the finest level of active instances.
// res[i * kResStride + 4] = 0 for every instance (a deferred p shift applied)
void launch_clear_pshift(double* res, int n_inst, hipStream_t st);
void launch_shift_p(const Batch<double>& b, const CellTask* t, int nt, const double* res,
                    hipStream_t st);
// Energy partials over the finest level: ws != 0 takes phi = u, q = phi^m and
// the flow terms from mu, p, phi_* of the workspace; else the packed caller
// arrays phi and q and no flow terms.  partial[block][0..8]: sum phi, phi^2,
// phi^4, |D phi|^2 h^2, (phi-q)^2, |D(phi-q)|^2 h^2, |D mu|^2 h^2, |u|^2 h^2,
// max |phi| (interior faces only).
// The step's copy into the caller's packed arrays, fused into the energy pass
// over the workspace: phi_prev <- phi^m, phi_cur <- phi, mu <- mu, p <- p minus
// the pending shift (b.pshift), as launch_copy_out.
struct CopyOut {
    double *phi_prev, *phi_cur, *mu, *p;
};
void launch_energy_partials(int dim, const Batch<double>& b, const CellTask* t, int nt,
                            const InstInfo* info, int ws, const double* phi, const double* q,
                            double* partial, hipStream_t st, const CopyOut* copy = nullptr);
// Per instance: out[i*kResStride + 0..5] = mass, E_h, F_h, s||grad mu||^2,
// (s/gamma)||u||^2, max |phi|.
void launch_energy_reduce(const double* partial, const Range* ranges, const InstInfo* info,
                          double* out, int n_inst, hipStream_t st);
// State rotation into packed caller arrays: phi_prev <- phi_cur, phi_cur <- phi,
// mu <- mu, p <- p (finest level, current copy).
void launch_copy_out(const Batch<double>& b, const CellTask* t, int nt, const InstInfo* info,
                     double* phi_prev, double* phi_cur, double* mu, double* p, hipStream_t st);
// Finest-level iterate into packed caller arrays (any may be null).
void launch_get_solution(const Batch<double>& b, const CellTask* t, int nt, const InstInfo* info,
                         double* phi, double* mu, double* p, hipStream_t st);
void launch_fill_int(int* dst, int n, int value, hipStream_t st);
void launch_copy_int(int* dst, const int* src, int n, hipStream_t st);
// last <- cur, cur <- next (per-instance flags)
void launch_roll_flags(int* last, int* cur, const int* next, int n, hipStream_t st);

// ---- tiled 2D smoothing (chhs_tile2d.hip) ------------------------------------------
// Tiles are 64 x 16 cells, or on coarse levels 64 x 8 or 64 x 4 (more,
// smaller blocks: on levels with few tiles the time of one block is the time
// of the launch), or on the FP32 finest level 64 x 32 (fewer cells of the
// halo recomputed per cell of the tile).
constexpr int kTileX = 64;
constexpr int kTileY = 16;
constexpr int kTileYSmall = 8;
constexpr int kTileYTiny = 4;
constexpr int kTileYTall = 32;
// ns fused smoothing steps on level b.level of every tasked instance, read from
// copy b.cur and written to the other copy; epi 0 none, 1 residual + restriction
// into level + 1 (copy b.cur_c), 2 residual-norm partials (4 per block, in task
// order); pro: prolongation of level + 1's correction first; level0: f_phi =
// phi^m and f_p = 0 implied; threads: 256, 512 or 1024 per block (four, two
// or one pair of cells per thread);
// rhs: first pre-smoothing launch on a coarse level, which first forms the FAS
// right-hand side f += N(u) (not with level0, pro or epi 2); ty: tile height,
// kTileY or (not with level0) kTileYSmall or kTileYTiny, as the tasks were cut,
// or (FP32, not with rhs) kTileYTall;
// zero (FP32 only, the finest level's first launch of a correction cycle, 64 x
// 16 or 64 x 32 tiles, not with pro, rhs or epi 2): u is taken as zero instead of read.
template <typename T>
void launch_tile2d(const Batch<T>& b, const TileTask* t, int nt, bool level0, int ns, int epi,
                   bool pro, int threads, bool rhs, int ty, bool zero, double* partial,
                   hipStream_t st);

// ---- row-streaming 2D smoothing (chhs_stream2d.hip) ---------------------------------
// Strip sx owns columns [sx kStripWO, (sx + 1) kStripWO) and stages kStripW
// columns from sx kStripWO - kStripHX.  Segments start at even rows.
constexpr int kStripW = 128;
constexpr int kStripHX = 6;
constexpr int kStripWO = kStripW - 2 * kStripHX;
// Same contract as launch_tile2d over strip tasks; partial gets 4 sums per task.
template <typename T>
void launch_stream2d(const Batch<T>& b, const StripTask* t, int nt, bool level0, int ns, int epi,
                     bool pro, bool zero, double* partial, hipStream_t st);

// ---- fused 3D smoothing steps by z marching (chhs_step3d.hip) ----------------------
// One red-black smoothing step on level b.level of every tasked instance, read
// from copy b.cur and written to the other copy.  Tiles of (x, y) columns:
// 16 x 16 in FP64, 32 x 8 in FP32 (correction form).
constexpr int kStep3TX64 = 16, kStep3TY64 = 16;
constexpr int kStep3TX32 = 32, kStep3TY32 = 8;
// Residual of a 3D level by z marching over the level's fused-step tasks:
// norm partials of the finest FP64 level (one per task, as the per-cell
// residual partials) or residual + restriction into level b.level + 1 (copy
// b.cur_c): u_c, ub_c, fr_c (and b_c in the correction form).
void launch_residual3d_partials(const Batch<double>& b, const Step3Task* t, int nt, double* partial,
                                hipStream_t st);
void launch_restrict3d(const Batch<double>& b, const Step3Task* t, int nt, hipStream_t st);
void launch_restrict3d(const Batch<float>& b, const Step3Task* t, int nt, hipStream_t st);
// The FP64 refinement step of the mixed path on the finest 3D level over its
// fused-step tasks (as launch_mixed_residual; partials one per task).
void launch_refine3d(const Batch<double>& b64, const Batch<float>& b32, const Step3Task* t, int nt,
                     int add, const int* was_active, double* partial, hipStream_t st);
// pro: 0 no prolongation, 1 piecewise-constant, 2 trilinear coarse correction
// added to u (from level + 1, copy cur_c) as the launch loads it; zero: u is
// the zero correction (not read); b.pshift: the pending mean of p subtracted
// as p is loaded
void launch_step3d(const Batch<double>& b, const Step3Task* t, int nt, int pro, int zero,
                   hipStream_t st);
void launch_step3d(const Batch<float>& b, const Step3Task* t, int nt, int pro, int zero,
                   hipStream_t st);

// ---- single-workgroup coarse tail (chhs_tail.hip) ----------------------------------
// The cycle's shape: smoothing steps before / after the coarse correction on
// the finest level (f) and on the coarser ones (c), steps on the coarsest
// grid, and the prolongation (bilinear != 0: bi/trilinear, else piecewise
// constant).
struct CycleShape {
    int nu1f, nu2f, nu1c, nu2c, coarse, bilinear;
};
size_t tail_lds_bytes(const int* cells, int nlev, size_t elem, int nfields);
template <typename T, bool CORR>
int prepare_tail(int dim, size_t lds_bytes);
// One workgroup per listed instance: the V-cycle over levels info.tail ..
// info.nlev - 1 of that instance; bit l of cur_mask = current copy of u on
// level l.
template <typename T, bool CORR>
void launch_tail(int dim, const LevelDesc<T>* desc, const InstInfo* info, const int* insts,
                 int ninst, const int* active, unsigned cur_mask, const CycleShape& shape,
                 double* pend, size_t lds_bytes, hipStream_t st);

}  // namespace chhs
