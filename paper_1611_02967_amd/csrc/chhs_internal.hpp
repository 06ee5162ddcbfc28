// Internal declarations shared by the host driver and the kernels of libchhs.
//
// Grid conventions (App. A of arXiv 1611.02967): cell-centred fields over an
// nx x ny (x nz) box of one spacing h, interior cells only, x fastest.
// Homogeneous Neumann data (eqn:nbc1-3) are applied by leaving boundary faces
// out of every stencil sum: a missing neighbour contributes no flux.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace chhs {

// Device view of one multigrid level of one instance.
//   u      = (phi, mu, p), the current iterate
//   ub     = u as restricted from the finer level before the coarse solve (FAS)
//   f      = right-hand side of the three rows of (2.5)-(2.7)
//   pstar  = phi_* of (2.4) (cell average of the finer level's on coarse levels)
//   psi    = phi^m, the second argument of chi
//   phi_alt, mu_alt, p_alt = second copy of u: out-of-place kernels (the tiled
//          2D smoother) read u and write u_alt, and the host then swaps the
//          two, so that no block reads a halo another block already updated
// lam = s/h^2, kap = 3/4 eps^2 / h^2, gamma as in (1.3).
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
    T* pstar;
    T* psi;
    T* phi_alt;
    T* mu_alt;
    T* p_alt;
    int nx, ny, nz, n;
    T lam, kap, gamma, h;
};

constexpr int kBlock = 256;          // threads per block of the cell kernels
constexpr int kMaxTailLevels = 8;    // levels handled by the single-workgroup tail
constexpr size_t kTailLdsBudget = 150 * 1024;   // LDS bytes the tail may stage
constexpr int kMaxPartials = 1024;   // blocks of the two-pass reductions
constexpr int kPartialStride = 16;   // doubles per block in the partial buffer

// ---- launchers (chhs_kernels.hip); dim is 2 or 3 ------------------------------
void launch_setup(int dim, const Level<double>& L, const double* phi_prev,
                  const double* phi_cur, const double* mu, const double* p,
                  double quarter_eps2_over_h2, hipStream_t st);
void launch_restrict_frozen(int dim, const Level<double>& F, const Level<double>& C,
                            hipStream_t st);
void launch_smooth(int dim, const Level<double>& L, int color, hipStream_t st);
void launch_restrict_residual(int dim, const Level<double>& F, const Level<double>& C,
                              hipStream_t st);
void launch_coarse_rhs(int dim, const Level<double>& C, hipStream_t st);
void launch_prolong(int dim, const Level<double>& F, const Level<double>& C, hipStream_t st);

// Residual reduction: partial[b][0..3] = sum R_phi^2, R_mu^2, R_p^2, p over the
// cells of block b; returns the number of blocks used.
int launch_residual_partials(int dim, const Level<double>& L, double* partial, hipStream_t st);
// out[c] = sum over blocks of partial[b][c] for c < ncomp (fixed order).
void launch_reduce_final(const double* partial, int nblocks, int ncomp, double* out,
                         hipStream_t st);
// p -= sum_p / n with sum_p read from device memory.
void launch_shift_p(const Level<double>& L, const double* sum_p, hipStream_t st);

// Energy reduction over (phi, q[, mu, p, pstar]): partial[b][0..8] =
//   sum phi, phi^2, phi^4, |D phi|^2 h^2, (phi-q)^2, |D(phi-q)|^2 h^2,
//   |D mu|^2 h^2, |u|^2 h^2, and max |phi| in slot 8.
// Face sums run over interior faces; mu == nullptr skips the two flow terms.
int launch_energy_partials(int dim, int nx, int ny, int nz, const double* phi,
                           const double* q, const double* mu, const double* p,
                           const double* pstar, double gamma, double* partial,
                           hipStream_t st);
void launch_reduce_energy(const double* partial, int nblocks, double* out, hipStream_t st);

// ---- tiled 2D smoothing (chhs_tile2d.hip) ----------------------------------------
// Blocks of one tiled launch on an nx x ny level.
int tile2d_blocks(int nx, int ny);
// ns fused smoothing steps on L; epi 0 none, 1 residual + restriction into C,
// 2 residual-norm partials (4 per block); pro: prolongation of C's correction
// first; level0: f_phi = phi^m and f_p = 0 implied.  Returns blocks launched.
template <typename T>
int launch_tile2d(const Level<T>& L, const Level<T>& C, bool level0, int ns, int epi, bool pro,
                  double* partial, hipStream_t st);

// ---- single-workgroup coarse tail (chhs_tail.hip) ---------------------------------
size_t tail_lds_bytes(const int* cells, int nlev, size_t elem);
template <typename T>
int prepare_tail(int dim, size_t lds_bytes);
// V(nu1, nu2) cycle over levels[0..nlev-1] (levels[0] = the tail's top level,
// whose iterate is updated in global memory).
template <typename T>
void launch_tail(int dim, const Level<T>* levels, int nlev, int nu1, int nu2, int coarse_sweeps,
                 size_t lds_bytes, hipStream_t st);

}  // namespace chhs
