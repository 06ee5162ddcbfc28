// Per-cell kernels of the FAS solve for one step of the CHHS scheme (2.4)-(2.7),
// batched over independent instances.
//
// A block covers kBlock consecutive cells of one level of one instance, named
// by its CellTask; neighbours are read straight from global memory.  The
// stencils are the App. A.2 operators with boundary faces left out (zero flux,
// App. A.1).  FP64 throughout.
#include "chhs_cell.hpp"

namespace chhs {
namespace {

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// The task of this workgroup: XCD x = b mod 8 takes a contiguous range of the
// tasks (a bijection on [0, gridDim.x)), so the neighbouring rows and planes
// that consecutive tasks' stencils share are read through one L2.
__device__ __forceinline__ int xcd_task() {
    const int n = int(gridDim.x), bid = int(blockIdx.x);
    const int q8 = n / 8, rem = n % 8;
    const int xcd = bid % 8, jj = bid / 8;
    return xcd * q8 + (xcd < rem ? xcd : rem) + jj;
}

__device__ __forceinline__ bool inactive(const int* active, int inst) {
    return active != nullptr && active[inst] == 0;
}

template <typename T>
__device__ __forceinline__ Level<T> view_at(const Batch<T>& b, int inst, int level, int cur) {
    return make_view(b.desc[inst * kMaxLevels + level], cur);
}

template <int NC, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[NC], double* out);

// Per-step setup of the finest level, and with `partial` the residual of the
// initial guess u = (phi^m, mu, p) in the same pass: its norm partials (R_phi^2,
// R_mu^2, R_p^2, p) per block, as k_residual_partials gives them, formed from
// the caller's arrays (the values the level receives here), with N(u) written
// as cell_operator writes it.  With e32 (mixed precision): the FP32 copies of
// phi_* and phi^m, and with `partial` also the residual rounded to FP32 as the
// first correction cycle's right-hand side and b = phi (what a refinement step
// without a correction writes).
//
// kPairThreads threads per 256-cell task.  Where the instance's x extent is
// even and its arrays allow 2-element accesses (FP64 ones 16-byte aligned,
// FP32 ones 8-byte), a thread takes a pair of x-adjacent cells (2-element loads and stores, the pair's inner faces read
// from registers); otherwise cells q and q + kPairThreads of the task.  Both
// forms sum each cell's faces in the order of for_each_face.
constexpr int kPairThreads = kBlock / 2;

template <int DIM>
__global__ __launch_bounds__(kPairThreads) void k_setup(Batch<double> b,
                                                        const CellTask* __restrict__ t,
                                                        const InstInfo* __restrict__ info,
                                                        const double* __restrict__ phi_prev,
                                                        const double* __restrict__ phi_cur,
                                                        const double* __restrict__ mu,
                                                        const double* __restrict__ p,
                                                        double* partial, Batch<float> e32) {
    typedef double D2 __attribute__((ext_vector_type(2)));
    typedef float F2 __attribute__((ext_vector_type(2)));
    const int task = xcd_task();
    const CellTask tk = t[task];
    const Level<double> L = view_at(b, tk.inst, 0, b.cur);
    const InstInfo in = info[tk.inst];
    const bool res = partial != nullptr;
    const bool mixed = e32.desc != nullptr;
    const Level<float> E = mixed ? view_at(e32, tk.inst, 0, 0) : Level<float>{};
    // the first-order step (order 1): phi_* := phi^m and f_mu = -phi^m
    const bool first = in.order == 1;
    const double q = 0.25 * in.eps * in.eps / (in.h * in.h);
    double v[4] = {0.0, 0.0, 0.0, 0.0};

    // One face of a cell (values pm, pc, ps, muc, pp) with the neighbour
    // (pmn, pcn, mun, pn): the Laplacian of phi^{m-1} and N(u)'s face sums.
    struct Acc {
        double lap = 0, smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
    };
    auto face = [&](Acc& s, bool h, double pm, double pc, double ps, double muc, double pp,
                    double pmn, double pcn, double mun, double pn) {
        const double d = pmn - pm;
        s.lap = h ? s.lap + d : s.lap;
        if (res) {
            const double a = 0.5 * (ps + (first ? pcn : 1.5 * pcn - 0.5 * pmn));
            const double m = 1.0 + L.gamma * a * a;
            const double dmu = mun - muc;
            const double dp = pn - pp;
            const double dphi = pcn - pc;
            s.smm = h ? s.smm + m * dmu : s.smm;
            s.sap = h ? s.sap + a * dp : s.sap;
            s.sphi = h ? s.sphi + dphi : s.sphi;
            s.sp = h ? s.sp + dp : s.sp;
            s.samu = h ? s.samu + a * dmu : s.samu;
        }
    };
    // phi_* (2.4), f_mu (2.6), and the residual of the initial guess
    auto finish = [&](const Acc& s, double pc, double ps, double muc, double pp, double& f1,
                      double& r0, double& r1, double& r2) {
        f1 = first ? -pc : -ps - q * s.lap;
        if (res) {
            const double chi = first ? pc * pc * pc : nonlin<double, false>(pc, pc, 0.0);
            const double n0 = pc - L.lam * s.smm - L.lam * s.sap;
            const double n1 = muc - chi + L.kap * s.sphi;
            const double n2 = L.lam * s.sp + L.lam * L.gamma * s.samu;
            r0 = pc - n0;
            r1 = f1 - n1;
            r2 = -n2;
            v[0] += r0 * r0;
            v[1] += r1 * r1;
            v[2] += r2 * r2;
            v[3] += pp;
        }
    };
    auto phistar = [&](double pm, double pc) { return first ? pc : 1.5 * pc - 0.5 * pm; };

    const uintptr_t bits64 =
        uintptr_t(phi_prev) | uintptr_t(phi_cur) | uintptr_t(mu) | uintptr_t(p) |
        uintptr_t(L.pstar) | uintptr_t(L.psi) | uintptr_t(L.f0) | uintptr_t(L.f1) |
        uintptr_t(L.f2) | uintptr_t(L.phi) | uintptr_t(L.mu) | uintptr_t(L.p);
    const uintptr_t bits32 =
        mixed ? uintptr_t(E.pstar) | uintptr_t(E.psi) | uintptr_t(E.f0) | uintptr_t(E.f1) |
                    uintptr_t(E.f2) | uintptr_t(E.b)
              : uintptr_t(0);
    // (FP64 pairs take 16-byte alignment, FP32 pairs 8-byte)
    const bool pairs =
        (L.nx & 1) == 0 && (in.off & 1) == 0 && (bits64 & 15) == 0 && (bits32 & 7) == 0;

    if (pairs) {
        const int idx = tk.cell0 + 2 * int(threadIdx.x);   // first cell of the pair
        if (idx < L.n) {
            int i, j, k;
            decode<DIM>(idx, L.nx, L.ny, i, j, k);
            const int g = in.off + idx;
            auto ld2 = [&](const double* a, int c) {
                return gload(reinterpret_cast<const D2*>(a), c >> 1);
            };
            const D2 pm = ld2(phi_prev, g), pc = ld2(phi_cur, g);
            const D2 muc = ld2(mu, g), pp = ld2(p, g);
            const D2 ps = {phistar(pm.x, pc.x), phistar(pm.y, pc.y)};
            // outer x neighbours (the cell itself across a boundary face)
            const bool hl = i > 0, hr = i + 2 < L.nx;
            const int ql = hl ? g - 1 : g, qr = hr ? g + 2 : g + 1;
            const double pml = gload(phi_prev, ql), pmr = gload(phi_prev, qr);
            const double pcl = res ? gload(phi_cur, ql) : 0.0, pcr = res ? gload(phi_cur, qr) : 0.0;
            const double mul = res ? gload(mu, ql) : 0.0, mur = res ? gload(mu, qr) : 0.0;
            const double pl = res ? gload(p, ql) : 0.0, pr = res ? gload(p, qr) : 0.0;
            Acc sa, sb;
            face(sa, hl, pm.x, pc.x, ps.x, muc.x, pp.x, pml, pcl, mul, pl);
            face(sa, true, pm.x, pc.x, ps.x, muc.x, pp.x, pm.y, pc.y, muc.y, pp.y);
            face(sb, true, pm.y, pc.y, ps.y, muc.y, pp.y, pm.x, pc.x, muc.x, pp.x);
            face(sb, hr, pm.y, pc.y, ps.y, muc.y, pp.y, pmr, pcr, mur, pr);
            // y (and z) neighbour pairs: -y, +y (, -z, +z)
            const int sz = L.nx * L.ny;
            const int off[4] = {-L.nx, L.nx, -sz, sz};
            const bool has[4] = {j > 0, j < L.ny - 1, k > 0, k < L.nz - 1};
#pragma unroll
            for (int f = 0; f < 2 * (DIM - 1); ++f) {
                const int qn = has[f] ? g + off[f] : g;
                const D2 pmn = ld2(phi_prev, qn);
                const D2 pcn = res ? ld2(phi_cur, qn) : D2{0.0, 0.0};
                const D2 mun = res ? ld2(mu, qn) : D2{0.0, 0.0};
                const D2 pn = res ? ld2(p, qn) : D2{0.0, 0.0};
                face(sa, has[f], pm.x, pc.x, ps.x, muc.x, pp.x, pmn.x, pcn.x, mun.x, pn.x);
                face(sb, has[f], pm.y, pc.y, ps.y, muc.y, pp.y, pmn.y, pcn.y, mun.y, pn.y);
            }
            double fa, fb, ra0 = 0, ra1 = 0, ra2 = 0, rb0 = 0, rb1 = 0, rb2 = 0;
            finish(sa, pc.x, ps.x, muc.x, pp.x, fa, ra0, ra1, ra2);
            finish(sb, pc.y, ps.y, muc.y, pp.y, fb, rb0, rb1, rb2);
            const int hw = idx >> 1;
            auto st2 = [&](double* a, D2 x) { gstore(reinterpret_cast<D2*>(a), hw, x); };
            auto st2f = [&](float* a, double x, double y) {
                gstore(reinterpret_cast<F2*>(a), hw, F2{float(x), float(y)});
            };
            st2(L.pstar, ps);
            st2(L.psi, pc);
            st2(L.f0, pc);                                 // (2.5): phi^m
            st2(L.f1, D2{fa, fb});                         // (2.6)
            st2(L.f2, D2{0.0, 0.0});                       // (2.7)
            st2(L.phi, pc);                                // initial guess phi^m
            st2(L.mu, muc);
            st2(L.p, pp);
            if (mixed) {
                st2f(E.pstar, ps.x, ps.y);
                st2f(E.psi, pc.x, pc.y);
                if (res) {
                    st2f(E.f0, ra0, rb0);
                    st2f(E.f1, ra1, rb1);
                    st2f(E.f2, ra2, rb2);
                    st2f(E.b, pc.x, pc.y);
                }
            }
        }
    } else {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int idx = tk.cell0 + int(threadIdx.x) + half * kPairThreads;
            if (idx >= L.n) continue;
            const int g = in.off + idx;
            int i, j, k;
            decode<DIM>(idx, L.nx, L.ny, i, j, k);
            const double pm = gload(phi_prev, g), pc = gload(phi_cur, g);
            const double muc = gload(mu, g), pp = gload(p, g);
            const double ps = phistar(pm, pc);
            Acc s;
            for_each_face<DIM>(i, j, k, L.nx, L.ny, L.nz, idx, [&](bool h, int nb) {
                const int gn = in.off + nb;
                face(s, h, pm, pc, ps, muc, pp, gload(phi_prev, gn),
                     res ? gload(phi_cur, gn) : 0.0, res ? gload(mu, gn) : 0.0,
                     res ? gload(p, gn) : 0.0);
            });
            double f1, r0 = 0, r1 = 0, r2 = 0;
            finish(s, pc, ps, muc, pp, f1, r0, r1, r2);
            gstore(L.pstar, idx, ps);
            gstore(L.psi, idx, pc);
            gstore(L.f0, idx, pc);
            gstore(L.f1, idx, f1);
            gstore(L.f2, idx, 0.0);
            gstore(L.phi, idx, pc);
            gstore(L.mu, idx, muc);
            gstore(L.p, idx, pp);
            if (mixed) {
                gstore(E.pstar, idx, float(ps));
                gstore(E.psi, idx, float(pc));
                if (res) {
                    gstore(E.f0, idx, float(r0));
                    gstore(E.f1, idx, float(r1));
                    gstore(E.f2, idx, float(r2));
                    gstore(E.b, idx, float(pc));
                }
            }
        }
    }
    if (!res) return;
    double out[4];
    block_sum<4, kPairThreads>(v, out);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) partial[task * kPartialStride + c] = out[c];
}

// tasks over coarse cells (level b.level + 1)
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_frozen(Batch<T> b,
                                                            const CellTask* __restrict__ t) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    const Level<T> F = view_at(b, tk.inst, b.level, 0);
    const Level<T> C = view_at(b, tk.inst, b.level + 1, 0);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= C.n) return;
    int ci, cj, ck;
    decode<DIM>(idx, C.nx, C.ny, ci, cj, ck);
    T sps = 0, sph = 0;
    for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int f = ((2 * ck + dz) * F.ny + (2 * cj + dy)) * F.nx + 2 * ci + dx;
                sps += F.pstar[f];
                sph += F.psi[f];
            }
    const T w = DIM == 3 ? T(0.125) : T(0.25);
    C.pstar[idx] = sps * w;
    C.psi[idx] = sph * w;
}

constexpr int kChainThreads = 1024;

template <int DIM, typename T>
__global__ __launch_bounds__(kChainThreads) void k_restrict_frozen_chain(
    const LevelDesc<T>* __restrict__ desc, const InstInfo* __restrict__ info, int from) {
    const int nlev = info[blockIdx.x].nlev;
    const LevelDesc<T>* d = desc + blockIdx.x * kMaxLevels;
    for (int l = from; l + 1 < nlev; ++l) {
        const Level<T> F = make_view(d[l], 0);
        const Level<T> C = make_view(d[l + 1], 0);
        for (int idx = threadIdx.x; idx < C.n; idx += blockDim.x) {
            int ci, cj, ck;
            decode<DIM>(idx, C.nx, C.ny, ci, cj, ck);
            T sps = 0, sph = 0;
            for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        const int f = ((2 * ck + dz) * F.ny + (2 * cj + dy)) * F.nx + 2 * ci + dx;
                        sps += F.pstar[f];
                        sph += F.psi[f];
                    }
            const T w = DIM == 3 ? T(0.125) : T(0.25);
            C.pstar[idx] = sps * w;
            C.psi[idx] = sph * w;
        }
        __syncthreads();
    }
}

// L0 (FP64 finest level): f_phi = phi^m and f_p = 0 are not loaded.
template <int DIM, typename T, bool CORR, bool L0 = false>
__global__ __launch_bounds__(kBlock) void k_smooth(Batch<T> b, const CellTask* __restrict__ t,
                                                   int color) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    if (inactive(b.active, tk.inst)) return;
    const Level<T> L = view_at(b, tk.inst, b.level, b.cur);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= L.n) return;
    int i, j, k;
    decode<DIM>(idx, L.nx, L.ny, i, j, k);
    if (((i + j + k) & 1) != color) return;
    T phi, mu, p;
    cell_solve<DIM, T, CORR, L0>(L, idx, i, j, k, T(1) / L.lam, phi, mu, p);
    L.phi[idx] = phi;
    L.mu[idx] = mu;
    L.p[idx] = p;
}

// The same update with threads mapped to the cells of one color only (levels
// with an even x extent: every row holds nx / 2 cells of each color), so that
// no lane of a launch idles on the other color.  Task cell0 counts cells of
// the color.
template <int DIM, typename T, bool CORR, bool L0 = false>
__global__ __launch_bounds__(kBlock) void k_smooth_color(Batch<T> b, const CellTask* __restrict__ t,
                                                         int color) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    if (inactive(b.active, tk.inst)) return;
    const Level<T> L = view_at(b, tk.inst, b.level, b.cur);
    const int q = tk.cell0 + threadIdx.x;
    if (q >= L.n / 2) return;
    const int hx = L.nx / 2;
    const int row = q / hx;                       // row index over (j, k)
    const int m = q - row * hx;
    const int j = DIM == 2 ? row : row % L.ny;
    const int k = DIM == 2 ? 0 : row / L.ny;
    const int i = 2 * m + ((j + k + color) & 1);
    const int idx = row * L.nx + i;
    T phi, mu, p;
    cell_solve<DIM, T, CORR, L0>(L, idx, i, j, k, T(1) / L.lam, phi, mu, p);
    L.phi[idx] = phi;
    L.mu[idx] = mu;
    L.p[idx] = p;
}

// The seven values a fine cell contributes to its coarse cell: the residual
// f - N(u) of the three rows, u, and (CORR) the base state b.
template <int DIM, typename T, bool CORR>
__device__ __forceinline__ void child_values(const Level<T>& F, int fi, int fj, int fk,
                                             T (&v)[7]) {
    const int f = (fk * F.ny + fj) * F.nx + fi;
    T n0, n1, n2;
    cell_operator<DIM, T, CORR>(F, f, fi, fj, fk, n0, n1, n2);
    v[0] = F.f0[f] - n0;
    v[1] = F.f1[f] - n1;
    v[2] = F.f2[f] - n2;
    v[3] = F.phi[f];
    v[4] = F.mu[f];
    v[5] = F.p[f];
    v[6] = CORR ? F.b[f] : T(0);
}

// Per coarse cell: u_c = R u, ub_c = u_c, f_c = R(f - N(u)) (the N_c(u_c) part
// is added by k_coarse_rhs once all of u_c is written).  Child c = dx + 2 dy
// + 4 dz; the children are added in the tree ((c0 + c1) + (c2 + c3)) [+ ((c4
// + c5) + (c6 + c7)) in 3D], the order of the lane exchanges of
// k_restrict_residual_lanes, so that both kernels give the same bits and an
// instance's restriction does not depend on which one its batch launches.
template <int DIM, typename T, bool CORR>
__global__ __launch_bounds__(kBlock) void k_restrict_residual(Batch<T> b,
                                                              const CellTask* __restrict__ t) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    if (inactive(b.active, tk.inst)) return;
    const Level<T> F = view_at(b, tk.inst, b.level, b.cur);
    const Level<T> C = view_at(b, tk.inst, b.level + 1, b.cur_c);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= C.n) return;
    int ci, cj, ck;
    decode<DIM>(idx, C.nx, C.ny, ci, cj, ck);
    T acc[7], half[7];
#pragma unroll 1
    for (int q = 0; q < (DIM == 3 ? 4 : 2); ++q) {    // q = 2 dz + dy: one x pair
        const int dy = q & 1, dz = q >> 1;
        T a[7], c[7];
        child_values<DIM, T, CORR>(F, 2 * ci, 2 * cj + dy, 2 * ck + dz, a);
        child_values<DIM, T, CORR>(F, 2 * ci + 1, 2 * cj + dy, 2 * ck + dz, c);
#pragma unroll
        for (int k = 0; k < 7; ++k) a[k] = a[k] + c[k];
        if (dy == 0) {
#pragma unroll
            for (int k = 0; k < 7; ++k) half[k] = a[k];
        } else {
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                const T s = half[k] + a[k];
                acc[k] = dz == 0 ? s : acc[k] + s;
            }
        }
    }
    const T w = DIM == 3 ? T(0.125) : T(0.25);
    if (CORR) C.b[idx] = acc[6] * w;
    C.phi[idx] = C.ub0[idx] = acc[3] * w;
    C.mu[idx] = C.ub1[idx] = acc[4] * w;
    C.p[idx] = C.ub2[idx] = acc[5] * w;
    C.fr0[idx] = acc[0] * w;
    C.fr1[idx] = acc[1] * w;
    C.fr2[idx] = acc[2] * w;
}

// Launches of at most this many tasks use the lane-parallel restriction below
// (3D 128^3 FP64: the launches into 32^3, 16^3 and 8^3 take 10.5, 4.8 and 5.0
// us against 15.1, 13.6 and 12.5 with the serial loop; into 64^3, 1024 tasks,
// the serial loop is faster).
constexpr int kLaneRestrictTasks = 256;

// The same for levels with few coarse cells, where the serial loop over the
// children above is the latency of the launch.  One thread per
// (coarse cell, child): the 2^DIM children of a coarse cell are consecutive
// lanes, summed by lane exchanges in the fixed order ((c0 + c1) + (c2 + c3))
// [+ the same for c4 .. c7 in 3D].  A workgroup covers 256 / 2^DIM coarse
// cells of a task, so a launch has 2^DIM workgroups per task.
template <int DIM, typename T, bool CORR>
__global__ __launch_bounds__(kBlock) void k_restrict_residual_lanes(Batch<T> b,
                                                                    const CellTask* __restrict__ t) {
    constexpr int NCH = DIM == 3 ? 8 : 4;
    const int w = xcd_task();
    const CellTask tk = t[w / NCH];
    if (inactive(b.active, tk.inst)) return;
    const Level<T> F = view_at(b, tk.inst, b.level, b.cur);
    const Level<T> C = view_at(b, tk.inst, b.level + 1, b.cur_c);
    const int q = tk.cell0 + (w % NCH) * (kBlock / NCH) + int(threadIdx.x) / NCH;
    const int ch = int(threadIdx.x) % NCH;
    // every lane of a child group computes (a group past the level's end on
    // coarse cell 0), so that the exchanges read only computing lanes
    const bool live = q < C.n;
    const int idx = live ? q : 0;
    int ci, cj, ck;
    decode<DIM>(idx, C.nx, C.ny, ci, cj, ck);
    const int fi = 2 * ci + (ch & 1), fj = 2 * cj + ((ch >> 1) & 1), fk = 2 * ck + (ch >> 2);
    T v[7];
    child_values<DIM, T, CORR>(F, fi, fj, fk, v);
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        if (!CORR && c == 6) continue;
        v[c] += __shfl_xor(v[c], 1, 64);
        v[c] += __shfl_xor(v[c], 2, 64);
        if (DIM == 3) v[c] += __shfl_xor(v[c], 4, 64);
    }
    if (!live || ch != 0) return;
    const T wt = DIM == 3 ? T(0.125) : T(0.25);
    if (CORR) C.b[idx] = v[6] * wt;
    C.phi[idx] = C.ub0[idx] = v[3] * wt;
    C.mu[idx] = C.ub1[idx] = v[4] * wt;
    C.p[idx] = C.ub2[idx] = v[5] * wt;
    C.fr0[idx] = v[0] * wt;
    C.fr1[idx] = v[1] * wt;
    C.fr2[idx] = v[2] * wt;
}

// tasks over coarse cells: f_c += N_c(u_c)
template <int DIM, typename T, bool CORR>
__global__ __launch_bounds__(kBlock) void k_coarse_rhs(Batch<T> b,
                                                       const CellTask* __restrict__ t) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    if (inactive(b.active, tk.inst)) return;
    const Level<T> C = view_at(b, tk.inst, b.level + 1, b.cur_c);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= C.n) return;
    int i, j, k;
    decode<DIM>(idx, C.nx, C.ny, i, j, k);
    T n0, n1, n2;
    cell_operator<DIM, T, CORR>(C, idx, i, j, k, n0, n1, n2);
    C.f0[idx] = C.fr0[idx] + n0;
    C.f1[idx] = C.fr1[idx] + n1;
    C.f2[idx] = C.fr2[idx] + n2;
}

// tasks over fine cells: u += P(u_c - ub_c), P piecewise-constant injection
// or (BIL) cell-centred bi/trilinear interpolation
template <int DIM, typename T, bool BIL>
__global__ __launch_bounds__(kBlock) void k_prolong(Batch<T> b, const CellTask* __restrict__ t) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    if (inactive(b.active, tk.inst)) return;
    const Level<T> F = view_at(b, tk.inst, b.level, b.cur);
    const Level<T> C = view_at(b, tk.inst, b.level + 1, b.cur_c);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= F.n) return;
    int i, j, k;
    decode<DIM>(idx, F.nx, F.ny, i, j, k);
    if (BIL) {
        F.phi[idx] += bilinear_corr<DIM>(C.phi, C.ub0, C.nx, C.ny, C.nz, i, j, k);
        F.mu[idx] += bilinear_corr<DIM>(C.mu, C.ub1, C.nx, C.ny, C.nz, i, j, k);
        F.p[idx] += bilinear_corr<DIM>(C.p, C.ub2, C.nx, C.ny, C.nz, i, j, k);
        return;
    }
    const int c = ((k >> 1) * C.ny + (j >> 1)) * C.nx + (i >> 1);
    F.phi[idx] += C.phi[c] - C.ub0[c];
    F.mu[idx] += C.mu[c] - C.ub1[c];
    F.p[idx] += C.p[c] - C.ub2[c];
}

// ---- mixed precision: FP64 outer work around the FP32 correction solve ---------------

// Zero correction on the FP32 finest level (current copy).
__global__ __launch_bounds__(kBlock) void k_zero_correction(Batch<float> b32,
                                                            const CellTask* __restrict__ t) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    if (inactive(b32.active, tk.inst)) return;
    const Level<float> E = view_at(b32, tk.inst, 0, b32.cur);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= E.n) return;
    E.phi[idx] = 0.0f;
    E.mu[idx] = 0.0f;
    E.p[idx] = 0.0f;
}

// Outer step of the iterative refinement on the finest level, in FP64:
//   u' = u + e (add != 0; e the FP32 correction of the last inner cycle),
//   R  = f - N(u') with the plain (2.5)-(2.7) operator,
// written as u' into the other FP64 copy, R and b = u'_phi rounded to FP32
// into the FP32 finest level's right-hand side and base state, and the block
// partial sums of R^2 and p'.  An instance inactive in this refinement but
// active in the previous one (was_active) copies its iterate into the other
// copy, so that both copies hold it from then on and the alternation of the
// copies leaves it current; later refinements skip it.
// A thread takes a pair of x-adjacent cells (2 q, 2 q + 1): the finest level
// has a coarser one, so its x extent is even and a task's 256 cells are 128
// whole pairs of one row each.  The pair's own values and its y (and z)
// neighbours load as 2-element vectors, the pair's outer x neighbours as
// single values; each cell sums its faces in the order of for_each_face.

template <int DIM>
__global__ __launch_bounds__(kPairThreads) void k_mixed_residual(Batch<double> b64,
                                                                 Batch<float> b32,
                                                                 const CellTask* __restrict__ t,
                                                                 int add, const int* was_active,
                                                                 double* partial) {
    typedef double D2 __attribute__((ext_vector_type(2)));
    typedef float F2 __attribute__((ext_vector_type(2)));
    const int task = xcd_task();
    const CellTask tk = t[task];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int idx = tk.cell0 + 2 * int(threadIdx.x);      // first cell of the pair
    const Level<double> L = view_at(b64, tk.inst, 0, b64.cur);
    if (!inactive(b64.active, tk.inst)) {
        const Level<float> E = view_at(b32, tk.inst, 0, b32.cur);
        if (idx < L.n) {
            int i, j, k;
            decode<DIM>(idx, L.nx, L.ny, i, j, k);
            // u + e of the pair at q (even), and of the single cell q
            auto u_pair = [&](int q, D2& ph, D2& m, D2& pp) {
                ph = gload(reinterpret_cast<const D2*>(L.phi), q >> 1);
                m = gload(reinterpret_cast<const D2*>(L.mu), q >> 1);
                pp = gload(reinterpret_cast<const D2*>(L.p), q >> 1);
                if (add) {
                    const F2 e0 = gload(reinterpret_cast<const F2*>(E.phi), q >> 1);
                    const F2 e1 = gload(reinterpret_cast<const F2*>(E.mu), q >> 1);
                    const F2 e2 = gload(reinterpret_cast<const F2*>(E.p), q >> 1);
                    ph.x += double(e0.x);
                    ph.y += double(e0.y);
                    m.x += double(e1.x);
                    m.y += double(e1.y);
                    pp.x += double(e2.x);
                    pp.y += double(e2.y);
                }
            };
            auto u_one = [&](int q, double& ph, double& m, double& pp) {
                ph = gload(L.phi, q);
                m = gload(L.mu, q);
                pp = gload(L.p, q);
                if (add) {
                    ph += double(gload(E.phi, q));
                    m += double(gload(E.mu, q));
                    pp += double(gload(E.p, q));
                }
            };
            D2 phc, muc, pc;
            u_pair(idx, phc, muc, pc);
            const D2 psc = gload(reinterpret_cast<const D2*>(L.pstar), idx >> 1);
            // outer x neighbours (the cell itself across a boundary face)
            const bool hl = i > 0, hr = i + 2 < L.nx;
            const int ql = hl ? idx - 1 : idx, qr = hr ? idx + 2 : idx + 1;
            double phl, mul, pl, phr, mur, pr;
            u_one(ql, phl, mul, pl);
            u_one(qr, phr, mur, pr);
            const double psl = gload(L.pstar, ql), psr = gload(L.pstar, qr);
            // y (and z) neighbour pairs: -y, +y (, -z, +z)
            constexpr int NP = 2 * (DIM - 1);
            D2 phn[NP], mun[NP], pn[NP], psn[NP];
            bool hn[NP];
            {
                const int sz = L.nx * L.ny;
                const int off[4] = {-L.nx, L.nx, -sz, sz};
                const bool has[4] = {j > 0, j < L.ny - 1, k > 0, k < L.nz - 1};
#pragma unroll
                for (int f = 0; f < NP; ++f) {
                    hn[f] = has[f];
                    const int q = has[f] ? idx + off[f] : idx;
                    u_pair(q, phn[f], mun[f], pn[f]);
                    psn[f] = gload(reinterpret_cast<const D2*>(L.pstar), q >> 1);
                }
            }
            struct Sums {
                double smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
            };
            auto face = [&](Sums& s, bool h, double ph0, double mu0, double p0, double ps0,
                            double ph1, double mu1, double p1, double ps1) {
                const double a = 0.5 * (ps0 + ps1);
                const double m = 1.0 + L.gamma * a * a;
                const double dmu = mu1 - mu0;
                const double dp = p1 - p0;
                const double dphi = ph1 - ph0;
                s.smm = h ? s.smm + m * dmu : s.smm;
                s.sap = h ? s.sap + a * dp : s.sap;
                s.sphi = h ? s.sphi + dphi : s.sphi;
                s.sp = h ? s.sp + dp : s.sp;
                s.samu = h ? s.samu + a * dmu : s.samu;
            };
            Sums sa, sb;
            face(sa, hl, phc.x, muc.x, pc.x, psc.x, phl, mul, pl, psl);
            face(sa, true, phc.x, muc.x, pc.x, psc.x, phc.y, muc.y, pc.y, psc.y);
            face(sb, true, phc.y, muc.y, pc.y, psc.y, phc.x, muc.x, pc.x, psc.x);
            face(sb, hr, phc.y, muc.y, pc.y, psc.y, phr, mur, pr, psr);
#pragma unroll
            for (int f = 0; f < NP; ++f) {
                face(sa, hn[f], phc.x, muc.x, pc.x, psc.x, phn[f].x, mun[f].x, pn[f].x, psn[f].x);
                face(sb, hn[f], phc.y, muc.y, pc.y, psc.y, phn[f].y, mun[f].y, pn[f].y, psn[f].y);
            }
            const D2 psi = gload(reinterpret_cast<const D2*>(L.psi), idx >> 1);
            const D2 f1 = gload(reinterpret_cast<const D2*>(L.f1), idx >> 1);
            auto resid = [&](const Sums& s, double ph, double mu, double pp, double ps, double f,
                             double& r0, double& r1, double& r2) {
                r0 = ps - (ph - L.lam * s.smm - L.lam * s.sap);
                r1 = f - (mu - nonlin<double, false>(ph, ps, 0.0) + L.kap * s.sphi);
                r2 = -(L.lam * s.sp + L.lam * L.gamma * s.samu);
            };
            double ra0, ra1, ra2, rb0, rb1, rb2;
            resid(sa, phc.x, muc.x, pc.x, psi.x, f1.x, ra0, ra1, ra2);
            resid(sb, phc.y, muc.y, pc.y, psi.y, f1.y, rb0, rb1, rb2);
            const int h = idx >> 1;
            gstore(reinterpret_cast<D2*>(L.phi_alt), h, phc);
            gstore(reinterpret_cast<D2*>(L.mu_alt), h, muc);
            gstore(reinterpret_cast<D2*>(L.p_alt), h, pc);
            gstore(reinterpret_cast<F2*>(E.f0), h, F2{float(ra0), float(rb0)});
            gstore(reinterpret_cast<F2*>(E.f1), h, F2{float(ra1), float(rb1)});
            gstore(reinterpret_cast<F2*>(E.f2), h, F2{float(ra2), float(rb2)});
            gstore(reinterpret_cast<F2*>(E.b), h, F2{float(phc.x), float(phc.y)});
            v[0] = ra0 * ra0 + rb0 * rb0;
            v[1] = ra1 * ra1 + rb1 * rb1;
            v[2] = ra2 * ra2 + rb2 * rb2;
            v[3] = pc.x + pc.y;
        }
    } else if (add && idx < L.n && (was_active == nullptr || was_active[tk.inst] != 0)) {
        // an instance that has just converged keeps its iterate in both copies,
        // so that it is still the current one after the step flips the copies
        const int h = idx >> 1;
        gstore(reinterpret_cast<D2*>(L.phi_alt), h, gload(reinterpret_cast<const D2*>(L.phi), h));
        gstore(reinterpret_cast<D2*>(L.mu_alt), h, gload(reinterpret_cast<const D2*>(L.mu), h));
        gstore(reinterpret_cast<D2*>(L.p_alt), h, gload(reinterpret_cast<const D2*>(L.p), h));
    }
    double out[4];
    block_sum<4, kPairThreads>(v, out);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) partial[task * kPartialStride + c] = out[c];
}

// ---- deterministic reductions --------------------------------------------------------

template <int NC, int NT>
__device__ __forceinline__ void block_sum(double (&v)[NC], double* out) {
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < NC; ++c) v[c] += __shfl_xor(v[c], off, 64);
    __shared__ double sh[NC][NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < NC; ++c) sh[c][wid] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
            for (int w = 0; w < NT / 64; ++w) s += sh[c][w];
            out[c] = s;
        }
    __syncthreads();
}

template <int NT = kBlock>
__device__ __forceinline__ double block_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    __shared__ double shm[NT / 64];
    if ((threadIdx.x & 63) == 0) shm[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = 0.0;
    for (int w = 0; w < NT / 64; ++w) m = fmax(m, shm[w]);
    __syncthreads();
    return m;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_residual_partials(Batch<double> b,
                                                              const CellTask* __restrict__ t,
                                                              double* partial) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (!inactive(b.active, tk.inst)) {
        const Level<double> L = view_at(b, tk.inst, 0, b.cur);
        const int idx = tk.cell0 + threadIdx.x;
        if (idx < L.n) {
            int i, j, k;
            decode<DIM>(idx, L.nx, L.ny, i, j, k);
            double n0, n1, n2;
            cell_operator<DIM>(L, idx, i, j, k, n0, n1, n2);
            // the finest level: f_phi = phi^m, f_p = 0 ((2.5), (2.7))
            const double r0 = L.psi[idx] - n0, r1 = L.f1[idx] - n1, r2 = -n2;
            v[0] = r0 * r0;
            v[1] = r1 * r1;
            v[2] = r2 * r2;
            v[3] = L.p[idx];
        }
    }
    double out[4];
    block_sum<4>(v, out);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) partial[task * kPartialStride + c] = out[c];
}

// Sums runs of consecutive norm partials of one instance into one partial, so
// that the per-instance reduction (one workgroup per instance) reads a few
// partials instead of thousands of scattered ones.
__global__ __launch_bounds__(kBlock) void k_fold_partials(const double* __restrict__ src,
                                                          const FoldTask* __restrict__ t,
                                                          const int* active, double* dst) {
    const FoldTask ft = t[blockIdx.x];
    if (inactive(active, ft.inst)) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int q = ft.begin + threadIdx.x; q < ft.end; q += kBlock)
        for (int c = 0; c < 4; ++c) v[c] += src[q * kPartialStride + c];
    double s[4];
    block_sum<4>(v, s);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) dst[blockIdx.x * kPartialStride + c] = s[c];
}

// The same for the energy partials: eight sums and a maximum per partial.
__global__ __launch_bounds__(kBlock) void k_fold_energy(const double* __restrict__ src,
                                                        const FoldTask* __restrict__ t, double* dst) {
    const FoldTask ft = t[blockIdx.x];
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double vmax = 0.0;
#pragma unroll 4
    for (int q = ft.begin + threadIdx.x; q < ft.end; q += kBlock) {
        for (int c = 0; c < 8; ++c) v[c] += src[q * kPartialStride + c];
        vmax = fmax(vmax, src[q * kPartialStride + 8]);
    }
    double s[8];
    block_sum<8>(v, s);
    const double m = block_max(vmax);
    if (threadIdx.x == 0) {
        for (int c = 0; c < 8; ++c) dst[blockIdx.x * kPartialStride + c] = s[c];
        dst[blockIdx.x * kPartialStride + 8] = m;
    }
}

__global__ __launch_bounds__(kBlock) void k_inst_reduce(const double* __restrict__ partial,
                                                        const Range* __restrict__ ranges,
                                                        const double* __restrict__ partial_t,
                                                        const Range* __restrict__ ranges_t,
                                                        int use_fused,
                                                        const InstInfo* __restrict__ info,
                                                        const int* active, int* act_next,
                                                        int* cycles, double* res, double tol,
                                                        int max_cycles, int count) {
    const int i = blockIdx.x;
    if (inactive(active, i)) return;
    const InstInfo in = info[i];
    const bool fused = use_fused && in.fused;
    const Range rg = fused ? ranges_t[i] : ranges[i];
    const double* src = fused ? partial_t : partial;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    // unrolled so that the loads of several partials are in flight together
    // (the sums keep their order)
#pragma unroll 8
    for (int q = rg.begin + threadIdx.x; q < rg.end; q += kBlock)
        for (int c = 0; c < 4; ++c) v[c] += src[q * kPartialStride + c];
    double s[4];
    block_sum<4>(v, s);
    if (threadIdx.x != 0) return;
    double hd = in.h * in.h;
    if (in.dim == 3) hd *= in.h;
    const double a = s[0] * hd, bb = s[1] * hd, c = s[2] * hd;
    const double tot = sqrt(a + bb + c);
    double* r = res + i * kResStride;
    r[0] = sqrt(a);
    r[1] = sqrt(bb);
    r[2] = sqrt(c);
    r[3] = tot;
    r[4] = s[3] / double(in.n0);
    const bool finite = tot == tot && tot < 1e300;
    r[5] = finite ? 0.0 : 1.0;
    int cyc = cycles[i];
    if (count) cycles[i] = ++cyc;
    act_next[i] = (finite && tot > tol && cyc < max_cycles) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_shift_p(Batch<double> b, const CellTask* __restrict__ t,
                                                    const double* __restrict__ res) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    if (inactive(b.active, tk.inst)) return;
    const Level<double> L = view_at(b, tk.inst, 0, b.cur);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= L.n) return;
    L.p[idx] -= res[tk.inst * kResStride + 4];
}

// Half a task's width of threads, each taking two cells of the task: a pair of
// x-adjacent cells (2-element loads and stores, the pair's inner face from
// registers) where the instance's x extent is even and its arrays are 16-byte
// aligned, otherwise cells q and q + kEnergyThreads.
constexpr int kEnergyThreads = kBlock / 2;

template <int DIM>
__global__ __launch_bounds__(kEnergyThreads) void k_energy_partials(Batch<double> b,
                                                            const CellTask* __restrict__ t,
                                                            const InstInfo* __restrict__ info,
                                                            int ws, const double* __restrict__ phi_c,
                                                            const double* __restrict__ q_c,
                                                            double* partial, CopyOut co) {
    typedef double D2 __attribute__((ext_vector_type(2)));
    const int task = xcd_task();
    const CellTask tk = t[task];
    const Level<double> L = view_at(b, tk.inst, 0, b.cur);
    const int off = info[tk.inst].off;
    const double gamma = L.gamma;
    const double* phi = ws ? L.phi : phi_c + off;
    const double* q = ws ? L.psi : q_c + off;
    const bool copy = ws && co.phi_cur != nullptr;
    // the copy-out of the step (phi^m is the workspace's psi); the instance's
    // own base pointers keep the 32-bit offsets in range
    double* const cp_prev = copy ? co.phi_prev + off : nullptr;
    double* const cp_cur = copy ? co.phi_cur + off : nullptr;
    double* const cp_mu = copy ? co.mu + off : nullptr;
    double* const cp_p = copy ? co.p + off : nullptr;
    const double psh = copy && b.pshift != nullptr ? b.pshift[tk.inst * kResStride + 4] : 0.0;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double vmax = 0.0;
    // a cell's own terms (phi, phi^m): mass, the two potentials, |phi - phi^m|^2
    auto own = [&](double f, double qc) {
        const double d = f - qc;
        v[0] += f;
        v[1] += f * f;
        v[2] += f * f * f * f;
        v[4] += d * d;
        vmax = fmax(vmax, fabs(f));
    };
    // a forward face (every interior face counted once): the cell (f, phi^m
    // difference d, mu, p, phi_*) and its neighbour (fn, qn, mun, pn, psn)
    auto face = [&](double f, double d, double muc, double pc, double psc, double fn,
                    double qn, double mun, double pn, double psn) {
        const double df = fn - f;
        const double dd = (fn - qn) - d;
        v[3] += df * df;
        v[5] += dd * dd;
        if (ws) {
            const double dm = mun - muc;
            const double a = 0.5 * (psc + psn);
            const double u = -(pn - pc) - gamma * a * dm;
            v[6] += dm * dm;
            v[7] += u * u;
        }
    };
    const uintptr_t bits = uintptr_t(phi) | uintptr_t(q) |
                           (ws ? uintptr_t(L.mu) | uintptr_t(L.p) | uintptr_t(L.pstar) : 0) |
                           (copy ? uintptr_t(cp_prev) | uintptr_t(cp_cur) | uintptr_t(cp_mu) |
                                       uintptr_t(cp_p)
                                 : 0);
    // (global-address-space loads: the block reductions below wait on LDS
    // without also waiting for outstanding global accesses)
    if ((L.nx & 1) == 0 && (bits & 15) == 0) {
        const int idx = tk.cell0 + 2 * int(threadIdx.x);   // first cell of the pair
        if (idx < L.n) {
            int i, j, k;
            decode<DIM>(idx, L.nx, L.ny, i, j, k);
            auto ld2 = [&](const double* a, int c) {
                return gload(reinterpret_cast<const D2*>(a), c >> 1);
            };
            const D2 z2 = {0.0, 0.0};
            const D2 f = ld2(phi, idx), qc = ld2(q, idx);
            const D2 muc = ws ? ld2(L.mu, idx) : z2, pc = ws ? ld2(L.p, idx) : z2;
            const D2 psc = ws ? ld2(L.pstar, idx) : z2;
            const D2 d = f - qc;
            own(f.x, qc.x);
            own(f.y, qc.y);
            face(f.x, d.x, muc.x, pc.x, psc.x, f.y, qc.y, muc.y, pc.y, psc.y);
            if (i + 2 < L.nx) {
                const int r = idx + 2;
                face(f.y, d.y, muc.y, pc.y, psc.y, gload(phi, r), gload(q, r),
                     ws ? gload(L.mu, r) : 0.0, ws ? gload(L.p, r) : 0.0,
                     ws ? gload(L.pstar, r) : 0.0);
            }
            auto face2 = [&](int nb) {
                const D2 fn = ld2(phi, nb), qn = ld2(q, nb);
                const D2 mun = ws ? ld2(L.mu, nb) : z2, pn = ws ? ld2(L.p, nb) : z2;
                const D2 psn = ws ? ld2(L.pstar, nb) : z2;
                face(f.x, d.x, muc.x, pc.x, psc.x, fn.x, qn.x, mun.x, pn.x, psn.x);
                face(f.y, d.y, muc.y, pc.y, psc.y, fn.y, qn.y, mun.y, pn.y, psn.y);
            };
            if (j < L.ny - 1) face2(idx + L.nx);
            if (DIM == 3 && k < L.nz - 1) face2(idx + L.nx * L.ny);
            if (copy) {
                const int h = idx >> 1;
                gstore(reinterpret_cast<D2*>(cp_prev), h, qc);
                gstore(reinterpret_cast<D2*>(cp_cur), h, f);
                gstore(reinterpret_cast<D2*>(cp_mu), h, muc);
                gstore(reinterpret_cast<D2*>(cp_p), h, D2{pc.x - psh, pc.y - psh});
            }
        }
    } else {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int idx = tk.cell0 + int(threadIdx.x) + half * kEnergyThreads;
            if (idx >= L.n) continue;
            int i, j, k;
            decode<DIM>(idx, L.nx, L.ny, i, j, k);
            const double f = gload(phi, idx);
            const double qc = gload(q, idx);
            const double d = f - qc;
            own(f, qc);
            const double muc = ws ? gload(L.mu, idx) : 0.0;
            const double pc = ws ? gload(L.p, idx) : 0.0;
            const double psc = ws ? gload(L.pstar, idx) : 0.0;
            auto face1 = [&](int nb) {
                face(f, d, muc, pc, psc, gload(phi, nb), gload(q, nb),
                     ws ? gload(L.mu, nb) : 0.0, ws ? gload(L.p, nb) : 0.0,
                     ws ? gload(L.pstar, nb) : 0.0);
            };
            if (i < L.nx - 1) face1(idx + 1);
            if (j < L.ny - 1) face1(idx + L.nx);
            if (DIM == 3 && k < L.nz - 1) face1(idx + L.nx * L.ny);
            if (copy) {
                gstore(cp_prev, idx, qc);
                gstore(cp_cur, idx, f);
                gstore(cp_mu, idx, muc);
                gstore(cp_p, idx, pc - psh);
            }
        }
    }
    double out[8];
    block_sum<8, kEnergyThreads>(v, out);
    const double m = block_max<kEnergyThreads>(vmax);
    if (threadIdx.x == 0) {
        double* pp = partial + task * kPartialStride;
        for (int c = 0; c < 8; ++c) pp[c] = out[c];
        pp[8] = m;
    }
}

__global__ __launch_bounds__(kBlock) void k_energy_reduce(const double* __restrict__ partial,
                                                          const Range* __restrict__ ranges,
                                                          const InstInfo* __restrict__ info,
                                                          double* out) {
    const int i = blockIdx.x;
    const Range rg = ranges[i];
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double vmax = 0.0;
    for (int q = rg.begin + threadIdx.x; q < rg.end; q += kBlock) {
        for (int c = 0; c < 8; ++c) v[c] += partial[q * kPartialStride + c];
        vmax = fmax(vmax, partial[q * kPartialStride + 8]);
    }
    double s[8];
    block_sum<8>(v, s);
    const double m = block_max(vmax);
    if (threadIdx.x != 0) return;
    const InstInfo in = info[i];
    double hd = in.h * in.h;
    if (in.dim == 3) hd *= in.h;
    const double e2 = in.eps * in.eps, ih2 = 1.0 / (in.h * in.h);
    const double E = hd * (0.25 * s[2] - 0.5 * s[1] + 0.5 * e2 * s[3] * ih2);
    double* o = out + i * kResStride;
    o[0] = hd * s[0];
    o[1] = E;
    o[2] = E + hd * (0.25 * s[4] + 0.125 * e2 * s[5] * ih2);
    o[3] = in.dt * hd * s[6] * ih2;
    o[4] = in.gamma > 0.0 ? in.dt / in.gamma * hd * s[7] * ih2 : 0.0;
    o[5] = m;
}

__global__ __launch_bounds__(kBlock) void k_copy_out(Batch<double> b, const CellTask* __restrict__ t,
                                                     const InstInfo* __restrict__ info,
                                                     double* phi_prev, double* phi_cur, double* mu,
                                                     double* p) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    const Level<double> L = view_at(b, tk.inst, 0, b.cur);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= L.n) return;
    const int g = info[tk.inst].off + idx;
    const double psh = b.pshift != nullptr ? b.pshift[tk.inst * kResStride + 4] : 0.0;
    phi_prev[g] = phi_cur[g];
    phi_cur[g] = L.phi[idx];
    mu[g] = L.mu[idx];
    p[g] = L.p[idx] - psh;
}

__global__ void k_clear_pshift(double* res, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) res[i * kResStride + 4] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_get_solution(Batch<double> b,
                                                         const CellTask* __restrict__ t,
                                                         const InstInfo* __restrict__ info,
                                                         double* phi, double* mu, double* p) {
    const int task = xcd_task();
    const CellTask tk = t[task];
    const Level<double> L = view_at(b, tk.inst, 0, b.cur);
    const int idx = tk.cell0 + threadIdx.x;
    if (idx >= L.n) return;
    const int g = info[tk.inst].off + idx;
    if (phi) phi[g] = L.phi[idx];
    if (mu) mu[g] = L.mu[idx];
    if (p) p[g] = L.p[idx] - (b.pshift != nullptr ? b.pshift[tk.inst * kResStride + 4] : 0.0);
}

__global__ __launch_bounds__(kBlock) void k_fill_int(int* dst, int n, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_copy_int(int* dst, const int* src, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void k_roll_flags(int* last, int* cur, const int* next, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        last[i] = cur[i];
        cur[i] = next[i];
    }
}

inline int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

#define CHHS_DISPATCH(dim, KERNEL, GRID, ...)                                             \
    do {                                                                                  \
        if ((GRID) <= 0) break;                                                           \
        if ((dim) == 2)                                                                   \
            hipLaunchKernelGGL(KERNEL<2>, dim3(GRID), dim3(kBlock), 0, st, __VA_ARGS__);  \
        else                                                                              \
            hipLaunchKernelGGL(KERNEL<3>, dim3(GRID), dim3(kBlock), 0, st, __VA_ARGS__);  \
    } while (0)

void launch_setup(int dim, const Batch<double>& b, const CellTask* t, int nt, const InstInfo* info,
                  const double* phi_prev, const double* phi_cur, const double* mu,
                  const double* p, double* partial, const Batch<float>* frozen32,
                  hipStream_t st) {
    Batch<float> e32{};
    if (frozen32 != nullptr) e32 = *frozen32;
    if (nt <= 0) return;
    if (dim == 2)
        hipLaunchKernelGGL(k_setup<2>, dim3(nt), dim3(kPairThreads), 0, st, b, t, info, phi_prev,
                           phi_cur, mu, p, partial, e32);
    else
        hipLaunchKernelGGL(k_setup<3>, dim3(nt), dim3(kPairThreads), 0, st, b, t, info, phi_prev,
                           phi_cur, mu, p, partial, e32);
}

#define CHHS_DISPATCH_T(dim, KERNEL, GRID, ...)                                           \
    do {                                                                                  \
        if ((GRID) <= 0) break;                                                           \
        if ((dim) == 2)                                                                   \
            hipLaunchKernelGGL((KERNEL<2, CHHS_TARGS>), dim3(GRID), dim3(kBlock), 0, st,     \
                               __VA_ARGS__);                                              \
        else                                                                              \
            hipLaunchKernelGGL((KERNEL<3, CHHS_TARGS>), dim3(GRID), dim3(kBlock), 0, st,     \
                               __VA_ARGS__);                                              \
    } while (0)

#define CHHS_TARGS double
template <typename T>
void chain_launch(int dim, const LevelDesc<T>* desc, const InstInfo* info, int n_inst, int from,
                  hipStream_t st) {
    if (n_inst <= 0) return;
    if (dim == 2)
        hipLaunchKernelGGL((k_restrict_frozen_chain<2, T>), dim3(n_inst), dim3(kChainThreads), 0,
                           st, desc, info, from);
    else
        hipLaunchKernelGGL((k_restrict_frozen_chain<3, T>), dim3(n_inst), dim3(kChainThreads), 0,
                           st, desc, info, from);
}
void launch_restrict_frozen_chain(int dim, const LevelDesc<double>* desc, const InstInfo* info,
                                  int n_inst, int from, hipStream_t st) {
    chain_launch(dim, desc, info, n_inst, from, st);
}
void launch_restrict_frozen_chain(int dim, const LevelDesc<float>* desc, const InstInfo* info,
                                  int n_inst, int from, hipStream_t st) {
    chain_launch(dim, desc, info, n_inst, from, st);
}

void launch_restrict_frozen(int dim, const Batch<double>& b, const CellTask* t, int nt,
                            hipStream_t st) {
    CHHS_DISPATCH_T(dim, k_restrict_frozen, nt, b, t);
}
#undef CHHS_TARGS
#define CHHS_TARGS float
void launch_restrict_frozen(int dim, const Batch<float>& b, const CellTask* t, int nt,
                            hipStream_t st) {
    CHHS_DISPATCH_T(dim, k_restrict_frozen, nt, b, t);
}
#undef CHHS_TARGS
#define CHHS_TARGS double, false
void launch_prolong(int dim, const Batch<double>& b, const CellTask* t, int nt, bool bilinear,
                    hipStream_t st) {
    if (bilinear) {
#undef CHHS_TARGS
#define CHHS_TARGS double, true
        CHHS_DISPATCH_T(dim, k_prolong, nt, b, t);
        return;
    }
#undef CHHS_TARGS
#define CHHS_TARGS double, false
    CHHS_DISPATCH_T(dim, k_prolong, nt, b, t);
}
#undef CHHS_TARGS
#define CHHS_TARGS float, false
void launch_prolong(int dim, const Batch<float>& b, const CellTask* t, int nt, bool bilinear,
                    hipStream_t st) {
    if (bilinear) {
#undef CHHS_TARGS
#define CHHS_TARGS float, true
        CHHS_DISPATCH_T(dim, k_prolong, nt, b, t);
        return;
    }
#undef CHHS_TARGS
#define CHHS_TARGS float, false
    CHHS_DISPATCH_T(dim, k_prolong, nt, b, t);
}
#undef CHHS_TARGS
#define CHHS_TARGS double, false
// (the finest level takes the form that does not load f_phi, f_p)
#define CHHS_SMOOTH_LAUNCH(KERNEL)                                                             \
    do {                                                                                       \
        if (nt <= 0) break;                                                                    \
        const bool l0 = b.level == 0;                                                          \
        if (dim == 2 && l0)                                                                    \
            hipLaunchKernelGGL((KERNEL<2, double, false, true>), dim3(nt), dim3(kBlock), 0, st, \
                               b, t, color);                                                   \
        else if (dim == 2)                                                                     \
            hipLaunchKernelGGL((KERNEL<2, double, false, false>), dim3(nt), dim3(kBlock), 0, st, \
                               b, t, color);                                                   \
        else if (l0)                                                                           \
            hipLaunchKernelGGL((KERNEL<3, double, false, true>), dim3(nt), dim3(kBlock), 0, st, \
                               b, t, color);                                                   \
        else                                                                                   \
            hipLaunchKernelGGL((KERNEL<3, double, false, false>), dim3(nt), dim3(kBlock), 0, st, \
                               b, t, color);                                                   \
    } while (0)
void launch_smooth(int dim, const Batch<double>& b, const CellTask* t, int nt, int color,
                   hipStream_t st) {
    CHHS_SMOOTH_LAUNCH(k_smooth);
}
void launch_smooth_color(int dim, const Batch<double>& b, const CellTask* t, int nt, int color,
                         hipStream_t st) {
    CHHS_SMOOTH_LAUNCH(k_smooth_color);
}
#undef CHHS_SMOOTH_LAUNCH
void launch_restrict_residual(int dim, const Batch<double>& b, const CellTask* t, int nt,
                              hipStream_t st) {
    if (nt <= kLaneRestrictTasks)
        CHHS_DISPATCH_T(dim, k_restrict_residual_lanes, nt * (dim == 3 ? 8 : 4), b, t);
    else
        CHHS_DISPATCH_T(dim, k_restrict_residual, nt, b, t);
}
void launch_coarse_rhs(int dim, const Batch<double>& b, const CellTask* t, int nt, hipStream_t st) {
    CHHS_DISPATCH_T(dim, k_coarse_rhs, nt, b, t);
}
#undef CHHS_TARGS
#define CHHS_TARGS float, true
void launch_smooth(int dim, const Batch<float>& b, const CellTask* t, int nt, int color,
                   hipStream_t st) {
    CHHS_DISPATCH_T(dim, k_smooth, nt, b, t, color);
}
void launch_smooth_color(int dim, const Batch<float>& b, const CellTask* t, int nt, int color,
                         hipStream_t st) {
    CHHS_DISPATCH_T(dim, k_smooth_color, nt, b, t, color);
}
void launch_restrict_residual(int dim, const Batch<float>& b, const CellTask* t, int nt,
                              hipStream_t st) {
    if (nt <= kLaneRestrictTasks)
        CHHS_DISPATCH_T(dim, k_restrict_residual_lanes, nt * (dim == 3 ? 8 : 4), b, t);
    else
        CHHS_DISPATCH_T(dim, k_restrict_residual, nt, b, t);
}
void launch_coarse_rhs(int dim, const Batch<float>& b, const CellTask* t, int nt, hipStream_t st) {
    CHHS_DISPATCH_T(dim, k_coarse_rhs, nt, b, t);
}
#undef CHHS_TARGS


void launch_zero_correction(const Batch<float>& b32, const CellTask* t, int nt, hipStream_t st) {
    if (nt > 0) hipLaunchKernelGGL(k_zero_correction, dim3(nt), dim3(kBlock), 0, st, b32, t);
}

void launch_mixed_residual(int dim, const Batch<double>& b64, const Batch<float>& b32,
                           const CellTask* t, int nt, int add, const int* was_active,
                           double* partial, hipStream_t st) {
    if (nt <= 0) return;
    if (dim == 2)
        hipLaunchKernelGGL(k_mixed_residual<2>, dim3(nt), dim3(kPairThreads), 0, st, b64, b32, t,
                           add, was_active, partial);
    else
        hipLaunchKernelGGL(k_mixed_residual<3>, dim3(nt), dim3(kPairThreads), 0, st, b64, b32, t,
                           add, was_active, partial);
}

void launch_residual_partials(int dim, const Batch<double>& b, const CellTask* t, int nt,
                              double* partial, hipStream_t st) {
    CHHS_DISPATCH(dim, k_residual_partials, nt, b, t, partial);
}

void launch_fold_partials(const double* src, const FoldTask* t, int nt, const int* active,
                          double* dst, hipStream_t st) {
    if (nt <= 0) return;
    hipLaunchKernelGGL(k_fold_partials, dim3(nt), dim3(kBlock), 0, st, src, t, active, dst);
}

void launch_fold_energy(const double* src, const FoldTask* t, int nt, double* dst, hipStream_t st) {
    if (nt > 0) hipLaunchKernelGGL(k_fold_energy, dim3(nt), dim3(kBlock), 0, st, src, t, dst);
}

void launch_inst_reduce(const double* partial, const Range* ranges, const double* partial_t,
                        const Range* ranges_t, int use_fused, const InstInfo* info,
                        const int* active, int* act_next, int* cycles, double* res, int n_inst,
                        double tol, int max_cycles, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_inst_reduce, dim3(n_inst), dim3(kBlock), 0, st, partial, ranges,
                       partial_t, ranges_t, use_fused, info, active, act_next, cycles, res, tol,
                       max_cycles, count);
}

void launch_clear_pshift(double* res, int n_inst, hipStream_t st) {
    hipLaunchKernelGGL(k_clear_pshift, dim3(blocks_for(n_inst)), dim3(kBlock), 0, st, res, n_inst);
}

void launch_shift_p(const Batch<double>& b, const CellTask* t, int nt, const double* res,
                    hipStream_t st) {
    if (nt > 0) hipLaunchKernelGGL(k_shift_p, dim3(nt), dim3(kBlock), 0, st, b, t, res);
}

void launch_energy_partials(int dim, const Batch<double>& b, const CellTask* t, int nt,
                            const InstInfo* info, int ws, const double* phi, const double* q,
                            double* partial, hipStream_t st, const CopyOut* copy) {
    const CopyOut co = copy != nullptr ? *copy : CopyOut{nullptr, nullptr, nullptr, nullptr};
    if (nt <= 0) return;
    if (dim == 2)
        hipLaunchKernelGGL(k_energy_partials<2>, dim3(nt), dim3(kEnergyThreads), 0, st, b, t, info,
                           ws, phi, q, partial, co);
    else
        hipLaunchKernelGGL(k_energy_partials<3>, dim3(nt), dim3(kEnergyThreads), 0, st, b, t, info,
                           ws, phi, q, partial, co);
}

void launch_energy_reduce(const double* partial, const Range* ranges, const InstInfo* info,
                          double* out, int n_inst, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_reduce, dim3(n_inst), dim3(kBlock), 0, st, partial, ranges, info,
                       out);
}

void launch_copy_out(const Batch<double>& b, const CellTask* t, int nt, const InstInfo* info,
                     double* phi_prev, double* phi_cur, double* mu, double* p, hipStream_t st) {
    if (nt > 0)
        hipLaunchKernelGGL(k_copy_out, dim3(nt), dim3(kBlock), 0, st, b, t, info, phi_prev,
                           phi_cur, mu, p);
}

void launch_get_solution(const Batch<double>& b, const CellTask* t, int nt, const InstInfo* info,
                         double* phi, double* mu, double* p, hipStream_t st) {
    if (nt > 0)
        hipLaunchKernelGGL(k_get_solution, dim3(nt), dim3(kBlock), 0, st, b, t, info, phi, mu, p);
}

void launch_fill_int(int* dst, int n, int value, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n)), dim3(kBlock), 0, st, dst, n, value);
}

void launch_copy_int(int* dst, const int* src, int n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(n)), dim3(kBlock), 0, st, dst, src, n);
}

void launch_roll_flags(int* last, int* cur, const int* next, int n, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_roll_flags, dim3(blocks_for(n)), dim3(kBlock), 0, st, last, cur, next, n);
}

}  // namespace chhs
