// The residual f - N(u) of a 3D level (the three rows of (2.5)-(2.7), as
// cell_operator evaluates it) by marching up z, for the two uses that read a
// whole level once per V-cycle:
//   MODE 0: the norm partials of the finest FP64 level (sum of R^2 per row and
//           of p per workgroup), as the per-cell residual kernel forms them;
//   MODE 1: residual and restriction into the next coarser level: u_c = ub_c =
//           R u, fr_c = R(f - N(u)) (and, in the correction form, b_c = R b),
//           R the average of the 8 children summed in the tree order of the
//           per-cell restriction ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 +
//           c7)), child c = dx + 2 dy + 4 dz.
//
// and, with the same layout of the work, the FP64 refinement step of the mixed
// path on the finest 3D level (k_refine3d, below).
//
// A workgroup of 256 threads owns a TX x TY tile of (x, y) columns (one cell
// per thread and plane) and a segment [z0, z1) of planes of one instance (a
// Step3Task of the level's fused-step table, so z0 is even).  It stages the
// tile with a halo of one cell, plane by plane, in an LDS ring of 4 planes of
// the fields neighbours read (phi, mu, p, phi_*); in iteration t it forms the
// residual of its cells of plane t from planes t - 1 .. t + 1.  Plane t + 3
// and the own data of plane t + 2 (f, phi^m, b) are loaded into one of two
// register sets at the end of iteration t, so a load's latency overlaps a
// whole iteration (region cells outside the grid load cell 0 of the level:
// finite values that no face reads; no operation follows a load before its
// value is stored to LDS).  In MODE 1 the 2 x 2 in-plane sums are lane exchanges (the
// x neighbour is lane ^ 1, the y neighbour lane ^ TX) and the z pair is summed
// in registers over two iterations.
#include "chhs_cell.hpp"

namespace chhs {
namespace {

constexpr int kThreads = 256;
constexpr int kRing = 4;          // planes t - 1 .. t + 2 are live in iteration t
constexpr int PHI = 0, MU = 1, P = 2, PS = 3, NRF = 4;

// L0: the finest level of the plain form, whose right-hand side is f_phi =
// phi^m (psi) and f_p = 0 ((2.5), (2.7)): neither is loaded.
template <typename T, bool CORR, int MODE, int TX, int TY, bool L0>
__global__ __launch_bounds__(kThreads) void k_resid3d(Batch<T> bt, const Step3Task* __restrict__ tasks,
                                                      int ntasks, double* __restrict__ partial) {
    static_assert(TX * TY == kThreads, "one cell per thread and plane");
    static_assert(64 % TX == 0, "a wave holds whole rows of the tile");
    constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;
    constexpr int KR = (NR + kThreads - 1) / kThreads;
    __shared__ T s[kRing][NRF][NR];

    const int bid = blockIdx.x;
    const int xcd = bid % 8, jj = bid / 8;
    const int q8 = ntasks / 8, rem = ntasks % 8;
    const int task = xcd * q8 + (xcd < rem ? xcd : rem) + jj;
    const Step3Task tk = tasks[task];
    if (bt.active != nullptr && bt.active[tk.inst] == 0) return;
    const Level<T> L = make_view(bt.desc[tk.inst * kMaxLevels + bt.level], bt.cur);
    const Level<T> C =
        make_view(bt.desc[tk.inst * kMaxLevels + bt.level + (MODE == 1 ? 1 : 0)], bt.cur_c);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int sxy = nx * ny;
    const int x0 = tk.bx * TX - 1, y0 = tk.by * TY - 1;    // region origin
    const int z0 = tk.z0, z1 = tk.z1;
    const int tid = threadIdx.x;
    const int ox = tid % TX, oy = tid / TX;
    const int gx = tk.bx * TX + ox, gy = tk.by * TY + oy;   // the thread's cell column
    const bool own_ok = gx < nx && gy < ny;
    const int w = (oy + 1) * RX + ox + 1;
    const T lam = L.lam, kap = L.kap, gam = L.gamma;

    using Regs = T[KR][NRF];
    auto load_plane = [&](int z, Regs& rv) {
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int q = tid + k * kThreads;
            const int ry = q / RX, rx = q - ry * RX;
            const int x = x0 + rx, y = y0 + ry;
            const bool ok = q < NR && x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
            const int g = ok ? z * sxy + y * nx + x : 0;
            rv[k][PHI] = gload(L.phi, g);
            rv[k][MU] = gload(L.mu, g);
            rv[k][P] = gload(L.p, g);
            rv[k][PS] = gload(L.pstar, g);
        }
    };
    auto store_plane = [&](int z, const Regs& rv) {
        const int sl = z % kRing;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int q = tid + k * kThreads;
            if (q < NR)
#pragma unroll
                for (int f = 0; f < NRF; ++f) s[sl][f][q] = rv[k][f];
        }
    };
    struct Own {
        T f0, f1, f2, psi, b;
    };
    auto load_own = [&](int z, Own& o) {
        const bool ok = own_ok && z >= 0 && z < nz;
        const int g = ok ? z * sxy + gy * nx + gx : 0;
        o.psi = gload(L.psi, g);
        o.f0 = L0 ? o.psi : gload(L.f0, g);
        o.f1 = gload(L.f1, g);
        o.f2 = L0 ? T(0) : gload(L.f2, g);
        o.b = CORR ? gload(L.b, g) : T(0);
    };

    // residual of the thread's cell in plane z (faces in the order x - 1,
    // x + 1, y - 1, y + 1, z - 1, z + 1, as cell_operator)
    auto residual = [&](int z, const Own& o, T& r0, T& r1, T& r2, T& phic, T& muc, T& pc) {
        const int sc = z % kRing, sd = (z + kRing - 1) % kRing, su = (z + 1) % kRing;
        phic = s[sc][PHI][w];
        muc = s[sc][MU][w];
        pc = s[sc][P][w];
        const T psc = s[sc][PS][w];
        T smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
        auto face = [&](bool h, int sl, int wn) {
            const T a = T(0.5) * (psc + s[sl][PS][wn]);
            const T m = T(1) + gam * a * a;
            const T dmu = s[sl][MU][wn] - muc;
            const T dp = s[sl][P][wn] - pc;
            const T dphi = s[sl][PHI][wn] - phic;
            smm = h ? smm + m * dmu : smm;
            sap = h ? sap + a * dp : sap;
            sphi = h ? sphi + dphi : sphi;
            sp = h ? sp + dp : sp;
            samu = h ? samu + a * dmu : samu;
        };
        face(gx > 0, sc, w - 1);
        face(gx < nx - 1, sc, w + 1);
        face(gy > 0, sc, w - RX);
        face(gy < ny - 1, sc, w + RX);
        face(z > 0, sd, w);
        face(z < nz - 1, su, w);
        const T chi = nonlin<T, CORR>(phic, o.psi, o.b);
        const T n0 = phic - lam * smm - lam * sap;
        const T n1 = muc - chi + kap * sphi;
        const T n2 = lam * sp + lam * gam * samu;
        r0 = o.f0 - n0;
        r1 = o.f1 - n1;
        r2 = o.f2 - n2;
    };

    const int plo = z0 - 1 > 0 ? z0 - 1 : 0;          // planes loaded: plo .. zhi
    const int zhi = z1 < nz - 1 ? z1 : nz - 1;
    Regs rvA, rvB;
    Own oA, oB;
    for (int z = plo; z <= z0; ++z) {
        load_plane(z, rvA);
        store_plane(z, rvA);
    }
    if (z0 + 1 <= zhi) load_plane(z0 + 1, rvA);
    if (z0 + 2 <= zhi) load_plane(z0 + 2, rvB);
    load_own(z0, oA);
    load_own(z0 + 1, oB);

    double v[4] = {0.0, 0.0, 0.0, 0.0};     // MODE 0: sums of R^2 per row and of p
    T acc[7];                               // MODE 1: the even plane's 2 x 2 sums
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[c] = T(0);

    // iteration t takes register set t & 1: plane t + 1 (stored first) and the
    // own data of plane t; afterwards the same set receives plane t + 3 and
    // the own data of plane t + 2
    auto iteration = [&](int t, Regs& rv, Own& o) {
        if (t + 1 <= zhi) store_plane(t + 1, rv);
        __syncthreads();
        T r0, r1, r2, phic, muc, pc;
        residual(t, o, r0, r1, r2, phic, muc, pc);
        if (MODE == 0) {
            if (own_ok) {
                v[0] += double(r0) * double(r0);
                v[1] += double(r1) * double(r1);
                v[2] += double(r2) * double(r2);
                v[3] += double(pc);
            }
        } else {
            T c[7] = {r0, r1, r2, phic, muc, pc, o.b};
            if (!own_ok)
#pragma unroll
                for (int k = 0; k < 7; ++k) c[k] = T(0);
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                if (!CORR && k == 6) continue;
                c[k] = c[k] + __shfl_xor(c[k], 1, 64);      // x pair
                c[k] = c[k] + __shfl_xor(c[k], TX, 64);     // (x pair) + (x pair) along y
            }
            if (((t - z0) & 1) == 0) {
#pragma unroll
                for (int k = 0; k < 7; ++k) acc[k] = c[k];
            } else if (own_ok && (ox & 1) == 0 && (oy & 1) == 0) {
                const T wt = T(0.125);
                const int ci = ((t >> 1) * C.ny + (gy >> 1)) * C.nx + (gx >> 1);
                T tot[7];
#pragma unroll
                for (int k = 0; k < 7; ++k) tot[k] = acc[k] + c[k];
                if (CORR) C.b[ci] = tot[6] * wt;
                C.phi[ci] = C.ub0[ci] = tot[3] * wt;
                C.mu[ci] = C.ub1[ci] = tot[4] * wt;
                C.p[ci] = C.ub2[ci] = tot[5] * wt;
                C.fr0[ci] = tot[0] * wt;
                C.fr1[ci] = tot[1] * wt;
                C.fr2[ci] = tot[2] * wt;
            }
        }
        if (t + 3 <= zhi) load_plane(t + 3, rv);
        load_own(t + 2, o);
    };
    for (int t = z0; t < z1; t += 2) {
        iteration(t, rvA, oA);
        if (t + 1 < z1) iteration(t + 1, rvB, oB);
    }

    if (MODE == 0) {
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += __shfl_xor(v[c], off, 64);
        __shared__ double sh[4][kThreads / 64];
        const int lane = tid & 63, wid = tid >> 6;
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < 4; ++c) sh[c][wid] = v[c];
        __syncthreads();
        if (tid == 0)
            for (int c = 0; c < 4; ++c) {
                double sum = 0.0;
                for (int k = 0; k < kThreads / 64; ++k) sum += sh[c][k];
                partial[size_t(task) * kPartialStride + c] = sum;
            }
    }
}

// The FP64 refinement step of the mixed path on the finest 3D level over the
// level's fused-step tasks: u' = u + e (add; e the FP32 correction of the last
// inner cycles), R = f - N(u') of (2.5)-(2.7) (f_phi = phi^m, f_p = 0 on the
// finest level), u' written into the other FP64 copy, R and b = phi' rounded
// to FP32 into the FP32 finest level's right-hand side and base state, and the
// partial sums of R^2 and p' of the task (the arithmetic per cell of the
// per-cell refinement kernel; faces in the order x - 1, x + 1, y - 1, y + 1,
// z - 1, z + 1).  The ring holds u' and phi_*, formed as each plane is loaded.
// An instance inactive in this refinement but active in the previous one
// (was_active) copies its iterate into the other copy.
template <int TX, int TY>
__global__ __launch_bounds__(kThreads) void k_refine3d(Batch<double> b64, Batch<float> b32,
                                                       const Step3Task* __restrict__ tasks, int ntasks,
                                                       int add, const int* __restrict__ was_active,
                                                       double* __restrict__ partial) {
    static_assert(TX * TY == kThreads, "one cell per thread and plane");
    constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;
    constexpr int KR = (NR + kThreads - 1) / kThreads;
    __shared__ double s[kRing][NRF][NR];

    const int bid = blockIdx.x;
    const int xcd = bid % 8, jj = bid / 8;
    const int q8 = ntasks / 8, rem = ntasks % 8;
    const int task = xcd * q8 + (xcd < rem ? xcd : rem) + jj;
    const Step3Task tk = tasks[task];
    const Level<double> L = make_view(b64.desc[tk.inst * kMaxLevels], b64.cur);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int sxy = nx * ny;
    const int z0 = tk.z0, z1 = tk.z1;
    const int tid = threadIdx.x;
    const int ox = tid % TX, oy = tid / TX;
    const int gx = tk.bx * TX + ox, gy = tk.by * TY + oy;
    const bool own_ok = gx < nx && gy < ny;
    if (b64.active != nullptr && b64.active[tk.inst] == 0) {
        // an instance that has just converged keeps its iterate in both copies
        if (add && own_ok && (was_active == nullptr || was_active[tk.inst] != 0))
            for (int z = z0; z < z1; ++z) {
                const int g = z * sxy + gy * nx + gx;
                gstore(L.phi_alt, g, gload(L.phi, g));
                gstore(L.mu_alt, g, gload(L.mu, g));
                gstore(L.p_alt, g, gload(L.p, g));
            }
        return;
    }
    const Level<float> E = make_view(b32.desc[tk.inst * kMaxLevels], b32.cur);
    const int x0 = tk.bx * TX - 1, y0 = tk.by * TY - 1;
    const int w = (oy + 1) * RX + ox + 1;
    const double lam = L.lam, kap = L.kap, gam = L.gamma;

    struct Raw {
        double ph, mu, p, ps;
        float e0, e1, e2;
    };
    using Regs = Raw[KR];
    auto load_plane = [&](int z, Regs& rv) {
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int q = tid + k * kThreads;
            const int ry = q / RX, rx = q - ry * RX;
            const int x = x0 + rx, y = y0 + ry;
            const bool ok = q < NR && x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz;
            const int g = ok ? z * sxy + y * nx + x : 0;
            rv[k].ph = gload(L.phi, g);
            rv[k].mu = gload(L.mu, g);
            rv[k].p = gload(L.p, g);
            rv[k].ps = gload(L.pstar, g);
            if (add) {
                rv[k].e0 = gload(E.phi, g);
                rv[k].e1 = gload(E.mu, g);
                rv[k].e2 = gload(E.p, g);
            }
        }
    };
    auto store_plane = [&](int z, const Regs& rv) {
        const int sl = z % kRing;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int q = tid + k * kThreads;
            if (q >= NR) continue;
            double ph = rv[k].ph, mu = rv[k].mu, p = rv[k].p;
            if (add) {
                ph += double(rv[k].e0);
                mu += double(rv[k].e1);
                p += double(rv[k].e2);
            }
            s[sl][PHI][q] = ph;
            s[sl][MU][q] = mu;
            s[sl][P][q] = p;
            s[sl][PS][q] = rv[k].ps;
        }
    };
    struct Own {
        double psi, f1;
    };
    auto load_own = [&](int z, Own& o) {
        const bool ok = own_ok && z >= 0 && z < nz;
        const int g = ok ? z * sxy + gy * nx + gx : 0;
        o.psi = gload_stream(L.psi, g);
        o.f1 = gload_stream(L.f1, g);
    };

    const int plo = z0 - 1 > 0 ? z0 - 1 : 0;
    const int zhi = z1 < nz - 1 ? z1 : nz - 1;
    Regs rvA, rvB;
    Own oA, oB;
    for (int z = plo; z <= z0; ++z) {
        load_plane(z, rvA);
        store_plane(z, rvA);
    }
    if (z0 + 1 <= zhi) load_plane(z0 + 1, rvA);
    if (z0 + 2 <= zhi) load_plane(z0 + 2, rvB);
    load_own(z0, oA);
    load_own(z0 + 1, oB);
    double v[4] = {0.0, 0.0, 0.0, 0.0};

    auto iteration = [&](int t, Regs& rv, Own& o) {
        if (t + 1 <= zhi) store_plane(t + 1, rv);
        __syncthreads();
        const int sc = t % kRing, sd = (t + kRing - 1) % kRing, su = (t + 1) % kRing;
        const double phc = s[sc][PHI][w], muc = s[sc][MU][w], pc = s[sc][P][w];
        const double psc = s[sc][PS][w];
        double smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
        auto face = [&](bool h, int sl, int wn) {
            const double a = 0.5 * (psc + s[sl][PS][wn]);
            const double m = 1.0 + gam * a * a;
            const double dmu = s[sl][MU][wn] - muc;
            const double dp = s[sl][P][wn] - pc;
            const double dphi = s[sl][PHI][wn] - phc;
            smm = h ? smm + m * dmu : smm;
            sap = h ? sap + a * dp : sap;
            sphi = h ? sphi + dphi : sphi;
            sp = h ? sp + dp : sp;
            samu = h ? samu + a * dmu : samu;
        };
        face(gx > 0, sc, w - 1);
        face(gx < nx - 1, sc, w + 1);
        face(gy > 0, sc, w - RX);
        face(gy < ny - 1, sc, w + RX);
        face(t > 0, sd, w);
        face(t < nz - 1, su, w);
        const double r0 = o.psi - (phc - lam * smm - lam * sap);
        const double r1 = o.f1 - (muc - nonlin<double, false>(phc, o.psi, 0.0) + kap * sphi);
        const double r2 = -(lam * sp + lam * gam * samu);
        if (own_ok) {
            const int g = t * sxy + gy * nx + gx;
            gstore(L.phi_alt, g, phc);
            gstore(L.mu_alt, g, muc);
            gstore(L.p_alt, g, pc);
            gstore(E.f0, g, float(r0));
            gstore(E.f1, g, float(r1));
            gstore(E.f2, g, float(r2));
            gstore(E.b, g, float(phc));
            v[0] += r0 * r0;
            v[1] += r1 * r1;
            v[2] += r2 * r2;
            v[3] += pc;
        }
        if (t + 3 <= zhi) load_plane(t + 3, rv);
        load_own(t + 2, o);
    };
    for (int t = z0; t < z1; t += 2) {
        iteration(t, rvA, oA);
        if (t + 1 < z1) iteration(t + 1, rvB, oB);
    }
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] += __shfl_xor(v[c], off, 64);
    __shared__ double sh[4][kThreads / 64];
    const int lane = tid & 63, wid = tid >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[c][wid] = v[c];
    __syncthreads();
    if (tid == 0)
        for (int c = 0; c < 4; ++c) {
            double sum = 0.0;
            for (int k = 0; k < kThreads / 64; ++k) sum += sh[c][k];
            partial[size_t(task) * kPartialStride + c] = sum;
        }
}

}  // namespace

void launch_refine3d(const Batch<double>& b64, const Batch<float>& b32, const Step3Task* t, int nt,
                     int add, const int* was_active, double* partial, hipStream_t st) {
    if (nt > 0)
        hipLaunchKernelGGL((k_refine3d<kStep3TX64, kStep3TY64>), dim3(nt), dim3(kThreads), 0, st,
                           b64, b32, t, nt, add, was_active, partial);
}

void launch_residual3d_partials(const Batch<double>& b, const Step3Task* t, int nt, double* partial,
                                hipStream_t st) {
    if (nt <= 0) return;
    if (b.level == 0)
        hipLaunchKernelGGL((k_resid3d<double, false, 0, kStep3TX64, kStep3TY64, true>), dim3(nt),
                           dim3(kThreads), 0, st, b, t, nt, partial);
    else
        hipLaunchKernelGGL((k_resid3d<double, false, 0, kStep3TX64, kStep3TY64, false>), dim3(nt),
                           dim3(kThreads), 0, st, b, t, nt, partial);
}

void launch_restrict3d(const Batch<double>& b, const Step3Task* t, int nt, hipStream_t st) {
    if (nt <= 0) return;
    if (b.level == 0)
        hipLaunchKernelGGL((k_resid3d<double, false, 1, kStep3TX64, kStep3TY64, true>), dim3(nt),
                           dim3(kThreads), 0, st, b, t, nt, nullptr);
    else
        hipLaunchKernelGGL((k_resid3d<double, false, 1, kStep3TX64, kStep3TY64, false>), dim3(nt),
                           dim3(kThreads), 0, st, b, t, nt, nullptr);
}

void launch_restrict3d(const Batch<float>& b, const Step3Task* t, int nt, hipStream_t st) {
    if (nt > 0)
        hipLaunchKernelGGL((k_resid3d<float, true, 1, kStep3TX32, kStep3TY32, false>), dim3(nt),
                           dim3(kThreads), 0, st, b, t, nt, nullptr);
}

}  // namespace chhs
