// One fused smoothing step (red then black collective (phi, mu, p) cell
// updates, the update of cell_solve) on a 3D level, batched over instances,
// by marching up z.
//
// A workgroup owns a TX x TY tile of (x, y) columns and a segment [z0, z1) of
// planes of one instance (a Step3Task).  It stages the tile with a halo of two
// cells in x and y, plane by plane, in an LDS ring of kRing planes of the four
// fields that neighbours read (phi, mu, p, phi_*).  At iteration t the red
// phase updates plane t and the black phase plane t - 2: the black cells of
// plane t - 2 need the red cells of planes t - 3 .. t - 1, all updated in
// earlier iterations, and the red cells of plane t need black cells of planes
// t - 1 .. t + 1, none of which the black phase has reached; the two phases of
// an iteration touch disjoint planes, so one barrier per iteration orders
// everything.  The red phase covers the tile and one ring of halo cells (what
// the black phase reads); the outer halo ring is only read.  Plane t - 3, done,
// is written to the other copy of u (out of place: no workgroup reads a halo
// another one has already overwritten).  Loads run two iterations ahead: plane
// t + 3 is loaded in iteration t into one of two register sets and stored to
// LDS at the start of iteration t + 2, and a cell's own data (phi^m, the
// right-hand sides, the base state of the correction form) is loaded two
// iterations before its update by the thread that makes it, so a load's
// latency overlaps a whole iteration of work.
//
// With ZERO (the first pre-smoothing launch of a correction cycle on the
// finest level) the iterate is taken as the zero correction and not read.
// With b.pshift set (the first pre-smoothing launch on the finest FP64 level)
// the pending mean of p (res slot 4 of the instance) is subtracted from p as
// it is loaded, so that p's normalisation after a cycle costs no pass.
//
// With PRO != 0 the launch first prolongs the coarse correction: every
// region cell's iterate is loaded as u + P(u_c - ub_c) (PRO = 1 piecewise-
// constant injection, 2 cell-centred trilinear interpolation), the update the
// prolongation kernel makes, so the first post-smoothing step needs no pass of
// its own over the fine level.  Halo cells get the same corrected values as in
// the workgroup that owns them.
//
// Compared with one launch per color, every value is read once per step from
// HBM (halo columns and planes aside) and the neighbours of the other color
// come from LDS rather than from L2.
#include "chhs_cell.hpp"

namespace chhs {
namespace {

constexpr int kThreads = 256;
constexpr int kRing = 6;          // planes t - 3 .. t + 2 are live in iteration t
constexpr int kHalo = 2;
constexpr int PHI = 0, MU = 1, P = 2, PS = 3, NRF = 4;

template <int TX, int TY>
struct Geo {
    static constexpr int RX = TX + 2 * kHalo, RY = TY + 2 * kHalo;
    static constexpr int NR = RX * RY;                 // region cells of a plane
    static constexpr int KR = (NR + kThreads - 1) / kThreads;
    // red cells per plane: the tile and one ring of halo ((TX + 2)(TY + 2) / 2)
    static constexpr int WRX = TX + 2, WRY = TY + 2;
    static constexpr int NRED = WRX * WRY / 2;
    static constexpr int KRED = (NRED + kThreads - 1) / kThreads;
    // black cells per plane: the tile
    static constexpr int NBLK = TX * TY / 2;
    static constexpr int KBLK = (NBLK + kThreads - 1) / kThreads;
    static constexpr int NOWN = TX * TY;
    static constexpr int KOWN = (NOWN + kThreads - 1) / kThreads;
};

template <typename T>
struct Own {
    T psi, f0, f1, f2, b;
};

// PRO and ZERO are template arguments: a branch around the region loads
// would make the compiler wait for every load in flight where the branches
// join, and the loads would no longer overlap an iteration.  L0: the finest
// level of the plain form, whose right-hand side is f_phi = phi^m (psi) and
// f_p = 0 ((2.5), (2.7)): neither is loaded.
template <typename T, bool CORR, int TX, int TY, int PRO, bool ZERO, bool L0>
__global__ __launch_bounds__(kThreads) void k_step3d(Batch<T> bt, const Step3Task* __restrict__ tasks,
                                                     int ntasks) {
    using G = Geo<TX, TY>;
    constexpr int RX = G::RX, RY = G::RY, NR = G::NR;
    __shared__ T s[kRing][NRF][NR];

    const int bid = blockIdx.x;
    const int xcd = bid % 8, jj = bid / 8;
    const int q8 = ntasks / 8, rem = ntasks % 8;
    const Step3Task tk = tasks[xcd * q8 + (xcd < rem ? xcd : rem) + jj];
    if (bt.active != nullptr && bt.active[tk.inst] == 0) return;
    const Level<T> L = make_view(bt.desc[tk.inst * kMaxLevels + bt.level], bt.cur);
    // the coarse level of the prolongation (PRO != 0 only)
    const Level<T> C = make_view(bt.desc[tk.inst * kMaxLevels + bt.level + (PRO != 0 ? 1 : 0)],
                                 bt.cur_c);
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    const int sxy = nx * ny;
    const int x0 = tk.bx * TX - kHalo, y0 = tk.by * TY - kHalo;   // region origin
    const int z0 = tk.z0, z1 = tk.z1;
    const int plo = z0 - 2 > 0 ? z0 - 2 : 0;                        // planes loaded
    const int zhi = z1 + 1 < nz - 1 ? z1 + 1 : nz - 1;
    const int rlo = z0 - 1 > 0 ? z0 - 1 : 0;                        // planes red updates
    const int rhi = z1 < nz - 1 ? z1 : nz - 1;
    const int tid = threadIdx.x;
    const T lam = L.lam, kap = L.kap, gam = L.gamma;
    const T inv_lam = T(1) / lam;
    const T psh = bt.pshift != nullptr ? T(bt.pshift[tk.inst * kResStride + 4]) : T(0);

    // ---- region loads: thread takes region cells tid + k kThreads ----------------------
    // Loaded values are only stored to LDS two iterations later, and every
    // operation on them (the pending p shift, the coarse correction) is done
    // there: an operation right after a load would wait for it (and for every
    // load issued before it).  Region cells outside the grid load cell 0 of the
    // level (finite values that no face reads: boundary faces are dropped).
    // (PRO 1: u_c and ub_c of the coarse parent in six more slots, unused otherwise)
    using Regs = T[G::KR][NRF + 6];
    auto load_plane = [&](int z, Regs& rv) {
#pragma unroll
        for (int k = 0; k < G::KR; ++k) {
            const int q = tid + k * kThreads;
            const int ry = q / RX, rx = q - ry * RX;
            const int gx = x0 + rx, gy = y0 + ry;
            const bool ok = q < NR && gx >= 0 && gx < nx && gy >= 0 && gy < ny && z >= 0 && z < nz;
            const int g = ok ? z * sxy + gy * nx + gx : 0;
            if (ZERO) {
                rv[k][PHI] = rv[k][MU] = rv[k][P] = T(0);
            } else {
                rv[k][PHI] = gload(L.phi, g);
                rv[k][MU] = gload(L.mu, g);
                rv[k][P] = gload(L.p, g);
            }
            rv[k][PS] = gload(L.pstar, g);
            if (PRO == 1) {
                const int c = ok ? ((z >> 1) * C.ny + (gy >> 1)) * C.nx + (gx >> 1) : 0;
                rv[k][NRF + 0] = gload(C.phi, c);
                rv[k][NRF + 1] = gload(C.mu, c);
                rv[k][NRF + 2] = gload(C.p, c);
                rv[k][NRF + 3] = gload(C.ub0, c);
                rv[k][NRF + 4] = gload(C.ub1, c);
                rv[k][NRF + 5] = gload(C.ub2, c);
            } else if (PRO == 2 && ok) {
                rv[k][PHI] += bilinear_corr<3>(C.phi, C.ub0, C.nx, C.ny, C.nz, gx, gy, z);
                rv[k][MU] += bilinear_corr<3>(C.mu, C.ub1, C.nx, C.ny, C.nz, gx, gy, z);
                rv[k][P] += bilinear_corr<3>(C.p, C.ub2, C.nx, C.ny, C.nz, gx, gy, z);
            }
        }
    };
    auto store_plane = [&](int z, const Regs& rv) {
        const int sl = z % kRing;
#pragma unroll
        for (int k = 0; k < G::KR; ++k) {
            const int q = tid + k * kThreads;
            if (q >= NR) continue;
            T ph = rv[k][PHI], mu = rv[k][MU], p = rv[k][P] - psh;
            if (PRO == 1) {
                ph += rv[k][NRF + 0] - rv[k][NRF + 3];
                mu += rv[k][NRF + 1] - rv[k][NRF + 4];
                p += rv[k][NRF + 2] - rv[k][NRF + 5];
            }
            s[sl][PHI][q] = ph;
            s[sl][MU][q] = mu;
            s[sl][P][q] = p;
            s[sl][PS][q] = rv[k][PS];
        }
    };

    // ---- cells of a phase: red = the (TX + 2) x (TY + 2) box, black = the tile -------------
    // i-th cell of the color (color 0 red, 1 black) at plane z in a box of
    // width w, height hgt starting at region (bx0, by0); w even
    auto cell_of = [&](int i, int w, int bx0, int by0, int color, int z, int& rx, int& ry) {
        const int hw = w >> 1;
        const int row = i / hw;
        const int m = i - row * hw;
        ry = by0 + row;
        const int gy = y0 + ry;
        // (gx + gy + z) & 1 == color with gx = x0 + bx0 + 2m + e
        const int e = (x0 + bx0 + gy + z + color) & 1;
        rx = bx0 + 2 * m + e;
    };
    auto load_own = [&](int rx, int ry, int z, Own<T>& o) {
        const int gx = x0 + rx, gy = y0 + ry;
        const bool ok = gx >= 0 && gx < nx && gy >= 0 && gy < ny && z >= 0 && z < nz;
        const int g = ok ? z * sxy + gy * nx + gx : 0;
        o.psi = gload(L.psi, g);
        o.f0 = L0 ? o.psi : gload(L.f0, g);
        o.f1 = gload(L.f1, g);
        o.f2 = L0 ? T(0) : gload(L.f2, g);
        o.b = CORR ? gload(L.b, g) : T(0);
    };

    // the collective update of cell (rx, ry) of plane z from LDS (faces in the
    // order x - 1, x + 1, y - 1, y + 1, z - 1, z + 1, as cell_solve)
    auto update = [&](int rx, int ry, int z, const Own<T>& o) {
        const int gx = x0 + rx, gy = y0 + ry;
        if (gx < 0 || gx >= nx || gy < 0 || gy >= ny || z < 0 || z >= nz) return;
        const int sc = z % kRing;
        const int sd = (z + kRing - 1) % kRing, su = (z + 1) % kRing;
        const int w = ry * RX + rx;
        const T psc = s[sc][PS][w];
        int nf = 0;
        T sa = 0, sa2 = 0, smmu = 0, sphi = 0, sp = 0, sap = 0, samu = 0;
        auto face = [&](bool h, int sl, int wn) {
            const T a = T(0.5) * (psc + s[sl][PS][wn]);
            const T m = T(1) + gam * a * a;
            const T munb = s[sl][MU][wn];
            const T pnb = s[sl][P][wn];
            const T phinb = s[sl][PHI][wn];
            nf += h ? 1 : 0;
            sa = h ? sa + a : sa;
            sa2 = h ? sa2 + a * a : sa2;
            smmu = h ? smmu + m * munb : smmu;
            sphi = h ? sphi + phinb : sphi;
            sp = h ? sp + pnb : sp;
            sap = h ? sap + a * pnb : sap;
            samu = h ? samu + a * munb : samu;
        };
        face(gx > 0, sc, w - 1);
        face(gx < nx - 1, sc, w + 1);
        face(gy > 0, sc, w - RX);
        face(gy < ny - 1, sc, w + RX);
        face(z > 0, sd, w);
        face(z < nz - 1, su, w);
        const T fnf = T(nf);
        const T inv_nf = nf == 6 ? T(1) / T(6)
                       : (nf == 5 ? T(1) / T(5)
                       : (nf == 4 ? T(0.25) : (nf == 3 ? T(1) / T(3) : (nf == 2 ? T(0.5) : T(1)))));
        const T phit = s[sc][PHI][w];
        const T dchi = dnonlin<T, CORR>(phit, o.psi, o.b);
        const T chi = nonlin<T, CORR>(phit, o.psi, o.b);
        const T b1 = o.f0 + lam * smmu + lam * sap;
        const T b2 = o.f1 + chi - dchi * phit - kap * sphi;
        const T b3 = o.f2 - lam * sp - lam * gam * samu;
        const T ared = lam * (fnf + gam * (sa2 - sa * sa * inv_nf));
        const T b1r = b1 + (sa * inv_nf) * b3;
        const T bb = dchi + kap * fnf;
        const T inv_det = recip_ge1(T(1) + ared * bb);
        const T mun = (b2 + bb * b1r) * inv_det;
        s[sc][PHI][w] = (b1r - ared * b2) * inv_det;
        s[sc][MU][w] = mun;
        s[sc][P][w] = -(b3 * inv_lam + gam * sa * mun) * inv_nf;
    };

    // the thread's k-th red / black cell of plane z (a function of z's parity)
    auto red_cell = [&](int k, int z, int& rx, int& ry) {
        const int i = tid + k * kThreads;
        cell_of(i < G::NRED ? i : 0, G::WRX, kHalo - 1, kHalo - 1, 0, z, rx, ry);
    };
    auto blk_cell = [&](int k, int z, int& rx, int& ry) {
        const int i = tid + k * kThreads;
        cell_of(i < G::NBLK ? i : 0, TX, kHalo, kHalo, 1, z, rx, ry);
    };
    // own data of the thread's red cells of plane z and black cells of plane z
    using OwnRed = Own<T>[G::KRED];
    using OwnBlk = Own<T>[G::KBLK];
    auto prefetch_red = [&](int z, OwnRed& o) {
#pragma unroll
        for (int k = 0; k < G::KRED; ++k) {
            int rx, ry;
            red_cell(k, z, rx, ry);
            load_own(rx, ry, z, o[k]);
        }
    };
    auto prefetch_blk = [&](int z, OwnBlk& o) {
#pragma unroll
        for (int k = 0; k < G::KBLK; ++k) {
            int rx, ry;
            blk_cell(k, z, rx, ry);
            load_own(rx, ry, z, o[k]);
        }
    };

    // ---- the pipeline ---------------------------------------------------------------------
    // Iteration t takes register set t & 1: it holds plane t + 1 (stored to
    // LDS first), the red own data of plane t and the black own data of plane
    // t - 2; afterwards the same set receives plane t + 3, red t + 2, black t.
    Regs rvA, rvB;
    OwnRed oredA, oredB;
    OwnBlk oblkA, oblkB;
    load_plane(plo, rvA);
    store_plane(plo, rvA);
    if (plo + 1 <= zhi) load_plane(plo + 1, rvA);
    if (plo + 2 <= zhi) load_plane(plo + 2, rvB);
    prefetch_red(plo, oredA);
    prefetch_blk(plo - 2, oblkA);
    prefetch_red(plo + 1, oredB);
    prefetch_blk(plo - 1, oblkB);
    const int t_last = z1 + 2;              // plane z1 - 1 is stored in iteration z1 + 2
    auto iteration = [&](int t, Regs& rv, OwnRed& ored, OwnBlk& oblk) {
        if (t + 1 <= zhi) store_plane(t + 1, rv);
        __syncthreads();
        if (t >= rlo && t <= rhi)
#pragma unroll
            for (int k = 0; k < G::KRED; ++k)
                if (tid + k * kThreads < G::NRED) {
                    int rx, ry;
                    red_cell(k, t, rx, ry);
                    update(rx, ry, t, ored[k]);
                }
        const int tb = t - 2;
        if (tb >= z0 && tb < z1)
#pragma unroll
            for (int k = 0; k < G::KBLK; ++k)
                if (tid + k * kThreads < G::NBLK) {
                    int rx, ry;
                    blk_cell(k, tb, rx, ry);
                    update(rx, ry, tb, oblk[k]);
                }
        // plane t - 3 is final: write the tile into the other copy of u
        const int to = t - 3;
        if (to >= z0 && to < z1) {
            const int sl = to % kRing;
#pragma unroll
            for (int k = 0; k < G::KOWN; ++k) {
                const int q = tid + k * kThreads;
                if (q >= G::NOWN) continue;
                const int oy = q / TX, ox = q - oy * TX;
                const int gx = x0 + kHalo + ox, gy = y0 + kHalo + oy;
                if (gx >= nx || gy >= ny) continue;
                const int w = (oy + kHalo) * RX + ox + kHalo;
                const int g = to * sxy + gy * nx + gx;
                gstore(L.phi_alt, g, s[sl][PHI][w]);
                gstore(L.mu_alt, g, s[sl][MU][w]);
                gstore(L.p_alt, g, s[sl][P][w]);
            }
        }
        // loads for iteration t + 2: plane t + 3, own data of red t + 2 and
        // black t
        if (t + 3 <= zhi) load_plane(t + 3, rv);
        prefetch_red(t + 2, ored);
        prefetch_blk(t, oblk);
    };
    for (int t = plo; t <= t_last; t += 2) {
        iteration(t, rvA, oredA, oblkA);
        if (t + 1 <= t_last) iteration(t + 1, rvB, oredB, oblkB);
    }
}

template <typename T, bool CORR, int TX, int TY, bool L0>
void launch_tiles(const Batch<T>& b, const Step3Task* t, int nt, int pro, int zero, hipStream_t st) {
    if (pro == 1)
        hipLaunchKernelGGL((k_step3d<T, CORR, TX, TY, 1, false, L0>), dim3(nt), dim3(kThreads), 0,
                           st, b, t, nt);
    else if (pro == 2)
        hipLaunchKernelGGL((k_step3d<T, CORR, TX, TY, 2, false, L0>), dim3(nt), dim3(kThreads), 0,
                           st, b, t, nt);
    else if (zero && CORR)
        hipLaunchKernelGGL((k_step3d<T, CORR, TX, TY, 0, CORR, L0>), dim3(nt), dim3(kThreads), 0,
                           st, b, t, nt);
    else
        hipLaunchKernelGGL((k_step3d<T, CORR, TX, TY, 0, false, L0>), dim3(nt), dim3(kThreads), 0,
                           st, b, t, nt);
}

}  // namespace

void launch_step3d(const Batch<double>& b, const Step3Task* t, int nt, int pro, int zero,
                   hipStream_t st) {
    if (nt <= 0) return;
    if (b.level == 0)
        launch_tiles<double, false, kStep3TX64, kStep3TY64, true>(b, t, nt, pro, zero, st);
    else
        launch_tiles<double, false, kStep3TX64, kStep3TY64, false>(b, t, nt, pro, zero, st);
}

void launch_step3d(const Batch<float>& b, const Step3Task* t, int nt, int pro, int zero,
                   hipStream_t st) {
    if (nt > 0) launch_tiles<float, true, kStep3TX32, kStep3TY32, false>(b, t, nt, pro, zero, st);
}

}  // namespace chhs
