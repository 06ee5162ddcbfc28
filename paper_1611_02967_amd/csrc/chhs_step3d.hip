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
// another one has already overwritten).  A cell's own data (phi^m, the
// right-hand sides, the base state of the correction form) is loaded one
// iteration ahead into registers by the thread that updates it.
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

template <typename T, bool CORR, int TX, int TY>
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

    // ---- region loads: thread takes region cells tid + k kThreads ----------------------
    T rv[G::KR][NRF];
    auto load_plane = [&](int z) {
#pragma unroll
        for (int k = 0; k < G::KR; ++k) {
            const int q = tid + k * kThreads;
            const int ry = q / RX, rx = q - ry * RX;
            const int gx = x0 + rx, gy = y0 + ry;
            const bool ok = q < NR && gx >= 0 && gx < nx && gy >= 0 && gy < ny && z >= 0 && z < nz;
            const int g = ok ? z * sxy + gy * nx + gx : 0;
            rv[k][PHI] = gload(L.phi, g);
            rv[k][MU] = gload(L.mu, g);
            rv[k][P] = gload(L.p, g);
            rv[k][PS] = gload(L.pstar, g);
            if (!ok) rv[k][PHI] = rv[k][MU] = rv[k][P] = rv[k][PS] = T(0);
        }
    };
    auto store_plane = [&](int z) {
        const int sl = z % kRing;
#pragma unroll
        for (int k = 0; k < G::KR; ++k) {
            const int q = tid + k * kThreads;
            if (q < NR)
#pragma unroll
                for (int f = 0; f < NRF; ++f) s[sl][f][q] = rv[k][f];
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
        o.f0 = gload(L.f0, g);
        o.f1 = gload(L.f1, g);
        o.f2 = gload(L.f2, g);
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

    // own data of the thread's red cells of plane z and black cells of plane z
    Own<T> ored[G::KRED], oblk[G::KBLK];
    int rxr[G::KRED], ryr[G::KRED], rxb[G::KBLK], ryb[G::KBLK];
    auto prefetch_red = [&](int z) {
#pragma unroll
        for (int k = 0; k < G::KRED; ++k) {
            const int i = tid + k * kThreads;
            cell_of(i < G::NRED ? i : 0, G::WRX, kHalo - 1, kHalo - 1, 0, z, rxr[k], ryr[k]);
            load_own(rxr[k], ryr[k], z, ored[k]);
        }
    };
    auto prefetch_blk = [&](int z) {
#pragma unroll
        for (int k = 0; k < G::KBLK; ++k) {
            const int i = tid + k * kThreads;
            cell_of(i < G::NBLK ? i : 0, TX, kHalo, kHalo, 1, z, rxb[k], ryb[k]);
            load_own(rxb[k], ryb[k], z, oblk[k]);
        }
    };

    // ---- the pipeline ---------------------------------------------------------------------
    load_plane(plo);
    store_plane(plo);
    if (plo + 1 <= zhi) load_plane(plo + 1);
    prefetch_red(plo);
    prefetch_blk(plo - 2);
    const int t_last = z1 + 2;              // plane z1 - 1 is stored in iteration z1 + 2
    for (int t = plo; t <= t_last; ++t) {
        if (t + 1 <= zhi) store_plane(t + 1);
        __syncthreads();
        if (t >= rlo && t <= rhi)
#pragma unroll
            for (int k = 0; k < G::KRED; ++k)
                if (tid + k * kThreads < G::NRED) update(rxr[k], ryr[k], t, ored[k]);
        const int tb = t - 2;
        if (tb >= z0 && tb < z1)
#pragma unroll
            for (int k = 0; k < G::KBLK; ++k)
                if (tid + k * kThreads < G::NBLK) update(rxb[k], ryb[k], tb, oblk[k]);
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
        // loads for the next iteration: plane t + 2, own data of red t + 1 and
        // black t - 1
        if (t + 2 <= zhi) load_plane(t + 2);
        prefetch_red(t + 1);
        prefetch_blk(t - 1);
    }
}

template <typename T, bool CORR, int TX, int TY>
void launch_tiles(const Batch<T>& b, const Step3Task* t, int nt, hipStream_t st) {
    hipLaunchKernelGGL((k_step3d<T, CORR, TX, TY>), dim3(nt), dim3(kThreads), 0, st, b, t, nt);
}

}  // namespace

void launch_step3d(const Batch<double>& b, const Step3Task* t, int nt, hipStream_t st) {
    if (nt > 0) launch_tiles<double, false, kStep3TX64, kStep3TY64>(b, t, nt, st);
}

void launch_step3d(const Batch<float>& b, const Step3Task* t, int nt, hipStream_t st) {
    if (nt > 0) launch_tiles<float, true, kStep3TX32, kStep3TY32>(b, t, nt, st);
}

}  // namespace chhs
