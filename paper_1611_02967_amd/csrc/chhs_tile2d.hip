// LDS-tiled smoothing kernels for 2D levels, batched over instances.
//
// One workgroup owns a TX x TY block of cells of one instance (a TileTask) and
// stages it in LDS together with a halo of H cells.  It runs NS fused smoothing
// steps (each a red and a black collective (phi, mu, p) cell update, the same
// update as k_smooth) on shrinking rings: phase q of the 2 NS phases updates
// every cell of its color within ring X + 2 NS - 1 - q of the block, so after
// the last phase the block and X extra rings hold exactly what two-launch
// red-black sweeps would produce.  Halo cells are recomputed redundantly by the
// neighbouring blocks with identical arithmetic.
//
// The kernel is out of place: it reads u = (phi, mu, p) and writes the block
// into the other copy of u, so a block never loads a halo that another block
// has already overwritten; the host then makes the written copy current.
//
// Optional fused parts:
//   PRO    prologue: u += P(u_c - ub_c) (piecewise-constant prolongation of the
//          coarse correction) applied while loading, halo included.
//   EPI 1  epilogue: residual R = f - N(u) on the block (X = 1) restricted by
//          cell averaging to the coarse level: u_c = ub_c = R u, fr_c = R R
//          (f_c = fr_c + N_c(u_c) is formed by the coarse level's first
//          launch, the coarse tail, or a coarse kernel).
//   EPI 2  epilogue: per-block partial sums of R_phi^2, R_mu^2, R_p^2 and p.
//   CORR   correction form of the mixed-precision inner solve (chhs_cell.hpp):
//          the base state b is read per cell and restricted with u.
//   RHS    prologue of the first smoothing launch on a coarse level: the FAS
//          right-hand side f += N(u) (u = the restricted iterate, f = the
//          restricted residual) on every cell a phase may update, the block's
//          cells written back; replaces a separate launch over the level.
//   ZERO   the first launch of an inner correction cycle on the finest level
//          (CORR): the correction starts at zero, so u is not read but taken
//          as 0 (and no pass clears it beforehand).
//
// Threads own pairs of horizontally adjacent cells (x even, x + 1) so that
// exactly one cell of every pair has the color of a phase: all lanes work in
// every phase, and a wave's loads cover 128 consecutive values of a row.  In
// LDS each row is stored as its even columns followed by its odd columns; all
// pairs of a row update the same member in a phase, so the lanes of a wave
// touch consecutive LDS words.
#include "chhs_cell.hpp"

#include <type_traits>

namespace chhs {
namespace {

constexpr int kTX = kTileX;     // block width (cells)

// NT threads per block: 256, 512 or 1024 (four, two or one pair per thread),
// chosen per level by the autotuner; without it 1024 on levels with fewer
// tiles than compute units, where the time of one block is the time of the
// launch, and 256 elsewhere.
template <int NS, int EPI, int NT, int TY>
struct Geometry {
    static constexpr int X = EPI ? 1 : 0;          // extra valid rings after the last phase
    static constexpr int H = X + 2 * NS;           // halo depth needed by phase 0
    static constexpr int HX = (H + 1) & ~1;        // x halo padded to keep pairs aligned
    static constexpr int W = kTX + 2 * HX;         // region width
    static constexpr int R = TY + 2 * H;           // region height
    static constexpr int PW = W / 2;               // pairs per row
    static constexpr int NP = PW * R;              // pairs in the region
    static constexpr int KP = (NP + NT - 1) / NT;   // pairs per thread
};

// LDS word of region cell (r, x): even columns of row r, then odd columns.
template <int PW>
__device__ __forceinline__ int lds(int r, int x) { return (2 * r + (x & 1)) * PW + (x >> 1); }

template <typename T, bool LEVEL0, int NS, int EPI, bool PRO, bool CORR, int NT, bool RHS, int TY,
          bool ZERO>
__global__ __launch_bounds__(NT) void k_tile2d(Batch<T> bt, const TileTask* __restrict__ tasks,
                                               int ntiles, double* partial) {
    using G = Geometry<NS, EPI, NT, TY>;
    constexpr int kTY = TY;                        // block height (cells)
    constexpr int kSlots = kTX * kTY / 2;          // pairs of the block (epilogue work items)
    constexpr int kThreads = NT;
    constexpr int W = G::W, R = G::R, H = G::H, HX = G::HX;
    constexpr int PW = G::PW, KP = G::KP, NP = G::NP;
    __shared__ T s_phi[R * W];
    __shared__ T s_mu[R * W];
    __shared__ T s_p[R * W];
    __shared__ T s_ps[R * W];

    // Workgroups are dispatched round-robin over the 8 XCDs.  Give XCD x a
    // contiguous range of tasks (a bijection of [0, ntiles)) so that
    // neighbouring blocks share their halo through the same L2.
    const int bid = blockIdx.x;
    const int xcd = bid % 8, jj = bid / 8;
    const int q8 = ntiles / 8, rem = ntiles % 8;
    const int tile = xcd * q8 + (xcd < rem ? xcd : rem) + jj;
    const TileTask tk = tasks[tile];
    if (bt.active != nullptr && bt.active[tk.inst] == 0) return;
    const Level<T> L = make_view(bt.desc[tk.inst * kMaxLevels + bt.level], bt.cur);
    const Level<T> C = make_view(bt.desc[tk.inst * kMaxLevels + bt.level + 1], bt.cur_c);
    const int x0 = tk.bx * kTX - HX, y0 = tk.by * kTY - H;     // region origin in cells
    const int nx = L.nx, ny = L.ny;
    const int tid = threadIdx.x;
    // a deferred shift of p (Batch::pshift), subtracted as p loads
    const T psh = bt.pshift != nullptr ? T(bt.pshift[tk.inst * kResStride + 4]) : T(0);

    // A block whose whole region lies inside the grid (most blocks of a large
    // level) takes every position test as passed: no bounds tests on loads and
    // stores, no tests per face (nf = 4).  The arithmetic is the same in both
    // forms of the body.
    const bool inner = x0 >= 0 && y0 >= 0 && x0 + W <= nx && y0 + R <= ny;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};      // EPI 2 partial sums of the thread
    auto body = [&](auto kind) {
        constexpr bool kInner = decltype(kind)::value;
        // own-cell data of the thread's pairs, stored by color (index 0 = the red
        // member, 1 = the black member) so that every phase reads them with
        // compile-time indices: psi, f0, f1, f2
        T o_psi[2][KP], o_f0[2][KP], o_f1[2][KP], o_f2[2][KP], o_b[2][KP];
        // staged values of the pairs before they go to LDS
        T v_phi[KP][2], v_mu[KP][2], v_p[KP][2], v_ps[KP][2];

        // 1) issue every global load of the region first ...
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int q = tid + k * kThreads;
            const int r = q / PW, x = 2 * (q % PW);
            const int gy = y0 + r;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int gx = x0 + x + e;
                T phi = 0, mu = 0, p = 0, ps = 0, psi = 0, f0 = 0, f1 = 0, f2 = 0, bs = 0;
                if (q < NP && (kInner || (gx >= 0 && gx < nx && gy >= 0 && gy < ny))) {
                    const int g = gy * nx + gx;
                    phi = ZERO ? T(0) : gload(L.phi, g);
                    mu = ZERO ? T(0) : gload(L.mu, g);
                    p = ZERO ? T(0) : gload(L.p, g) - psh;
                    ps = gload(L.pstar, g);
                    psi = gload(L.psi, g);
                    // the first launch on a coarse level forms f from the restricted residual
                    f1 = gload(RHS ? L.fr1 : L.f1, g);
                    if (LEVEL0) {
                        f0 = psi;
                    } else {
                        f0 = gload(RHS ? L.fr0 : L.f0, g);
                        f2 = gload(RHS ? L.fr2 : L.f2, g);
                    }
                    if (CORR) bs = gload(L.b, g);
                    if (PRO) {
                        const int c = (gy >> 1) * C.nx + (gx >> 1);
                        phi += gload(C.phi, c) - gload(C.ub0, c);
                        mu += gload(C.mu, c) - gload(C.ub1, c);
                        p += gload(C.p, c) - gload(C.ub2, c);
                    }
                }
                v_phi[k][e] = phi;
                v_mu[k][e] = mu;
                v_p[k][e] = p;
                v_ps[k][e] = ps;
                // member e has color (e + gy) & 1 because x0 + x is even
                const bool red = ((e + gy) & 1) == 0;
                if (e == 0) {
                    o_psi[0][k] = o_psi[1][k] = psi;
                    o_f0[0][k] = o_f0[1][k] = f0;
                    o_f1[0][k] = o_f1[1][k] = f1;
                    o_f2[0][k] = o_f2[1][k] = f2;
                    o_b[0][k] = o_b[1][k] = bs;
                } else {
                    o_b[0][k] = red ? bs : o_b[0][k];
                    o_b[1][k] = red ? o_b[1][k] : bs;
                    o_psi[0][k] = red ? psi : o_psi[0][k];
                    o_f0[0][k] = red ? f0 : o_f0[0][k];
                    o_f1[0][k] = red ? f1 : o_f1[0][k];
                    o_f2[0][k] = red ? f2 : o_f2[0][k];
                    o_psi[1][k] = red ? o_psi[1][k] : psi;
                    o_f0[1][k] = red ? o_f0[1][k] : f0;
                    o_f1[1][k] = red ? o_f1[1][k] : f1;
                    o_f2[1][k] = red ? o_f2[1][k] : f2;
                }
            }
        }
        // 2) ... then stage them in LDS
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int q = tid + k * kThreads;
            if (q >= NP) continue;
            const int r = q / PW, x = 2 * (q % PW);
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int w = lds<PW>(r, x + e);
                s_phi[w] = v_phi[k][e];
                s_mu[w] = v_mu[k][e];
                s_p[w] = v_p[k][e];
                s_ps[w] = v_ps[k][e];
            }
        }
        __syncthreads();

        const T lam = L.lam, kap = L.kap, gam = L.gamma;
        const T inv_lam = T(1) / lam;

        if (RHS) {
            // f += N(u) on every cell within ring H - 1 of the block (the cells
            // the phases update; their neighbours are in the region)
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int q = tid + k * kThreads;
                if (q >= NP) continue;
                const int r = q / PW, xp = 2 * (q % PW);
                const int gy = y0 + r;
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int x = xp + e;
                    const int gx = x0 + x;
                    if (!kInner && (gx < 0 || gx >= nx || gy < 0 || gy >= ny)) continue;
                    const int dx = x < HX ? HX - x : (x >= HX + kTX ? x - (HX + kTX - 1) : 0);
                    const int dy = r < H ? H - r : (r >= H + kTY ? r - (H + kTY - 1) : 0);
                    if ((dx > dy ? dx : dy) > H - 1) continue;
                    const bool red = ((e + gy) & 1) == 0;
                    const int wc = lds<PW>(r, x);
                    const T phic = s_phi[wc], muc = s_mu[wc], pc = s_p[wc], psc = s_ps[wc];
                    T smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
                    auto nb_n = [&](int rr, int xx) {
                        const int w = lds<PW>(rr, xx);
                        const T a = T(0.5) * (psc + s_ps[w]);
                        const T m = T(1) + gam * a * a;
                        const T dmu = s_mu[w] - muc;
                        const T dp = s_p[w] - pc;
                        smm += m * dmu;
                        sap += a * dp;
                        sphi += s_phi[w] - phic;
                        sp += dp;
                        samu += a * dmu;
                    };
                    if (kInner || gx > 0) nb_n(r, x - 1);
                    if (kInner || gx < nx - 1) nb_n(r, x + 1);
                    if (kInner || gy > 0) nb_n(r - 1, x);
                    if (kInner || gy < ny - 1) nb_n(r + 1, x);
                    // select values, not addresses, so that the arrays stay in registers
                    const T psi0 = o_psi[0][k], psi1 = o_psi[1][k], b0 = o_b[0][k], b1 = o_b[1][k];
                    const T fa0 = o_f0[0][k], fb0 = o_f0[1][k], fa1 = o_f1[0][k], fb1 = o_f1[1][k];
                    const T fa2 = o_f2[0][k], fb2 = o_f2[1][k];
                    const T psi = red ? psi0 : psi1;
                    const T bg = red ? b0 : b1;
                    const T n0 = phic - lam * smm - lam * sap;
                    const T n1 = muc - nonlin<T, CORR>(phic, psi, bg) + kap * sphi;
                    const T n2 = lam * sp + lam * gam * samu;
                    const T f0 = (red ? fa0 : fb0) + n0;
                    const T f1 = (red ? fa1 : fb1) + n1;
                    const T f2 = (red ? fa2 : fb2) + n2;
                    o_f0[0][k] = red ? f0 : fa0;
                    o_f0[1][k] = red ? fb0 : f0;
                    o_f1[0][k] = red ? f1 : fa1;
                    o_f1[1][k] = red ? fb1 : f1;
                    o_f2[0][k] = red ? f2 : fa2;
                    o_f2[1][k] = red ? fb2 : f2;
                    if (r >= H && r < H + kTY && x >= HX && x < HX + kTX) {
                        const int g = gy * nx + gx;
                        gstore(L.f0, g, f0);
                        gstore(L.f1, g, f1);
                        gstore(L.f2, g, f2);
                    }
                }
            }
            // the first phase overwrites cells whose values other waves still read here
            __syncthreads();
        }

        // Per pair and color, once for all phases: the LDS word of the member with
        // that color, the word of its x - 1 neighbour (the x + 1 neighbour is the
        // next word: an even member's x neighbours are odd columns, stored after
        // the row's even ones, and the other way round), its ring distance from the
        // block (more than any ring outside the grid) and which of its faces are
        // interior (bits x - 1, x + 1, y - 1, y + 1).  A phase then needs no
        // geometry of its own.
        int wcol[2][KP], wlcol[2][KP], dcol[2][KP], fcol[2][KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int q = tid + k * kThreads;
            const int r = q / PW, xp = 2 * (q % PW);
            const int gy = y0 + r;
#pragma unroll
            for (int color = 0; color < 2; ++color) {
                const int e = (gy & 1) ^ color;         // the pair member with this color
                const int x = xp + e;
                const int gx = x0 + x;
                const bool in = q < NP && (kInner || (gx >= 0 && gx < nx && gy >= 0 && gy < ny));
                const int dx = x < HX ? HX - x : (x >= HX + kTX ? x - (HX + kTX - 1) : 0);
                const int dy = r < H ? H - r : (r >= H + kTY ? r - (H + kTY - 1) : 0);
                dcol[color][k] = in ? (dx > dy ? dx : dy) : H + 1;
                wcol[color][k] = lds<PW>(r, x);
                wlcol[color][k] = wcol[color][k] + (e ? -PW : PW - 1);
                fcol[color][k] = (gx > 0 ? 1 : 0) | (gx < nx - 1 ? 2 : 0) | (gy > 0 ? 4 : 0) |
                                 (gy < ny - 1 ? 8 : 0);
            }
        }

#pragma unroll
        for (int ph = 0; ph < 2 * NS; ++ph) {
            const int color = ph & 1;
            const int ring = G::X + 2 * NS - 1 - ph;
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                if (dcol[color][k] > ring) continue;
                const int wc = wcol[color][k], wl = wlcol[color][k], fl = fcol[color][k];
                const T psc = s_ps[wc];
                int nf = 0;
                T sa = 0, sa2 = 0, smmu = 0, sphi = 0, sp = 0, sap = 0, samu = 0;
                auto nb_acc = [&](int w) {
                    const T a = T(0.5) * (psc + s_ps[w]);
                    const T m = T(1) + gam * a * a;
                    const T munb = s_mu[w];
                    const T pnb = s_p[w];
                    nf += 1;
                    sa += a;
                    sa2 += a * a;
                    smmu += m * munb;
                    sphi += s_phi[w];
                    sp += pnb;
                    sap += a * pnb;
                    samu += a * munb;
                };
                // faces in the order x - 1, x + 1, y - 1, y + 1
                if (kInner) {
                    nb_acc(wl);
                    nb_acc(wl + 1);
                    nb_acc(wc - 2 * PW);
                    nb_acc(wc + 2 * PW);
                } else {
                    if (fl & 1) nb_acc(wl);
                    if (fl & 2) nb_acc(wl + 1);
                    if (fl & 4) nb_acc(wc - 2 * PW);
                    if (fl & 8) nb_acc(wc + 2 * PW);
                }
                const T fnf = T(nf);
                const T inv_nf = nf == 4 ? T(0.25) : (nf == 3 ? T(1) / T(3) : (nf == 2 ? T(0.5) : T(1)));
                const T phit = s_phi[wc];
                const T psi = o_psi[color][k];
                const T f0 = o_f0[color][k];
                const T f1 = o_f1[color][k];
                const T f2 = o_f2[color][k];
                const T base = o_b[color][k];
                const T dchi = dnonlin<T, CORR>(phit, psi, base);
                const T chi = nonlin<T, CORR>(phit, psi, base);
                const T b1 = f0 + lam * smmu + lam * sap;
                const T b2 = f1 + chi - dchi * phit - kap * sphi;
                const T b3 = f2 - lam * sp - lam * gam * samu;
                const T ared = lam * (fnf + gam * (sa2 - sa * sa * inv_nf));
                const T b1r = b1 + (sa * inv_nf) * b3;
                const T bb = dchi + kap * fnf;
                const T inv_det = recip_ge1(T(1) + ared * bb);
                const T mun = (b2 + bb * b1r) * inv_det;
                s_phi[wc] = (b1r - ared * b2) * inv_det;
                s_mu[wc] = mun;
                s_p[wc] = -(b3 * inv_lam + gam * sa * mun) * inv_nf;
            }
            __syncthreads();
        }

        // write the block into the other copy of u
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int q = tid + k * kThreads;
            if (q >= NP) continue;
            const int r = q / PW, xp = 2 * (q % PW);
            if (r < H || r >= H + kTY || xp < HX || xp >= HX + kTX) continue;
            const int gy = y0 + r;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int gx = x0 + xp + e;
                if (!kInner && (gx >= nx || gy >= ny)) continue;
                const int g = gy * nx + gx;
                const int w = lds<PW>(r, xp + e);
                gstore(L.phi_alt, g, s_phi[w]);
                gstore(L.mu_alt, g, s_mu[w]);
                gstore(L.p_alt, g, s_p[w]);
            }
        }

        if (EPI == 0) return;

        // residual on the block.  Slot s (512 per block) is the pair of
        // horizontally adjacent fine cells in row cy of coarse cell (cxl, cyl);
        // slots s and s ^ 32 -- lanes l and l ^ 32 of one wave -- are the two rows
        // of the same coarse cell.
#pragma unroll
        for (int j = 0; j < (kSlots + kThreads - 1) / kThreads; ++j) {
            const int slot = tid + j * kThreads;
            if (slot >= kSlots) break;      // whole waves
            const int cxl = slot & 31, cy = (slot >> 5) & 1, cyl = slot >> 6;   // 32 x 8 coarse cells
            T su[3] = {0, 0, 0}, sr[3] = {0, 0, 0}, sb = 0;
            const int gcx = (x0 + HX) / 2 + cxl, gcy = (y0 + H) / 2 + cyl;
            const bool live = kInner || (2 * gcx < nx && 2 * gcy < ny);
            if (live) {
                for (int cx = 0; cx < 2; ++cx) {
                    const int r = H + 2 * cyl + cy, x = HX + 2 * cxl + cx;
                    const int gx = x0 + x, gy = y0 + r;
                    const int g = gy * nx + gx;
                    const int wc = lds<PW>(r, x);
                    const T phic = s_phi[wc], muc = s_mu[wc], pc = s_p[wc], psc = s_ps[wc];
                    T smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
                    auto nb_res = [&](int rr, int xx) {
                        const int w = lds<PW>(rr, xx);
                        const T a = T(0.5) * (psc + s_ps[w]);
                        const T m = T(1) + gam * a * a;
                        const T dmu = s_mu[w] - muc;
                        const T dp = s_p[w] - pc;
                        smm += m * dmu;
                        sap += a * dp;
                        sphi += s_phi[w] - phic;
                        sp += dp;
                        samu += a * dmu;
                    };
                    if (kInner || gx > 0) nb_res(r, x - 1);
                    if (kInner || gx < nx - 1) nb_res(r, x + 1);
                    if (kInner || gy > 0) nb_res(r - 1, x);
                    if (kInner || gy < ny - 1) nb_res(r + 1, x);
                    const T psi = gload(L.psi, g);
                    const T f0 = LEVEL0 ? psi : gload(L.f0, g);
                    const T f1 = gload(L.f1, g);
                    const T f2 = LEVEL0 ? T(0) : gload(L.f2, g);
                    const T bg = CORR ? gload(L.b, g) : T(0);
                    const T r0 = f0 - (phic - lam * smm - lam * sap);
                    const T r1 = f1 - (muc - nonlin<T, CORR>(phic, psi, bg) + kap * sphi);
                    const T r2 = f2 - (lam * sp + lam * gam * samu);
                    if (EPI == 1) {
                        sr[0] += r0;
                        sr[1] += r1;
                        sr[2] += r2;
                        su[0] += phic;
                        su[1] += muc;
                        su[2] += pc;
                        sb += bg;
                    } else {
                        acc[0] += double(r0) * double(r0);
                        acc[1] += double(r1) * double(r1);
                        acc[2] += double(r2) * double(r2);
                        acc[3] += double(pc);
                    }
                }
            }
            if (EPI == 1) {
                // combine the two rows (lane ^ 32), two fields per exchange: lanes
                // 0-31 then hold r0, r2, mu and lanes 32-63 r1, phi, p of the coarse cell
                const T w = T(0.25);
                const T q0 = swap_sum(sr[0], sr[1], true) * w;
                const T q1 = swap_sum(sr[2], su[0], true) * w;
                const T q2 = swap_sum(su[1], su[2], true) * w;
                const T qb = CORR ? rows_sum(sb, true) * w : T(0);
                if (live) {
                    const int c = gcy * C.nx + gcx;
                    // separate conditions, so that no two stores merge into one
                    // through a selected address
                    if (cy == 0) gstore(C.fr0, c, q0);
                    if (cy == 1) gstore(C.fr1, c, q0);
                    if (cy == 0) gstore(C.fr2, c, q1);
                    if (cy == 1) gstore(C.phi, c, q1);
                    if (cy == 1) gstore(C.ub0, c, q1);
                    if (cy == 0) gstore(C.mu, c, q2);
                    if (cy == 0) gstore(C.ub1, c, q2);
                    if (cy == 1) gstore(C.p, c, q2);
                    if (cy == 1) gstore(C.ub2, c, q2);
                    if (CORR && cy == 0) gstore(C.b, c, qb);
                }
            }
        }
        if (EPI == 1) return;
    };
    if (inner)
        body(std::true_type{});
    else
        body(std::false_type{});
    if (EPI != 2) return;
    // EPI == 2: block partial sums in a fixed order
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < 4; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    __shared__ double red[4][kThreads / 64];
    if ((tid & 63) == 0)
        for (int c = 0; c < 4; ++c) red[c][tid >> 6] = acc[c];
    __syncthreads();
    if (tid == 0)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) s += red[c][w];
            gstore(partial, tile * kPartialStride + c, s);
        }
}

template <typename T, bool LEVEL0, int NS, int EPI, bool PRO, bool CORR, bool RHS, int TY,
          bool ZERO>
void launch_ty(const Batch<T>& b, const TileTask* t, int nt, int threads, double* partial,
               hipStream_t st) {
    if (threads == 1024)
        hipLaunchKernelGGL((k_tile2d<T, LEVEL0, NS, EPI, PRO, CORR, 1024, RHS, TY, ZERO>), dim3(nt),
                           dim3(1024), 0, st, b, t, nt, partial);
    else if (threads == 512)
        hipLaunchKernelGGL((k_tile2d<T, LEVEL0, NS, EPI, PRO, CORR, 512, RHS, TY, ZERO>), dim3(nt),
                           dim3(512), 0, st, b, t, nt, partial);
    else
        hipLaunchKernelGGL((k_tile2d<T, LEVEL0, NS, EPI, PRO, CORR, 256, RHS, TY, ZERO>), dim3(nt),
                           dim3(256), 0, st, b, t, nt, partial);
}

// 64 x 32 tiles exist for the FP32 (CORR) finest level only (no RHS form);
// the finest-level variants (LEVEL0, ZERO) for 64 x 16 and 64 x 32 tiles only.
template <typename T, bool LEVEL0, int NS, int EPI, bool PRO, bool CORR, bool RHS = false,
          bool ZERO = false>
void launch_one(const Batch<T>& b, const TileTask* t, int nt, int threads, int ty, double* partial,
                hipStream_t st) {
    if constexpr (CORR && !RHS) {
        if (ty == kTileYTall) {
            launch_ty<T, LEVEL0, NS, EPI, PRO, CORR, RHS, kTileYTall, ZERO>(b, t, nt, threads,
                                                                           partial, st);
            return;
        }
    }
    if constexpr (!LEVEL0 && !ZERO) {
        if (ty == kTileYSmall) {
            launch_ty<T, LEVEL0, NS, EPI, PRO, CORR, RHS, kTileYSmall, false>(b, t, nt, threads,
                                                                             partial, st);
            return;
        }
        if (ty == kTileYTiny) {
            launch_ty<T, LEVEL0, NS, EPI, PRO, CORR, RHS, kTileYTiny, false>(b, t, nt, threads,
                                                                            partial, st);
            return;
        }
    }
    launch_ty<T, LEVEL0, NS, EPI, PRO, CORR, RHS, kTileY, ZERO>(b, t, nt, threads, partial, st);
}

}  // namespace

template <>
void launch_tile2d<double>(const Batch<double>& b, const TileTask* t, int nt, bool level0, int ns,
                           int epi, bool pro, int threads, bool rhs, int ty, bool zero,
                           double* partial, hipStream_t st) {
    (void)zero;
    if (nt <= 0) return;
    if (rhs) {
        // first pre-smoothing launch of a coarse level (no prolongation)
        if (level0 || pro || epi == 2) return;
#define CHHS_TILE_RHS(NS, EPI)                                                    \
    if (ns == NS && epi == EPI) {                                                 \
        launch_one<double, false, NS, EPI, false, false, true>(b, t, nt, threads, ty, partial, st); \
        return;                                                                   \
    }
        CHHS_TILE_RHS(1, 0)
        CHHS_TILE_RHS(1, 1)
        CHHS_TILE_RHS(2, 0)
        CHHS_TILE_RHS(2, 1)
#undef CHHS_TILE_RHS
        return;
    }
#define CHHS_TILE_CASE(L0, NS, EPI, PRO)                                          \
    if (level0 == L0 && ns == NS && epi == EPI && pro == PRO) {                   \
        launch_one<double, L0, NS, EPI, PRO, false>(b, t, nt, threads, ty, partial, st); \
        return;                                                                   \
    }
#define CHHS_TILE_PRO(L0, NS, EPI) CHHS_TILE_CASE(L0, NS, EPI, false) CHHS_TILE_CASE(L0, NS, EPI, true)
#define CHHS_TILE_EPI(L0, NS) CHHS_TILE_PRO(L0, NS, 0) CHHS_TILE_PRO(L0, NS, 1) CHHS_TILE_PRO(L0, NS, 2)
    CHHS_TILE_EPI(true, 1)
    CHHS_TILE_EPI(true, 2)
    CHHS_TILE_EPI(false, 1)
    CHHS_TILE_EPI(false, 2)
#undef CHHS_TILE_EPI
#undef CHHS_TILE_PRO
#undef CHHS_TILE_CASE
}

// FP32 correction form (mixed-precision inner solve): general right-hand
// sides, no norm epilogue.
template <>
void launch_tile2d<float>(const Batch<float>& b, const TileTask* t, int nt, bool level0, int ns,
                          int epi, bool pro, int threads, bool rhs, int ty, bool zero,
                          double* partial, hipStream_t st) {
    (void)level0;
    if (nt <= 0) return;
    if (zero) {
        // first launch of a correction cycle on the finest level (64 x 16 or
        // 64 x 32 tiles)
        if (pro || rhs || epi == 2 || (ty != kTileY && ty != kTileYTall)) return;
#define CHHS_TILE_ZERO(NS, EPI)                                                   \
    if (ns == NS && epi == EPI) {                                                 \
        launch_one<float, false, NS, EPI, false, true, false, true>(b, t, nt, threads, ty, partial, st); \
        return;                                                                   \
    }
        CHHS_TILE_ZERO(1, 0)
        CHHS_TILE_ZERO(1, 1)
        CHHS_TILE_ZERO(2, 0)
        CHHS_TILE_ZERO(2, 1)
#undef CHHS_TILE_ZERO
        return;
    }
    if (rhs) {
        if (pro || epi == 2) return;
#define CHHS_TILE_RHS(NS, EPI)                                                    \
    if (ns == NS && epi == EPI) {                                                 \
        launch_one<float, false, NS, EPI, false, true, true>(b, t, nt, threads, ty, partial, st); \
        return;                                                                   \
    }
        CHHS_TILE_RHS(1, 0)
        CHHS_TILE_RHS(1, 1)
        CHHS_TILE_RHS(2, 0)
        CHHS_TILE_RHS(2, 1)
#undef CHHS_TILE_RHS
        return;
    }
#define CHHS_TILE_CASE(NS, EPI, PRO)                                              \
    if (ns == NS && epi == EPI && pro == PRO) {                                   \
        launch_one<float, false, NS, EPI, PRO, true>(b, t, nt, threads, ty, partial, st); \
        return;                                                                   \
    }
    CHHS_TILE_CASE(1, 0, false)
    CHHS_TILE_CASE(1, 0, true)
    CHHS_TILE_CASE(1, 1, false)
    CHHS_TILE_CASE(2, 0, false)
    CHHS_TILE_CASE(2, 0, true)
    CHHS_TILE_CASE(2, 1, false)
#undef CHHS_TILE_CASE
}

}  // namespace chhs
