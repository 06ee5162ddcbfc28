// Row-streaming smoothing kernels for 2D levels, batched over instances.
//
// A workgroup owns a strip of kStripWO columns and a segment [y0, y1) of rows
// of one instance (a StripTask).  It stages a 128-column region (the strip and
// kStripHX halo columns on each side) row by row in an LDS ring buffer and
// marches upwards.  The 2 NS phases of NS fused smoothing steps (each a red and
// a black collective (phi, mu, p) cell update, the update of k_smooth) run
// concurrently, one wave per phase: at iteration t wave q updates the cells of
// its color in row t - 2 q.  Two rows of lag per phase are exactly what
// ordered red-black sweeps need: phase q at row r reads rows r - 1 .. r + 1,
// which phase q - 1 finished in earlier iterations, and touches nothing that
// phase q - 1 or q + 1 writes in the same iteration.  One barrier per
// iteration orders the phases.  Rows leave the pipeline 4 NS + 1 iterations
// after they enter; the residual, the restriction and the write-back then
// read them from the ring.
//
// Compared with square tiles, halo cells are recomputed only in x (128 loaded
// columns for kStripWO = 116 owned) and in the few rows that overlap the
// neighbouring segments, global loads are issued at least two rows ahead of
// their use, and every wave reads consecutive LDS words.
//
// Only the fields that neighbours read (phi, mu, p, phi_*) live in the ring;
// a cell's own data (phi^m and the right-hand sides) is loaded by the wave
// that updates it, kU iterations ahead, as pairs of adjacent cells.  The ring
// of 4 NS + 5 rows then takes 52 KB in FP64, so that three workgroups share
// a compute unit.
//
// The kernel is out of place: it reads u = (phi, mu, p) from copy b.cur and
// writes the owned cells into the other copy.
//
// Optional fused parts, as in the tiled kernel:
//   PRO    u += P(u_c - ub_c) applied while loading (halo included).
//   EPI 1  residual R = f - N(u) on the owned cells restricted by cell
//          averaging: u_c = ub_c = R u, fr_c = R R on level + 1 (copy b.cur_c).
//   EPI 2  per-task partial sums of R_phi^2, R_mu^2, R_p^2 and p.
//   CORR   correction form of the mixed-precision inner solve.
//   ZERO   first launch of a correction cycle on the finest level (CORR): the
//          correction starts at zero and is not read.
#include <type_traits>

#include "chhs_cell.hpp"

namespace chhs {
namespace {

constexpr int kW = kStripW;          // region columns: one pair per lane of a wave
constexpr int kHalf = kW / 2;
constexpr int kThreads = 256;        // four waves
constexpr int kD = 2;                // rows per register bank of ring loads in flight
constexpr int kU = 2 * kD;           // iterations per loop body; own data is kU rows ahead

// Ring fields (read by neighbours).
constexpr int PHI = 0, MU = 1, P = 2, PS = 3, NRF = 4;

// Own fields of a cell, in load order: the finest level has f_phi = phi^m and
// f_p = 0 implied.
template <bool LEVEL0, bool CORR>
struct Own {
    static constexpr int N = LEVEL0 ? 2 : (CORR ? 5 : 4);
    // index of psi, f0, f1, f2, b in the load order (-1: implied)
    static constexpr int PSI = 0;
    static constexpr int F0 = LEVEL0 ? 0 : 1;
    static constexpr int F1 = LEVEL0 ? 1 : 2;
    static constexpr int F2 = LEVEL0 ? -1 : 3;
    static constexpr int B = CORR ? 4 : -1;
};

template <typename T>
struct Pair {
    T a, b;
};

// Pair k (cells 2 k, 2 k + 1) of a field: one 2-element vector load.
template <typename T>
__device__ __forceinline__ Pair<T> gload_pair(const T* p, int k) {
    typedef T V __attribute__((ext_vector_type(2)));
    const V v = gload(reinterpret_cast<const V*>(p), k);
    return Pair<T>{v.x, v.y};
}

// LDS word of region column c within a row: even columns, then odd columns.
__device__ __forceinline__ int col(int c) { return (c & 1) * kHalf + (c >> 1); }

// Three workgroups per compute unit (the LDS ring allows it) need at most 168
// VGPRs: requested for the finest-level variants.
template <typename T, bool LEVEL0, int NS, int EPI, bool PRO, bool CORR, bool ZERO>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(LEVEL0 || CORR ? 3 : 1))) void k_stream2d(Batch<T> bt,
                                                       const StripTask* __restrict__ tasks,
                                                       int ntasks, double* partial) {
    using O = Own<LEVEL0, CORR>;
    constexpr int NO = O::N;
    constexpr int X = EPI ? 1 : 0;
    constexpr int H = X + 2 * NS;          // halo rows
    constexpr int NPH = 2 * NS;            // phases = waves with phase work
    constexpr int LAG = 4 * NS + 1;        // rows (t - LAG, t - LAG + 1) leave at iteration t
    constexpr int RING = 4 * NS + 5;       // rows t - LAG - 1 .. t + 2 are live
    static_assert(kStripHX >= 2 * NS + 2, "halo columns must cover the phases and the residual");
    __shared__ T s[RING][NRF][kW];

    // XCD-aware order: XCD x runs a contiguous range of tasks (a bijection)
    const int bid = blockIdx.x;
    const int xcd = bid % 8, jj = bid / 8;
    const int q8 = ntasks / 8, rem = ntasks % 8;
    const int task = xcd * q8 + (xcd < rem ? xcd : rem) + jj;
    const StripTask tk = tasks[task];
    if (bt.active != nullptr && bt.active[tk.inst] == 0) return;
    const Level<T> L = make_view(bt.desc[tk.inst * kMaxLevels + bt.level], bt.cur);
    const Level<T> C = make_view(bt.desc[tk.inst * kMaxLevels + bt.level + 1], bt.cur_c);
    const int nx = L.nx, ny = L.ny;
    const int x0 = tk.sx * kStripWO - kStripHX;       // even
    const int y0 = tk.y0, y1 = tk.y1;                  // y0 even
    const int ys = y0 - H > 0 ? y0 - H : 0;
    const int ye = y1 + H < ny ? y1 + H : ny;          // loaded rows [ys, ye)
    const int rlo = ys == 0 ? 0 : ys + 1;              // rows a phase may update
    const int rhi = ye == ny ? ny - 1 : ye - 2;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);    // uniform per wave
    // every region column but the outermost two has both x neighbours in the grid
    const bool xin = x0 >= 0 && x0 + kW - 1 <= nx - 1;

    const T* own_src[NO];
    if (LEVEL0) {
        own_src[0] = L.psi;
        own_src[1] = L.f1;
    } else {
        own_src[0] = L.psi;
        own_src[1] = L.f0;
        own_src[2] = L.f1;
        own_src[3] = L.f2;
        if (CORR) own_src[NO - 1] = L.b;
    }

    // ---- ring loader: thread owns region column lc, fields 2 j + half ---------------
    // lanes 0-31 of a wave take even columns, 32-63 odd ones: a load covers 64
    // consecutive values of a row and a store 2 x 32 consecutive LDS words
    const int half = wave >> 1;
    const int lc = 2 * ((lane & 31) + 32 * (wave & 1)) + (lane >> 5);
    const int lgx = x0 + lc;
    const bool lcol = lgx >= 0 && lgx < nx;
    // j = 0: phi | mu, j = 1: p | phi_*
    const T* src[2] = {half ? L.mu : L.phi, half ? L.pstar : L.p};
    // a deferred shift of p (Batch::pshift), subtracted from field p as it
    // enters the ring (not at the load, which would wait for the load at once)
    const T psh = bt.pshift != nullptr && half == 0 ? T(bt.pshift[tk.inst * kResStride + 4]) : T(0);
    const T* csrc[2] = {nullptr, nullptr};
    const T* cbar[2] = {nullptr, nullptr};
    if (PRO) {
        csrc[0] = half ? C.mu : C.phi;
        cbar[0] = half ? C.ub1 : C.ub0;
        csrc[1] = C.p;
        cbar[1] = C.ub2;
    }
    T rv[2][kD][2], rc[2][kD][2], rb[2][kD][2];

    // Loads are unconditional (cells outside the loaded rows or the grid read
    // element 0 and are dropped) so that the compiler can wait for exactly the
    // row it stores, not for every load in flight.
    auto load_row = [&](T (&v)[2], T (&vc)[2], T (&vb)[2], int r) {
        const bool ok = lcol && r >= ys && r < ye;
        const int g = ok ? r * nx + lgx : 0;
        // ZERO: only phi_* is read (by both halves, so that every wave issues
        // the same loads; the second read of a row hits the cache)
        if (ZERO) {
            v[0] = T(0);
            v[1] = gload_stream(L.pstar, g);
        } else {
#pragma unroll
            for (int j = 0; j < 2; ++j) v[j] = gload_stream(src[j], g);
        }
        if (PRO) {
            const int cg = ok ? (r >> 1) * C.nx + (lgx >> 1) : 0;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                vc[j] = gload(csrc[j], cg);
                vb[j] = gload(cbar[j], cg);
            }
        }
    };
    auto store_row = [&](const T (&v)[2], const T (&vc)[2], const T (&vb)[2], int r) {
        if (r >= ye) return;
        const int slot = r % RING;
        const int w = col(lc);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            T x = lcol ? (j == 1 ? v[j] - psh : v[j]) : T(0);
            if (ZERO && (j == 0 || half == 0)) x = T(0);
            // prolongation of the correction onto phi, mu, p (not phi_*)
            if (PRO && lcol && (j == 0 || half == 0)) x += vc[j] - vb[j];
            s[slot][2 * j + half][w] = x;
        }
    };

    // ---- own data of the rows a phase wave updates: pairs (2 lane, 2 lane + 1) ---------
    // prefetch distance in iterations (and slots): kU, or 2 when the
    // prolongation's coarse loads also wait in registers
    constexpr int KO = PRO ? 2 : kU;
    Pair<T> od[KO][NO];
    const int pgx = x0 + 2 * lane;
    const bool pcol = pgx >= 0 && pgx < nx;            // nx is even on these levels
    auto load_own = [&](Pair<T> (&o)[NO], int r) {
        const bool ok = pcol && r >= rlo && r <= rhi;
        const int g2 = ok ? (r * nx + pgx) >> 1 : 0;
#pragma unroll
        for (int k = 0; k < NO; ++k) o[k] = gload_pair(own_src[k], g2);
    };

    const T lam = L.lam, kap = L.kap, gam = L.gamma;
    const T inv_lam = T(1) / lam;

    // sums over the faces of a cell, in the order x - 1, x + 1, y - 1, y + 1
    struct Sums {
        int nf;
        T sa, sa2, smmu, sphi, sp, sap, samu;
    };
    auto face = [&](Sums& q, T psc, T psn, T mun, T pn, T phin) {
        const T a = T(0.5) * (psc + psn);
        const T m = T(1) + gam * a * a;
        q.nf += 1;
        q.sa += a;
        q.sa2 += a * a;
        q.smmu += m * mun;
        q.sphi += phin;
        q.sp += pn;
        q.sap += a * pn;
        q.samu += a * mun;
    };
    auto face_if = [&](Sums& q, bool h, T psc, T psn, T mun, T pn, T phin) {
        Sums t = q;
        face(t, psc, psn, mun, pn, phin);
        q.nf = h ? t.nf : q.nf;
        q.sa = h ? t.sa : q.sa;
        q.sa2 = h ? t.sa2 : q.sa2;
        q.smmu = h ? t.smmu : q.smmu;
        q.sphi = h ? t.sphi : q.sphi;
        q.sp = h ? t.sp : q.sp;
        q.sap = h ? t.sap : q.sap;
        q.samu = h ? t.samu : q.samu;
    };

    // ---- phase q on row r: the collective update of the q & 1 colored cells ----------
    // XIN (strips away from the x boundaries): every cell the phase updates has
    // both x faces, so the face count is the same for the whole row
    auto phase = [&](auto xin_c, int q, int r, const Pair<T> (&o)[NO]) {
        constexpr bool XIN = decltype(xin_c)::value;
        if (r < rlo || r > rhi) return;
        const int e = (r & 1) ^ (q & 1);           // pair member with this color
        const int c = 2 * lane + e;
        const int gx = x0 + c;
        // Away from the x boundaries every lane updates its cell, the two
        // outermost columns with an in-bounds word of the row as their missing
        // neighbour: the error spreads one column per phase and reaches column
        // 2 NS from the edge with the residual, inside the kStripHX >= 2 NS + 2
        // halo columns (owned cells never depend on it).  The words are
        // col(c - 1), col(c), col(c + 1), wrapped within the row at the edges.
        if (!XIN && (c < 1 || c > kW - 2 || gx < 0 || gx >= nx)) return;
        const int sc = r % RING, sd = (r + RING - 1) % RING, su = (r + 1) % RING;
        // (e is uniform: the offsets are scalar selects)
        const int wc = XIN ? lane + (e ? kHalf : 0) : col(c);
        const int wl = XIN ? lane + (e ? 0 : kHalf - 1) : col(c - 1);
        const int wr = XIN ? lane + (e ? 1 : kHalf) : col(c + 1);
        const T psc = s[sc][PS][wc];
        // every neighbour is read (rows across the boundary read in-bounds ring
        // words) so that the reads issue together; missing faces add nothing
        const T lps = s[sc][PS][wl], lmu = s[sc][MU][wl], lp = s[sc][P][wl], lphi = s[sc][PHI][wl];
        const T rps = s[sc][PS][wr], rmu = s[sc][MU][wr], rp = s[sc][P][wr], rphi = s[sc][PHI][wr];
        const T dps = s[sd][PS][wc], dmu = s[sd][MU][wc], dp = s[sd][P][wc], dphi = s[sd][PHI][wc];
        const T ups = s[su][PS][wc], umu = s[su][MU][wc], up = s[su][P][wc], uphi = s[su][PHI][wc];
        const T phit = s[sc][PHI][wc];
        Sums q4{0, 0, 0, 0, 0, 0, 0, 0};
        if (XIN) {
            face(q4, psc, lps, lmu, lp, lphi);
            face(q4, psc, rps, rmu, rp, rphi);
        } else {
            face_if(q4, gx > 0, psc, lps, lmu, lp, lphi);
            face_if(q4, gx < nx - 1, psc, rps, rmu, rp, rphi);
        }
        if (r > 0) face(q4, psc, dps, dmu, dp, dphi);
        if (r < ny - 1) face(q4, psc, ups, umu, up, uphi);
        const int nf = XIN ? 2 + (r > 0 ? 1 : 0) + (r < ny - 1 ? 1 : 0) : q4.nf;
        const T fnf = T(nf);
        const T inv_nf = nf == 4 ? T(0.25) : (nf == 3 ? T(1) / T(3) : (nf == 2 ? T(0.5) : T(1)));
        // select values, not member addresses, so that the pairs stay in registers
        auto pick = [&](int k) {
            if (k < 0) return T(0);
            const T va = o[k].a, vb = o[k].b;
            return e ? vb : va;
        };
        const T psi = pick(O::PSI);
        const T f0 = pick(O::F0);
        const T f1 = pick(O::F1);
        const T f2 = pick(O::F2);
        const T base = pick(O::B);
        const T dchi = dnonlin<T, CORR>(phit, psi, base);
        const T chi = nonlin<T, CORR>(phit, psi, base);
        const T b1 = f0 + lam * q4.smmu + lam * q4.sap;
        const T b2 = f1 + chi - dchi * phit - kap * q4.sphi;
        const T b3 = f2 - lam * q4.sp - lam * gam * q4.samu;
        const T ared = lam * (fnf + gam * (q4.sa2 - q4.sa * q4.sa * inv_nf));
        const T b1r = b1 + (q4.sa * inv_nf) * b3;
        const T bb = dchi + kap * fnf;
        const T inv_det = recip_ge1(T(1) + ared * bb);
        const T mun = (b2 + bb * b1r) * inv_det;
        s[sc][PHI][wc] = (b1r - ared * b2) * inv_det;
        s[sc][MU][wc] = mun;
        s[sc][P][wc] = -(b3 * inv_lam + gam * q4.sa * mun) * inv_nf;
    };

    // ---- rows (k2, k2 + 1) leave: write-back, residual, restriction / norm -----------
    // thread -> fine cell: lanes 0-15 even columns of row k2, 16-31 odd columns,
    // 32-47 / 48-63 the same in row k2 + 1; coarse column cl = 16 wave + (lane & 15),
    // so the four children of a coarse cell are lanes l, l ^ 16, l ^ 32, l ^ 48.
    const int odx = (lane >> 4) & 1, ody = lane >> 5;
    const int ocl = wave * 16 + (lane & 15);
    const int oc = 2 * ocl + odx;
    const int ogx = x0 + oc;
    const bool own_col = oc >= kStripHX && oc < kStripHX + kStripWO && ogx < nx;
    const bool ocol = ogx >= 0 && ogx < nx;
    // the coarse cell of lane column ocl (its children's columns are owned together)
    const bool own_coarse = 2 * ocl >= kStripHX && 2 * ocl < kStripHX + kStripWO && x0 + 2 * ocl < nx;
    const int orow = (ody ? nx : 0) + ogx;             // offset of the cell from row k2
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    T lo[NO];                                          // own data of the leaving cell

    auto load_leave = [&](int k2) {
        const int r = k2 + ody;
        const int g = (ocol && r >= 0 && r < ny) ? k2 * nx + orow : 0;
#pragma unroll
        for (int k = 0; k < NO; ++k) lo[k] = gload(own_src[k], g);
    };

    auto leave = [&](int k2) {
        const int r = k2 + ody;
        const bool own = own_col && r < ny;
        // ring slots of rows k2 - 1 .. k2 + 2 (uniform), then per lane row
        const int sl_m = (k2 + RING - 1) % RING, sl_0 = k2 % RING;
        const int sl_1 = (k2 + 1) % RING, sl_2 = (k2 + 2) % RING;
        const int sc = ody ? sl_1 : sl_0;
        const int wc = col(oc);
        const T phic = s[sc][PHI][wc], muc = s[sc][MU][wc], pc = s[sc][P][wc];
        const int g = k2 * nx + orow;
        if (own) {
            gstore_stream(L.phi_alt, g, phic);
            gstore_stream(L.mu_alt, g, muc);
            gstore_stream(L.p_alt, g, pc);
        }
        if (EPI == 0) return;
        // computed by every lane (halo lanes read clamped, in-bounds words);
        // only owned cells are stored or summed
        const int sd = ody ? sl_0 : sl_m, su = ody ? sl_2 : sl_1;
        const int wl = col(oc > 0 ? oc - 1 : 0), wr = col(oc < kW - 1 ? oc + 1 : kW - 1);
        const T psc = s[sc][PS][wc];
        T nps[4], nmu[4], np[4], nphi[4];
        const int nsl[4] = {sc, sc, sd, su};
        const int nw[4] = {wl, wr, wc, wc};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            nps[k] = s[nsl[k]][PS][nw[k]];
            nmu[k] = s[nsl[k]][MU][nw[k]];
            np[k] = s[nsl[k]][P][nw[k]];
            nphi[k] = s[nsl[k]][PHI][nw[k]];
        }
        T smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
        auto rface = [&](int k) {
            const T a = T(0.5) * (psc + nps[k]);
            const T m = T(1) + gam * a * a;
            const T dmu = nmu[k] - muc;
            const T dp = np[k] - pc;
            smm += m * dmu;
            sap += a * dp;
            sphi += nphi[k] - phic;
            sp += dp;
            samu += a * dmu;
        };
        if (xin && k2 > 0 && k2 + 2 < ny) {
#pragma unroll
            for (int k = 0; k < 4; ++k) rface(k);
        } else {
            const bool nh[4] = {ogx > 0, ogx < nx - 1, r > 0, r < ny - 1};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T s0 = smm, s1 = sap, s2 = sphi, s3 = sp, s4 = samu;
                rface(k);
                smm = nh[k] ? smm : s0;
                sap = nh[k] ? sap : s1;
                sphi = nh[k] ? sphi : s2;
                sp = nh[k] ? sp : s3;
                samu = nh[k] ? samu : s4;
            }
        }
        const T psi = lo[O::PSI];
        const T f0 = lo[O::F0];
        const T f1 = lo[O::F1];
        const T f2 = O::F2 < 0 ? T(0) : lo[O::F2 < 0 ? 0 : O::F2];
        const T bg = O::B < 0 ? T(0) : lo[O::B < 0 ? 0 : O::B];
        const T r0 = f0 - (phic - lam * smm - lam * sap);
        const T r1 = f1 - (muc - nonlin<T, CORR>(phic, psi, bg) + kap * sphi);
        const T r2 = f2 - (lam * sp + lam * gam * samu);
        if (EPI == 2) {
            if (own) {
                acc[0] += double(r0) * double(r0);
                acc[1] += double(r1) * double(r1);
                acc[2] += double(r2) * double(r2);
                acc[3] += double(pc);
            }
            return;
        }
        // EPI 1: sum the children, columns (lanes l, l ^ 16) first, then rows
        // (l, l ^ 32), two fields per exchange.  Rows of 16 lanes after the
        // column sums: (r0, r1, r0, r1), (r2, phi, r2, phi), (mu, p, mu, p),
        // the last two rows being fine row k2 + 1; after the row sums:
        // (r0, r1, r2, phi) and (mu, p, mu, p) for coarse column ocl.
        const T w = T(0.25);
        const T c01 = swap_sum(r0, r1, false);
        const T c2u = swap_sum(r2, phic, false);
        const T cmp = swap_sum(muc, pc, false);
        const T q1 = swap_sum(c01, c2u, true) * w;
        const T q2 = swap_sum(cmp, cmp, true) * w;
        const T qb = CORR ? rows_sum(rows_sum(bg, false), true) * w : T(0);
        if (own_coarse && k2 < ny) {
            const int cgi = (k2 >> 1) * C.nx + (x0 >> 1) + ocl;
            // one store per destination, each by the lanes of one row
            // (separate conditions, so that no store is merged into one
            // through a selected address)
            const int rw = lane >> 4;
            if (rw == 0) gstore(C.fr0, cgi, q1);
            if (rw == 1) gstore(C.fr1, cgi, q1);
            if (rw == 2) gstore(C.fr2, cgi, q1);
            if (rw == 3) gstore(C.phi, cgi, q1);
            if (rw == 3) gstore(C.ub0, cgi, q1);
            if (rw == 0) gstore(C.mu, cgi, q2);
            if (rw == 1) gstore(C.p, cgi, q2);
            if (rw == 2) gstore(C.ub1, cgi, q2);
            if (rw == 3) gstore(C.ub2, cgi, q2);
            if (CORR && rw == 0) gstore(C.b, cgi, qb);
        }
    };

    // ---- the pipeline -------------------------------------------------------------------
    // Ring rows wait in two register banks of kD rows each.  At the first
    // iteration that drains bank b the other bank is refilled with the rows
    // needed kD iterations later, after the wait for the row being stored,
    // so that this wait does not cover them.  (Global stores share the
    // vector-memory counter with loads: after the leave's stores the compiler
    // waits for every outstanding load at the next use of loaded data.)  A
    // phase wave's own data for iteration t + KO is loaded at iteration t
    // into the slot it just used.
    {
        T v[2], vc[2], vb[2];
        load_row(v, vc, vb, ys);
        store_row(v, vc, vb, ys);
        load_row(v, vc, vb, ys + 1);
        store_row(v, vc, vb, ys + 1);
    }
#pragma unroll
    for (int u = 0; u < kD; ++u) load_row(rv[0][u], rc[0][u], rb[0][u], ys + 2 + u);
    if (wave < NPH) {
#pragma unroll
        for (int i = 0; i < KO; ++i) load_own(od[i], ys + i - 2 * wave);
    }
    if (EPI != 0) load_leave(y0);
    __syncthreads();

    const int t_last = y0 + 2 * ((y1 - y0 + 1) / 2 - 1) + LAG;   // the last pair of rows leaves
    for (int tb = ys; tb <= t_last; tb += kU) {
#pragma unroll
        for (int i = 0; i < kU; ++i) {
            const int b = i / kD, u = i % kD;
            const int t = tb + i;
            if (t > t_last) goto drained;
            const int k2 = t - LAG;
            const bool lv = k2 >= y0 && ((k2 - y0) & 1) == 0;
            store_row(rv[b][u], rc[b][u], rb[b][u], t + 2);
            if (u == 0) {
#pragma unroll
                for (int w = 0; w < kD; ++w)
                    load_row(rv[b ^ 1][w], rc[b ^ 1][w], rb[b ^ 1][w], t + 2 + kD + w);
            }
            if (wave < NPH) {
                if (xin)
                    phase(std::true_type{}, wave, t - 2 * wave, od[i % KO]);
                else
                    phase(std::false_type{}, wave, t - 2 * wave, od[i % KO]);
                load_own(od[i % KO], t + KO - 2 * wave);
            }
            if (lv) {
                leave(k2);
                // own data of the next pair of rows to leave, two iterations ahead
                if (EPI != 0) load_leave(k2 + 2);
            }
            __syncthreads();
        }
    }
drained:

    if (EPI != 2) return;
    // per-task partial sums in a fixed order
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < 4; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    __shared__ double red[4][kThreads / 64];
    if (lane == 0)
        for (int c = 0; c < 4; ++c) red[c][wave] = acc[c];
    __syncthreads();
    if (tid == 0)
        for (int c = 0; c < 4; ++c) {
            double sum = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) sum += red[c][w];
            gstore(partial, task * kPartialStride + c, sum);
        }
}

template <typename T, bool LEVEL0, int NS, int EPI, bool PRO, bool CORR, bool ZERO = false>
void launch_one(const Batch<T>& b, const StripTask* t, int nt, double* partial, hipStream_t st) {
    hipLaunchKernelGGL((k_stream2d<T, LEVEL0, NS, EPI, PRO, CORR, ZERO>), dim3(nt), dim3(kThreads),
                       0, st, b, t, nt, partial);
}

}  // namespace

template <>
void launch_stream2d<double>(const Batch<double>& b, const StripTask* t, int nt, bool level0,
                             int ns, int epi, bool pro, bool zero, double* partial, hipStream_t st) {
    (void)zero;
    if (nt <= 0) return;
#define CHHS_STRIP_CASE(L0, NS, EPI, PRO)                                         \
    if (level0 == L0 && ns == NS && epi == EPI && pro == PRO) {                   \
        launch_one<double, L0, NS, EPI, PRO, false>(b, t, nt, partial, st);       \
        return;                                                                   \
    }
#define CHHS_STRIP_PRO(L0, NS, EPI) CHHS_STRIP_CASE(L0, NS, EPI, false) CHHS_STRIP_CASE(L0, NS, EPI, true)
#define CHHS_STRIP_EPI(L0, NS) CHHS_STRIP_PRO(L0, NS, 0) CHHS_STRIP_PRO(L0, NS, 1) CHHS_STRIP_PRO(L0, NS, 2)
    CHHS_STRIP_EPI(true, 1)
    CHHS_STRIP_EPI(true, 2)
    CHHS_STRIP_EPI(false, 1)
    CHHS_STRIP_EPI(false, 2)
#undef CHHS_STRIP_EPI
#undef CHHS_STRIP_PRO
#undef CHHS_STRIP_CASE
}

template <>
void launch_stream2d<float>(const Batch<float>& b, const StripTask* t, int nt, bool level0, int ns,
                            int epi, bool pro, bool zero, double* partial, hipStream_t st) {
    (void)level0;
    if (nt <= 0) return;
    if (zero) {
        if (pro || epi == 2) return;
#define CHHS_STRIP_ZERO(NS, EPI)                                                  \
    if (ns == NS && epi == EPI) {                                                 \
        launch_one<float, false, NS, EPI, false, true, true>(b, t, nt, partial, st); \
        return;                                                                   \
    }
        CHHS_STRIP_ZERO(1, 0)
        CHHS_STRIP_ZERO(1, 1)
        CHHS_STRIP_ZERO(2, 0)
        CHHS_STRIP_ZERO(2, 1)
#undef CHHS_STRIP_ZERO
        return;
    }
#define CHHS_STRIP_CASE(NS, EPI, PRO)                                             \
    if (ns == NS && epi == EPI && pro == PRO) {                                   \
        launch_one<float, false, NS, EPI, PRO, true>(b, t, nt, partial, st);      \
        return;                                                                   \
    }
    CHHS_STRIP_CASE(1, 0, false)
    CHHS_STRIP_CASE(1, 0, true)
    CHHS_STRIP_CASE(1, 1, false)
    CHHS_STRIP_CASE(2, 0, false)
    CHHS_STRIP_CASE(2, 0, true)
    CHHS_STRIP_CASE(2, 1, false)
#undef CHHS_STRIP_CASE
}

}  // namespace chhs
