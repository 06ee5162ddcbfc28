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
// The kernel is out of place: it reads u = (phi, mu, p) from copy b.cur and
// writes the owned cells into the other copy.
//
// Optional fused parts, as in the tiled kernel:
//   PRO    u += P(u_c - ub_c) applied while loading (halo included).
//   EPI 1  residual R = f - N(u) on the owned cells restricted by cell
//          averaging: u_c = ub_c = R u, f_c = R R on level + 1 (copy b.cur_c).
//   EPI 2  per-task partial sums of R_phi^2, R_mu^2, R_p^2 and p.
//   CORR   correction form of the mixed-precision inner solve.
#include "chhs_cell.hpp"

namespace chhs {
namespace {

constexpr int kW = kStripW;          // region columns: one pair per lane of a wave
constexpr int kHalf = kW / 2;
constexpr int kThreads = 256;        // four waves
constexpr int kD = 2;                // rows per register bank of loads in flight

// Field slots of the LDS ring.  On the finest level f_phi = phi^m (slot PSI)
// and f_p = 0 are implied.
template <bool LEVEL0, bool CORR>
struct Slots {
    static constexpr int PHI = 0, MU = 1, P = 2, PS = 3, PSI = 4, F1 = 5;
    static constexpr int F0 = LEVEL0 ? PSI : 6;
    static constexpr int F2 = LEVEL0 ? -1 : 7;
    static constexpr int B = CORR ? (LEVEL0 ? 6 : 8) : -1;
    static constexpr int N = 6 + (LEVEL0 ? 0 : 2) + (CORR ? 1 : 0);
};

// LDS word of region column c within a row: even columns, then odd columns.
__device__ __forceinline__ int col(int c) { return (c & 1) * kHalf + (c >> 1); }

template <typename T, bool LEVEL0, int NS, int EPI, bool PRO, bool CORR>
__global__ __launch_bounds__(kThreads) void k_stream2d(Batch<T> bt,
                                                       const StripTask* __restrict__ tasks,
                                                       int ntasks, double* partial) {
    using S = Slots<LEVEL0, CORR>;
    constexpr int NF = S::N;
    constexpr int X = EPI ? 1 : 0;
    constexpr int H = X + 2 * NS;          // halo rows
    constexpr int NPH = 2 * NS;            // phases = waves with phase work
    constexpr int LAG = 4 * NS + 1;        // rows (t - LAG, t - LAG + 1) leave at iteration t
    constexpr int RING = 4 * NS + 5;       // rows t - LAG - 1 .. t + 2 are live
    constexpr int JL = (NF + 1) / 2;       // fields a thread loads per row
    __shared__ T s[RING][NF][kW];

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

    // ---- loader: thread owns region column lc, fields 2 j + half -------------------
    // lanes 0-31 of a wave take even columns, 32-63 odd ones: a load covers 64
    // consecutive values of a row and a store 2 x 32 consecutive LDS words
    const int half = wave >> 1;
    const int lc = 2 * ((lane & 31) + 32 * (wave & 1)) + (lane >> 5);
    const int lgx = x0 + lc;
    const bool lcol = lgx >= 0 && lgx < nx;
    const T* src[JL];
#pragma unroll
    for (int j = 0; j < JL; ++j) {
        const T* fp[2];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int f = 2 * j + hh;
            const T* p = nullptr;
            if (f == S::PHI) p = L.phi;
            if (f == S::MU) p = L.mu;
            if (f == S::P) p = L.p;
            if (f == S::PS) p = L.pstar;
            if (f == S::PSI) p = L.psi;
            if (f == S::F1) p = L.f1;
            if (!LEVEL0 && f == S::F0) p = L.f0;
            if (!LEVEL0 && f == S::F2) p = L.f2;
            if (CORR && f == S::B) p = L.b;
            fp[hh] = p;
        }
        // a missing field (odd field count) reads the other half's and drops it
        src[j] = (half && fp[1] != nullptr) ? fp[1] : fp[0];
    }
    // prolongation sources for the u fields (slots 0..2): j = 0 (phi | mu), j = 1 (p)
    const T* csrc[2] = {nullptr, nullptr};
    const T* cbar[2] = {nullptr, nullptr};
    if (PRO) {
        csrc[0] = half ? C.mu : C.phi;
        cbar[0] = half ? C.ub1 : C.ub0;
        csrc[1] = C.p;
        cbar[1] = C.ub2;
    }
    T rv[2][kD][JL], rc[2][kD][2], rb[2][kD][2];

    // Loads are unconditional (cells outside the loaded rows or the grid read
    // element 0 and are dropped) so that the compiler can wait for exactly the
    // row it stores, not for every load in flight.
    auto load_row = [&](T (&v)[JL], T (&vc)[2], T (&vb)[2], int r) {
        const bool ok = lcol && r >= ys && r < ye;
        const int g = ok ? r * nx + lgx : 0;
#pragma unroll
        for (int j = 0; j < JL; ++j) v[j] = gload(src[j], g);
        if (PRO) {
            const int cg = ok ? (r >> 1) * C.nx + (lgx >> 1) : 0;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                vc[j] = gload(csrc[j], cg);
                vb[j] = gload(cbar[j], cg);
            }
        }
    };
    auto store_row = [&](const T (&v)[JL], const T (&vc)[2], const T (&vb)[2], int r) {
        if (r >= ye) return;
        const bool ok = lcol;
        const int slot = r % RING;
        const int w = col(lc);
#pragma unroll
        for (int j = 0; j < JL; ++j) {
            const int f = 2 * j + half;
            if (f >= NF) continue;
            T x = ok ? v[j] : T(0);
            if (PRO && j < 2 && f < 3 && ok) x += vc[j] - vb[j];
            s[slot][f][w] = x;
        }
    };

    const T lam = L.lam, kap = L.kap, gam = L.gamma;
    const T inv_lam = T(1) / lam;

    // ---- phase q on row r: the collective update of the q & 1 colored cells ----------
    auto phase = [&](int q, int r) {
        if (r < rlo || r > rhi) return;
        const int e = (r & 1) ^ (q & 1);           // pair member with this color
        const int c = 2 * lane + e;
        const int gx = x0 + c;
        if (c < 1 || c > kW - 2 || gx < 0 || gx >= nx) return;
        const int sc = r % RING, sd = (r + RING - 1) % RING, su = (r + 1) % RING;
        const int wc = col(c);
        const T psc = s[sc][S::PS][wc];
        // the four neighbours (x - 1, x + 1, y - 1, y + 1) are read without
        // branches so that their LDS reads issue together; a neighbour across
        // the boundary reads in-bounds ring words whose terms the selects drop
        const int nsl[4] = {sc, sc, sd, su};
        const int nw[4] = {col(c - 1), col(c + 1), wc, wc};
        const bool nh[4] = {gx > 0, gx < nx - 1, r > 0, r < ny - 1};
        T vps[4], vmu[4], vp[4], vphi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            vps[k] = s[nsl[k]][S::PS][nw[k]];
            vmu[k] = s[nsl[k]][S::MU][nw[k]];
            vp[k] = s[nsl[k]][S::P][nw[k]];
            vphi[k] = s[nsl[k]][S::PHI][nw[k]];
        }
        int nf = 0;
        T sa = 0, sa2 = 0, smmu = 0, sphi = 0, sp = 0, sap = 0, samu = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T a = T(0.5) * (psc + vps[k]);
            const T m = T(1) + gam * a * a;
            const bool h = nh[k];
            nf += h ? 1 : 0;
            sa = h ? sa + a : sa;
            sa2 = h ? sa2 + a * a : sa2;
            smmu = h ? smmu + m * vmu[k] : smmu;
            sphi = h ? sphi + vphi[k] : sphi;
            sp = h ? sp + vp[k] : sp;
            sap = h ? sap + a * vp[k] : sap;
            samu = h ? samu + a * vmu[k] : samu;
        }
        const T fnf = T(nf);
        const T inv_nf = nf == 4 ? T(0.25) : (nf == 3 ? T(1) / T(3) : (nf == 2 ? T(0.5) : T(1)));
        const T phit = s[sc][S::PHI][wc];
        const T psi = s[sc][S::PSI][wc];
        const T f0 = s[sc][S::F0][wc];
        const T f1 = s[sc][S::F1][wc];
        const T f2 = LEVEL0 ? T(0) : s[sc][S::F2 < 0 ? 0 : S::F2][wc];
        const T base = CORR ? s[sc][S::B < 0 ? 0 : S::B][wc] : T(0);
        const T dchi = dnonlin<T, CORR>(phit, psi, base);
        const T chi = nonlin<T, CORR>(phit, psi, base);
        const T b1 = f0 + lam * smmu + lam * sap;
        const T b2 = f1 + chi - dchi * phit - kap * sphi;
        const T b3 = f2 - lam * sp - lam * gam * samu;
        const T ared = lam * (fnf + gam * (sa2 - sa * sa * inv_nf));
        const T b1r = b1 + (sa * inv_nf) * b3;
        const T bb = dchi + kap * fnf;
        const T inv_det = T(1) / (T(1) + ared * bb);
        const T mun = (b2 + bb * b1r) * inv_det;
        s[sc][S::PHI][wc] = (b1r - ared * b2) * inv_det;
        s[sc][S::MU][wc] = mun;
        s[sc][S::P][wc] = -(b3 * inv_lam + gam * sa * mun) * inv_nf;
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
    double acc[4] = {0.0, 0.0, 0.0, 0.0};

    auto leave = [&](int k2) {
        const int r = k2 + ody;
        const bool own = own_col && r < ny;
        const int sc = r % RING;
        const int wc = col(oc);
        const T phic = s[sc][S::PHI][wc], muc = s[sc][S::MU][wc], pc = s[sc][S::P][wc];
        const int g = r * nx + ogx;
        if (own) {
            gstore(L.phi_alt, g, phic);
            gstore(L.mu_alt, g, muc);
            gstore(L.p_alt, g, pc);
        }
        if (EPI == 0) return;
        // computed by every lane (halo lanes read clamped, in-bounds words);
        // only owned cells are stored or summed
        T r0 = 0, r1 = 0, r2 = 0, bg = 0;
        {
            const T psc = s[sc][S::PS][wc];
            const int nsl[4] = {sc, sc, (r + RING - 1) % RING, (r + 1) % RING};
            const int nw[4] = {col(oc > 0 ? oc - 1 : 0), col(oc < kW - 1 ? oc + 1 : kW - 1), wc, wc};
            const bool nh[4] = {ogx > 0, ogx < nx - 1, r > 0, r < ny - 1};
            T vps[4], vmu[4], vp[4], vphi[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                vps[k] = s[nsl[k]][S::PS][nw[k]];
                vmu[k] = s[nsl[k]][S::MU][nw[k]];
                vp[k] = s[nsl[k]][S::P][nw[k]];
                vphi[k] = s[nsl[k]][S::PHI][nw[k]];
            }
            T smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T a = T(0.5) * (psc + vps[k]);
                const T m = T(1) + gam * a * a;
                const T dmu = vmu[k] - muc;
                const T dp = vp[k] - pc;
                const bool h = nh[k];
                smm = h ? smm + m * dmu : smm;
                sap = h ? sap + a * dp : sap;
                sphi = h ? sphi + (vphi[k] - phic) : sphi;
                sp = h ? sp + dp : sp;
                samu = h ? samu + a * dmu : samu;
            }
            const T psi = s[sc][S::PSI][wc];
            const T f0 = s[sc][S::F0][wc];
            const T f1 = s[sc][S::F1][wc];
            const T f2 = LEVEL0 ? T(0) : s[sc][S::F2 < 0 ? 0 : S::F2][wc];
            bg = CORR ? s[sc][S::B < 0 ? 0 : S::B][wc] : T(0);
            r0 = f0 - (phic - lam * smm - lam * sap);
            r1 = f1 - (muc - nonlin<T, CORR>(phic, psi, bg) + kap * sphi);
            r2 = f2 - (lam * sp + lam * gam * samu);
        }
        if (EPI == 2) {
            if (own) {
                acc[0] += double(r0) * double(r0);
                acc[1] += double(r1) * double(r1);
                acc[2] += double(r2) * double(r2);
                acc[3] += double(pc);
            }
            return;
        }
        // EPI 1: sum the children, columns first, then rows
        T v[7] = {r0, r1, r2, phic, muc, pc, bg};
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            if (!CORR && c == 6) continue;
            v[c] += __shfl_xor(v[c], 16, 64);
            v[c] += __shfl_xor(v[c], 32, 64);
        }
        if (own && odx == 0 && ody == 0) {
            const int cgi = (k2 >> 1) * C.nx + (ogx >> 1);
            const T w = T(0.25);
            gstore(C.phi, cgi, v[3] * w);
            gstore(C.ub0, cgi, v[3] * w);
            gstore(C.mu, cgi, v[4] * w);
            gstore(C.ub1, cgi, v[4] * w);
            gstore(C.p, cgi, v[5] * w);
            gstore(C.ub2, cgi, v[5] * w);
            gstore(C.f0, cgi, v[0] * w);
            gstore(C.f1, cgi, v[1] * w);
            gstore(C.f2, cgi, v[2] * w);
            if (CORR) gstore(C.b, cgi, v[6] * w);
        }
    };

    // ---- the pipeline -------------------------------------------------------------------
    // Loaded rows wait in two register banks of kD rows each.  At the first
    // iteration that drains bank b the other bank is refilled with the rows
    // needed kD iterations later, after the wait for the row being stored:
    // whatever the compiler waits for at the loop head, the loads it waits
    // for were issued kD iterations earlier.
    {
        T v[JL], vc[2], vb[2];
        load_row(v, vc, vb, ys);
        store_row(v, vc, vb, ys);
        load_row(v, vc, vb, ys + 1);
        store_row(v, vc, vb, ys + 1);
    }
#pragma unroll
    for (int u = 0; u < kD; ++u) load_row(rv[0][u], rc[0][u], rb[0][u], ys + 2 + u);
    __syncthreads();

    const int t_last = y0 + 2 * ((y1 - y0 + 1) / 2 - 1) + LAG;   // the last pair of rows leaves
    for (int tb = ys; tb <= t_last; tb += 2 * kD) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int u = 0; u < kD; ++u) {
                const int t = tb + b * kD + u;
                if (t > t_last) goto drained;
                store_row(rv[b][u], rc[b][u], rb[b][u], t + 2);
                if (u == 0) {
#pragma unroll
                    for (int w = 0; w < kD; ++w)
                        load_row(rv[b ^ 1][w], rc[b ^ 1][w], rb[b ^ 1][w], t + 2 + kD + w);
                }
                if (wave < NPH) phase(wave, t - 2 * wave);
                const int k2 = t - LAG;
                if (k2 >= y0 && ((k2 - y0) & 1) == 0) leave(k2);
                __syncthreads();
            }
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

template <typename T, bool LEVEL0, int NS, int EPI, bool PRO, bool CORR>
void launch_one(const Batch<T>& b, const StripTask* t, int nt, double* partial, hipStream_t st) {
    hipLaunchKernelGGL((k_stream2d<T, LEVEL0, NS, EPI, PRO, CORR>), dim3(nt), dim3(kThreads), 0,
                       st, b, t, nt, partial);
}

}  // namespace

template <>
void launch_stream2d<double>(const Batch<double>& b, const StripTask* t, int nt, bool level0,
                             int ns, int epi, bool pro, double* partial, hipStream_t st) {
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
                            int epi, bool pro, double* partial, hipStream_t st) {
    (void)level0;
    if (nt <= 0) return;
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
