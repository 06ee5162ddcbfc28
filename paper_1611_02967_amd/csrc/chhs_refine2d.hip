// The FP64 refinement step of the mixed-precision path on 2D finest levels,
// batched over instances: u' = u + e, the residual R = f - N(u') of
// (2.5)-(2.7) (the pressure row times s), R and b = phi' rounded to FP32 for the
// next inner correction cycle, and the partial sums of R^2 and p' of each task.
// It is the same arithmetic per cell as the per-cell refinement kernel; the
// layout of the work is what differs (row marching, below).
#include "chhs_cell.hpp"

namespace chhs {
namespace {

__device__ __forceinline__ int xcd_block() {
    const int n = int(gridDim.x), bid = int(blockIdx.x);
    const int q8 = n / 8, rem = n % 8;
    const int xcd = bid % 8, jj = bid / 8;
    return xcd * q8 + (xcd < rem ? xcd : rem) + jj;
}

// Row marching.  A wave owns a
// window of kMarchW columns (lane l: the pair of columns 2 l, 2 l + 1 of the
// window) and a segment [y0, y1) of rows of one instance (a StripTask whose sx
// is the window) and walks up the segment holding u' = u + e and phi_* of the
// rows below, at and above the current one in registers: each row of every
// field is read once, y neighbours come from registers and x neighbours from
// the adjacent lanes (lane 0 and lane 63 read the cell beyond the window with
// one extra load per field).  The arithmetic per cell is that of
// k_mixed_residual (faces in the order x - 1, x + 1, y - 1, y + 1); each wave
// writes the partial sums of its task.
constexpr int kMarchW = kMarchCols;
constexpr int kMarchWaves = 4;      // waves per block, each with a task of its own

__global__ __launch_bounds__(kMarchWaves * 64) void k_mixed_residual_rows(
    Batch<double> b64, Batch<float> b32, const StripTask* __restrict__ t, int nt, int add,
    const int* was_active, double* partial) {
    typedef double D2 __attribute__((ext_vector_type(2)));
    typedef float F2 __attribute__((ext_vector_type(2)));
    const int lane = int(threadIdx.x) & 63;
    const int task = xcd_block() * kMarchWaves + (int(threadIdx.x) >> 6);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (task < nt) {
        const StripTask tk = t[task];
        const Level<double> L = make_view(b64.desc[tk.inst * kMaxLevels], b64.cur);
        const int nx = L.nx, ny = L.ny;
        const int ca = tk.sx * kMarchW + 2 * lane;          // column of the pair's first cell
        const bool live = ca < nx;                           // nx is even: pairs are whole
        const int cal = live ? ca : 0;
        const int y0 = tk.y0, y1 = tk.y1;
        if (b64.active != nullptr && b64.active[tk.inst] == 0) {
            // an instance that has just converged keeps its iterate in both copies
            if (add && live && (was_active == nullptr || was_active[tk.inst] != 0))
                for (int r = y0; r < y1; ++r) {
                    const int h = (r * nx + ca) >> 1;
                    gstore(reinterpret_cast<D2*>(L.phi_alt), h, gload(reinterpret_cast<const D2*>(L.phi), h));
                    gstore(reinterpret_cast<D2*>(L.mu_alt), h, gload(reinterpret_cast<const D2*>(L.mu), h));
                    gstore(reinterpret_cast<D2*>(L.p_alt), h, gload(reinterpret_cast<const D2*>(L.p), h));
                }
        } else {
            const Level<float> E = make_view(b32.desc[tk.inst * kMaxLevels], b32.cur);
            // the cell beyond the window for lanes 0 and 63, the lane's own cell
            // for the others (a load of lines the pair loads already fetch)
            const int ce = lane == 0 ? ca - 1 : (lane == 63 ? ca + 2 : ca);
            const int cel = (ce >= 0 && ce < nx) ? ce : cal;
            struct Raw {
                D2 ph, mu, p, ps;
                F2 e0, e1, e2;
                double xph, xmu, xp, xps;
                float xe0, xe1, xe2;
            };
            // u' = u + e and phi_* of a pair and of the edge cell
            struct Row {
                double pa, pb, ma, mb, qa, qb, sa, sb;
                double xph, xmu, xp, xps;
            };
            auto load = [&](int r, Raw& w) {
                const int rr = r < 0 ? 0 : (r >= ny ? ny - 1 : r);   // clamped rows are not used
                const int h = (rr * nx + cal) >> 1;
                const int g = rr * nx + cel;
                w.ph = gload(reinterpret_cast<const D2*>(L.phi), h);
                w.mu = gload(reinterpret_cast<const D2*>(L.mu), h);
                w.p = gload(reinterpret_cast<const D2*>(L.p), h);
                w.ps = gload(reinterpret_cast<const D2*>(L.pstar), h);
                w.xph = gload(L.phi, g);
                w.xmu = gload(L.mu, g);
                w.xp = gload(L.p, g);
                w.xps = gload(L.pstar, g);
                if (add) {
                    w.e0 = gload(reinterpret_cast<const F2*>(E.phi), h);
                    w.e1 = gload(reinterpret_cast<const F2*>(E.mu), h);
                    w.e2 = gload(reinterpret_cast<const F2*>(E.p), h);
                    w.xe0 = gload(E.phi, g);
                    w.xe1 = gload(E.mu, g);
                    w.xe2 = gload(E.p, g);
                }
            };
            auto finish = [&](const Raw& w, Row& u) {
                u.pa = w.ph.x;
                u.pb = w.ph.y;
                u.ma = w.mu.x;
                u.mb = w.mu.y;
                u.qa = w.p.x;
                u.qb = w.p.y;
                u.sa = w.ps.x;
                u.sb = w.ps.y;
                u.xph = w.xph;
                u.xmu = w.xmu;
                u.xp = w.xp;
                u.xps = w.xps;
                if (add) {
                    u.pa += double(w.e0.x);
                    u.pb += double(w.e0.y);
                    u.ma += double(w.e1.x);
                    u.mb += double(w.e1.y);
                    u.qa += double(w.e2.x);
                    u.qb += double(w.e2.y);
                    u.xph += double(w.xe0);
                    u.xmu += double(w.xe1);
                    u.xp += double(w.xe2);
                }
            };
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
            auto resid = [&](const Sums& s, double ph, double mu, double ps, double f,
                             double& r0, double& r1, double& r2) {
                r0 = ps - (ph - L.lam * s.smm - L.lam * s.sap);
                r1 = f - (mu - nonlin<double, false>(ph, ps, 0.0) + L.kap * s.sphi);
                r2 = -(L.lam * s.sp + L.lam * L.gamma * s.samu);
            };
            // row r from the rows below (D), at (C) and above (U) it
            auto row = [&](int r, const Row& D, const Row& C, const Row& U, D2 psi, D2 f1) {
                // x neighbours: the previous lane's second cell, the next lane's first
                double lph = __shfl_up(C.pb, 1, 64), lmu = __shfl_up(C.mb, 1, 64);
                double lp = __shfl_up(C.qb, 1, 64), lps = __shfl_up(C.sb, 1, 64);
                double rph = __shfl_down(C.pa, 1, 64), rmu = __shfl_down(C.ma, 1, 64);
                double rp = __shfl_down(C.qa, 1, 64), rps = __shfl_down(C.sa, 1, 64);
                if (lane == 0) {
                    lph = C.xph;
                    lmu = C.xmu;
                    lp = C.xp;
                    lps = C.xps;
                }
                if (lane == 63) {
                    rph = C.xph;
                    rmu = C.xmu;
                    rp = C.xp;
                    rps = C.xps;
                }
                const bool hd = r > 0, hu = r < ny - 1;
                Sums sa, sb;
                face(sa, ca > 0, C.pa, C.ma, C.qa, C.sa, lph, lmu, lp, lps);
                face(sa, true, C.pa, C.ma, C.qa, C.sa, C.pb, C.mb, C.qb, C.sb);
                face(sa, hd, C.pa, C.ma, C.qa, C.sa, D.pa, D.ma, D.qa, D.sa);
                face(sa, hu, C.pa, C.ma, C.qa, C.sa, U.pa, U.ma, U.qa, U.sa);
                face(sb, true, C.pb, C.mb, C.qb, C.sb, C.pa, C.ma, C.qa, C.sa);
                face(sb, ca + 2 < nx, C.pb, C.mb, C.qb, C.sb, rph, rmu, rp, rps);
                face(sb, hd, C.pb, C.mb, C.qb, C.sb, D.pb, D.mb, D.qb, D.sb);
                face(sb, hu, C.pb, C.mb, C.qb, C.sb, U.pb, U.mb, U.qb, U.sb);
                double ra0, ra1, ra2, rb0, rb1, rb2;
                resid(sa, C.pa, C.ma, psi.x, f1.x, ra0, ra1, ra2);
                resid(sb, C.pb, C.mb, psi.y, f1.y, rb0, rb1, rb2);
                if (!live) return;
                const int h = (r * nx + ca) >> 1;
                gstore(reinterpret_cast<D2*>(L.phi_alt), h, D2{C.pa, C.pb});
                gstore(reinterpret_cast<D2*>(L.mu_alt), h, D2{C.ma, C.mb});
                gstore(reinterpret_cast<D2*>(L.p_alt), h, D2{C.qa, C.qb});
                gstore(reinterpret_cast<F2*>(E.f0), h, F2{float(ra0), float(rb0)});
                gstore(reinterpret_cast<F2*>(E.f1), h, F2{float(ra1), float(rb1)});
                gstore(reinterpret_cast<F2*>(E.f2), h, F2{float(ra2), float(rb2)});
                gstore(reinterpret_cast<F2*>(E.b), h, F2{float(C.pa), float(C.pb)});
                v[0] += ra0 * ra0 + rb0 * rb0;
                v[1] += ra1 * ra1 + rb1 * rb1;
                v[2] += ra2 * ra2 + rb2 * rb2;
                v[3] += C.qa + C.qb;
            };
            auto own = [&](int r, D2& psi, D2& f1) {
                const int rr = r < ny ? r : ny - 1;
                const int h = (rr * nx + cal) >> 1;
                psi = gload_stream(reinterpret_cast<const D2*>(L.psi), h);
                f1 = gload_stream(reinterpret_cast<const D2*>(L.f1), h);
            };
            Raw w;
            Row D, C, U;
            load(y0 - 1, w);
            finish(w, D);
            load(y0, w);
            finish(w, C);
            load(y0 + 1, w);
            finish(w, U);
            Raw wn;
            load(y0 + 2, wn);           // two rows ahead of the one being formed
            D2 psi, f1;
            own(y0, psi, f1);
            int r = y0;
            // rows whose next-but-one row is still inside the segment's reach
            for (; r + 3 <= y1; ++r) {
                Raw wf;
                load(r + 3, wf);
                D2 npsi, nf1;
                own(r + 1, npsi, nf1);
                row(r, D, C, U, psi, f1);
                D = C;
                C = U;
                finish(wn, U);
                wn = wf;
                psi = npsi;
                f1 = nf1;
            }
            for (; r < y1; ++r) {
                D2 npsi, nf1;
                own(r + 1, npsi, nf1);
                row(r, D, C, U, psi, f1);
                D = C;
                C = U;
                finish(wn, U);
                psi = npsi;
                f1 = nf1;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < 4; ++c) v[c] += __shfl_xor(v[c], off, 64);
    if (lane == 0 && task < nt)
        for (int c = 0; c < 4; ++c) partial[task * kPartialStride + c] = v[c];
}

}  // namespace

void launch_mixed_residual_rows(const Batch<double>& b64, const Batch<float>& b32,
                                const StripTask* t, int nt, int add, const int* was_active,
                                double* partial, hipStream_t st) {
    if (nt <= 0) return;
    const int blocks = (nt + kMarchWaves - 1) / kMarchWaves;
    hipLaunchKernelGGL(k_mixed_residual_rows, dim3(blocks), dim3(kMarchWaves * 64), 0, st, b64,
                       b32, t, nt, add, was_active, partial);
}

}  // namespace chhs
