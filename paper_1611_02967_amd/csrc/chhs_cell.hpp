// Cell arithmetic shared by the per-cell kernels and the single-workgroup
// coarse tail: the residual operator N(u) of (2.5)-(2.7) and the collective
// (phi, mu, p) update at one cell.  Level pointers may address global memory
// or LDS.
//
// CORR selects the correction form used by the mixed-precision inner solve:
// the unknown is a correction e to a base state b (held in Level::psi's
// companion b), and chi(phi, psi) is replaced by
//   g(e) = chi(b + e, psi) - chi(b, psi) = e (3b^2 + 2b psi + psi^2 + (3b + psi) e + e^2) / 4,
// written in product form so that no two nearly equal cubes are subtracted,
// with g'(e) = chi'(b + e, psi).  Every other term of N is linear in u and is
// unchanged.
#pragma once

#include "chhs_internal.hpp"

namespace chhs {

// Global-memory access through pointers read from device-side descriptors.
// Without the address-space cast they would be flat accesses, which the
// hardware counts together with LDS accesses, so that every wait for an LDS
// read would also wait for outstanding global loads and stores.  The element
// index becomes a 32-bit unsigned byte offset (every field is below 4 GiB), so
// that a wave-uniform base stays in scalar registers and the address is one
// 32-bit vector register.
template <typename T>
__device__ __forceinline__ T gload(const T* p, int i) {
    const unsigned off = unsigned(i) * unsigned(sizeof(T));
    return *(const __attribute__((address_space(1))) T*)((const __attribute__((address_space(1))) char*)p + off);
}
template <typename T>
__device__ __forceinline__ void gstore(T* p, int i, T v) {
    const unsigned off = unsigned(i) * unsigned(sizeof(T));
    *(__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)p + off) = v;
}
// Streaming variants (non-temporal hint).  Loads: data read once per launch,
// kept from displacing data that the launch reads again through L2.  Stores:
// results written once, without the line fills that partially written lines
// otherwise cause (measured on the strip kernel's write-back: less total
// traffic although the written bytes grow).
template <typename T>
__device__ __forceinline__ T gload_stream(const T* p, int i) {
    const unsigned off = unsigned(i) * unsigned(sizeof(T));
    return __builtin_nontemporal_load(
        (const __attribute__((address_space(1))) T*)((const __attribute__((address_space(1))) char*)p + off));
}
template <typename T>
__device__ __forceinline__ void gstore_stream(T* p, int i, T v) {
    const unsigned off = unsigned(i) * unsigned(sizeof(T));
    __builtin_nontemporal_store(
        v, (__attribute__((address_space(1))) T*)((__attribute__((address_space(1))) char*)p + off));
}

template <int DIM>
__device__ __forceinline__ void decode(int idx, int nx, int ny, int& i, int& j, int& k) {
    i = idx % nx;
    const int r = idx / nx;
    if (DIM == 2) {
        j = r;
        k = 0;
    } else {
        j = r % ny;
        k = r / ny;
    }
}

// Calls fn(has, nb) for the 2 DIM faces of cell (i, j, k) in the order x - 1,
// x + 1, y - 1, y + 1 (, z - 1, z + 1): has = the face is interior, nb = the
// neighbour's index (the cell's own index across a boundary face, so that
// every read stays in bounds).  Callers read every neighbour unconditionally,
// which lets all the reads be in flight together, and drop the terms of
// boundary faces with selects.
template <int DIM, typename Fn>
__device__ __forceinline__ void for_each_face(int i, int j, int k, int nx, int ny, int nz,
                                              int idx, Fn&& fn) {
    fn(i > 0, i > 0 ? idx - 1 : idx);
    fn(i < nx - 1, i < nx - 1 ? idx + 1 : idx);
    fn(j > 0, j > 0 ? idx - nx : idx);
    fn(j < ny - 1, j < ny - 1 ? idx + nx : idx);
    if (DIM == 3) {
        const int sz = nx * ny;
        fn(k > 0, k > 0 ? idx - sz : idx);
        fn(k < nz - 1, k < nz - 1 ? idx + sz : idx);
    }
}

// The nonlinear term of (2.6) at one cell and its derivative.
template <typename T, bool CORR>
__device__ __forceinline__ T nonlin(T x, T psi, T b) {
    if (CORR)
        return T(0.25) * x * (T(3) * b * b + T(2) * b * psi + psi * psi + (T(3) * b + psi) * x + x * x);
    return T(0.25) * (x * x + psi * psi) * (x + psi);
}
template <typename T, bool CORR>
__device__ __forceinline__ T dnonlin(T x, T psi, T b) {
    const T y = CORR ? b + x : x;
    return T(0.25) * (T(3) * y * y + T(2) * y * psi + psi * psi);
}

// Lane-row exchanges of gfx950 (VALU, no LDS traffic) summed: with rows of
// 16 lanes, v_permlane16_swap trades the odd rows of its first operand for
// the even rows of its second, and v_permlane32_swap the upper 32 lanes of the
// first for the lower 32 of the second.  Adding the two swapped registers gives
//   by32 = false: rows 0-3 hold x0 + x1, y0 + y1, x2 + x3, y2 + y3
//   by32 = true:  lanes 0-31 hold x_lo + x_hi, lanes 32-63 y_lo + y_hi
// (xi = x in row i, lane by lane), so one exchange sums two values across
// lanes l, l ^ 16 (or l ^ 32) at once.  With x = y every lane gets
// v + (v of lane l ^ 16 or ^ 32): rows_sum.  Every lane of the wave must be
// active.
__device__ __forceinline__ double swap_sum(double x, double y, bool by32) {
    const unsigned long long bx = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long by = __builtin_bit_cast(unsigned long long, y);
    const unsigned xl = unsigned(bx), xh = unsigned(bx >> 32);
    const unsigned yl = unsigned(by), yh = unsigned(by >> 32);
    unsigned a0, a1, c0, c1;
    if (by32) {
        const auto l = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        a0 = l[0], a1 = h[0], c0 = l[1], c1 = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        a0 = l[0], a1 = h[0], c0 = l[1], c1 = h[1];
    }
    const double a = __builtin_bit_cast(double, (unsigned long long)a0 | ((unsigned long long)a1 << 32));
    const double c = __builtin_bit_cast(double, (unsigned long long)c0 | ((unsigned long long)c1 << 32));
    return a + c;
}
__device__ __forceinline__ float swap_sum(float x, float y, bool by32) {
    const unsigned xb = __builtin_bit_cast(unsigned, x), yb = __builtin_bit_cast(unsigned, y);
    unsigned a, c;
    if (by32) {
        const auto r = __builtin_amdgcn_permlane32_swap(xb, yb, false, false);
        a = r[0], c = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(xb, yb, false, false);
        a = r[0], c = r[1];
    }
    return __builtin_bit_cast(float, a) + __builtin_bit_cast(float, c);
}
template <typename T>
__device__ __forceinline__ T rows_sum(T v, bool by32) { return swap_sum(v, v, by32); }

// 1 / x for x >= 1 (the determinant of the collective cell solve): the
// hardware reciprocal estimate refined by Newton steps r <- r + r (1 - x r),
// each of which squares the relative error: two in FP64, one in FP32.  Within
// an ulp or so of the quotient, at half the instructions of a correctly
// rounded division; every kernel uses this same sequence.
__device__ __forceinline__ double recip_ge1(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip_ge1(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

// Cell-centred bi/trilinear interpolation of the coarse correction cv - cb at
// fine cell (i, j, k) (coarse extents cnx, cny, cnz): along each axis 3/4 of
// the parent and 1/4 of the parent's neighbour towards the cell, the parent
// itself standing in beyond the boundary (even continuation, as the Neumann
// ghost cells continue a field), applied axis by axis in the order z, y, x.
template <int DIM, typename T>
__device__ __forceinline__ T bilinear_corr(const T* cv, const T* cb, int cnx, int cny, int cnz,
                                           int i, int j, int k) {
    const int pi = i >> 1, pj = j >> 1, pk = k >> 1;
    const int si = pi + ((i & 1) ? 1 : -1), sj = pj + ((j & 1) ? 1 : -1), sk = pk + ((k & 1) ? 1 : -1);
    const int ni = si < 0 ? 0 : (si >= cnx ? cnx - 1 : si);
    const int nj = sj < 0 ? 0 : (sj >= cny ? cny - 1 : sj);
    const int nk = sk < 0 ? 0 : (sk >= cnz ? cnz - 1 : sk);
    auto d = [&](int kk, int jj, int ii) {
        const int c = (kk * cny + jj) * cnx + ii;
        return cv[c] - cb[c];
    };
    if (DIM == 2) {
        const T t0 = T(0.75) * d(0, pj, pi) + T(0.25) * d(0, nj, pi);
        const T t1 = T(0.75) * d(0, pj, ni) + T(0.25) * d(0, nj, ni);
        return T(0.75) * t0 + T(0.25) * t1;
    }
    auto tz = [&](int jj, int ii) { return T(0.75) * d(pk, jj, ii) + T(0.25) * d(nk, jj, ii); };
    const T y0 = T(0.75) * tz(pj, pi) + T(0.25) * tz(nj, pi);
    const T y1 = T(0.75) * tz(pj, ni) + T(0.25) * tz(nj, ni);
    return T(0.75) * y0 + T(0.25) * y1;
}

// N(u) at one cell for the three rows of (2.5)-(2.7), the pressure row times s:
//   N_phi = phi - lam sum M_f (mu_nb - mu) - lam sum a_f (p_nb - p)
//   N_mu  = mu - chi(phi, psi) + kap sum (phi_nb - phi)
//   N_p   = lam sum (p_nb - p) + lam gamma sum a_f (mu_nb - mu)
// with a_f = (phi_*,c + phi_*,nb)/2 and M_f = 1 + gamma a_f^2.
template <int DIM, typename T, bool CORR = false>
__device__ __forceinline__ void cell_operator(const Level<T>& L, int idx, int i, int j, int k,
                                              T& n0, T& n1, T& n2) {
    const T phic = L.phi[idx], muc = L.mu[idx], pc = L.p[idx], psc = L.pstar[idx];
    T smm = 0, sap = 0, sphi = 0, sp = 0, samu = 0;
    for_each_face<DIM>(i, j, k, L.nx, L.ny, L.nz, idx, [&](bool h, int nb) {
        const T a = T(0.5) * (psc + L.pstar[nb]);
        const T m = T(1) + L.gamma * a * a;
        const T dmu = L.mu[nb] - muc;
        const T dp = L.p[nb] - pc;
        const T dphi = L.phi[nb] - phic;
        smm = h ? smm + m * dmu : smm;
        sap = h ? sap + a * dp : sap;
        sphi = h ? sphi + dphi : sphi;
        sp = h ? sp + dp : sp;
        samu = h ? samu + a * dmu : samu;
    });
    const T psi = L.psi[idx];
    const T chi = !CORR && L.order == 1 ? phic * phic * phic
                                        : nonlin<T, CORR>(phic, psi, CORR ? L.b[idx] : T(0));
    n0 = phic - L.lam * smm - L.lam * sap;
    n1 = muc - chi + L.kap * sphi;
    n2 = L.lam * sp + L.lam * L.gamma * samu;
}

// Collective (phi, mu, p) update of one cell with its neighbours frozen and chi
// linearised at the current phi (one local Newton step).  The three local rows
//   phi + lam SM mu + lam Sa p        = b1
//   -(chi' + kap nF) phi + mu         = b2
//   -lam gamma Sa mu - lam nF p       = b3
// are solved by eliminating p; the reduced 2x2 determinant is
// 1 + lam (nF + gamma (Sa2 - Sa^2/nF)) (chi' + kap nF) >= 1.
//
// Written with one reciprocal of the determinant (recip_ge1) and 1/nF by cases, in the
// same operation order as the tiled and row-streaming 2D kernels, so that
// every path performs the same update; kernels differ at most in which
// products the compiler fuses into multiply-adds, i.e. they agree to
// rounding.  inv_lam = 1 / lam.
// L0: the finest level of the plain form, whose right-hand side is f_phi =
// phi^m (psi) and f_p = 0 ((2.5), (2.7)): neither is loaded.
template <int DIM, typename T, bool CORR = false, bool L0 = false>
__device__ __forceinline__ void cell_solve(const Level<T>& L, int idx, int i, int j, int k,
                                           T inv_lam, T& phi_o, T& mu_o, T& p_o) {
    const T psc = L.pstar[idx];
    const T lam = L.lam, kap = L.kap, gam = L.gamma;
    int nf = 0;
    T sa = 0, sa2 = 0, smmu = 0, sphi = 0, sp = 0, sap = 0, samu = 0;
    for_each_face<DIM>(i, j, k, L.nx, L.ny, L.nz, idx, [&](bool h, int nb) {
        const T a = T(0.5) * (psc + L.pstar[nb]);
        const T m = T(1) + gam * a * a;
        const T munb = L.mu[nb];
        const T pnb = L.p[nb];
        const T phinb = L.phi[nb];
        nf += h ? 1 : 0;
        sa = h ? sa + a : sa;
        sa2 = h ? sa2 + a * a : sa2;
        smmu = h ? smmu + m * munb : smmu;
        sphi = h ? sphi + phinb : sphi;
        sp = h ? sp + pnb : sp;
        sap = h ? sap + a * pnb : sap;
        samu = h ? samu + a * munb : samu;
    });
    const T fnf = T(nf);
    const T inv_nf = nf == 6 ? T(1) / T(6)
                   : (nf == 5 ? T(1) / T(5)
                   : (nf == 4 ? T(0.25) : (nf == 3 ? T(1) / T(3) : (nf == 2 ? T(0.5) : T(1)))));
    const T phit = L.phi[idx];
    const T psi = L.psi[idx];
    const T base = CORR ? L.b[idx] : T(0);
    // the first-order step (order 1): chi(phi) = phi^3, implicit
    const bool cubic = !CORR && L.order == 1;
    const T dchi = cubic ? T(3) * phit * phit : dnonlin<T, CORR>(phit, psi, base);
    const T chi = cubic ? phit * phit * phit : nonlin<T, CORR>(phit, psi, base);
    const T b1 = (L0 ? psi : L.f0[idx]) + lam * smmu + lam * sap;
    const T b2 = L.f1[idx] + chi - dchi * phit - kap * sphi;
    const T b3 = (L0 ? T(0) : L.f2[idx]) - lam * sp - lam * gam * samu;
    const T ared = lam * (fnf + gam * (sa2 - sa * sa * inv_nf));
    const T b1r = b1 + (sa * inv_nf) * b3;
    const T bb = dchi + kap * fnf;
    const T inv_det = recip_ge1(T(1) + ared * bb);
    mu_o = (b2 + bb * b1r) * inv_det;
    phi_o = (b1r - ared * b2) * inv_det;
    p_o = -(b3 * inv_lam + gam * sa * mu_o) * inv_nf;
}

}  // namespace chhs
