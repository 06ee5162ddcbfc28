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

// Calls fn(nb) for every neighbour across an interior face of cell (i, j, k).
template <int DIM, typename Fn>
__device__ __forceinline__ void for_each_nb(int i, int j, int k, int nx, int ny, int nz,
                                            int idx, Fn&& fn) {
    if (i > 0) fn(idx - 1);
    if (i < nx - 1) fn(idx + 1);
    if (j > 0) fn(idx - nx);
    if (j < ny - 1) fn(idx + nx);
    if (DIM == 3) {
        const int sz = nx * ny;
        if (k > 0) fn(idx - sz);
        if (k < nz - 1) fn(idx + sz);
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
    for_each_nb<DIM>(i, j, k, L.nx, L.ny, L.nz, idx, [&](int nb) {
        const T a = T(0.5) * (psc + L.pstar[nb]);
        const T m = T(1) + L.gamma * a * a;
        const T dmu = L.mu[nb] - muc;
        const T dp = L.p[nb] - pc;
        smm += m * dmu;
        sap += a * dp;
        sphi += L.phi[nb] - phic;
        sp += dp;
        samu += a * dmu;
    });
    const T psi = L.psi[idx];
    const T chi = nonlin<T, CORR>(phic, psi, CORR ? L.b[idx] : T(0));
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
template <int DIM, typename T, bool CORR = false>
__device__ __forceinline__ void cell_solve(const Level<T>& L, int idx, int i, int j, int k,
                                           T& phi_o, T& mu_o, T& p_o) {
    const T psc = L.pstar[idx];
    T nf = 0, sa = 0, sa2 = 0, smmu = 0, sphi = 0, sp = 0, sap = 0, samu = 0;
    for_each_nb<DIM>(i, j, k, L.nx, L.ny, L.nz, idx, [&](int nb) {
        const T a = T(0.5) * (psc + L.pstar[nb]);
        const T m = T(1) + L.gamma * a * a;
        const T munb = L.mu[nb];
        const T pnb = L.p[nb];
        nf += T(1);
        sa += a;
        sa2 += a * a;
        smmu += m * munb;
        sphi += L.phi[nb];
        sp += pnb;
        sap += a * pnb;
        samu += a * munb;
    });
    const T phit = L.phi[idx];
    const T psi = L.psi[idx];
    const T base = CORR ? L.b[idx] : T(0);
    const T dchi = dnonlin<T, CORR>(phit, psi, base);
    const T chi = nonlin<T, CORR>(phit, psi, base);
    const T b1 = L.f0[idx] + L.lam * smmu + L.lam * sap;
    const T b2 = L.f1[idx] + chi - dchi * phit - L.kap * sphi;
    const T b3 = L.f2[idx] - L.lam * sp - L.lam * L.gamma * samu;
    const T ared = L.lam * (nf + L.gamma * (sa2 - sa * sa / nf));
    const T b1r = b1 + (sa / nf) * b3;
    const T bb = dchi + L.kap * nf;
    const T det = T(1) + ared * bb;
    phi_o = (b1r - ared * b2) / det;
    mu_o = (b2 + bb * b1r) / det;
    p_o = -(b3 + L.lam * L.gamma * sa * mu_o) / (L.lam * nf);
}

}  // namespace chhs
