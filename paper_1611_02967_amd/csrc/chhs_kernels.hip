// Cell kernels of the FAS solve for one step of the CHHS scheme (2.4)-(2.7).
//
// One thread per cell; neighbours are read straight from global memory.  The
// stencils are the App. A.2 operators with boundary faces left out (zero flux,
// App. A.1).  The arithmetic is FP64 throughout.
#include "chhs_cell.hpp"

namespace chhs {
namespace {

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_setup(Level<double> L, const double* __restrict__ phi_prev,
                        const double* __restrict__ phi_cur, const double* __restrict__ mu,
                        const double* __restrict__ p, double q) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L.n) return;
    int i, j, k;
    decode<DIM>(idx, L.nx, L.ny, i, j, k);
    const double pm = phi_prev[idx];
    const double pc = phi_cur[idx];
    double lap = 0.0;
    for_each_nb<DIM>(i, j, k, L.nx, L.ny, L.nz, idx, [&](int nb) { lap += phi_prev[nb] - pm; });
    const double ps = 1.5 * pc - 0.5 * pm;           // phi_*, (2.4)
    L.pstar[idx] = ps;
    L.psi[idx] = pc;
    L.f0[idx] = pc;                                   // (2.5): phi^m
    L.f1[idx] = -ps - q * lap;                        // (2.6): -phi_* - eps^2/4 Lap phi^{m-1}
    L.f2[idx] = 0.0;                                  // (2.7)
    L.phi[idx] = pc;                                  // initial guess phi^m
    L.mu[idx] = mu[idx];
    L.p[idx] = p[idx];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict_frozen(Level<double> F, Level<double> C) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= C.n) return;
    int ci, cj, ck;
    decode<DIM>(idx, C.nx, C.ny, ci, cj, ck);
    double sps = 0.0, sph = 0.0;
    for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int f = ((2 * ck + dz) * F.ny + (2 * cj + dy)) * F.nx + 2 * ci + dx;
                sps += F.pstar[f];
                sph += F.psi[f];
            }
    const double w = DIM == 3 ? 0.125 : 0.25;
    C.pstar[idx] = sps * w;
    C.psi[idx] = sph * w;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_smooth(Level<double> L, int color) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L.n) return;
    int i, j, k;
    decode<DIM>(idx, L.nx, L.ny, i, j, k);
    if (((i + j + k) & 1) != color) return;
    double phi, mu, p;
    cell_solve<DIM>(L, idx, i, j, k, phi, mu, p);
    L.phi[idx] = phi;
    L.mu[idx] = mu;
    L.p[idx] = p;
}

// Per coarse cell: u_c = R u, ub_c = u_c, f_c = R(f - N(u)) (the N_c(u_c) part
// is added by k_coarse_rhs once all of u_c is written).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_restrict_residual(Level<double> F, Level<double> C) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= C.n) return;
    int ci, cj, ck;
    decode<DIM>(idx, C.nx, C.ny, ci, cj, ck);
    double su0 = 0, su1 = 0, su2 = 0, sr0 = 0, sr1 = 0, sr2 = 0;
#pragma unroll 1
    for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int fi = 2 * ci + dx, fj = 2 * cj + dy, fk = 2 * ck + dz;
                const int f = (fk * F.ny + fj) * F.nx + fi;
                double n0, n1, n2;
                cell_operator<DIM>(F, f, fi, fj, fk, n0, n1, n2);
                sr0 += F.f0[f] - n0;
                sr1 += F.f1[f] - n1;
                sr2 += F.f2[f] - n2;
                su0 += F.phi[f];
                su1 += F.mu[f];
                su2 += F.p[f];
            }
    const double w = DIM == 3 ? 0.125 : 0.25;
    C.phi[idx] = C.ub0[idx] = su0 * w;
    C.mu[idx] = C.ub1[idx] = su1 * w;
    C.p[idx] = C.ub2[idx] = su2 * w;
    C.f0[idx] = sr0 * w;
    C.f1[idx] = sr1 * w;
    C.f2[idx] = sr2 * w;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_coarse_rhs(Level<double> C) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= C.n) return;
    int i, j, k;
    decode<DIM>(idx, C.nx, C.ny, i, j, k);
    double n0, n1, n2;
    cell_operator<DIM>(C, idx, i, j, k, n0, n1, n2);
    C.f0[idx] += n0;
    C.f1[idx] += n1;
    C.f2[idx] += n2;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_prolong(Level<double> F, Level<double> C) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= F.n) return;
    int i, j, k;
    decode<DIM>(idx, F.nx, F.ny, i, j, k);
    const int c = ((k >> 1) * C.ny + (j >> 1)) * C.nx + (i >> 1);
    F.phi[idx] += C.phi[c] - C.ub0[c];
    F.mu[idx] += C.mu[c] - C.ub1[c];
    F.p[idx] += C.p[c] - C.ub2[c];
}

// ---- deterministic reductions --------------------------------------------------

template <int NC>
__device__ __forceinline__ void block_sum_store(double (&v)[NC], double* out) {
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < NC; ++c) v[c] += __shfl_xor(v[c], off, 64);
    __shared__ double sh[NC][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < NC; ++c) sh[c][wid] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) s += sh[c][w];
            out[c] = s;
        }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_residual_partials(Level<double> L, double* partial) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < L.n;
         idx += gridDim.x * blockDim.x) {
        int i, j, k;
        decode<DIM>(idx, L.nx, L.ny, i, j, k);
        double n0, n1, n2;
        cell_operator<DIM>(L, idx, i, j, k, n0, n1, n2);
        const double r0 = L.f0[idx] - n0, r1 = L.f1[idx] - n1, r2 = L.f2[idx] - n2;
        v[0] += r0 * r0;
        v[1] += r1 * r1;
        v[2] += r2 * r2;
        v[3] += L.p[idx];
    }
    block_sum_store<4>(v, partial + blockIdx.x * kPartialStride);
}

__global__ __launch_bounds__(kBlock) void k_reduce_final(const double* partial, int nblocks, int ncomp, double* out) {
    double v[8];
    for (int c = 0; c < 8; ++c) v[c] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int c = 0; c < 8; ++c)
            if (c < ncomp) v[c] += partial[b * kPartialStride + c];
    double res[8];
    block_sum_store<8>(v, res);
    if (threadIdx.x == 0)
        for (int c = 0; c < ncomp; ++c) out[c] = res[c];
}

__global__ __launch_bounds__(kBlock) void k_shift_p(double* p, int n, const double* sum_p) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    p[idx] -= sum_p[0] / double(n);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_energy_partials(int nx, int ny, int nz, const double* __restrict__ phi,
                                  const double* __restrict__ q, const double* __restrict__ mu,
                                  const double* __restrict__ p, const double* __restrict__ ps,
                                  double gamma, double* partial) {
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double vmax = 0.0;
    const int n = nx * ny * nz;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += gridDim.x * blockDim.x) {
        int i, j, k;
        decode<DIM>(idx, nx, ny, i, j, k);
        const double f = phi[idx];
        const double d = f - q[idx];
        v[0] += f;
        v[1] += f * f;
        v[2] += f * f * f * f;
        v[4] += d * d;
        vmax = fmax(vmax, fabs(f));
        // forward faces only: every interior face counted once
        auto face = [&](int nb) {
            const double df = phi[nb] - f;
            const double dd = (phi[nb] - q[nb]) - d;
            v[3] += df * df;
            v[5] += dd * dd;
            if (mu != nullptr) {
                const double dm = mu[nb] - mu[idx];
                const double a = 0.5 * (ps[idx] + ps[nb]);
                const double u = -(p[nb] - p[idx]) - gamma * a * dm;
                v[6] += dm * dm;
                v[7] += u * u;
            }
        };
        if (i < nx - 1) face(idx + 1);
        if (j < ny - 1) face(idx + nx);
        if (DIM == 3 && k < nz - 1) face(idx + nx * ny);
    }
    double* out = partial + blockIdx.x * kPartialStride;
    block_sum_store<8>(v, out);
    for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off, 64));
    __shared__ double shm[kBlock / 64];
    if ((threadIdx.x & 63) == 0) shm[threadIdx.x >> 6] = vmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) m = fmax(m, shm[w]);
        out[8] = m;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_energy(const double* partial, int nblocks, double* out) {
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double vmax = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        for (int c = 0; c < 8; ++c) v[c] += partial[b * kPartialStride + c];
        vmax = fmax(vmax, partial[b * kPartialStride + 8]);
    }
    double res[8];
    block_sum_store<8>(v, res);
    for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off, 64));
    __shared__ double shm[kBlock / 64];
    if ((threadIdx.x & 63) == 0) shm[threadIdx.x >> 6] = vmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) m = fmax(m, shm[w]);
        for (int c = 0; c < 8; ++c) out[c] = res[c];
        out[8] = m;
    }
}

inline int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }
inline int partial_blocks(int n) {
    const int b = blocks_for(n);
    return b < kMaxPartials ? b : kMaxPartials;
}

}  // namespace

#define CHHS_DISPATCH(dim, KERNEL, GRID, ...)                                         \
    do {                                                                              \
        if ((dim) == 2)                                                               \
            hipLaunchKernelGGL(KERNEL<2>, dim3(GRID), dim3(kBlock), 0, st, __VA_ARGS__); \
        else                                                                          \
            hipLaunchKernelGGL(KERNEL<3>, dim3(GRID), dim3(kBlock), 0, st, __VA_ARGS__); \
    } while (0)

void launch_setup(int dim, const Level<double>& L, const double* phi_prev, const double* phi_cur,
                  const double* mu, const double* p, double q, hipStream_t st) {
    CHHS_DISPATCH(dim, k_setup, blocks_for(L.n), L, phi_prev, phi_cur, mu, p, q);
}

void launch_restrict_frozen(int dim, const Level<double>& F, const Level<double>& C,
                            hipStream_t st) {
    CHHS_DISPATCH(dim, k_restrict_frozen, blocks_for(C.n), F, C);
}

void launch_smooth(int dim, const Level<double>& L, int color, hipStream_t st) {
    CHHS_DISPATCH(dim, k_smooth, blocks_for(L.n), L, color);
}

void launch_restrict_residual(int dim, const Level<double>& F, const Level<double>& C,
                              hipStream_t st) {
    CHHS_DISPATCH(dim, k_restrict_residual, blocks_for(C.n), F, C);
}

void launch_coarse_rhs(int dim, const Level<double>& C, hipStream_t st) {
    CHHS_DISPATCH(dim, k_coarse_rhs, blocks_for(C.n), C);
}

void launch_prolong(int dim, const Level<double>& F, const Level<double>& C, hipStream_t st) {
    CHHS_DISPATCH(dim, k_prolong, blocks_for(F.n), F, C);
}

int launch_residual_partials(int dim, const Level<double>& L, double* partial, hipStream_t st) {
    const int nb = partial_blocks(L.n);
    CHHS_DISPATCH(dim, k_residual_partials, nb, L, partial);
    return nb;
}

void launch_reduce_final(const double* partial, int nblocks, int ncomp, double* out,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, partial, nblocks, ncomp, out);
}

void launch_shift_p(const Level<double>& L, const double* sum_p, hipStream_t st) {
    hipLaunchKernelGGL(k_shift_p, dim3(blocks_for(L.n)), dim3(kBlock), 0, st, L.p, L.n, sum_p);
}

int launch_energy_partials(int dim, int nx, int ny, int nz, const double* phi, const double* q,
                           const double* mu, const double* p, const double* pstar, double gamma,
                           double* partial, hipStream_t st) {
    const int nb = partial_blocks(nx * ny * nz);
    CHHS_DISPATCH(dim, k_energy_partials, nb, nx, ny, nz, phi, q, mu, p, pstar, gamma, partial);
    return nb;
}

void launch_reduce_energy(const double* partial, int nblocks, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(kBlock), 0, st, partial, nblocks, out);
}

}  // namespace chhs
