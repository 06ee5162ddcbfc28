// Coarse tail of the V-cycle in one workgroup.
//
// Every level from the tail's top level down to the coarsest grid is staged in
// LDS (11 fields per level), and the V-cycle over those levels -- smoothing,
// residual + restriction, FAS coarse right-hand side, the coarsest-grid
// smoothing steps, prolongation + correction -- runs inside a single
// workgroup with a barrier between dependent phases.  Launch latency of the
// small levels disappears; the arithmetic is the shared cell code, so the
// result equals the per-level kernels'.
#include "chhs_cell.hpp"

namespace chhs {
namespace {

constexpr int kTailThreads = 1024;

template <typename T>
struct TailArgs {
    Level<T> lv[kMaxTailLevels];
    int nlev;
    int nu1, nu2, coarse_sweeps;
};

template <int DIM, typename T>
__device__ void tail_smooth(const Level<T>& L) {
    for (int color = 0; color < 2; ++color) {
        for (int idx = threadIdx.x; idx < L.n; idx += blockDim.x) {
            int i, j, k;
            decode<DIM>(idx, L.nx, L.ny, i, j, k);
            if (((i + j + k) & 1) != color) continue;
            T phi, mu, p;
            cell_solve<DIM>(L, idx, i, j, k, phi, mu, p);
            L.phi[idx] = phi;
            L.mu[idx] = mu;
            L.p[idx] = p;
        }
        __syncthreads();
    }
}

template <int DIM, typename T>
__device__ void tail_restrict(const Level<T>& F, const Level<T>& C) {
    for (int idx = threadIdx.x; idx < C.n; idx += blockDim.x) {
        int ci, cj, ck;
        decode<DIM>(idx, C.nx, C.ny, ci, cj, ck);
        T su0 = 0, su1 = 0, su2 = 0, sr0 = 0, sr1 = 0, sr2 = 0;
#pragma unroll 1
        for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll 1
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const int fi = 2 * ci + dx, fj = 2 * cj + dy, fk = 2 * ck + dz;
                    const int f = (fk * F.ny + fj) * F.nx + fi;
                    T n0, n1, n2;
                    cell_operator<DIM>(F, f, fi, fj, fk, n0, n1, n2);
                    sr0 += F.f0[f] - n0;
                    sr1 += F.f1[f] - n1;
                    sr2 += F.f2[f] - n2;
                    su0 += F.phi[f];
                    su1 += F.mu[f];
                    su2 += F.p[f];
                }
        const T w = DIM == 3 ? T(0.125) : T(0.25);
        C.phi[idx] = C.ub0[idx] = su0 * w;
        C.mu[idx] = C.ub1[idx] = su1 * w;
        C.p[idx] = C.ub2[idx] = su2 * w;
        C.f0[idx] = sr0 * w;
        C.f1[idx] = sr1 * w;
        C.f2[idx] = sr2 * w;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < C.n; idx += blockDim.x) {
        int i, j, k;
        decode<DIM>(idx, C.nx, C.ny, i, j, k);
        T n0, n1, n2;
        cell_operator<DIM>(C, idx, i, j, k, n0, n1, n2);
        C.f0[idx] += n0;
        C.f1[idx] += n1;
        C.f2[idx] += n2;
    }
    __syncthreads();
}

template <int DIM, typename T>
__device__ void tail_prolong(const Level<T>& F, const Level<T>& C) {
    for (int idx = threadIdx.x; idx < F.n; idx += blockDim.x) {
        int i, j, k;
        decode<DIM>(idx, F.nx, F.ny, i, j, k);
        const int c = ((k >> 1) * C.ny + (j >> 1)) * C.nx + (i >> 1);
        F.phi[idx] += C.phi[c] - C.ub0[c];
        F.mu[idx] += C.mu[c] - C.ub1[c];
        F.p[idx] += C.p[c] - C.ub2[c];
    }
    __syncthreads();
}

// LDS view of tail level l: the global descriptor with its 11 arrays placed
// one after another in LDS, levels one after another.
template <typename T>
__device__ __forceinline__ Level<T> lds_view(const TailArgs<T>& a, int l, T* base) {
    size_t off = 0;
    for (int k = 0; k < l; ++k) off += size_t(11) * a.lv[k].n;
    Level<T> v = a.lv[l];
    const int n = v.n;
    T* b = base + off;
    v.phi = b;
    v.mu = b + n;
    v.p = b + 2 * n;
    v.ub0 = b + 3 * n;
    v.ub1 = b + 4 * n;
    v.ub2 = b + 5 * n;
    v.f0 = b + 6 * n;
    v.f1 = b + 7 * n;
    v.f2 = b + 8 * n;
    v.pstar = b + 9 * n;
    v.psi = b + 10 * n;
    return v;
}

template <int DIM, typename T>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailArgs<T> a) {
    extern __shared__ __align__(16) unsigned char tail_lds[];
    T* base = reinterpret_cast<T*>(tail_lds);

    // stage the top level's iterate and right-hand side, and every level's
    // frozen data
    {
        const Level<T>& G = a.lv[0];
        const Level<T> S = lds_view(a, 0, base);
        for (int idx = threadIdx.x; idx < G.n; idx += blockDim.x) {
            S.phi[idx] = G.phi[idx];
            S.mu[idx] = G.mu[idx];
            S.p[idx] = G.p[idx];
            S.f0[idx] = G.f0[idx];
            S.f1[idx] = G.f1[idx];
            S.f2[idx] = G.f2[idx];
        }
        for (int l = 0; l < a.nlev; ++l) {
            const Level<T> V = lds_view(a, l, base);
            for (int idx = threadIdx.x; idx < V.n; idx += blockDim.x) {
                V.pstar[idx] = a.lv[l].pstar[idx];
                V.psi[idx] = a.lv[l].psi[idx];
            }
        }
    }
    __syncthreads();

    const int last = a.nlev - 1;
    for (int l = 0; l < last; ++l) {
        const Level<T> F = lds_view(a, l, base);
        for (int s = 0; s < a.nu1; ++s) tail_smooth<DIM>(F);
        tail_restrict<DIM>(F, lds_view(a, l + 1, base));
    }
    {
        const Level<T> B = lds_view(a, last, base);
        for (int s = 0; s < a.coarse_sweeps; ++s) tail_smooth<DIM>(B);
    }
    for (int l = last - 1; l >= 0; --l) {
        const Level<T> F = lds_view(a, l, base);
        tail_prolong<DIM>(F, lds_view(a, l + 1, base));
        for (int s = 0; s < a.nu2; ++s) tail_smooth<DIM>(F);
    }

    const Level<T>& G = a.lv[0];
    const Level<T> S = lds_view(a, 0, base);
    for (int idx = threadIdx.x; idx < G.n; idx += blockDim.x) {
        G.phi[idx] = S.phi[idx];
        G.mu[idx] = S.mu[idx];
        G.p[idx] = S.p[idx];
    }
}

}  // namespace

size_t tail_lds_bytes(const int* cells, int nlev, size_t elem) {
    size_t b = 0;
    for (int l = 0; l < nlev; ++l) b += size_t(cells[l]) * 11 * elem;
    return b;
}

template <typename T>
int prepare_tail(int dim, size_t lds_bytes) {
    hipError_t e;
    if (dim == 2)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tail<2, T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
    else
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tail<3, T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
    return e == hipSuccess ? 0 : -1;
}

template <typename T>
void launch_tail(int dim, const Level<T>* levels, int nlev, int nu1, int nu2, int coarse_sweeps,
                 size_t lds_bytes, hipStream_t st) {
    TailArgs<T> a{};
    for (int l = 0; l < nlev; ++l) a.lv[l] = levels[l];
    a.nlev = nlev;
    a.nu1 = nu1;
    a.nu2 = nu2;
    a.coarse_sweeps = coarse_sweeps;
    if (dim == 2)
        hipLaunchKernelGGL((k_tail<2, T>), dim3(1), dim3(kTailThreads), lds_bytes, st, a);
    else
        hipLaunchKernelGGL((k_tail<3, T>), dim3(1), dim3(kTailThreads), lds_bytes, st, a);
}

template int prepare_tail<double>(int, size_t);
template void launch_tail<double>(int, const Level<double>*, int, int, int, int, size_t,
                                  hipStream_t);

}  // namespace chhs
