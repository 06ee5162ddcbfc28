// Coarse tail of the V-cycle in one workgroup.
//
// One workgroup per instance.  Every level from the instance's tail level
// down to the coarsest grid is staged in LDS (11 fields per level), and the
// V-cycle over those levels -- smoothing,
// residual + restriction, FAS coarse right-hand side, the coarsest-grid
// smoothing steps, prolongation + correction -- runs inside a single
// workgroup with a barrier between dependent phases.  Launch latency of the
// small levels disappears; the arithmetic is the shared cell code, so the
// result equals the per-level kernels'.
#include "chhs_cell.hpp"

namespace chhs {
namespace {

constexpr int kTailThreads = 1024;

// (i, j, k) of cell idx of a tail level: a float reciprocal replaces the
// integer divisions; exact while idx < 2^20 (a tail level holds at most a few
// thousand cells), since (idx + 1/2) / n is never within 2^-21 of an integer.
template <int DIM>
__device__ __forceinline__ void tail_decode(int idx, int nx, int ny, float rnx, float rnxy, int& i,
                                            int& j, int& k) {
    if (DIM == 2) {
        j = int((float(idx) + 0.5f) * rnx);
        i = idx - j * nx;
        k = 0;
    } else {
        k = int((float(idx) + 0.5f) * rnxy);
        const int r = idx - k * nx * ny;
        j = int((float(r) + 0.5f) * rnx);
        i = r - j * nx;
    }
}

// In the FP32 correction form, levels of at most kWaveCells cells are worked
// by the first wave alone: its lanes take the cells with a stride of 64, and
// a wave-level fence replaces the workgroup barrier between dependent phases
// (LDS accesses of one wave are performed in the order issued), so the other
// waves do not take part (on the batch 0.4% per step; the FP64 tail built the
// same way needs more registers than its 1024-thread workgroup allows and
// was no faster).
constexpr int kWaveCells = 128;

// First work item and stride of a phase: the whole workgroup, or (W) the
// first wave's 64 lanes.
template <bool W>
__device__ __forceinline__ int phase_first() { return W ? int(threadIdx.x & 63) : int(threadIdx.x); }
template <bool W>
__device__ __forceinline__ int phase_stride() { return W ? 64 : int(blockDim.x); }
template <bool W>
__device__ __forceinline__ void phase_sync() {
    if (W) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int DIM, typename T, bool CORR, bool W = false>
__device__ void tail_smooth(const Level<T>& L) {
    const float rnx = 1.0f / float(L.nx), rnxy = 1.0f / float(L.nx * L.ny);
    const T inv_lam = T(1) / L.lam;
    const bool even = (L.nx & 1) == 0;
    const int hx = L.nx >> 1;
    const float rhx = 1.0f / float(hx > 0 ? hx : 1), rny = 1.0f / float(L.ny);
    for (int color = 0; color < 2; ++color) {
        if (even) {
            // thread q takes the q-th cell of the color: every active lane works
            #pragma unroll 1
            for (int q = phase_first<W>(); q < L.n / 2; q += phase_stride<W>()) {
                const int row = int((float(q) + 0.5f) * rhx);      // over (j, k)
                const int m = q - row * hx;
                int j = row, k = 0;
                if (DIM == 3) {
                    k = int((float(row) + 0.5f) * rny);
                    j = row - k * L.ny;
                }
                const int i = 2 * m + ((j + k + color) & 1);
                const int idx = row * L.nx + i;
                T phi, mu, p;
                cell_solve<DIM, T, CORR>(L, idx, i, j, k, inv_lam, phi, mu, p);
                L.phi[idx] = phi;
                L.mu[idx] = mu;
                L.p[idx] = p;
            }
        } else {
            #pragma unroll 1
            for (int idx = phase_first<W>(); idx < L.n; idx += phase_stride<W>()) {
                int i, j, k;
                tail_decode<DIM>(idx, L.nx, L.ny, rnx, rnxy, i, j, k);
                if (((i + j + k) & 1) != color) continue;
                T phi, mu, p;
                cell_solve<DIM, T, CORR>(L, idx, i, j, k, inv_lam, phi, mu, p);
                L.phi[idx] = phi;
                L.mu[idx] = mu;
                L.p[idx] = p;
            }
        }
        phase_sync<W>();
    }
}

template <int DIM, typename T, bool CORR, bool W = false>
__device__ void tail_restrict(const Level<T>& F, const Level<T>& C) {
    const float rnx = 1.0f / float(C.nx), rnxy = 1.0f / float(C.nx * C.ny);
    // one thread per (coarse cell, child): the 2^DIM children of a coarse cell
    // are consecutive lanes of one wave, summed by lane exchanges in the fixed
    // order ((c0 + c1) + (c2 + c3)) [+ the same for the upper four in 3D]
    constexpr int NCH = DIM == 3 ? 8 : 4;
    const int nwork = C.n * NCH;
    const int span = (nwork + 63) & ~63;               // whole waves take part
    #pragma unroll 1
    for (int q = phase_first<W>(); q < span; q += phase_stride<W>()) {
        const bool live = q < nwork;
        const int idx = live ? q / NCH : 0;
        const int ch = q % NCH;
        int ci, cj, ck;
        tail_decode<DIM>(idx, C.nx, C.ny, rnx, rnxy, ci, cj, ck);
        const int fi = 2 * ci + (ch & 1), fj = 2 * cj + ((ch >> 1) & 1), fk = 2 * ck + (ch >> 2);
        const int f = (fk * F.ny + fj) * F.nx + fi;
        T n0, n1, n2;
        cell_operator<DIM, T, CORR>(F, f, fi, fj, fk, n0, n1, n2);
        T v[7] = {F.f0[f] - n0, F.f1[f] - n1, F.f2[f] - n2, F.phi[f], F.mu[f], F.p[f],
                  CORR ? F.b[f] : T(0)};
#pragma unroll
        for (int c = 0; c < 7; ++c) {
            if (!CORR && c == 6) continue;
            v[c] += __shfl_xor(v[c], 1, 64);
            v[c] += __shfl_xor(v[c], 2, 64);
            if (DIM == 3) v[c] += __shfl_xor(v[c], 4, 64);
        }
        if (live && ch == 0) {
            const T w = DIM == 3 ? T(0.125) : T(0.25);
            if (CORR) C.b[idx] = v[6] * w;
            C.phi[idx] = C.ub0[idx] = v[3] * w;
            C.mu[idx] = C.ub1[idx] = v[4] * w;
            C.p[idx] = C.ub2[idx] = v[5] * w;
            C.f0[idx] = v[0] * w;
            C.f1[idx] = v[1] * w;
            C.f2[idx] = v[2] * w;
        }
    }
    phase_sync<W>();
    #pragma unroll 1
    for (int idx = phase_first<W>(); idx < C.n; idx += phase_stride<W>()) {
        int i, j, k;
        tail_decode<DIM>(idx, C.nx, C.ny, rnx, rnxy, i, j, k);
        T n0, n1, n2;
        cell_operator<DIM, T, CORR>(C, idx, i, j, k, n0, n1, n2);
        C.f0[idx] += n0;
        C.f1[idx] += n1;
        C.f2[idx] += n2;
    }
    phase_sync<W>();
}

template <int DIM, typename T, bool W = false>
__device__ void tail_prolong(const Level<T>& F, const Level<T>& C, bool bilinear) {
    const float rnx = 1.0f / float(F.nx), rnxy = 1.0f / float(F.nx * F.ny);
    #pragma unroll 1
    for (int idx = phase_first<W>(); idx < F.n; idx += phase_stride<W>()) {
        int i, j, k;
        tail_decode<DIM>(idx, F.nx, F.ny, rnx, rnxy, i, j, k);
        if (bilinear) {
            F.phi[idx] += bilinear_corr<DIM>(C.phi, C.ub0, C.nx, C.ny, C.nz, i, j, k);
            F.mu[idx] += bilinear_corr<DIM>(C.mu, C.ub1, C.nx, C.ny, C.nz, i, j, k);
            F.p[idx] += bilinear_corr<DIM>(C.p, C.ub2, C.nx, C.ny, C.nz, i, j, k);
            continue;
        }
        const int c = ((k >> 1) * C.ny + (j >> 1)) * C.nx + (i >> 1);
        F.phi[idx] += C.phi[c] - C.ub0[c];
        F.mu[idx] += C.mu[c] - C.ub1[c];
        F.p[idx] += C.p[c] - C.ub2[c];
    }
    phase_sync<W>();
}

// LDS view of tail level l (a level index of the instance, l >= tail): the
// level's descriptor with its 11 arrays (12 with the base state b of the
// correction form) placed one after another in LDS, levels one after another
// from the tail's top level.
template <typename T, bool CORR>
__device__ __forceinline__ Level<T> lds_view(const LevelDesc<T>* d, int tail, int l, T* base) {
    constexpr int NF = CORR ? 12 : 11;
    size_t off = 0;
    for (int k = tail; k < l; ++k) off += size_t(NF) * d[k].n;
    Level<T> v = make_view(d[l], 0);
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
    v.fr0 = v.fr1 = v.fr2 = nullptr;
    v.pstar = b + 9 * n;
    v.psi = b + 10 * n;
    v.b = CORR ? b + 11 * n : nullptr;
    v.phi_alt = v.mu_alt = v.p_alt = nullptr;
    return v;
}

template <int DIM, typename T, bool CORR>
__global__ __launch_bounds__(kTailThreads) void k_tail(const LevelDesc<T>* __restrict__ desc,
                                                       const InstInfo* __restrict__ info,
                                                       const int* __restrict__ insts,
                                                       const int* __restrict__ active,
                                                       unsigned cur_mask, CycleShape shape,
                                                       double* pend) {
    extern __shared__ __align__(16) unsigned char tail_lds[];
    T* base = reinterpret_cast<T*>(tail_lds);
    const int inst = insts[blockIdx.x];
    if (active != nullptr && active[inst] == 0) return;
    const InstInfo in = info[inst];
    const LevelDesc<T>* d = desc + inst * kMaxLevels;
    const int top = in.tail, nlev = in.nlev;

    // stage the top level's iterate and right-hand side, and every level's
    // frozen data
    const Level<T> G = make_view(d[top], (cur_mask >> top) & 1u);
    {
        // a top level below the finest one holds the restricted residual fr;
        // its FAS right-hand side f = fr + N(u) is formed below
        const Level<T> S = lds_view<T, CORR>(d, top, top, base);
        const T* g0 = top > 0 ? G.fr0 : G.f0;
        const T* g1 = top > 0 ? G.fr1 : G.f1;
        const T* g2 = top > 0 ? G.fr2 : G.f2;
        // a deferred shift of the finest p: subtracted here when the tail
        // holds the finest level, then cleared (the finest level's first
        // smoothing launch has already subtracted it otherwise)
        const T psh = pend != nullptr && top == 0 ? T(pend[inst * kResStride + 4]) : T(0);
        // Every global load of the first rounds is issued before any LDS
        // store, so the staging waits for memory once: two cells of the top
        // level per thread (the LDS budget keeps the top below 2 kTailThreads
        // cells) and one of each lower level (a quarter or an eighth of the
        // level above); any further cells by the loops after.
        const int t0 = threadIdx.x;
        T tv[2][9];
        T lv[kMaxTailLevels][2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int idx = t0 + k * kTailThreads;
            if (idx < G.n) {
                tv[k][0] = gload(G.phi, idx);
                tv[k][1] = gload(G.mu, idx);
                tv[k][2] = gload(G.p, idx);
                tv[k][3] = gload(g0, idx);
                tv[k][4] = gload(g1, idx);
                tv[k][5] = gload(g2, idx);
                tv[k][6] = CORR ? gload(G.b, idx) : T(0);
                tv[k][7] = gload(G.pstar, idx);
                tv[k][8] = gload(G.psi, idx);
            }
        }
#pragma unroll
        for (int m = 1; m < kMaxTailLevels; ++m) {
            const int l = top + m;
            if (l < nlev && t0 < d[l].n) {
                lv[m][0] = gload(d[l].pstar, t0);
                lv[m][1] = gload(d[l].psi, t0);
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int idx = t0 + k * kTailThreads;
            if (idx < G.n) {
                S.phi[idx] = tv[k][0];
                S.mu[idx] = tv[k][1];
                S.p[idx] = tv[k][2] - psh;
                S.f0[idx] = tv[k][3];
                S.f1[idx] = tv[k][4];
                S.f2[idx] = tv[k][5];
                if (CORR) S.b[idx] = tv[k][6];
                S.pstar[idx] = tv[k][7];
                S.psi[idx] = tv[k][8];
            }
        }
#pragma unroll
        for (int m = 1; m < kMaxTailLevels; ++m) {
            const int l = top + m;
            if (l < nlev && t0 < d[l].n) {
                const Level<T> V = lds_view<T, CORR>(d, top, l, base);
                V.pstar[t0] = lv[m][0];
                V.psi[t0] = lv[m][1];
            }
        }
        for (int idx = t0 + 2 * kTailThreads; idx < G.n; idx += blockDim.x) {
            S.phi[idx] = G.phi[idx];
            S.mu[idx] = G.mu[idx];
            S.p[idx] = G.p[idx] - psh;
            S.f0[idx] = g0[idx];
            S.f1[idx] = g1[idx];
            S.f2[idx] = g2[idx];
            if (CORR) S.b[idx] = G.b[idx];
            S.pstar[idx] = G.pstar[idx];
            S.psi[idx] = G.psi[idx];
        }
        for (int l = top + 1; l < nlev; ++l) {
            const Level<T> V = lds_view<T, CORR>(d, top, l, base);
            const LevelDesc<T>& D = d[l];
            for (int idx = t0 + kTailThreads; idx < V.n; idx += blockDim.x) {
                V.pstar[idx] = D.pstar[idx];
                V.psi[idx] = D.psi[idx];
            }
        }
    }
    __syncthreads();
    if (pend != nullptr && threadIdx.x == 0) pend[inst * kResStride + 4] = 0.0;
    if (top > 0) {
        const Level<T> S = lds_view<T, CORR>(d, top, top, base);
        const float rnx = 1.0f / float(S.nx), rnxy = 1.0f / float(S.nx * S.ny);
        for (int idx = threadIdx.x; idx < S.n; idx += blockDim.x) {
            int i, j, k;
            tail_decode<DIM>(idx, S.nx, S.ny, rnx, rnxy, i, j, k);
            T n0, n1, n2;
            cell_operator<DIM, T, CORR>(S, idx, i, j, k, n0, n1, n2);
            S.f0[idx] += n0;
            S.f1[idx] += n1;
            S.f2[idx] += n2;
        }
        __syncthreads();
    }

    // FP32: levels of at most kWaveCells cells (the coarse end of the cycle)
    // are worked by the first wave alone; a workgroup barrier follows the last
    // of them before any larger level is worked again.
    const int last = nlev - 1;
    auto small = [&](int l) { return CORR && d[l].n <= kWaveCells; };
    // (the wave index read as a scalar: the branch is uniform per wave)
    const bool wave0 = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6) == 0;
    for (int l = top; l < last; ++l) {
        const Level<T> F = lds_view<T, CORR>(d, top, l, base);
        const int nu1 = l == 0 ? shape.nu1f : shape.nu1c;
        if (small(l)) {
            if (wave0) {
                for (int s = 0; s < nu1; ++s) tail_smooth<DIM, T, CORR, true>(F);
                tail_restrict<DIM, T, CORR, true>(F, lds_view<T, CORR>(d, top, l + 1, base));
            }
        } else {
            for (int s = 0; s < nu1; ++s) tail_smooth<DIM, T, CORR>(F);
            tail_restrict<DIM, T, CORR>(F, lds_view<T, CORR>(d, top, l + 1, base));
        }
    }
    bool wave_only = small(last);
    {
        const Level<T> B = lds_view<T, CORR>(d, top, last, base);
        if (wave_only) {
            if (wave0)
                for (int s = 0; s < shape.coarse; ++s) tail_smooth<DIM, T, CORR, true>(B);
        } else {
            for (int s = 0; s < shape.coarse; ++s) tail_smooth<DIM, T, CORR>(B);
        }
    }
    for (int l = last - 1; l >= top; --l) {
        const Level<T> F = lds_view<T, CORR>(d, top, l, base);
        const int nu2 = l == 0 ? shape.nu2f : shape.nu2c;
        if (small(l)) {
            if (wave0) {
                tail_prolong<DIM, T, true>(F, lds_view<T, CORR>(d, top, l + 1, base),
                                           shape.bilinear != 0);
                for (int s = 0; s < nu2; ++s) tail_smooth<DIM, T, CORR, true>(F);
            }
            wave_only = true;
        } else {
            if (wave_only) __syncthreads();
            wave_only = false;
            tail_prolong<DIM>(F, lds_view<T, CORR>(d, top, l + 1, base), shape.bilinear != 0);
            for (int s = 0; s < nu2; ++s) tail_smooth<DIM, T, CORR>(F);
        }
    }
    // the write-back reads what the first wave alone may have written last
    if (wave_only) __syncthreads();

    const Level<T> S = lds_view<T, CORR>(d, top, top, base);
    for (int idx = threadIdx.x; idx < G.n; idx += blockDim.x) {
        gstore(G.phi, idx, S.phi[idx]);
        gstore(G.mu, idx, S.mu[idx]);
        gstore(G.p, idx, S.p[idx]);
    }
}

}  // namespace

size_t tail_lds_bytes(const int* cells, int nlev, size_t elem, int nfields) {
    size_t b = 0;
    for (int l = 0; l < nlev; ++l) b += size_t(cells[l]) * nfields * elem;
    return b;
}

template <typename T, bool CORR>
int prepare_tail(int dim, size_t lds_bytes) {
    hipError_t e;
    if (dim == 2)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tail<2, T, CORR>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
    else
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tail<3, T, CORR>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
    return e == hipSuccess ? 0 : -1;
}

template <typename T, bool CORR>
void launch_tail(int dim, const LevelDesc<T>* desc, const InstInfo* info, const int* insts,
                 int ninst, const int* active, unsigned cur_mask, const CycleShape& shape,
                 double* pend, size_t lds_bytes, hipStream_t st) {
    if (ninst <= 0) return;
    if (dim == 2)
        hipLaunchKernelGGL((k_tail<2, T, CORR>), dim3(ninst), dim3(kTailThreads), lds_bytes, st,
                           desc, info, insts, active, cur_mask, shape, pend);
    else
        hipLaunchKernelGGL((k_tail<3, T, CORR>), dim3(ninst), dim3(kTailThreads), lds_bytes, st,
                           desc, info, insts, active, cur_mask, shape, pend);
}

template int prepare_tail<double, false>(int, size_t);
template int prepare_tail<float, true>(int, size_t);
template void launch_tail<double, false>(int, const LevelDesc<double>*, const InstInfo*,
                                         const int*, int, const int*, unsigned,
                                         const CycleShape&, double*, size_t, hipStream_t);
template void launch_tail<float, true>(int, const LevelDesc<float>*, const InstInfo*, const int*,
                                       int, const int*, unsigned, const CycleShape&, double*,
                                       size_t, hipStream_t);

}  // namespace chhs
