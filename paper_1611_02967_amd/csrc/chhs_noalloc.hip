// chhs_energy_mass_noalloc: the discrete mass (phi, 1), E_h(phi) (2.8) and
// F_h(phi, phi_prev) (2.9) of caller arrays without a context and without any
// allocation, for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops).
//
// The per-block partial sums live in `scratch`, a file-scope device array of
// fixed size.  Host code never passes the array's name to a kernel: its
// address on each device is taken once with hipGetSymbolAddress, with that
// device current, and kept per device.  Every call on a device shares that
// device's array, so calls that overlap on one GPU race.  Nothing needs
// clearing between calls: every block of a launch writes its whole partial
// before the reduction reads it.
#include <mutex>

#include "chhs.h"
#include "chhs_internal.hpp"

namespace chhs {
namespace {

constexpr int kNaMaxInst = 32;        // instances per call
constexpr int kNaMaxBlocks = 256;     // blocks per instance at most (grid-stride loop)
constexpr int kNaThreads = 256;
constexpr int kNaVals = 6;            // partial sums per block
constexpr int kNaMaxDevices = 64;
// 32 x 256 partials of 8 doubles: 512 KiB
constexpr size_t kNaScratchDoubles = size_t(kNaMaxInst) * kNaMaxBlocks * 8;

static __device__ __align__(256) double scratch[kNaScratchDoubles];

struct NaInst {
    int nx, ny, nz, off;    // extents, offset in the packed arrays
    int block0, nblocks;    // the instance's blocks (and partials)
    double h, eps;
};
struct NaArgs {
    int n_inst, dim;
    NaInst in[kNaMaxInst];
};

// Per block: over its instance's cells (grid-stride within the instance)
// sum phi, phi^2, phi^4, |D phi|^2 h^2 and, with d = phi - q, d^2 and
// |D d|^2 h^2 over the forward interior faces (every interior face once).
template <int DIM>
__global__ __launch_bounds__(kNaThreads) void k_na_partials(NaArgs a, const double* __restrict__ phi,
                                                           const double* __restrict__ q,
                                                           double* __restrict__ part) {
    const int b = blockIdx.x;
    int i = 0;
    while (i + 1 < a.n_inst && b >= a.in[i + 1].block0) ++i;
    const NaInst in = a.in[i];
    const int n = in.nx * in.ny * in.nz;
    const double* f0 = phi + in.off;
    const double* q0 = q + in.off;
    double v[kNaVals] = {0, 0, 0, 0, 0, 0};
    const int stride = in.nblocks * kNaThreads;
    for (int idx = (b - in.block0) * kNaThreads + int(threadIdx.x); idx < n; idx += stride) {
        const int x = idx % in.nx;
        const int r = idx / in.nx;
        const int y = DIM == 2 ? r : r % in.ny;
        const int z = DIM == 2 ? 0 : r / in.ny;
        const double f = f0[idx];
        const double d = f - q0[idx];
        v[0] += f;
        v[1] += f * f;
        v[2] += f * f * f * f;
        v[4] += d * d;
        auto face = [&](int nb) {
            const double df = f0[nb] - f;
            const double dd = (f0[nb] - q0[nb]) - d;
            v[3] += df * df;
            v[5] += dd * dd;
        };
        if (x < in.nx - 1) face(idx + 1);
        if (y < in.ny - 1) face(idx + in.nx);
        if (DIM == 3 && z < in.nz - 1) face(idx + in.nx * in.ny);
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < kNaVals; ++c) v[c] += __shfl_xor(v[c], off, 64);
    __shared__ double sh[kNaVals][kNaThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < kNaVals; ++c) sh[c][wid] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < kNaVals; ++c) {
            double s = 0.0;
            for (int w = 0; w < kNaThreads / 64; ++w) s += sh[c][w];
            part[size_t(b) * 8 + c] = s;
        }
}

// One block per instance: its partials summed in order, then
// mass = h^d sum phi, E_h = h^d (sum phi^4 / 4 - sum phi^2 / 2 + eps^2 / 2 |grad phi|^2),
// F_h = E_h + h^d (sum d^2 / 4 + eps^2 / 8 |grad d|^2).
__global__ __launch_bounds__(kNaThreads) void k_na_reduce(NaArgs a, const double* __restrict__ part,
                                                         double* __restrict__ out) {
    const NaInst in = a.in[blockIdx.x];
    double v[kNaVals] = {0, 0, 0, 0, 0, 0};
    for (int k = int(threadIdx.x); k < in.nblocks; k += kNaThreads)
        for (int c = 0; c < kNaVals; ++c) v[c] += part[size_t(in.block0 + k) * 8 + c];
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < kNaVals; ++c) v[c] += __shfl_xor(v[c], off, 64);
    __shared__ double sh[kNaVals][kNaThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < kNaVals; ++c) sh[c][wid] = v[c];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double s[kNaVals];
    for (int c = 0; c < kNaVals; ++c) {
        s[c] = 0.0;
        for (int w = 0; w < kNaThreads / 64; ++w) s[c] += sh[c][w];
    }
    double hd = in.h * in.h;
    if (a.dim == 3) hd *= in.h;
    const double e2 = in.eps * in.eps, ih2 = 1.0 / (in.h * in.h);
    const double E = hd * (0.25 * s[2] - 0.5 * s[1] + 0.5 * e2 * s[3] * ih2);
    out[3 * blockIdx.x + 0] = hd * s[0];
    out[3 * blockIdx.x + 1] = E;
    out[3 * blockIdx.x + 2] = E + hd * (0.25 * s[4] + 0.125 * e2 * s[5] * ih2);
}

std::mutex g_scratch_mu;
double* g_scratch[kNaMaxDevices] = {};

// The device address of `scratch` on the current device, taken once per device.
double* scratch_address() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
            return nullptr;
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    return g_scratch[dev];
}

}  // namespace
}  // namespace chhs

extern "C" int chhs_energy_mass_noalloc(const chhs_problem* p, int32_t n_inst, const double* phi,
                                        const double* phi_prev, double* out_dev, void* hip_stream) {
    using namespace chhs;
    if (p == nullptr || phi == nullptr || phi_prev == nullptr || out_dev == nullptr)
        return CHHS_E_INVAL;
    if (n_inst < 1 || n_inst > kNaMaxInst) return CHHS_E_INVAL;
    NaArgs a{};
    a.n_inst = n_inst;
    a.dim = p[0].dim;
    long long total = 0;
    int blocks = 0;
    for (int i = 0; i < n_inst; ++i) {
        const chhs_problem& q = p[i];
        if (q.dim != a.dim || (q.dim != 2 && q.dim != 3)) return CHHS_E_INVAL;
        if (q.nx < 1 || q.ny < 1 || q.nz < 1 || (q.dim == 2 && q.nz != 1)) return CHHS_E_INVAL;
        if (!(q.h > 0.0) || !(q.eps > 0.0)) return CHHS_E_INVAL;
        const long long cells = (long long)q.nx * q.ny * q.nz;
        if (cells >= (1LL << 29)) return CHHS_E_INVAL;
        NaInst& in = a.in[i];
        in.nx = q.nx;
        in.ny = q.ny;
        in.nz = q.nz;
        in.off = int(total);
        in.h = q.h;
        in.eps = q.eps;
        in.block0 = blocks;
        const long long want = (cells + kNaThreads - 1) / kNaThreads;
        in.nblocks = int(want < kNaMaxBlocks ? want : kNaMaxBlocks);
        blocks += in.nblocks;
        total += cells;
        if (total > 2147483647LL) return CHHS_E_INVAL;
    }
    double* part = scratch_address();
    if (part == nullptr) return CHHS_E_HIP;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (a.dim == 2)
        hipLaunchKernelGGL(k_na_partials<2>, dim3(blocks), dim3(kNaThreads), 0, st, a, phi,
                           phi_prev, part);
    else
        hipLaunchKernelGGL(k_na_partials<3>, dim3(blocks), dim3(kNaThreads), 0, st, a, phi,
                           phi_prev, part);
    hipLaunchKernelGGL(k_na_reduce, dim3(n_inst), dim3(kNaThreads), 0, st, a, part, out_dev);
    return hipGetLastError() == hipSuccess ? CHHS_OK : CHHS_E_HIP;
}
