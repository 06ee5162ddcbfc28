// Host driver and C ABI of libchhs (declared in include/chhs.h).
//
// Owns the multigrid hierarchies of a batch of independent instances carved
// out of the caller's workspace, the task tables that let one launch per level
// cover every instance, the FAS V-cycle schedule (optionally replayed as a
// captured HIP graph), the per-instance stopping test (one small readback per
// cycle), the mixed-precision iterative refinement, and the time-step loop
// with its state rotation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <utility>
#include <vector>

#include "chhs.h"
#include "chhs_internal.hpp"

using chhs::Batch;
using chhs::CellTask;
using chhs::FoldTask;
using chhs::InstInfo;
using chhs::Level;
using chhs::LevelDesc;
using chhs::Range;
using chhs::Step3Task;
using chhs::StripTask;
using chhs::TileTask;
using chhs::kMaxLevels;

namespace {

constexpr size_t kAlign = 256;
// Limits of the 32-bit indexing: cells per instance (an FP64 field < 4 GiB)
// and cells of a whole batch (packed offsets are int).
constexpr long long kMaxCellsPerInstance = 1LL << 29;
constexpr long long kMaxPackedCells = 2147483647LL;
// Tiled launches of at most this many blocks (at most one per compute unit)
// use 1024-thread blocks: their time is the latency of one block.
constexpr int kWideTiles = 256;
constexpr long kSmallTileLevel = 128;
// Threads per tile block: the autotuned choice (256, 512 or 1024), else by
// the number of tiles.
int tile_block(int chosen, int ntiles) {
    return chosen > 0 ? chosen : (ntiles <= kWideTiles ? 1024 : 256);
}
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// A table of block tasks in device memory.
template <typename Task>
struct Table {
    Task* dev = nullptr;
    int n = 0;
};

// Everything the workspace holds, computed from the problems alone.
struct Layout {
    size_t bytes = 0;
    std::vector<LevelDesc<double>> desc;       // [inst * kMaxLevels + l] (device pointers)
    std::vector<LevelDesc<float>> desc32;      // FP32 correction hierarchy (mixed precision)
    std::vector<InstInfo> info;
    std::vector<std::vector<CellTask>> A, B, Bc, Bh, Bcs;
    std::vector<std::vector<TileTask>> T, Tall;
    std::vector<std::vector<StripTask>> S, Sall;
    // 3D: fused-step tiles per level (instances above their tail; FP64 and FP32
    // tile sizes) and z-segment height per level
    std::vector<std::vector<Step3Task>> Z64, Z32;
    // 3D restriction: z-marching tasks of the instances whose level is large
    // enough, per-cell coarse tasks of the others
    std::vector<std::vector<Step3Task>> ZR64, ZR32;
    std::vector<std::vector<CellTask>> BcS;
    int zseg64[kMaxLevels] = {}, zseg32[kMaxLevels] = {};
    // 3D level smoothed by the fused step (else by one launch per color)
    bool z3[kMaxLevels] = {};
    bool strip[kMaxLevels] = {};            // level smoothed by the row-streaming kernel
    int tile_threads[kMaxLevels] = {};      // tiles: threads per block, 0 = by the tile count
    int tile_threads_post[kMaxLevels] = {}; // ... of the post-smoothing launches (0 = the same)
    int tile_y[kMaxLevels] = {};            // tile height of the level's tasks (T)
    int tile_y_all[kMaxLevels] = {};        // tile height of the tasks over every instance (Tall)
    size_t cap_T[kMaxLevels] = {};          // capacity of T: tasks of the smallest tile height
    size_t cap_S[kMaxLevels] = {};          // capacity of S: tasks of the shortest tuned segment
    int seg[kMaxLevels] = {};               // rows per strip segment of S[l]
    // per level and instance: x / y extent of the grids in S[l] (-1: not listed)
    std::vector<std::vector<int>> snx, sny;
    std::vector<int> tail_insts;
    std::vector<CellTask> A0n;              // finest-level cells of instances without a fused norm
    std::vector<CellTask> A0t;              // finest-level cells of instances held by the tail
    std::vector<CellTask> A0x;              // 3D mixed: finest cells refined per cell
    std::vector<Range> rngA0x;
    std::vector<StripTask> M0;              // 2D mixed: row-marching refinement tasks
    std::vector<Range> rngM0, rngM0f;
    std::vector<FoldTask> FM0;
    int march_seg = 0;
    std::vector<Range> rngA0, rngT0, rngA0n;
    // folds of the partials over A[0] / A0n (empty when no instance has more
    // than kFold of them) and the per-instance ranges of the folded partials
    std::vector<FoldTask> FA0, FA0n;
    std::vector<Range> rngA0f, rngA0nf;
    int max_nlev = 0, depth = 0;
    // the setup's restriction of phi_* and phi^m runs level by level down to
    // chain_from, then in one workgroup per instance (levels of at most
    // kChainCells cells in every instance)
    int chain_from = 0;
    std::vector<int> max_cells;
    size_t tail_lds = 0, tail_lds32 = 0;
    // offsets into the workspace
    size_t off_desc = 0, off_desc32 = 0, off_info = 0, off_tail = 0, off_rngA0 = 0, off_rngT0 = 0,
           off_rngA0n = 0;
    size_t off_A0n = 0, off_A0t = 0, off_partial_t = 0, off_A0x = 0, off_rngA0x = 0;
    size_t off_M0 = 0, off_rngM0 = 0, off_rngM0f = 0, off_FM0 = 0;
    size_t off_FA0 = 0, off_FA0n = 0, off_rngA0f = 0, off_rngA0nf = 0, off_partial_f = 0;
    size_t off_partial = 0, off_res = 0, off_eres = 0, off_act_cycle = 0, off_act_next = 0,
           off_cycles = 0, off_act_last = 0;
    std::vector<size_t> off_A, off_B, off_Bc, off_Bh, off_Bcs, off_T, off_Tall, off_S, off_Sall,
        off_Z64, off_Z32, off_ZR64, off_ZR32, off_BcS;
    int partial_cap = 0, partial_t_cap = 0;
};

}  // namespace

struct chhs_ctx {
    std::vector<chhs_problem> prob;
    chhs_opts opts;
    int n_inst = 1;
    int dim = 2;
    bool mixed = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;        // created by chhs_init (no stream given)
    Layout lay;
    char* base = nullptr;
    // device views
    LevelDesc<double>* ddesc = nullptr;
    LevelDesc<float>* ddesc32 = nullptr;
    InstInfo* dinfo = nullptr;
    Table<CellTask> A[kMaxLevels], B[kMaxLevels], Bc[kMaxLevels], Bh[kMaxLevels],
        Bcs[kMaxLevels];
    Table<TileTask> T[kMaxLevels], Tall[kMaxLevels];
    Table<StripTask> S[kMaxLevels], Sall[kMaxLevels];
    Table<Step3Task> Z64[kMaxLevels], Z32[kMaxLevels], ZR64[kMaxLevels], ZR32[kMaxLevels];
    Table<CellTask> BcS[kMaxLevels];
    Table<CellTask> A0n, A0t, A0x;
    Range* rngA0x = nullptr;
    Table<StripTask> M0;
    Table<FoldTask> FM0;
    Range* rngM0 = nullptr;
    Range* rngM0f = nullptr;
    Table<FoldTask> FA0, FA0n;
    int* tail_insts = nullptr;
    Range* rngA0 = nullptr;
    Range* rngT0 = nullptr;
    Range* rngA0n = nullptr;
    Range* rngA0f = nullptr;
    Range* rngA0nf = nullptr;
    double* partial = nullptr;
    double* partial_f = nullptr;    // folded per-cell partials
    double* partial_t = nullptr;    // norm partials of the fused finest-level launch
    double* res = nullptr;          // [n_inst][kResStride]
    double* eres = nullptr;         // [n_inst][kResStride]
    int* act_cycle = nullptr;
    int* act_next = nullptr;
    int* act_last = nullptr;        // mixed: act_cycle of the previous refinement
    int* cycles = nullptr;
    // pinned host mirrors of the result block (res | act_next | cycles): two
    // that the cycles of the pipelined plain loop alternate between, a third
    // for the setup of a step that the loop reads with its first cycle, and
    // the current view into one of them; the energies follow the first
    double* hbuf[3] = {nullptr, nullptr, nullptr};
    double* hres = nullptr;
    double* heres = nullptr;
    // per-step energies of chhs_step_log (pinned, grown on demand)
    double* hlog = nullptr;
    size_t hlog_cap = 0;
    int* hact = nullptr;
    int* hcyc = nullptr;
    int cur[kMaxLevels] = {};       // current copy of u per FP64 level
    int cur32[kMaxLevels] = {};     // current copy of u per FP32 level
    bool fused_norm = false;
    // plain 2D path with pre-smoothing: p's mean is not subtracted by a launch
    // of its own after a cycle; the next cycle's first finest-level launch
    // (or the tail, holding that level) subtracts it as it loads p, and the
    // copy to the caller's arrays subtracts what is still pending
    bool defer_shift = false;
    bool loaded = false;
    // graph replay of one cycle; two slots in mixed precision (the FP64 finest
    // level alternates its copy once per refinement step)
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    bool graph_failed = false;
    int capturing = -1;             // slot being captured, -1 when none
    // kernel timing (opts.timing)
    struct Pending { hipEvent_t a, b; int cls; };
    std::vector<hipEvent_t> ev_pool;
    std::vector<Pending> pending;        // resolved and recycled after each sync
    std::vector<Pending> graph_pairs[2]; // recorded by every replay of a graph slot
    int last_slot = -1;                  // slot replayed since the last synchronisation
    hipEvent_t cycle_done[2] = {nullptr, nullptr};   // end of a pipelined cycle per slot
    double t_ms[CHHS_K_COUNT] = {};
    int64_t t_n[CHHS_K_COUNT] = {};
};

namespace {

bool valid_problem(const chhs_problem* p) {
    if (p == nullptr) return false;
    if (p->dim != 2 && p->dim != 3) return false;
    if (p->nx < 2 || p->ny < 2) return false;
    if (p->dim == 2 && p->nz != 1) return false;
    if (p->dim == 3 && p->nz < 2) return false;
    if (!(p->h > 0.0) || !(p->eps > 0.0) || !(p->gamma >= 0.0) || !(p->dt > 0.0)) return false;
    if (!std::isfinite(p->h) || !std::isfinite(p->eps) || !std::isfinite(p->gamma) ||
        !std::isfinite(p->dt))
        return false;
    // Kernels address a field with a 32-bit unsigned byte offset: an FP64 field
    // must stay below 4 GiB, i.e. below 2^29 cells.
    const double cells = double(p->nx) * p->ny * p->nz;
    return cells < double(kMaxCellsPerInstance);
}

// Cells of all instances together: packed caller arrays are indexed with
// 32-bit signed offsets.
bool valid_total(const chhs_problem* p, int n_inst) {
    double total = 0.0;
    for (int i = 0; i < n_inst; ++i) total += double(p[i].nx) * p[i].ny * p[i].nz;
    return total <= double(kMaxPackedCells);
}

bool valid_opts(const chhs_opts* o) {
    if (o == nullptr) return false;
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1) return false;
    if (o->max_vcycles < 1 || o->coarse_sweeps < 1) return false;
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return false;
    if (o->precision != 0 && o->precision != 1) return false;
    if (o->smoother < 0 || o->smoother > 4) return false;
    if (o->autotune < 0 || o->autotune > 1) return false;
    if (o->order < 0 || o->order > 2) return false;
    if (o->order == 1 && o->precision != 0) return false;
    if (o->tile_threads != 0 && o->tile_threads != 256 && o->tile_threads != 512 &&
        o->tile_threads != 1024)
        return false;
    if (o->tile_rows != 0 && o->tile_rows != chhs::kTileY && o->tile_rows != chhs::kTileYSmall &&
        o->tile_rows != chhs::kTileYTiny && o->tile_rows != chhs::kTileYTall)
        return false;
    // 32 rows: the finest level of the FP32 hierarchy (mixed precision) only
    if (o->tile_rows == chhs::kTileYTall && o->precision != 1)
        return false;
    if (o->nu1_coarse < 0 || o->nu2_coarse < 0) return false;
    if (o->prolong != 0 && o->prolong != 1) return false;
    if (o->inner_cycles < 0 || o->inner_cycles > 8) return false;
    return true;
}

// Smoothing steps before / after the coarse correction on level l.
int nu_pre(const chhs_opts& o, int l) { return l == 0 || o.nu1_coarse == 0 ? o.nu1 : o.nu1_coarse; }
int nu_post(const chhs_opts& o, int l) { return l == 0 || o.nu2_coarse == 0 ? o.nu2 : o.nu2_coarse; }

chhs::CycleShape cycle_shape(const chhs_opts& o) {
    return chhs::CycleShape{o.nu1, o.nu2, nu_pre(o, 1), nu_post(o, 1), o.coarse_sweeps, o.prolong};
}

// Extents of every level: halve all directions while every extent is even and
// at least 4; the coarsest extents must be at most 8 and there must be at least
// two levels.
bool level_extents(const chhs_problem* p, std::vector<int>& ext) {
    int nx = p->nx, ny = p->ny, nz = p->nz;
    ext.assign({nx, ny, nz});
    for (;;) {
        const bool even = nx % 2 == 0 && ny % 2 == 0 && (p->dim == 2 || nz % 2 == 0);
        const bool big = nx >= 4 && ny >= 4 && (p->dim == 2 || nz >= 4);
        if (!even || !big) break;
        nx /= 2;
        ny /= 2;
        if (p->dim == 3) nz /= 2;
        ext.insert(ext.end(), {nx, ny, nz});
    }
    const int nlev = int(ext.size() / 3);
    if (nlev < 2 || nlev > kMaxLevels) return false;
    return nx <= 8 && ny <= 8 && nz <= 8;
}

// First level of the one-workgroup tail: the finest level whose own and
// coarser levels' FP64 fields (and, in mixed precision, the 12 FP32 fields of
// the correction form) fit the LDS budget.
int pick_tail(const std::vector<int>& cells, bool mixed, size_t* bytes, size_t* bytes32) {
    const int nlev = int(cells.size());
    for (int l = 0; l < nlev; ++l) {
        if (nlev - l > chhs::kMaxTailLevels) continue;
        const size_t b = chhs::tail_lds_bytes(&cells[l], nlev - l, sizeof(double), 11);
        const size_t b32 = chhs::tail_lds_bytes(&cells[l], nlev - l, sizeof(float), 12);
        if (b <= chhs::kTailLdsBudget && (!mixed || b32 <= chhs::kTailLdsBudget)) {
            *bytes = b;
            *bytes32 = b32;
            return l;
        }
    }
    *bytes = chhs::tail_lds_bytes(&cells[nlev - 1], 1, sizeof(double), 11);
    *bytes32 = chhs::tail_lds_bytes(&cells[nlev - 1], 1, sizeof(float), 12);
    return nlev - 1;
}

void cell_tasks(std::vector<CellTask>& out, int inst, int n) {
    for (int c = 0; c < n; c += chhs::kBlock) out.push_back({inst, c});
}

void tile_tasks(std::vector<TileTask>& out, int inst, int nx, int ny, int tile_y) {
    const int tx = (nx + chhs::kTileX - 1) / chhs::kTileX;
    const int ty = (ny + tile_y - 1) / tile_y;
    for (int by = 0; by < ty; ++by)
        for (int bx = 0; bx < tx; ++bx) out.push_back({inst, bx, by});
}

// Strip tasks of one level over the instances listed (extents nx, ny, -1 =
// skip): strips of kStripWO columns, segments of seg rows.
void strip_tasks(std::vector<StripTask>& out, const std::vector<int>& nxs,
                 const std::vector<int>& nys, int seg) {
    for (size_t i = 0; i < nxs.size(); ++i) {
        if (nxs[i] < 0) continue;
        const int sxn = (nxs[i] + chhs::kStripWO - 1) / chhs::kStripWO;
        for (int sx = 0; sx < sxn; ++sx)
            for (int y0 = 0; y0 < nys[i]; y0 += seg)
                out.push_back({int(i), sx, y0, std::min(nys[i], y0 + seg)});
    }
}

// Segment height (even, >= 8) for one launch over the listed instances: the
// smallest that keeps the tasks within one wave of `slots` resident blocks,
// as short as possible otherwise (shorter segments mean more blocks in
// flight, taller ones fewer recomputed halo rows).
int strip_seg(const std::vector<int>& nxs, const std::vector<int>& nys, int slots) {
    int maxny = 8;
    for (size_t i = 0; i < nys.size(); ++i)
        if (nxs[i] >= 0) maxny = std::max(maxny, nys[i]);
    for (int seg = 8;; seg += 2) {
        long tasks = 0;
        for (size_t i = 0; i < nxs.size(); ++i) {
            if (nxs[i] < 0) continue;
            tasks += long((nxs[i] + chhs::kStripWO - 1) / chhs::kStripWO) *
                     ((nys[i] + seg - 1) / seg);
        }
        if (tasks <= slots || seg >= maxny) return seg;
    }
}

// Resident blocks of the row-streaming kernel across the device (256 compute
// units): three per unit for the finest FP64 variant (LDS ring and registers
// both allow it), four for the FP32 ones, two otherwise.
int strip_slots(bool finest_fp64, bool mixed) { return mixed ? 1024 : (finest_fp64 ? 768 : 512); }

void ranges_of(std::vector<Range>& r, int n_inst, const std::vector<CellTask>& t) {
    r.assign(n_inst, Range{0, 0});
    for (int q = 0; q < int(t.size()); ++q) {
        Range& x = r[t[q].inst];
        if (x.end == 0) x.begin = q;
        x.end = q + 1;
    }
}

// Per-cell norm partials per folded partial.  A single workgroup per instance
// sums an instance's partials; above this many it would spend tens of
// microseconds loading them one stride after another.
constexpr int kFold = 1024;

// Coarse levels whose frozen data the setup restricts in one workgroup per
// instance (four cells per thread at most).
constexpr int kChainCells = 4096;

// Runs of kFold partials within each instance's range (relative to the
// range's start, so an instance's sum does not depend on the batch), and the
// ranges of the folded partials; nothing when no range is longer than kFold.
void fold_of(const std::vector<Range>& r, std::vector<FoldTask>& t, std::vector<Range>& rf) {
    t.clear();
    rf.assign(r.size(), Range{0, 0});
    bool need = false;
    for (const Range& x : r) need = need || x.end - x.begin > kFold;
    if (!need) return;
    for (int i = 0; i < int(r.size()); ++i) {
        rf[i].begin = int(t.size());
        for (int q = r[i].begin; q < r[i].end; q += kFold)
            t.push_back(FoldTask{i, q, std::min(q + kFold, r[i].end)});
        rf[i].end = int(t.size());
    }
}

// Per-instance ranges of the finest level's smoothing tasks (strips or tiles)
// in the fused norm partials.
template <typename Task>
void task_ranges(std::vector<Range>& r, int n_inst, const std::vector<Task>& tasks) {
    r.assign(n_inst, Range{0, 0});
    for (int q = 0; q < int(tasks.size()); ++q) {
        Range& x = r[tasks[q].inst];
        if (x.end == 0) x.begin = q;
        x.end = q + 1;
    }
}

void fused_ranges(Layout& L, int n_inst) {
    if (L.strip[0])
        task_ranges(L.rngT0, n_inst, L.S[0]);
    else if (!L.T[0].empty())
        task_ranges(L.rngT0, n_inst, L.T[0]);
    else
        task_ranges(L.rngT0, n_inst, L.Z64[0]);     // 3D
}

// 3D levels above the tail may be smoothed by the fused z-marching step kernel
// (the second-order scheme, unless opts.smoother = 3 asks for the per-cell
// red-black kernels everywhere); which levels do is Layout::z3.
bool step3d_opts(int dim, const chhs_opts* o) { return dim == 3 && o->order != 1 && o->smoother != 3; }

// Cells of an instance's 3D level from which it restricts by z marching.
constexpr long kRes3MinCells = 1L << 20;

// Planes per segment below which a level is left to the per-color kernels by
// default: the segments of such levels are short (few planes per workgroup to
// amortise the four halo planes) or too few workgroups fill the device.
constexpr int kStep3MinSeg = 16;

// Fused-step tasks of one 3D level over the listed instances (extents, -1 =
// skip): tiles of tx x ty columns, z-segments of zs planes.
void step3_tasks(std::vector<Step3Task>& out, const std::vector<int>& nxs,
                 const std::vector<int>& nys, const std::vector<int>& nzs, int tx, int ty, int zs) {
    for (size_t i = 0; i < nxs.size(); ++i) {
        if (nxs[i] < 0) continue;
        for (int z0 = 0; z0 < nzs[i]; z0 += zs)
            for (int by = 0; by < (nys[i] + ty - 1) / ty; ++by)
                for (int bx = 0; bx < (nxs[i] + tx - 1) / tx; ++bx)
                    out.push_back({int(i), bx, by, z0, std::min(nzs[i], z0 + zs)});
    }
}

// z-segment height of one fused-step launch: the tallest (fewer halo planes
// loaded twice) that still gives kStep3Blocks workgroups over the batch, no
// shorter than 8 planes.
constexpr long kStep3Blocks = 2048;
int step3_seg(const std::vector<int>& nxs, const std::vector<int>& nys, const std::vector<int>& nzs,
              int tx, int ty) {
    for (int zs : {64, 32, 16}) {
        long blocks = 0;
        for (size_t i = 0; i < nxs.size(); ++i)
            if (nxs[i] >= 0)
                blocks += long((nxs[i] + tx - 1) / tx) * ((nys[i] + ty - 1) / ty) *
                          ((nzs[i] + zs - 1) / zs);
        if (blocks >= kStep3Blocks) return zs;
    }
    return 8;
}

// Rows per segment of the row-marching refinement tasks: the longest segment
// (fewer halo rows read twice) that still gives at least kMarchWavesWanted
// waves over the batch (enough resident waves to keep loads in flight), but
// no shorter than 16 rows.
constexpr long kMarchWavesWanted = 4096;
int march_seg(const std::vector<InstInfo>& info, const std::vector<LevelDesc<double>>& desc,
              int n_inst) {
    for (int seg : {64, 48, 32, 24}) {
        long waves = 0;
        for (int i = 0; i < n_inst; ++i) {
            const LevelDesc<double>& d = desc[size_t(i) * kMaxLevels];
            waves += long((d.nx + chhs::kMarchCols - 1) / chhs::kMarchCols) * ((d.ny + seg - 1) / seg);
        }
        if (waves >= kMarchWavesWanted) return seg;
    }
    (void)info;
    return 16;
}

// Builds the layout; base != nullptr fills the device pointers of the descriptors.
bool plan(const chhs_problem* p, int n_inst, const chhs_opts* o, char* base, Layout& L) {
    L = Layout();
    // every size check before any per-cell table is built
    for (int i = 0; i < n_inst; ++i)
        if (!valid_problem(&p[i])) return false;
    if (!valid_total(p, n_inst)) return false;
    const int dim = p[0].dim;
    // smoother 4 (the fused step on every level) is a 3D choice of the
    // second-order scheme
    if (o->smoother == 4 && (dim != 3 || o->order == 1)) return false;
    const bool mixed = o->precision == 1;
    L.A.resize(kMaxLevels);
    L.B.resize(kMaxLevels);
    L.Bc.resize(kMaxLevels);
    L.Bh.resize(kMaxLevels);
    L.Bcs.resize(kMaxLevels);
    L.T.resize(kMaxLevels);
    L.Tall.resize(kMaxLevels);
    L.S.resize(kMaxLevels);
    L.Sall.resize(kMaxLevels);
    L.Z64.resize(kMaxLevels);
    L.Z32.resize(kMaxLevels);
    L.ZR64.resize(kMaxLevels);
    L.ZR32.resize(kMaxLevels);
    L.BcS.resize(kMaxLevels);
    // level extents per instance (-1: no such level) for the strip planner
    std::vector<std::vector<int>> lnx(kMaxLevels, std::vector<int>(n_inst, -1));
    std::vector<std::vector<int>> lny(kMaxLevels, std::vector<int>(n_inst, -1));
    std::vector<std::vector<int>> lnx_t(kMaxLevels, std::vector<int>(n_inst, -1));
    std::vector<std::vector<int>> lnz(kMaxLevels, std::vector<int>(n_inst, -1));
    L.desc.assign(size_t(n_inst) * kMaxLevels, LevelDesc<double>{});
    if (mixed) L.desc32.assign(size_t(n_inst) * kMaxLevels, LevelDesc<float>{});
    size_t off = 0;
    auto take = [&](size_t bytes) -> size_t {
        const size_t o2 = off;
        off += align_up(bytes);
        return o2;
    };
    auto ptr = [&](size_t o2) -> double* {
        return base ? reinterpret_cast<double*>(base + o2) : nullptr;
    };
    auto ptr32 = [&](size_t o2) -> float* {
        return base ? reinterpret_cast<float*>(base + o2) : nullptr;
    };
    // tile height per 2D level: opts.tile_rows on coarse levels if given, else
    // 64 x 8 on coarse levels with at most kSmallTileLevel 64 x 16 tiles over
    // the batch (more, smaller blocks, each a shorter launch), 64 x 16
    // elsewhere; the autotuner may cut coarse levels anew
    for (int l = 0; l < kMaxLevels; ++l) L.tile_y[l] = chhs::kTileY;
    if (dim == 2) {
        std::vector<long> tiles16(kMaxLevels, 0);
        for (int i = 0; i < n_inst; ++i) {
            std::vector<int> ext;
            if (!valid_problem(&p[i]) || !level_extents(&p[i], ext)) continue;
            for (size_t l = 0; l < ext.size() / 3; ++l)
                tiles16[l] += long((ext[3 * l] + chhs::kTileX - 1) / chhs::kTileX) *
                              ((ext[3 * l + 1] + chhs::kTileY - 1) / chhs::kTileY);
        }
        const bool tall = o->tile_rows == chhs::kTileYTall;    // finest level only
        if (tall) L.tile_y[0] = chhs::kTileYTall;
        for (int l = 1; l < kMaxLevels; ++l)
            L.tile_y[l] = o->tile_rows != 0 && !tall
                              ? o->tile_rows
                              : (tiles16[l] <= kSmallTileLevel ? chhs::kTileYSmall : chhs::kTileY);
    }
    int packed = 0;
    for (int i = 0; i < n_inst; ++i) {
        if (!valid_problem(&p[i]) || p[i].dim != dim) return false;
        std::vector<int> ext;
        if (!level_extents(&p[i], ext)) return false;
        const int nlev = int(ext.size() / 3);
        std::vector<int> cells(nlev);
        for (int l = 0; l < nlev; ++l) cells[l] = ext[3 * l] * ext[3 * l + 1] * ext[3 * l + 2];
        size_t tb = 0, tb32 = 0;
        const int tail = pick_tail(cells, mixed, &tb, &tb32);
        L.tail_lds = std::max(L.tail_lds, tb);
        L.tail_lds32 = std::max(L.tail_lds32, tb32);
        InstInfo in{};
        in.dim = dim;
        in.nlev = nlev;
        in.tail = tail;
        in.off = packed;
        in.n0 = cells[0];
        const bool first = o->order == 1;
        in.order = first ? 1 : 2;
        // the finest level's norm partials: from the fused 2D post launch, or
        // (3D) from the z-marching residual kernel over the fused-step tasks
        // (the mixed 3D path: from the z-marching refinement step)
        in.fused = (!first && tail > 0 &&
                    ((dim == 2 && !mixed && o->nu2 > 0) || (dim == 3 && step3d_opts(dim, o))))
                       ? 1 : 0;
        in.h = p[i].h;
        in.eps = p[i].eps;
        in.gamma = p[i].gamma;
        in.dt = p[i].dt;
        L.info.push_back(in);
        packed += cells[0];
        L.max_nlev = std::max(L.max_nlev, nlev);
        L.depth = std::max(L.depth, tail);
        if (L.max_cells.size() < size_t(nlev)) L.max_cells.resize(nlev, 0);
        for (int l = 0; l < nlev; ++l) L.max_cells[l] = std::max(L.max_cells[l], cells[l]);
        double h = p[i].h;
        for (int l = 0; l < nlev; ++l) {
            const int n = cells[l];
            LevelDesc<double>& d = L.desc[size_t(i) * kMaxLevels + l];
            d.nx = ext[3 * l];
            d.ny = ext[3 * l + 1];
            d.nz = ext[3 * l + 2];
            d.n = n;
            const size_t nb = size_t(n) * sizeof(double);
            for (int k = 0; k < 3; ++k) d.u[0][k] = ptr(take(nb));
            // a second copy of u for out-of-place kernels: the tiled smoother
            // (2D) and the FP64 refinement step (mixed, finest level)
            const bool z3 = step3d_opts(dim, o) && l < tail;
            const bool two = dim == 2 || (mixed && l == 0) || z3;
            for (int k = 0; k < 3; ++k) d.u[1][k] = two ? ptr(take(nb)) : d.u[0][k];
            if (l > 0)
                for (int k = 0; k < 3; ++k) d.ub[k] = ptr(take(nb));
            for (int k = 0; k < 3; ++k) d.f[k] = ptr(take(nb));
            for (int k = 0; k < 3; ++k) d.fr[k] = l > 0 ? ptr(take(nb)) : nullptr;
            d.pstar = ptr(take(nb));
            d.psi = ptr(take(nb));
            d.b = nullptr;
            d.h = h;
            d.lam = p[i].dt / (h * h);
            // the whole eps^2 Lap phi is implicit in the first-order step
            d.kap = (first ? 1.0 : 0.75) * p[i].eps * p[i].eps / (h * h);
            d.order = in.order;
            d.gamma = p[i].gamma;
            if (mixed) {
                LevelDesc<float>& e = L.desc32[size_t(i) * kMaxLevels + l];
                e.nx = d.nx;
                e.ny = d.ny;
                e.nz = d.nz;
                e.n = n;
                const size_t nf = size_t(n) * sizeof(float);
                for (int k = 0; k < 3; ++k) e.u[0][k] = ptr32(take(nf));
                for (int k = 0; k < 3; ++k) e.u[1][k] = dim == 2 || z3 ? ptr32(take(nf)) : e.u[0][k];
                if (l > 0)
                    for (int k = 0; k < 3; ++k) e.ub[k] = ptr32(take(nf));
                for (int k = 0; k < 3; ++k) e.f[k] = ptr32(take(nf));
                for (int k = 0; k < 3; ++k) e.fr[k] = l > 0 ? ptr32(take(nf)) : nullptr;
                e.pstar = ptr32(take(nf));
                e.psi = ptr32(take(nf));
                e.b = ptr32(take(nf));
                e.h = float(h);
                e.lam = float(d.lam);
                e.kap = float(d.kap);
                e.order = d.order;
                e.gamma = float(d.gamma);
            }
            h *= 2.0;
            cell_tasks(L.A[l], i, n);
            if (l < tail) cell_tasks(L.B[l], i, n);
            // levels above the tail have even extents: n / 2 cells per color
            if (l < tail) cell_tasks(L.Bh[l], i, n / 2);
            if (dim == 2) tile_tasks(L.Tall[l], i, d.nx, d.ny, L.tile_y[l]);
            if (dim == 2 && l < tail) {
                tile_tasks(L.T[l], i, d.nx, d.ny, L.tile_y[l]);
                // the autotuner may cut coarse levels into shorter tiles
                const int ymin = l > 0 ? chhs::kTileYTiny : chhs::kTileY;
                L.cap_T[l] += size_t((d.nx + chhs::kTileX - 1) / chhs::kTileX) *
                              size_t((d.ny + ymin - 1) / ymin);
            }
            lnx[l][i] = d.nx;
            lny[l][i] = d.ny;
            lnz[l][i] = d.nz;
            if (l < tail) lnx_t[l][i] = d.nx;
        }
        for (int l = 0; l + 1 < nlev && l < tail; ++l) cell_tasks(L.Bc[l], i, cells[l + 1]);
        // coarse levels above the tail (the tail forms its top level's f itself)
        for (int l = 0; l + 1 < tail; ++l) cell_tasks(L.Bcs[l], i, cells[l + 1]);
        if (!in.fused) cell_tasks(L.A0n, i, cells[0]);
        if (!in.fused && mixed && dim == 3 && step3d_opts(dim, o)) cell_tasks(L.A0x, i, cells[0]);
        if (tail == 0) cell_tasks(L.A0t, i, cells[0]);
        L.tail_insts.push_back(i);
    }
    // 2D smoother per level: row-streaming strips or square tiles (the same
    // choice for the FP64 and the FP32 hierarchy)
    if (dim == 2)
        for (int l = 0; l < kMaxLevels; ++l) {
            const int slots = strip_slots(l == 0 && !mixed, mixed);
            strip_tasks(L.Sall[l], lnx[l], lny[l], strip_seg(lnx[l], lny[l], slots));
            L.seg[l] = strip_seg(lnx_t[l], lny[l], slots);
            strip_tasks(L.S[l], lnx_t[l], lny[l], L.seg[l]);
            {
                std::vector<StripTask> shortest;
                strip_tasks(shortest, lnx_t[l], lny[l], std::max(8, (L.seg[l] / 4) & ~1));
                L.cap_S[l] = shortest.size();
            }
            L.tile_threads[l] = o->tile_threads;
            // default: strips on the finest level (long segments, two blocks
            // per compute unit), tiles below, where more and shorter blocks
            // hide latency better
            // the strip kernel loads pairs of cells: every grid of the level
            // needs an even x extent
            bool even = true;
            for (int i = 0; i < n_inst; ++i) even = even && (lnx[l][i] < 0 || lnx[l][i] % 2 == 0);
            L.strip[l] = even && o->order != 1 &&
                         (o->smoother == 2 ? !L.Sall[l].empty()
                                                   : (o->smoother == 0 && l == 0 && !L.T[l].empty()));
        }
    L.snx = lnx_t;
    if (step3d_opts(dim, o))
        for (int l = 0; l < kMaxLevels; ++l) {
            L.zseg64[l] = step3_seg(lnx_t[l], lny[l], lnz[l], chhs::kStep3TX64, chhs::kStep3TY64);
            step3_tasks(L.Z64[l], lnx_t[l], lny[l], lnz[l], chhs::kStep3TX64, chhs::kStep3TY64,
                        L.zseg64[l]);
            if (mixed) {
                L.zseg32[l] = step3_seg(lnx_t[l], lny[l], lnz[l], chhs::kStep3TX32, chhs::kStep3TY32);
                step3_tasks(L.Z32[l], lnx_t[l], lny[l], lnz[l], chhs::kStep3TX32, chhs::kStep3TY32,
                            L.zseg32[l]);
            }
            // smoother 4: every level; default: levels with long enough segments
            // (the autotuner may choose anew)
            const int zs = mixed ? L.zseg32[l] : L.zseg64[l];
            L.z3[l] = o->smoother == 4 || zs >= kStep3MinSeg;
        }
    // 3D restriction per instance (never by what else the batch holds): the
    // z-marching residual kernel on levels of at least kRes3MinCells cells, the
    // per-cell kernel on smaller ones (where its short launches win)
    for (int l = 0; l < kMaxLevels; ++l) {
        auto big = [&](int i) {
            return step3d_opts(dim, o) && lnx_t[l][i] >= 0 &&
                   long(lnx[l][i]) * lny[l][i] * lnz[l][i] >= kRes3MinCells;
        };
        for (const Step3Task& t : L.Z64[l])
            if (big(t.inst)) L.ZR64[l].push_back(t);
        for (const Step3Task& t : L.Z32[l])
            if (big(t.inst)) L.ZR32[l].push_back(t);
        for (const CellTask& t : L.Bc[l])
            if (!big(t.inst)) L.BcS[l].push_back(t);
    }
    // 2D mixed precision: tasks of the row-marching refinement step over every
    // instance's finest level (instance, then row segment, then column window)
    if (dim == 2 && mixed) {
        L.march_seg = march_seg(L.info, L.desc, n_inst);
        for (int i = 0; i < n_inst; ++i) {
            const LevelDesc<double>& d = L.desc[size_t(i) * kMaxLevels];
            const int nw = (d.nx + chhs::kMarchCols - 1) / chhs::kMarchCols;
            for (int y0 = 0; y0 < d.ny; y0 += L.march_seg)
                for (int w = 0; w < nw; ++w)
                    L.M0.push_back({i, w, y0, std::min(d.ny, y0 + L.march_seg)});
        }
    }
    L.chain_from = L.max_nlev - 1;
    for (int l = 0; l + 1 < L.max_nlev; ++l)
        if (L.max_cells[l + 1] <= kChainCells) {
            L.chain_from = l;
            break;
        }
    L.sny = lny;
    // per-instance ranges of the finest-level partial buffers
    ranges_of(L.rngA0, n_inst, L.A[0]);
    task_ranges(L.rngM0, n_inst, L.M0);
    fold_of(L.rngM0, L.FM0, L.rngM0f);
    ranges_of(L.rngA0n, n_inst, L.A0n);
    ranges_of(L.rngA0x, n_inst, L.A0x);
    fold_of(L.rngA0, L.FA0, L.rngA0f);
    fold_of(L.rngA0n, L.FA0n, L.rngA0nf);
    fused_ranges(L, n_inst);
    L.partial_cap = int(std::max(L.A[0].size(), L.M0.size()));
    L.partial_t_cap =
        int(std::max<size_t>(1, std::max({L.T[0].size(), L.S[0].size(), L.Z64[0].size()})));
    L.off_desc = take(L.desc.size() * sizeof(LevelDesc<double>));
    L.off_desc32 = take(std::max<size_t>(1, L.desc32.size()) * sizeof(LevelDesc<float>));
    L.off_info = take(L.info.size() * sizeof(InstInfo));
    L.off_tail = take(L.tail_insts.size() * sizeof(int));
    L.off_rngA0 = take(n_inst * sizeof(Range));
    L.off_rngT0 = take(n_inst * sizeof(Range));
    L.off_rngA0n = take(n_inst * sizeof(Range));
    L.off_A0n = take(L.A0n.size() * sizeof(CellTask));
    L.off_A0t = take(L.A0t.size() * sizeof(CellTask));
    L.off_A0x = take(L.A0x.size() * sizeof(CellTask));
    L.off_rngA0x = take(n_inst * sizeof(Range));
    L.off_M0 = take(L.M0.size() * sizeof(StripTask));
    L.off_rngM0 = take(n_inst * sizeof(Range));
    L.off_rngM0f = take(n_inst * sizeof(Range));
    L.off_FM0 = take(L.FM0.size() * sizeof(FoldTask));
    L.off_FA0 = take(L.FA0.size() * sizeof(FoldTask));
    L.off_FA0n = take(L.FA0n.size() * sizeof(FoldTask));
    L.off_rngA0f = take(n_inst * sizeof(Range));
    L.off_rngA0nf = take(n_inst * sizeof(Range));
    for (int l = 0; l < kMaxLevels; ++l) {
        L.off_A.push_back(take(L.A[l].size() * sizeof(CellTask)));
        L.off_B.push_back(take(L.B[l].size() * sizeof(CellTask)));
        L.off_Bh.push_back(take(L.Bh[l].size() * sizeof(CellTask)));
        L.off_Bcs.push_back(take(L.Bcs[l].size() * sizeof(CellTask)));
        L.off_Bc.push_back(take(L.Bc[l].size() * sizeof(CellTask)));
        L.tile_y_all[l] = L.tile_y[l];
        L.off_T.push_back(take(std::max(L.T[l].size(), L.cap_T[l]) * sizeof(TileTask)));
        L.off_Tall.push_back(take(L.Tall[l].size() * sizeof(TileTask)));
        L.off_S.push_back(take(std::max(L.S[l].size(), L.cap_S[l]) * sizeof(StripTask)));
        L.off_Sall.push_back(take(L.Sall[l].size() * sizeof(StripTask)));
        L.off_Z64.push_back(take(L.Z64[l].size() * sizeof(Step3Task)));
        L.off_Z32.push_back(take(L.Z32[l].size() * sizeof(Step3Task)));
        L.off_ZR64.push_back(take(L.ZR64[l].size() * sizeof(Step3Task)));
        L.off_ZR32.push_back(take(L.ZR32[l].size() * sizeof(Step3Task)));
        L.off_BcS.push_back(take(L.BcS[l].size() * sizeof(CellTask)));
    }
    L.off_partial = take(size_t(L.partial_cap) * chhs::kPartialStride * sizeof(double));
    L.off_partial_t = take(size_t(L.partial_t_cap) * chhs::kPartialStride * sizeof(double));
    L.off_partial_f = take(std::max<size_t>(1, std::max({L.FA0.size(), L.FA0n.size(), L.FM0.size()})) *
                           chhs::kPartialStride * sizeof(double));
    // res | act_next | cycles contiguous: one readback per cycle
    L.off_res = take(size_t(n_inst) * chhs::kResStride * sizeof(double) + 2 * n_inst * sizeof(int));
    L.off_act_next = L.off_res + size_t(n_inst) * chhs::kResStride * sizeof(double);
    L.off_cycles = L.off_act_next + n_inst * sizeof(int);
    L.off_eres = take(size_t(n_inst) * chhs::kResStride * sizeof(double));
    L.off_act_cycle = take(n_inst * sizeof(int));
    L.off_act_last = take(n_inst * sizeof(int));
    L.bytes = off;
    return true;
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        if ((expr) != hipSuccess) return CHHS_E_HIP;   \
    } while (0)

int check_launch() { return hipGetLastError() == hipSuccess ? CHHS_OK : CHHS_E_HIP; }

template <typename Task>
int upload(Table<Task>& t, char* base, size_t off, const std::vector<Task>& v, hipStream_t st) {
    t.dev = reinterpret_cast<Task*>(base + off);
    t.n = int(v.size());
    if (!v.empty())
        HIP_TRY(hipMemcpyAsync(t.dev, v.data(), v.size() * sizeof(Task), hipMemcpyHostToDevice, st));
    return CHHS_OK;
}

// ---- kernel timing ---------------------------------------------------------------------

hipEvent_t pooled_event(chhs_ctx* c) {
    if (c->ev_pool.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
}

// opts.timing: 1 times every class, any other nonzero value is a mask of
// (1 << (class + 1)) bits.  Every event pair adds a few microseconds between
// launches, so timing only the classes of interest keeps the schedule close to
// the untimed one.
bool timed(const chhs_ctx* c, int cls) {
    const int t = c->opts.timing;
    return t == 1 || (t != 0 && ((t >> (cls + 1)) & 1));
}

// Brackets the launches issued during its lifetime with a pair of events on
// the context stream when timing is enabled (captured into the graph when a
// cycle is being captured).
class TimedScope {
  public:
    TimedScope(chhs_ctx* c, int cls) : c_(c), cls_(cls) {
        if (!timed(c_, cls_)) return;
        a_ = pooled_event(c_);
        if (a_) (void)hipEventRecord(a_, c_->stream);
    }
    ~TimedScope() {
        if (!timed(c_, cls_) || a_ == nullptr) return;
        hipEvent_t b = pooled_event(c_);
        if (b == nullptr) return;
        (void)hipEventRecord(b, c_->stream);
        if (c_->capturing >= 0)
            c_->graph_pairs[c_->capturing].push_back({a_, b, cls_});
        else
            c_->pending.push_back({a_, b, cls_});
    }

  private:
    chhs_ctx* c_;
    int cls_;
    hipEvent_t a_ = nullptr;
};

void accumulate(chhs_ctx* c, const chhs_ctx::Pending& pe) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
        c->t_ms[pe.cls] += ms;
        c->t_n[pe.cls] += 1;
    }
}

// After a stream synchronisation: accumulate the event pairs of the graph
// replayed since the last one, and accumulate and recycle the eager pairs.
void resolve_timing(chhs_ctx* c) {
    if (c->last_slot >= 0)
        for (auto& pe : c->graph_pairs[c->last_slot]) accumulate(c, pe);
    c->last_slot = -1;
    for (auto& pe : c->pending) {
        accumulate(c, pe);
        c->ev_pool.push_back(pe.a);
        c->ev_pool.push_back(pe.b);
    }
    c->pending.clear();
}

// ---- batched launches ------------------------------------------------------------------

template <typename T>
Batch<T> make_batch(const LevelDesc<T>* desc, const int* cur, int level, const int* active) {
    Batch<T> b;
    b.desc = desc;
    b.active = active;
    b.level = level;
    b.cur = cur[level];
    b.cur_c = 0;    // a coarser level is always at copy 0 when a transfer touches it
    b.pshift = nullptr;
    return b;
}

Batch<double> batch(chhs_ctx* c, int level, const int* active) {
    return make_batch(c->ddesc, c->cur, level, active);
}

Batch<float> batch32(chhs_ctx* c, int level, const int* active) {
    return make_batch(c->ddesc32, c->cur32, level, active);
}

// The hierarchy of one precision: device descriptors, host copies, current
// copies of u per level, tail LDS bytes.
template <typename T>
struct Hier {
    const LevelDesc<T>* dev;
    const std::vector<LevelDesc<T>>* host;
    int* cur;
    size_t tail_lds;
};

Hier<double> hier64(chhs_ctx* c) { return {c->ddesc, &c->lay.desc, c->cur, c->lay.tail_lds}; }
Hier<float> hier32(chhs_ctx* c) { return {c->ddesc32, &c->lay.desc32, c->cur32, c->lay.tail_lds32}; }

// One 2D smoothing launch on level l (row-streaming strips or tiles, as
// planned; all = every instance, else those whose tail starts below l);
// flips the level's current copy.
template <typename T>
void tiled(chhs_ctx* c, const Hier<T>& H, bool all, int l, int ns, int epi, bool pro,
           const int* active, int cls, bool rhs = false, const double* pshift = nullptr,
           bool zero = false, bool post = false) {
    Batch<T> b = make_batch(H.dev, H.cur, l, active);
    b.pshift = pshift;
    const bool level0 = std::is_same<T, double>::value && l == 0;
    double* part = epi == 2 ? c->partial_t : nullptr;
    {
        TimedScope t(c, cls);
        if (c->lay.strip[l]) {
            const Table<StripTask>& st = all ? c->Sall[l] : c->S[l];
            chhs::launch_stream2d<T>(b, st.dev, st.n, level0, ns, epi, pro, zero, part, c->stream);
        } else {
            const Table<TileTask>& tt = all ? c->Tall[l] : c->T[l];
            const int* thr = post && c->lay.tile_threads_post[l] > 0 ? c->lay.tile_threads_post
                                                                     : c->lay.tile_threads;
            chhs::launch_tile2d<T>(b, tt.dev, tt.n, level0, ns, epi, pro,
                                   tile_block(all ? 0 : thr[l], tt.n), rhs,
                                   all ? c->lay.tile_y_all[l] : c->lay.tile_y[l], zero, part,
                                   c->stream);
        }
    }
    H.cur[l] ^= 1;
}

// One fused 3D smoothing step on level l of a hierarchy (the instances above
// their tail); flips the level's current copy.
template <typename T>
void step3(chhs_ctx* c, const Hier<T>& H, int l, const int* active, int cls, int pro = 0,
           bool zero = false, const double* psh = nullptr) {
    Batch<T> b = make_batch(H.dev, H.cur, l, active);
    b.pshift = psh;
    const Table<Step3Task>& z = std::is_same<T, double>::value ? c->Z64[l] : c->Z32[l];
    {
        TimedScope t(c, cls);
        chhs::launch_step3d(b, z.dev, z.n, pro, zero ? 1 : 0, c->stream);
    }
    H.cur[l] ^= 1;
}

// An odd number of out-of-place launches on level l left copy 1 current: copy
// it back so that every level ends each V-cycle on copy 0.
template <typename T>
void restore_copy0(chhs_ctx* c, const Hier<T>& H, int l) {
    for (int i = 0; i < c->n_inst; ++i) {
        const LevelDesc<T>& d = (*H.host)[size_t(i) * kMaxLevels + l];
        if (d.u[1][0] == d.u[0][0] || d.n == 0) continue;
        const size_t nb = size_t(d.n) * sizeof(T);
        for (int k = 0; k < 3; ++k)
            (void)hipMemcpyAsync(d.u[0][k], d.u[1][k], nb, hipMemcpyDeviceToDevice, c->stream);
    }
    H.cur[l] = 0;
}

// 2D levels above the tail are smoothed by the fused tiled / strip kernels
// (the second-order scheme); otherwise by the per-cell red-black kernels.
bool tiled2d(const chhs_ctx* c) { return c->dim == 2 && c->opts.order != 1; }
bool fused3d(const chhs_ctx* c) { return step3d_opts(c->dim, &c->opts); }
// Level l of the smoothing hierarchy takes the fused 3D step.
bool z3_at(const chhs_ctx* c, int l) { return fused3d(c) && c->lay.z3[l]; }

// nsweeps smoothing steps on level l of the FP64 hierarchy (2D: tiled,
// including levels inside the tail for kernel tests; 3D and the first-order
// step: per-cell red-black).
void smooth_steps(chhs_ctx* c, int l, int nsweeps, const int* active, int cls) {
    if (tiled2d(c)) {
        while (nsweeps > 0) {
            const int k = nsweeps >= 2 ? 2 : 1;
            nsweeps -= k;
            tiled(c, hier64(c), true, l, k, 0, false, active, cls);
        }
        return;
    }
    if (z3_at(c, l) && c->Z64[l].n > 0) {
        for (int s = 0; s < nsweeps; ++s) step3(c, hier64(c), l, active, cls);
        return;
    }
    Batch<double> b = batch(c, l, active);
    for (int s = 0; s < nsweeps; ++s)
        for (int color = 0; color < 2; ++color) {
            TimedScope t(c, cls);
            chhs::launch_smooth(c->dim, b, c->A[l].dev, c->A[l].n, color, c->stream);
        }
}

// Enqueues one FAS V(nu1, nu2) cycle of one hierarchy over the batch for the
// instances in act_cycle.  FP64: the plain form, whose finest-level post
// launch also yields the fused norm partials; FP32: the correction form,
// starting from a zero correction (zero_corr; the tiled finest level's first
// launch then takes it as implied) or from the previous cycle's.
bool zero_start(const chhs_ctx* c);

template <typename T>
void enqueue_vcycle(chhs_ctx* c, const Hier<T>& H, bool zero_corr = true) {
    constexpr bool kPlain = std::is_same<T, double>::value;
    const int dim = c->dim;
    const int* act = c->act_cycle;
    const int depth = c->lay.depth;
    const chhs_opts& o = c->opts;
    for (int d = 0; d < depth; ++d) {
        const int pre_cls = d == 0 ? CHHS_K_PRE0 : CHHS_K_COARSE;
        const int xfer_cls = d == 0 ? CHHS_K_TRANSFER0 : CHHS_K_COARSE;
        const int nu1 = nu_pre(o, d);
        if (tiled2d(c) && nu1 > 0) {
            // on a tiled coarse level the first launch forms f = fr + N(u)
            const bool rhs = d > 0 && !c->lay.strip[d];
            // ... and on the finest level it subtracts a deferred p shift, or,
            // for a correction cycle, takes the zero starting correction as
            // implied
            const double* psh = kPlain && d == 0 && c->defer_shift ? c->res : nullptr;
            const bool zero = !kPlain && d == 0 && zero_corr;
            bool first = true;
            int rem = nu1;
            while (rem > 2) {
                tiled(c, H, false, d, 2, 0, false, act, pre_cls, rhs && first, first ? psh : nullptr,
                      zero && first);
                first = false;
                rem -= 2;
            }
            tiled(c, H, false, d, rem, 1, false, act, pre_cls, rhs && first, first ? psh : nullptr,
                  zero && first);
        } else {
            if (z3_at(c, d)) {
                // on the finest level the first step takes the zero correction
                // as implied (correction cycles) or subtracts a deferred p shift
                const bool zero = !kPlain && d == 0 && zero_corr && zero_start(c);
                const double* psh = kPlain && d == 0 && c->defer_shift ? c->res : nullptr;
                for (int s = 0; s < nu1; ++s)
                    step3(c, H, d, act, pre_cls, 0, zero && s == 0, s == 0 ? psh : nullptr);
            }
            else if (!tiled2d(c))
                for (int s = 0; s < nu1; ++s)
                    for (int color = 0; color < 2; ++color) {
                        TimedScope t(c, pre_cls);
                        chhs::launch_smooth_color(dim, make_batch(H.dev, H.cur, d, act),
                                                  c->Bh[d].dev, c->Bh[d].n, color, c->stream);
                    }
            TimedScope t(c, xfer_cls);
            // z marching for the instances whose level is large, per cell for
            // the others (a batched instance restricts as it does alone)
            const Table<Step3Task>& zt = kPlain ? c->ZR64[d] : c->ZR32[d];
            if (zt.n > 0)
                chhs::launch_restrict3d(make_batch(H.dev, H.cur, d, act), zt.dev, zt.n, c->stream);
            if (c->BcS[d].n > 0)
                chhs::launch_restrict_residual(dim, make_batch(H.dev, H.cur, d, act), c->BcS[d].dev,
                                               c->BcS[d].n, c->stream);
        }
        // level d + 1's right-hand side f = fr + N(u), unless its first tiled
        // launch forms it (tail levels: the tail does)
        const bool fused_next =
            tiled2d(c) && nu_pre(o, d + 1) > 0 && d + 1 < depth && !c->lay.strip[d + 1];
        if (!fused_next && c->Bcs[d].n > 0) {
            TimedScope t(c, xfer_cls);
            chhs::launch_coarse_rhs(dim, make_batch(H.dev, H.cur, d, act), c->Bcs[d].dev,
                                    c->Bcs[d].n, c->stream);
        }
    }
    {
        // an instance's tail level is only ever written by the restriction into
        // it (copy 0) and by the tail itself: it is always read from copy 0
        TimedScope t(c, depth == 0 ? CHHS_K_PRE0 : CHHS_K_COARSE);
        chhs::launch_tail<T, !kPlain>(dim, H.dev, c->dinfo, c->tail_insts, c->n_inst, act, 0u,
                                      cycle_shape(o),
                                      kPlain && c->defer_shift ? c->res : nullptr, H.tail_lds,
                                      c->stream);
    }
    const bool bil = o.prolong == 1;
    for (int d = depth - 1; d >= 0; --d) {
        const int post_cls = d == 0 ? CHHS_K_POST0 : CHHS_K_COARSE;
        const int xfer_cls = d == 0 ? CHHS_K_TRANSFER0 : CHHS_K_COARSE;
        const int nu2 = nu_post(o, d);
        if (tiled2d(c) && nu2 > 0) {
            // the fused kernels prolong by injection while they load; the
            // bilinear prolongation is a launch of its own before them
            if (bil) {
                TimedScope t(c, xfer_cls);
                chhs::launch_prolong(dim, make_batch(H.dev, H.cur, d, act), c->B[d].dev, c->B[d].n,
                                     true, c->stream);
            }
            int rem = nu2;
            bool first = !bil;
            while (rem > 0) {
                const int k = rem >= 2 ? 2 : 1;
                rem -= k;
                const bool norm = kPlain && d == 0 && rem == 0 && c->fused_norm;
                tiled(c, H, false, d, k, norm ? 2 : 0, first, act, post_cls, false, nullptr, false,
                      true);
                first = false;
            }
        } else {
            // the fused 3D step takes the prolongation into its first launch
            const bool pro3 = z3_at(c, d) && nu2 > 0;
            if (!pro3) {
                TimedScope t(c, xfer_cls);
                chhs::launch_prolong(dim, make_batch(H.dev, H.cur, d, act), c->B[d].dev, c->B[d].n,
                                     bil, c->stream);
            }
            if (z3_at(c, d))
                for (int s = 0; s < nu2; ++s) step3(c, H, d, act, post_cls, s == 0 ? (bil ? 2 : 1) : 0);
            else if (!tiled2d(c))
                for (int s = 0; s < nu2; ++s)
                    for (int color = 0; color < 2; ++color) {
                        TimedScope t(c, post_cls);
                        chhs::launch_smooth_color(dim, make_batch(H.dev, H.cur, d, act),
                                                  c->Bh[d].dev, c->Bh[d].n, color, c->stream);
                    }
        }
        if (H.cur[d] != 0) restore_copy0(c, H, d);
    }
}

// ---- autotuning of the 2D smoothing kernels ----------------------------------------------

// Keeps the device busy for about `ticks` periods of the constant-rate wall
// clock (bounded wait, one wave).  Launched before a timed sequence, it lets the
// host enqueue the whole sequence before the device reaches it, so the events
// time the kernels back to back (as a captured graph replays them) rather than
// the host's launch rate.
__global__ __launch_bounds__(64) void k_spin(long long ticks) {
    const long long t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

// Enqueues ~200 us of k_spin on the context's stream.
int spin_ahead(chhs_ctx* c) {
    static thread_local int rate_khz = 0;
    if (rate_khz <= 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
            rate_khz <= 0)
            rate_khz = 100000;      // the 100 MHz clock of gfx9
    }
    hipLaunchKernelGGL(k_spin, dim3(1), dim3(64), 0, c->stream, (long long)rate_khz / 5);
    return check_launch();
}

// Device time (ms) of one level's pre- and post-smoothing launches as a V-cycle
// issues them, the best of `reps` repetitions; *pre and *post get the best
// time of each part.
template <typename T>
float time_level(chhs_ctx* c, const Hier<T>& H, int l, int reps, hipEvent_t ea, hipEvent_t em,
                 hipEvent_t eb, float* pre, float* post) {
    const chhs_opts& o = c->opts;
    const bool norm = std::is_same<T, double>::value && l == 0 && c->fused_norm;
    float best = 1e30f;
    *pre = *post = 1e30f;
    for (int r = 0; r < reps; ++r) {
        if (spin_ahead(c) != CHHS_OK || hipEventRecord(ea, c->stream) != hipSuccess) return -1.0f;
        // the level's right-hand side: formed by its first tiled launch, or
        // by a separate launch before strips
        const bool rhs = l > 0 && !c->lay.strip[l];
        if (l > 0 && c->lay.strip[l] && c->Bcs[l - 1].n > 0)
            chhs::launch_coarse_rhs(2, make_batch(H.dev, H.cur, l - 1, nullptr), c->Bcs[l - 1].dev,
                                    c->Bcs[l - 1].n, c->stream);
        // the FP32 finest level's first launch takes a zero correction as implied
        const bool zero = !std::is_same<T, double>::value && l == 0;
        bool first = true;
        int rem = nu_pre(o, l);
        while (rem > 2) {
            tiled(c, H, false, l, 2, 0, false, nullptr, CHHS_K_PRE0, rhs && first, nullptr,
                  zero && first);
            first = false;
            rem -= 2;
        }
        tiled(c, H, false, l, rem, 1, false, nullptr, CHHS_K_PRE0, rhs && first, nullptr,
              zero && first);
        if (hipEventRecord(em, c->stream) != hipSuccess) return -1.0f;
        rem = nu_post(o, l);
        bool pro = o.prolong != 1;
        while (rem > 0) {
            const int k = rem >= 2 ? 2 : 1;
            rem -= k;
            tiled(c, H, false, l, k, norm && rem == 0 ? 2 : 0, pro, nullptr, CHHS_K_POST0, false,
                  nullptr, false, true);
            pro = false;
        }
        if (hipEventRecord(eb, c->stream) != hipSuccess || hipEventSynchronize(eb) != hipSuccess)
            return -1.0f;
        float ms = 0.0f, m1 = 0.0f, m2 = 0.0f;
        if (hipEventElapsedTime(&ms, ea, eb) != hipSuccess ||
            hipEventElapsedTime(&m1, ea, em) != hipSuccess ||
            hipEventElapsedTime(&m2, em, eb) != hipSuccess)
            return -1.0f;
        best = std::min(best, ms);
        *pre = std::min(*pre, m1);
        *post = std::min(*post, m2);
    }
    if (H.cur[l] != 0) restore_copy0(c, H, l);
    return best;
}

// Device time (ms) of nu1 + nu2 smoothing steps on 3D level l of hierarchy H
// with the level's current kernel choice, the best of `reps`.
template <typename T>
float time_level3(chhs_ctx* c, const Hier<T>& H, int l, int reps, hipEvent_t ea, hipEvent_t eb) {
    const int n1 = nu_pre(c->opts, l), n2 = nu_post(c->opts, l);
    const bool bil = c->opts.prolong == 1;
    float best = 1e30f;
    for (int r = 0; r < reps; ++r) {
        if (spin_ahead(c) != CHHS_OK || hipEventRecord(ea, c->stream) != hipSuccess) return -1.0f;
        // nu1 steps, the prolongation (a launch of its own unless the first
        // fused post step takes it), nu2 steps
        for (int s = 0; s < n1 + n2; ++s) {
            const bool first_post = s == n1;
            if (z3_at(c, l)) {
                step3(c, H, l, nullptr, CHHS_K_PRE0, first_post ? (bil ? 2 : 1) : 0);
            } else {
                if (first_post)
                    chhs::launch_prolong(3, make_batch(H.dev, H.cur, l, nullptr), c->B[l].dev,
                                         c->B[l].n, bil, c->stream);
                for (int color = 0; color < 2; ++color)
                    chhs::launch_smooth_color(3, make_batch(H.dev, H.cur, l, nullptr), c->Bh[l].dev,
                                              c->Bh[l].n, color, c->stream);
            }
        }
        if (hipEventRecord(eb, c->stream) != hipSuccess || hipEventSynchronize(eb) != hipSuccess)
            return -1.0f;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ea, eb) != hipSuccess) return -1.0f;
        best = std::min(best, ms);
    }
    if (H.cur[l] != 0) restore_copy0(c, H, l);
    return best;
}

// 3D: per level above the tail, the fused step or one launch per color,
// whichever smooths faster on the problem at hand.
int autotune3(chhs_ctx* c) {
    hipEvent_t ea = nullptr, eb = nullptr;
    if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
        if (ea) (void)hipEventDestroy(ea);
        return CHHS_E_HIP;
    }
    const chhs_opts saved = c->opts;
    c->opts.timing = 0;
    int rc = CHHS_OK;
    for (int l = 0; l < c->lay.depth && rc == CHHS_OK; ++l) {
        if ((c->mixed ? c->Z32[l].n : c->Z64[l].n) == 0) continue;
        float t[2];
        for (int k = 0; k < 2 && rc == CHHS_OK; ++k) {
            c->lay.z3[l] = k == 1;
            t[k] = c->mixed ? time_level3(c, hier32(c), l, 3, ea, eb)
                            : time_level3(c, hier64(c), l, 3, ea, eb);
            if (t[k] < 0.0f) rc = CHHS_E_HIP;
        }
        if (rc == CHHS_OK) c->lay.z3[l] = t[1] < t[0];
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    c->opts = saved;
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return check_launch();
}

// Picks, per 2D level above the tail, the fastest of: tiles with 256, 512 or
// 1024 threads (on coarse levels each also 16, 8 and 4 rows high; on the FP32
// finest level also 64 x 32), the pre- and the post-smoothing launches each
// with the block size that is fastest for it, or strips with 1/4, 1/2, 1, 2 or 4
// times the default segment height.  Runs the
// candidates on the workspace as it is (its contents do not matter for the
// timing and are rewritten by the next setup).
int autotune(chhs_ctx* c) {
    Layout& L = c->lay;
    hipEvent_t ea = nullptr, em = nullptr, eb = nullptr;
    if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&em) != hipSuccess ||
        hipEventCreate(&eb) != hipSuccess) {
        if (ea) (void)hipEventDestroy(ea);
        if (em) (void)hipEventDestroy(em);
        return CHHS_E_HIP;
    }
    const chhs_opts saved = c->opts;
    c->opts.timing = 0;
    int rc = CHHS_OK;
    for (int l = 0; l < L.depth && rc == CHHS_OK; ++l) {
        if (c->T[l].n == 0) continue;
        struct Cand {
            bool strip;
            int threads, seg, ty;
        };
        std::vector<Cand> cands;
        for (int ty : {chhs::kTileY, chhs::kTileYSmall, chhs::kTileYTiny}) {
            if (l == 0 && ty != chhs::kTileY) continue;     // the finest level has 64 x 16 tiles
            for (int nt : {256, 512, 1024}) cands.push_back({false, nt, 0, ty});
        }
        // ... or, on the FP32 finest level (mixed precision), 64 x 32 (on
        // coarse FP32 levels they were never faster)
        if (l == 0 && c->mixed)
            for (int nt : {512, 1024}) cands.push_back({false, nt, 0, chhs::kTileYTall});
        bool even = true;
        int maxny = 0;
        for (int i = 0; i < c->n_inst; ++i)
            if (L.snx[l][i] >= 0) {
                even = even && L.snx[l][i] % 2 == 0;
                maxny = std::max(maxny, L.sny[l][i]);
            }
        const int seg0 = L.seg[l];
        if (even && c->S[l].n > 0) {
            // segments of a quarter, half, one, two and four times the default
            // height (even, at least 8 rows; the strip table holds the tasks of
            // the shortest)
            for (int d : {4, 2}) {
                const int sg = std::max(8, (seg0 / d) & ~1);
                if (sg < seg0 && (cands.empty() || !cands.back().strip || sg > cands.back().seg))
                    cands.push_back({true, 0, sg, 0});
            }
            for (int m = 1; m <= 4; m *= 2) {
                const int sg = std::min(seg0 * m, (maxny + 1) & ~1);
                if (m == 1 || sg > cands.back().seg) cands.push_back({true, 0, sg, 0});
            }
        }
        const size_t cap = std::max(L.cap_S[l], size_t(c->S[l].n));
        auto apply = [&](const Cand& k) -> int {
            L.strip[l] = k.strip;
            L.tile_threads[l] = k.threads;
            L.tile_threads_post[l] = 0;
            if (!k.strip) {
                if (k.ty == L.tile_y[l]) return CHHS_OK;
                // re-cut the level's tiles (same instance order as the plan)
                L.T[l].clear();
                for (int i = 0; i < c->n_inst; ++i)
                    if (L.snx[l][i] >= 0) tile_tasks(L.T[l], i, L.snx[l][i], L.sny[l][i], k.ty);
                if (L.T[l].size() > L.cap_T[l]) return CHHS_E_INVAL;
                L.tile_y[l] = k.ty;
                c->T[l].n = int(L.T[l].size());
                HIP_TRY(hipMemcpyAsync(c->T[l].dev, L.T[l].data(), L.T[l].size() * sizeof(TileTask),
                                       hipMemcpyHostToDevice, c->stream));
                return CHHS_OK;
            }
            L.seg[l] = k.seg;
            L.S[l].clear();
            strip_tasks(L.S[l], L.snx[l], L.sny[l], k.seg);
            if (L.S[l].size() > cap) return CHHS_E_INVAL;
            c->S[l].n = int(L.S[l].size());
            HIP_TRY(hipMemcpyAsync(c->S[l].dev, L.S[l].data(), L.S[l].size() * sizeof(StripTask),
                                   hipMemcpyHostToDevice, c->stream));
            return CHHS_OK;
        };
        std::vector<float> t_pre(cands.size()), t_post(cands.size());
        for (int k = 0; k < int(cands.size()) && rc == CHHS_OK; ++k) {
            rc = apply(cands[k]);
            if (rc) break;
            const float ms = c->mixed
                                 ? time_level(c, hier32(c), l, 3, ea, em, eb, &t_pre[k], &t_post[k])
                                 : time_level(c, hier64(c), l, 3, ea, em, eb, &t_pre[k], &t_post[k]);
            if (ms < 0.0f) rc = CHHS_E_HIP;
        }
        if (rc) break;
        // strips by their pre + post time; tiles per height by the fastest
        // pre-smoothing block size plus the fastest post-smoothing one (the
        // same tasks, so the two launches may take different block sizes)
        float best = 1e30f;
        int pick = 0, pick_post = -1;
        for (int k = 0; k < int(cands.size()); ++k) {
            if (cands[k].strip) {
                if (t_pre[k] + t_post[k] < best) {
                    best = t_pre[k] + t_post[k];
                    pick = k;
                    pick_post = -1;
                }
                continue;
            }
            int kq = k;
            for (int j = 0; j < int(cands.size()); ++j)
                if (!cands[j].strip && cands[j].ty == cands[k].ty && t_post[j] < t_post[kq]) kq = j;
            if (t_pre[k] + t_post[kq] < best) {
                best = t_pre[k] + t_post[kq];
                pick = k;
                pick_post = kq;
            }
        }
        rc = apply(cands[pick]);
        if (rc == CHHS_OK && pick_post >= 0) L.tile_threads_post[l] = cands[pick_post].threads;
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(em);
    (void)hipEventDestroy(eb);
    c->opts = saved;
    if (rc) return rc;
    fused_ranges(L, c->n_inst);
    HIP_TRY(hipMemcpyAsync(c->rngT0, L.rngT0.data(), c->n_inst * sizeof(Range),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return check_launch();
}

// The partials of a task table for the per-instance reduction: folded first
// when an instance has more than kFold of them (F non-empty).
void fold_table(chhs_ctx* c, const Table<FoldTask>& F, const Range* rng, const Range* rngf,
                const int* act, const double** src, const Range** out) {
    *src = c->partial;
    *out = rng;
    if (F.n == 0) return;
    chhs::launch_fold_partials(c->partial, F.dev, F.n, act, c->partial_f, c->stream);
    *src = c->partial_f;
    *out = rngf;
}

// The partials that the per-instance reduction reads for the finest level's
// per-cell tasks (n_only: the tasks of instances without a fused norm, else
// every instance's), folded first when an instance has more than kFold.
void fold_cells(chhs_ctx* c, bool n_only, const int* act, const double** src, const Range** rng) {
    const Table<FoldTask>& F = n_only ? c->FA0n : c->FA0;
    *src = c->partial;
    *rng = n_only ? c->rngA0n : c->rngA0;
    if (F.n == 0) return;
    chhs::launch_fold_partials(c->partial, F.dev, F.n, act, c->partial_f, c->stream);
    *src = c->partial_f;
    *rng = n_only ? c->rngA0nf : c->rngA0f;
}

// Plain FP64: one V-cycle, the residual norms (p normalised to mean zero).
void enqueue_plain_cycle(chhs_ctx* c, bool count) {
    const int* act = c->act_cycle;
    const chhs_opts& o = c->opts;
    chhs::launch_copy_int(c->act_cycle, c->act_next, c->n_inst, c->stream);
    enqueue_vcycle(c, hier64(c));
    TimedScope t(c, CHHS_K_NORM);
    // 3D: the z-marching residual over the finest level's fused-step tasks
    if (c->dim == 3 && c->Z64[0].n > 0)
        chhs::launch_residual3d_partials(batch(c, 0, act), c->Z64[0].dev, c->Z64[0].n,
                                         c->partial_t, c->stream);
    // instances without a fused finest-level norm: per-cell residual partials
    chhs::launch_residual_partials(c->dim, batch(c, 0, act), c->A0n.dev, c->A0n.n, c->partial,
                                   c->stream);
    const double* src;
    const Range* rng;
    fold_cells(c, true, act, &src, &rng);
    chhs::launch_inst_reduce(src, rng, c->partial_t, c->rngT0, 1, c->dinfo, act,
                             c->act_next, c->cycles, c->res, c->n_inst, o.tol,
                             count ? o.max_vcycles : 1 << 30, count ? 1 : 0, c->stream);
    if (!c->defer_shift)
        chhs::launch_shift_p(batch(c, 0, act), c->A[0].dev, c->A[0].n, c->res, c->stream);
}

// Applies a deferred p shift to the finest level's p and clears it.
void apply_pshift(chhs_ctx* c) {
    chhs::launch_shift_p(batch(c, 0, nullptr), c->A[0].dev, c->A[0].n, c->res, c->stream);
    chhs::launch_clear_pshift(c->res, c->n_inst, c->stream);
}

// Mixed precision, one refinement step: zero FP32 correction, inner_cycles FP32
// correction-form V-cycles, then in FP64 u += e, the residual of the full
// system (into the FP32 right-hand side) and its norms.
// The first FP32 launch of a correction cycle on the finest level is a tiled
// (2D) or fused 3D pre-smoothing launch that takes the zero starting
// correction as implied (nu1 > 0); otherwise the correction is cleared by a
// pass of its own, as it is for instances whose finest level the
// one-workgroup tail holds.
bool zero_start(const chhs_ctx* c) {
    return c->opts.nu1 > 0 && (tiled2d(c) || z3_at(c, 0));
}

// p's mean is not subtracted here: N(u) depends on p through differences only,
// so the residual and the cycle do not change; res slot 4 holds the mean of the
// stored p (the reduction of p'), and the copy to the caller's arrays (or
// apply_pshift) subtracts it.
void enqueue_refinement(chhs_ctx* c, bool count, bool add) {
    const int* act = c->act_cycle;
    const chhs_opts& o = c->opts;
    // this refinement's flags from the last reduction; the previous ones kept
    // for the instances that have just converged
    chhs::launch_roll_flags(c->act_last, c->act_cycle, c->act_next, c->n_inst, c->stream);
    if (add) {
        const Table<CellTask>& z = zero_start(c) ? c->A0t : c->A[0];
        chhs::launch_zero_correction(batch32(c, 0, act), z.dev, z.n, c->stream);
        enqueue_vcycle(c, hier32(c));
        for (int k = 1; k < o.inner_cycles; ++k) enqueue_vcycle(c, hier32(c), false);
    }
    const bool rows = c->M0.n > 0;       // 2D: the row-marching kernel
    // 3D: z marching over the finest level's fused-step tasks (partials into
    // the fused buffer), per cell for instances whose finest level is the tail
    const bool zm = c->dim == 3 && c->Z64[0].n > 0;
    {
        TimedScope t(c, CHHS_K_REFINE);
        if (rows) {
            chhs::launch_mixed_residual_rows(batch(c, 0, add ? act : nullptr), batch32(c, 0, act),
                                             c->M0.dev, c->M0.n, add ? 1 : 0,
                                             add ? c->act_last : nullptr, c->partial, c->stream);
        } else if (zm) {
            chhs::launch_refine3d(batch(c, 0, add ? act : nullptr), batch32(c, 0, act), c->Z64[0].dev,
                                  c->Z64[0].n, add ? 1 : 0, add ? c->act_last : nullptr,
                                  c->partial_t, c->stream);
            if (c->A0x.n > 0)
                chhs::launch_mixed_residual(c->dim, batch(c, 0, add ? act : nullptr),
                                            batch32(c, 0, act), c->A0x.dev, c->A0x.n, add ? 1 : 0,
                                            add ? c->act_last : nullptr, c->partial, c->stream);
        } else {
            chhs::launch_mixed_residual(c->dim, batch(c, 0, add ? act : nullptr),
                                        batch32(c, 0, act), c->A[0].dev, c->A[0].n, add ? 1 : 0,
                                        add ? c->act_last : nullptr, c->partial, c->stream);
        }
    }
    TimedScope t(c, CHHS_K_NORM);
    c->cur[0] ^= 1;
    const double* src;
    const Range* rng;
    if (rows) {
        fold_table(c, c->FM0, c->rngM0, c->rngM0f, add ? act : nullptr, &src, &rng);
    } else if (zm) {
        src = c->partial;
        rng = c->rngA0x;
    } else {
        fold_cells(c, false, add ? act : nullptr, &src, &rng);
    }
    chhs::launch_inst_reduce(src, rng, zm ? c->partial_t : nullptr, zm ? c->rngT0 : nullptr,
                             zm ? 1 : 0, c->dinfo, add ? act : nullptr, c->act_next, c->cycles,
                             c->res, c->n_inst, o.tol, count ? o.max_vcycles : 1 << 30,
                             count ? 1 : 0, c->stream);
}

void enqueue_cycle(chhs_ctx* c, bool count) {
    if (c->mixed)
        enqueue_refinement(c, count, true);
    else
        enqueue_plain_cycle(c, count);
}

// Readback of res | act_next | cycles (contiguous on both sides) into pinned
// mirror `buf` (enqueued).
int enqueue_readback(chhs_ctx* c, int buf = 0) {
    const int n = c->n_inst;
    const size_t bytes = size_t(n) * chhs::kResStride * sizeof(double) + 2 * n * sizeof(int);
    HIP_TRY(hipMemcpyAsync(c->hbuf[buf], c->res, bytes, hipMemcpyDeviceToHost, c->stream));
    return CHHS_OK;
}

// Points the host view (hres, hact, hcyc) at mirror `buf`.
void view_results(chhs_ctx* c, int buf) {
    const size_t nres = size_t(c->n_inst) * chhs::kResStride;
    c->hres = c->hbuf[buf];
    c->hact = reinterpret_cast<int*>(c->hres + nres);
    c->hcyc = c->hact + c->n_inst;
}

int sync_results(chhs_ctx* c) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    resolve_timing(c);
    return CHHS_OK;
}

void drop_graphs(chhs_ctx* c) {
    for (int s = 0; s < 2; ++s) {
        if (c->gexec[s]) (void)hipGraphExecDestroy(c->gexec[s]);
        if (c->graph[s]) (void)hipGraphDestroy(c->graph[s]);
        c->gexec[s] = nullptr;
        c->graph[s] = nullptr;
        for (auto& pe : c->graph_pairs[s]) {
            c->ev_pool.push_back(pe.a);
            c->ev_pool.push_back(pe.b);
        }
        c->graph_pairs[s].clear();
    }
}

// Captures the counted cycle into graph slot `slot` (reading back into mirror
// `buf`) unless already captured; on failure graphs are disabled for the
// context and the eager path is used.  Timed contexts are not captured (event
// records inside a capture are not reliable here); they launch directly.
void ensure_graph(chhs_ctx* c, int slot, int buf) {
    if (!c->opts.use_graph || c->opts.timing != 0 || c->graph_failed || c->gexec[slot] != nullptr)
        return;
    c->capturing = slot;
    const int saved_cur0 = c->cur[0];
    bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    hipGraph_t g = nullptr;
    if (ok) {
        enqueue_cycle(c, true);
        ok = enqueue_readback(c, buf) == CHHS_OK;
        ok = (hipStreamEndCapture(c->stream, &g) == hipSuccess) && ok && g != nullptr;
    }
    c->capturing = -1;
    if (ok && hipGraphInstantiate(&c->gexec[slot], g, nullptr, nullptr, 0) != hipSuccess) {
        c->gexec[slot] = nullptr;
        ok = false;
    }
    c->graph[slot] = g;
    (void)hipGetLastError();
    c->cur[0] = saved_cur0;   // the capture did not run anything
    if (!ok) {
        c->graph_failed = true;
        drop_graphs(c);
    }
}

// One cycle (plain V-cycle or mixed refinement step) with norms and readback
// into mirror 0, launched directly; returns after the results are on the host.
int run_cycle(chhs_ctx* c, bool count) {
    view_results(c, 0);
    enqueue_cycle(c, count);
    int rc = check_launch();
    if (rc) return rc;
    rc = enqueue_readback(c);
    if (rc) return rc;
    return sync_results(c);
}

bool any_active(chhs_ctx* c) {
    for (int i = 0; i < c->n_inst; ++i)
        if (c->hact[i]) return true;
    return false;
}

// Whether the cycle in flight is expected to leave some instance unconverged:
// its residual after the last cycle read, times the contraction that cycle
// showed (rho, per instance), still more than three times the tolerance.
bool expect_more(const chhs_ctx* c, const std::vector<double>& rho) {
    for (int i = 0; i < c->n_inst; ++i) {
        if (!c->hact[i]) continue;
        const double r = c->hres[size_t(i) * chhs::kResStride + 3];
        if (r * rho[i] > 3.0 * c->opts.tol) return true;
    }
    return false;
}

// The counted cycles of one step until no instance is active: while the cycle
// in flight is not expected to converge, the next one is
// enqueued before the host reads its results (two pinned mirrors, cycles
// alternating between them), so the device does not wait for the host's
// stopping test; near convergence the host reads each cycle first, so that
// no cycle runs for nothing.  A cycle enqueued all the same after the last
// one finds every instance inactive on the device and does nothing; its timing
// events are dropped.  Cycles replay captured graphs (one per mirror) when
// the stream can be captured and no class is timed, else launch directly.
// Mixed precision: a refinement step flips the FP64 finest level's two copies,
// so slot s is the step that starts from copy s, captured with that copy
// current and reading back into mirror s; successive steps alternate slots
// and mirrors as plain cycles do.
// setup_pending: the step's setup was enqueued without waiting, its norms
// arriving in the third mirror; the first cycle is then enqueued at once (it
// does nothing for an instance that is converged already).
int run_cycles(chhs_ctx* c, bool setup_pending = false) {
    if (!setup_pending && !any_active(c)) return CHHS_OK;
    for (int s = 0; s < 2; ++s)
        if (c->cycle_done[s] == nullptr && hipEventCreateWithFlags(&c->cycle_done[s],
                                                                    hipEventDisableTiming) != hipSuccess)
            return CHHS_E_HIP;
    const int cur0 = c->cur[0];
    for (int s = 0; s < 2; ++s) {
        if (c->mixed) c->cur[0] = s;
        ensure_graph(c, s, s);
    }
    c->cur[0] = cur0;
    const bool graphs = c->gexec[0] != nullptr && c->gexec[1] != nullptr;
    // last residual read and the contraction of the last cycle per instance
    // (a typical V-cycle contraction until one has been measured)
    std::vector<double> prev(c->n_inst, 0.0), rho(c->n_inst, 0.1);
    if (!setup_pending)
        for (int i = 0; i < c->n_inst; ++i) prev[i] = c->hres[size_t(i) * chhs::kResStride + 3];
    size_t mark[2] = {0, 0};       // pending timing pairs before each mirror's latest cycle
    int queue[2], nq = 0, next = c->mixed ? c->cur[0] : 0;
    auto launch = [&]() -> int {
        const int s = next;
        mark[s] = c->pending.size();
        if (graphs) {
            HIP_TRY(hipGraphLaunch(c->gexec[s], c->stream));
            if (c->mixed) c->cur[0] ^= 1;    // as the captured step does
        } else {
            enqueue_cycle(c, true);
            int rc = check_launch();
            if (rc == CHHS_OK) rc = enqueue_readback(c, s);
            if (rc) return rc;
        }
        HIP_TRY(hipEventRecord(c->cycle_done[s], c->stream));
        queue[nq++] = s;
        next ^= 1;
        return CHHS_OK;
    };
    int rc = launch();
    if (rc) return rc;
    for (;;) {
        if (nq == 1 && (setup_pending || expect_more(c, rho))) {
            rc = launch();
            if (rc) return rc;
        }
        const int s = queue[0];
        queue[0] = queue[1];
        --nq;
        HIP_TRY(hipEventSynchronize(c->cycle_done[s]));
        if (graphs)
            for (auto& pe : c->graph_pairs[s]) accumulate(c, pe);
        view_results(c, s);
        if (setup_pending) {
            // the setup ran before this cycle: its norms are on the host now
            for (int i = 0; i < c->n_inst; ++i) prev[i] = c->hbuf[2][size_t(i) * chhs::kResStride + 3];
            setup_pending = false;
        }
        for (int i = 0; i < c->n_inst; ++i) {
            const double r = c->hres[size_t(i) * chhs::kResStride + 3];
            if (prev[i] > 0.0 && std::isfinite(r)) rho[i] = r / prev[i];
            prev[i] = r;
        }
        if (!any_active(c)) {
            if (nq == 1) {
                // enqueued before this result: it runs with no active instance
                const int d = queue[0];
                HIP_TRY(hipEventSynchronize(c->cycle_done[d]));
                for (size_t i = mark[d]; i < c->pending.size(); ++i) {
                    c->ev_pool.push_back(c->pending[i].a);
                    c->ev_pool.push_back(c->pending[i].b);
                }
                c->pending.resize(mark[d]);
            }
            break;
        }
        if (nq == 0) {
            rc = launch();
            if (rc) return rc;
        }
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->last_slot = -1;
    resolve_timing(c);
    return CHHS_OK;
}

// Setup of every instance's step system, p normalised to mean zero, and the
// norms of the initial guess on the host.
// defer: leave the mean of the initial p pending (the step loop) rather than
// subtract it at once (callers that read the level's fields).  wait = false
// (the step loop, the cycle tuner): the norms go to the third mirror and nothing is
// synchronised; the cycle loop reads them with its first cycle.
int setup(chhs_ctx* c, const double* phi_prev, const double* phi_cur, const double* mu,
          const double* p, bool defer = false, bool wait = true) {
    const int dim = c->dim;
    {
        TimedScope t(c, CHHS_K_SETUP);
        chhs::launch_fill_int(c->act_next, c->n_inst, 1, c->stream);
        chhs::launch_fill_int(c->cycles, c->n_inst, 0, c->stream);
        chhs::launch_copy_int(c->act_cycle, c->act_next, c->n_inst, c->stream);
        // the initial residual's norm partials in the same pass (mixed
        // precision: also the FP32 frozen fields of the finest level and the
        // residual as the first correction cycle's right-hand side)
        const Batch<float> f32 = c->mixed ? batch32(c, 0, nullptr) : Batch<float>{};
        chhs::launch_setup(dim, batch(c, 0, nullptr), c->A[0].dev, c->A[0].n, c->dinfo, phi_prev,
                           phi_cur, mu, p, c->partial, c->mixed ? &f32 : nullptr, c->stream);
        if (c->mixed) {
            for (int l = 0; l < c->lay.chain_from; ++l)
                chhs::launch_restrict_frozen(dim, batch32(c, l, nullptr), c->A[l + 1].dev,
                                             c->A[l + 1].n, c->stream);
            chhs::launch_restrict_frozen_chain(dim, c->ddesc32, c->dinfo, c->n_inst,
                                               c->lay.chain_from, c->stream);
        } else {
            for (int l = 0; l < c->lay.chain_from; ++l)
                chhs::launch_restrict_frozen(dim, batch(c, l, nullptr), c->A[l + 1].dev,
                                             c->A[l + 1].n, c->stream);
            chhs::launch_restrict_frozen_chain(dim, c->ddesc, c->dinfo, c->n_inst,
                                               c->lay.chain_from, c->stream);
        }
    }
    if (c->mixed) {
        // the residual of the initial guess came with the setup pass: its
        // norms and the flags, as a refinement step without a correction
        // would leave them (u stays in the current FP64 copy)
        TimedScope t(c, CHHS_K_NORM);
        chhs::launch_roll_flags(c->act_last, c->act_cycle, c->act_next, c->n_inst, c->stream);
        const double* src;
        const Range* rng;
        fold_cells(c, false, nullptr, &src, &rng);
        chhs::launch_inst_reduce(src, rng, nullptr, nullptr, 0, c->dinfo, nullptr, c->act_next,
                                 c->cycles, c->res, c->n_inst, c->opts.tol, 1 << 30, 0, c->stream);
    } else {
        TimedScope t(c, CHHS_K_NORM);
        const double* src;
        const Range* rng;
        fold_cells(c, false, nullptr, &src, &rng);
        chhs::launch_inst_reduce(src, rng, nullptr, nullptr, 0, c->dinfo, nullptr,
                                 c->act_next, c->cycles, c->res, c->n_inst, c->opts.tol,
                                 c->opts.max_vcycles, 0, c->stream);
        if (!c->defer_shift)
            chhs::launch_shift_p(batch(c, 0, nullptr), c->A[0].dev, c->A[0].n, c->res, c->stream);
    }
    if (c->defer_shift && !defer) apply_pshift(c);
    int rc = check_launch();
    if (rc) return rc;
    c->loaded = true;
    if (!wait) return enqueue_readback(c, 2);
    view_results(c, 0);
    rc = enqueue_readback(c, 0);
    if (rc) return rc;
    return sync_results(c);
}

const double* hres_of(chhs_ctx* c, int i) { return c->hres + size_t(i) * chhs::kResStride; }

// Enqueues the energies (per instance, kResStride doubles each) and their
// copy into pinned host memory `dst`: workspace mode (ws != 0: the finest
// level's iterate, phi^m and the flow terms) or caller arrays.
// copy (ws only): the step's copy into the caller's arrays in the same pass.
int enqueue_energies(chhs_ctx* c, int ws, const double* phi, const double* q, double* dst,
                     const chhs::CopyOut* copy = nullptr) {
    {
        TimedScope t(c, CHHS_K_SETUP);
        Batch<double> b = batch(c, 0, nullptr);
        b.pshift = c->defer_shift ? c->res : nullptr;
        chhs::launch_energy_partials(c->dim, b, c->A[0].dev, c->A[0].n, c->dinfo, ws, phi, q,
                                     c->partial, c->stream, copy);
        // instances with more than kFold partials: folded in runs first, so
        // that one workgroup per instance reads a few partials
        if (c->FA0.n > 0) {
            chhs::launch_fold_energy(c->partial, c->FA0.dev, c->FA0.n, c->partial_f, c->stream);
            chhs::launch_energy_reduce(c->partial_f, c->rngA0f, c->dinfo, c->eres, c->n_inst,
                                       c->stream);
        } else {
            chhs::launch_energy_reduce(c->partial, c->rngA0, c->dinfo, c->eres, c->n_inst,
                                       c->stream);
        }
    }
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(dst, c->eres, size_t(c->n_inst) * chhs::kResStride * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    return CHHS_OK;
}

// Energies into heres (per instance), waited for.
int energies(chhs_ctx* c, int ws, const double* phi, const double* q) {
    const int rc = enqueue_energies(c, ws, phi, q, c->heres);
    if (rc) return rc;
    return sync_results(c);
}

// Pinned host records of the per-step energies of nsteps steps (kept by the
// context and grown on demand).
// Pinned host allocation and release synchronise the device: the log grows at
// least twofold, and chhs_init reserves kLogSteps0 steps of it (at most
// kLogBytes0), so that a call with a modest step count allocates nothing.
constexpr int kLogSteps0 = 64;
constexpr size_t kLogBytes0 = size_t(1) << 20;
int reserve_log(chhs_ctx* c, int nsteps) {
    size_t need = size_t(nsteps) * size_t(c->n_inst) * chhs::kResStride;
    if (need <= c->hlog_cap) return CHHS_OK;
    need = std::max(need, 2 * c->hlog_cap);
    if (c->hlog != nullptr) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        (void)hipHostFree(c->hlog);
        c->hlog = nullptr;
        c->hlog_cap = 0;
    }
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&c->hlog), need * sizeof(double),
                          hipHostMallocDefault));
    c->hlog_cap = need;
    return CHHS_OK;
}

void fill_energies(chhs_stats& s, const double* e) {
    s.mass = e[0];
    s.E_h = e[1];
    s.F_h = e[2];
    s.diss_mu = e[3];
    s.diss_u = e[4];
    s.max_abs_phi = e[5];
}

// The time-step loop of chhs_step / chhs_step_log.  last: n_inst records of
// the last step (energies of that step), or null; log: nsteps x n_inst records,
// one per step with that step's energies (enqueued after each step's solve,
// read once at the end), or null.
int step_loop(chhs_ctx* c, double* phi_prev, double* phi_cur, double* mu, double* p,
              int nsteps, chhs_stats* last, chhs_stats* log) {
    const int n = c->n_inst;
    std::vector<chhs_stats> st(n);
    for (auto& s : st) std::memset(&s, 0, sizeof(s));
    if (log != nullptr) std::memset(log, 0, size_t(nsteps) * n * sizeof(chhs_stats));
    int rc = log != nullptr ? reserve_log(c, nsteps) : CHHS_OK;
    int done = 0;
    for (int m = 0; m < nsteps && rc == CHHS_OK; ++m) {
        // the setup is not waited for; its norms come with the first cycle
        rc = setup(c, phi_prev, phi_cur, mu, p, true, false);
        if (rc) break;
        rc = run_cycles(c, true);
        if (rc) break;
        for (int i = 0; i < n; ++i) st[i].res0 = c->hbuf[2][size_t(i) * chhs::kResStride + 3];
        for (int i = 0; i < n; ++i) {
            const double* r = hres_of(c, i);
            st[i].vcycles = c->hcyc[i];
            st[i].total_vcycles += c->hcyc[i];
            for (int k = 0; k < 3; ++k) st[i].res[k] = r[k];
            st[i].res_norm = r[3];
            st[i].status = CHHS_OK;
            if (!std::isfinite(r[3]))
                st[i].status = CHHS_E_NONFINITE;
            else if (r[3] > c->opts.tol)
                st[i].status = CHHS_E_NOCONV;
            if (st[i].status != CHHS_OK && rc == CHHS_OK) rc = st[i].status;
        }
        if (rc) {
            if (log != nullptr)
                for (int i = 0; i < n; ++i) log[size_t(m) * n + i] = st[i];
            break;
        }
        // rotate: (phi^{m-1}, phi^m) <- (phi^m, phi^{m+1}); mu, p <- this step's
        // (in the energy pass when the step's energies are wanted)
        const chhs::CopyOut co{phi_prev, phi_cur, mu, p};
        if (log != nullptr) {
            rc = enqueue_energies(c, 1, nullptr, nullptr,
                                  c->hlog + size_t(m) * n * chhs::kResStride, &co);
            if (rc) break;
        } else if (m == nsteps - 1 && last != nullptr) {
            rc = enqueue_energies(c, 1, nullptr, nullptr, c->heres, &co);
            if (rc == CHHS_OK) rc = sync_results(c);
            if (rc) break;
            for (int i = 0; i < n; ++i) fill_energies(st[i], c->heres + size_t(i) * chhs::kResStride);
        } else {
            Batch<double> bo = batch(c, 0, nullptr);
            bo.pshift = c->defer_shift ? c->res : nullptr;
            chhs::launch_copy_out(bo, c->A[0].dev, c->A[0].n, c->dinfo, phi_prev, phi_cur, mu, p,
                                  c->stream);
        }
        rc = check_launch();
        if (rc) break;
        for (int i = 0; i < n; ++i) {
            ++st[i].steps_done;
            if (log != nullptr) log[size_t(m) * n + i] = st[i];
        }
        done = m + 1;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == CHHS_OK) rc = CHHS_E_HIP;
    if (log != nullptr)
        for (int m = 0; m < done; ++m)
            for (int i = 0; i < n; ++i)
                fill_energies(log[size_t(m) * n + i], c->hlog + (size_t(m) * n + i) * chhs::kResStride);
    if (last != nullptr) {
        if (log != nullptr && done > 0)
            for (int i = 0; i < n; ++i) fill_energies(st[i], c->hlog + (size_t(done - 1) * n + i) * chhs::kResStride);
        for (int i = 0; i < n; ++i) last[i] = st[i];
    }
    return rc;
}



}  // namespace
extern "C" {

void chhs_default_opts(chhs_opts* o) {
    if (o == nullptr) return;
    std::memset(o, 0, sizeof(*o));
    o->nu1 = 2;
    o->nu2 = 2;
    o->max_vcycles = 100;
    o->coarse_sweeps = 4;
    o->tol = 1e-10;
    o->precision = 0;
    o->use_graph = 1;
    o->timing = 0;
    o->order = 2;
}

size_t chhs_workspace_bytes(const chhs_problem* p, int32_t n_inst, const chhs_opts* o) {
    if (p == nullptr || n_inst < 1 || !valid_opts(o)) return 0;
    Layout L;
    if (!plan(p, n_inst, o, nullptr, L)) return 0;
    return L.bytes;
}

int chhs_init(const chhs_problem* p, int32_t n_inst, const chhs_opts* o, void* workspace_dev,
              size_t ws_bytes, void* hip_stream, chhs_ctx** out) {
    if (out == nullptr) return CHHS_E_INVAL;
    *out = nullptr;
    if (p == nullptr || n_inst < 1 || !valid_opts(o) || workspace_dev == nullptr)
        return CHHS_E_INVAL;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign != 0) return CHHS_E_INVAL;
    Layout probe;
    if (!plan(p, n_inst, o, nullptr, probe)) return CHHS_E_INVAL;
    if (ws_bytes < probe.bytes) return CHHS_E_NOMEM;
    chhs_ctx* c = new chhs_ctx();
    c->prob.assign(p, p + n_inst);
    c->opts = *o;
    c->n_inst = n_inst;
    c->dim = p[0].dim;
    c->mixed = o->precision == 1;
    c->stream = static_cast<hipStream_t>(hip_stream);
    // The legacy null stream cannot be captured into a graph: without a stream
    // from the caller the context makes one with default flags, which keeps
    // its work ordered with the caller's work on the null stream.
    if (c->stream == nullptr) {
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return CHHS_E_HIP;
        }
        c->own_stream = true;
    }
    c->base = static_cast<char*>(workspace_dev);
    plan(p, n_inst, o, c->base, c->lay);
    Layout& L = c->lay;
    char* b = c->base;
    int rc = CHHS_OK;
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(c->stream);
        for (int k = 0; k < 3; ++k)
            if (c->hbuf[k]) (void)hipHostFree(c->hbuf[k]);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return code;
    };
    if (chhs::prepare_tail<double, false>(c->dim, L.tail_lds) != 0) return fail(CHHS_E_HIP);
    if (c->mixed && chhs::prepare_tail<float, true>(c->dim, L.tail_lds32) != 0)
        return fail(CHHS_E_HIP);
    c->ddesc = reinterpret_cast<LevelDesc<double>*>(b + L.off_desc);
    c->ddesc32 = reinterpret_cast<LevelDesc<float>*>(b + L.off_desc32);
    c->dinfo = reinterpret_cast<InstInfo*>(b + L.off_info);
    c->tail_insts = reinterpret_cast<int*>(b + L.off_tail);
    c->rngA0 = reinterpret_cast<Range*>(b + L.off_rngA0);
    c->rngT0 = reinterpret_cast<Range*>(b + L.off_rngT0);
    c->rngA0n = reinterpret_cast<Range*>(b + L.off_rngA0n);
    c->rngA0x = reinterpret_cast<Range*>(b + L.off_rngA0x);
    c->partial_t = reinterpret_cast<double*>(b + L.off_partial_t);
    c->partial = reinterpret_cast<double*>(b + L.off_partial);
    c->partial_f = reinterpret_cast<double*>(b + L.off_partial_f);
    c->rngA0f = reinterpret_cast<Range*>(b + L.off_rngA0f);
    c->rngA0nf = reinterpret_cast<Range*>(b + L.off_rngA0nf);
    c->res = reinterpret_cast<double*>(b + L.off_res);
    c->eres = reinterpret_cast<double*>(b + L.off_eres);
    c->act_cycle = reinterpret_cast<int*>(b + L.off_act_cycle);
    c->act_last = reinterpret_cast<int*>(b + L.off_act_last);
    c->act_next = reinterpret_cast<int*>(b + L.off_act_next);
    c->cycles = reinterpret_cast<int*>(b + L.off_cycles);
    hipStream_t st = c->stream;
    if (c->mixed && hipMemcpyAsync(c->ddesc32, L.desc32.data(),
                                   L.desc32.size() * sizeof(LevelDesc<float>),
                                   hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(CHHS_E_HIP);
    if (hipMemcpyAsync(c->ddesc, L.desc.data(), L.desc.size() * sizeof(LevelDesc<double>),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(c->dinfo, L.info.data(), L.info.size() * sizeof(InstInfo),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(c->tail_insts, L.tail_insts.data(), L.tail_insts.size() * sizeof(int),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(c->rngA0, L.rngA0.data(), n_inst * sizeof(Range), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(c->rngT0, L.rngT0.data(), n_inst * sizeof(Range), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(c->rngA0n, L.rngA0n.data(), n_inst * sizeof(Range), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(c->rngA0x, L.rngA0x.data(), n_inst * sizeof(Range), hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return fail(CHHS_E_HIP);
    for (int l = 0; l < kMaxLevels; ++l) {
        rc |= upload(c->A[l], b, L.off_A[l], L.A[l], st);
        rc |= upload(c->B[l], b, L.off_B[l], L.B[l], st);
        rc |= upload(c->Bh[l], b, L.off_Bh[l], L.Bh[l], st);
        rc |= upload(c->Bcs[l], b, L.off_Bcs[l], L.Bcs[l], st);
        rc |= upload(c->Bc[l], b, L.off_Bc[l], L.Bc[l], st);
        rc |= upload(c->T[l], b, L.off_T[l], L.T[l], st);
        rc |= upload(c->Tall[l], b, L.off_Tall[l], L.Tall[l], st);
        rc |= upload(c->S[l], b, L.off_S[l], L.S[l], st);
        rc |= upload(c->Sall[l], b, L.off_Sall[l], L.Sall[l], st);
        rc |= upload(c->Z64[l], b, L.off_Z64[l], L.Z64[l], st);
        rc |= upload(c->Z32[l], b, L.off_Z32[l], L.Z32[l], st);
        rc |= upload(c->ZR64[l], b, L.off_ZR64[l], L.ZR64[l], st);
        rc |= upload(c->ZR32[l], b, L.off_ZR32[l], L.ZR32[l], st);
        rc |= upload(c->BcS[l], b, L.off_BcS[l], L.BcS[l], st);
    }
    rc |= upload(c->A0n, b, L.off_A0n, L.A0n, st);
    rc |= upload(c->A0t, b, L.off_A0t, L.A0t, st);
    rc |= upload(c->A0x, b, L.off_A0x, L.A0x, st);
    rc |= upload(c->M0, b, L.off_M0, L.M0, st);
    rc |= upload(c->FM0, b, L.off_FM0, L.FM0, st);
    c->rngM0 = reinterpret_cast<Range*>(b + L.off_rngM0);
    c->rngM0f = reinterpret_cast<Range*>(b + L.off_rngM0f);
    if (hipMemcpyAsync(c->rngM0, L.rngM0.data(), n_inst * sizeof(Range), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(c->rngM0f, L.rngM0f.data(), n_inst * sizeof(Range),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        rc = CHHS_E_HIP;
    rc |= upload(c->FA0, b, L.off_FA0, L.FA0, st);
    rc |= upload(c->FA0n, b, L.off_FA0n, L.FA0n, st);
    if (hipMemcpyAsync(c->rngA0f, L.rngA0f.data(), n_inst * sizeof(Range), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        hipMemcpyAsync(c->rngA0nf, L.rngA0nf.data(), n_inst * sizeof(Range),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        rc = CHHS_E_HIP;
    if (rc) return fail(CHHS_E_HIP);
    // pinned mirror, same layout as the device result block: res | act_next |
    // cycles, then the energies
    const size_t nres = size_t(n_inst) * chhs::kResStride;
    const size_t nint = (2 * size_t(n_inst) * sizeof(int) + sizeof(double) - 1) / sizeof(double);
    const size_t hbytes = (2 * nres + nint) * sizeof(double);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->hbuf[0]), hbytes, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->hbuf[1]), (nres + nint) * sizeof(double),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->hbuf[2]), (nres + nint) * sizeof(double),
                      hipHostMallocDefault) != hipSuccess)
        return fail(CHHS_E_HIP);
    view_results(c, 0);
    c->heres = c->hbuf[0] + nres + nint;
    c->fused_norm = !c->mixed && c->dim == 2 && o->nu2 > 0 && o->order != 1;
    // the mixed path never subtracts p's mean inside its cycles
    c->defer_shift = c->mixed || (tiled2d(c) && o->nu1 > 0);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(CHHS_E_HIP);
    if (o->autotune && o->smoother == 0 && c->dim == 2 && o->nu1 > 0 && o->nu2 > 0 &&
        o->order != 1) {
        const int arc = autotune(c);
        if (arc) return fail(arc);
    }
    if (o->autotune && o->smoother == 0 && fused3d(c)) {
        const int arc = autotune3(c);
        if (arc) return fail(arc);
    }
    // 3D plain FP64 with the fused step on the finest level: its first
    // pre-smoothing launch subtracts p's pending mean as it loads p
    if (!c->mixed && z3_at(c, 0) && o->nu1 > 0) c->defer_shift = true;
    {
        // the per-step log of chhs_step_log, reserved up front
        const size_t per_step = size_t(n_inst) * chhs::kResStride * sizeof(double);
        const size_t steps0 = std::max<size_t>(1, std::min<size_t>(kLogSteps0, kLogBytes0 / per_step));
        const int lrc = reserve_log(c, int(steps0));
        if (lrc) return fail(lrc);
    }
    *out = c;
    return CHHS_OK;
}

int chhs_setup_step(chhs_ctx* c, const double* phi_prev, const double* phi_cur,
                    const double* mu, const double* p) {
    if (c == nullptr || phi_prev == nullptr || phi_cur == nullptr || mu == nullptr ||
        p == nullptr)
        return CHHS_E_INVAL;
    return setup(c, phi_prev, phi_cur, mu, p);
}

int chhs_fas_vcycle(chhs_ctx* c, double* res_norm_host) {
    if (c == nullptr) return CHHS_E_INVAL;
    if (!c->loaded) return CHHS_E_STATE;
    // every instance takes part, whatever its convergence state
    chhs::launch_fill_int(c->act_next, c->n_inst, 1, c->stream);
    int rc = run_cycle(c, false);
    if (rc) return rc;
    // the level's fields after this call hold the normalised p
    if (c->defer_shift) {
        apply_pshift(c);
        rc = check_launch();
        if (rc) return rc;
    }
    bool finite = true;
    for (int i = 0; i < c->n_inst; ++i) {
        if (res_norm_host) res_norm_host[i] = hres_of(c, i)[3];
        finite = finite && std::isfinite(hres_of(c, i)[3]);
    }
    return finite ? CHHS_OK : CHHS_E_NONFINITE;
}

int chhs_residual_norms(chhs_ctx* c, double* out_host) {
    if (c == nullptr || out_host == nullptr) return CHHS_E_INVAL;
    if (!c->loaded) return CHHS_E_STATE;
    chhs::launch_residual_partials(c->dim, batch(c, 0, nullptr), c->A[0].dev, c->A[0].n,
                                   c->partial, c->stream);
    const double* src;
    const Range* rng;
    fold_cells(c, false, nullptr, &src, &rng);
    chhs::launch_inst_reduce(src, rng, nullptr, nullptr, 0, c->dinfo, nullptr,
                             c->act_next, c->cycles, c->res, c->n_inst, c->opts.tol, 1 << 30, 0,
                             c->stream);
    int rc = check_launch();
    if (rc) return rc;
    rc = enqueue_readback(c);
    if (rc) return rc;
    rc = sync_results(c);
    if (rc) return rc;
    for (int i = 0; i < c->n_inst; ++i) std::memcpy(out_host + 4 * i, hres_of(c, i), 4 * sizeof(double));
    return CHHS_OK;
}

int chhs_get_solution(chhs_ctx* c, double* phi, double* mu, double* p) {
    if (c == nullptr) return CHHS_E_INVAL;
    if (!c->loaded) return CHHS_E_STATE;
    Batch<double> b = batch(c, 0, nullptr);
    b.pshift = c->defer_shift ? c->res : nullptr;
    chhs::launch_get_solution(b, c->A[0].dev, c->A[0].n, c->dinfo, phi, mu, p, c->stream);
    return check_launch();
}

int chhs_step(chhs_ctx* c, double* phi_prev, double* phi_cur, double* mu, double* p,
              int32_t nsteps, chhs_stats* stats_host) {
    if (c == nullptr || phi_prev == nullptr || phi_cur == nullptr || mu == nullptr ||
        p == nullptr || nsteps < 0)
        return CHHS_E_INVAL;
    return step_loop(c, phi_prev, phi_cur, mu, p, nsteps, stats_host, nullptr);
}

int chhs_step_log(chhs_ctx* c, double* phi_prev, double* phi_cur, double* mu, double* p,
                  int32_t nsteps, chhs_stats* per_step_host) {
    if (c == nullptr || phi_prev == nullptr || phi_cur == nullptr || mu == nullptr ||
        p == nullptr || nsteps < 0 || (nsteps > 0 && per_step_host == nullptr))
        return CHHS_E_INVAL;
    return step_loop(c, phi_prev, phi_cur, mu, p, nsteps, nullptr, per_step_host);
}

int chhs_energy_mass(chhs_ctx* c, const double* phi, const double* phi_prev, double* out_host) {
    if (c == nullptr || phi == nullptr || phi_prev == nullptr || out_host == nullptr)
        return CHHS_E_INVAL;
    int rc = energies(c, 0, phi, phi_prev);
    if (rc) return rc;
    for (int i = 0; i < c->n_inst; ++i) {
        const double* e = c->heres + size_t(i) * chhs::kResStride;
        out_host[3 * i + 0] = e[0];
        out_host[3 * i + 1] = e[1];
        out_host[3 * i + 2] = e[2];
    }
    return CHHS_OK;
}

int chhs_level_count(chhs_ctx* c, int32_t* levels) {
    if (c == nullptr || levels == nullptr || c->n_inst != 1) return CHHS_E_INVAL;
    *levels = c->lay.info[0].nlev;
    return CHHS_OK;
}

int chhs_level_shape(chhs_ctx* c, int32_t level, int32_t* nxyz3) {
    if (c == nullptr || nxyz3 == nullptr || c->n_inst != 1 || level < 0 ||
        level >= c->lay.info[0].nlev)
        return CHHS_E_INVAL;
    const LevelDesc<double>& d = c->lay.desc[level];
    nxyz3[0] = d.nx;
    nxyz3[1] = d.ny;
    nxyz3[2] = d.nz;
    return CHHS_OK;
}

int chhs_graph_count(chhs_ctx* c, int32_t* graphs) {
    if (c == nullptr || graphs == nullptr) return CHHS_E_INVAL;
    *graphs = (c->gexec[0] != nullptr ? 1 : 0) + (c->gexec[1] != nullptr ? 1 : 0);
    return CHHS_OK;
}

int chhs_level_kernel(chhs_ctx* c, int32_t level, int32_t* out3) {
    if (c == nullptr || out3 == nullptr || level < 0 || level >= c->lay.max_nlev)
        return CHHS_E_INVAL;
    if (level >= c->lay.depth) {
        out3[0] = 3;
        out3[1] = 0;
        out3[2] = 0;
    } else if (z3_at(c, level)) {
        out3[0] = 4;
        out3[1] = c->mixed ? c->lay.zseg32[level] : c->lay.zseg64[level];
        out3[2] = c->mixed ? c->Z32[level].n : c->Z64[level].n;
    } else if (!tiled2d(c)) {
        out3[0] = 2;
        out3[1] = chhs::kBlock;
        out3[2] = c->Bh[level].n;
    } else if (c->lay.strip[level]) {
        out3[0] = 1;
        out3[1] = c->lay.seg[level];
        out3[2] = c->S[level].n;
    } else {
        out3[0] = 0;
        out3[1] = tile_block(c->lay.tile_threads[level], c->T[level].n);
        out3[2] = c->T[level].n;
    }
    return CHHS_OK;
}

int chhs_copy_field(chhs_ctx* c, int32_t level, int32_t field, double* dev, int32_t dir) {
    if (c == nullptr || dev == nullptr || c->n_inst != 1 || level < 0 ||
        level >= c->lay.info[0].nlev || field < 0 || field > 7 || (dir != 0 && dir != 1))
        return CHHS_E_INVAL;
    const LevelDesc<double>& d = c->lay.desc[level];
    const int cu = c->cur[level];
    double* f[8] = {d.u[cu][0], d.u[cu][1], d.u[cu][2], d.f[0], d.f[1], d.f[2], d.pstar, d.psi};
    const size_t bytes = size_t(d.n) * sizeof(double);
    if (dir == 0)
        HIP_TRY(hipMemcpyAsync(dev, f[field], bytes, hipMemcpyDeviceToDevice, c->stream));
    else
        HIP_TRY(hipMemcpyAsync(f[field], dev, bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return CHHS_OK;
}

int chhs_smooth(chhs_ctx* c, int32_t level, int32_t nsweeps) {
    if (c == nullptr || c->n_inst != 1 || level < 0 || level >= c->lay.info[0].nlev ||
        nsweeps < 0)
        return CHHS_E_INVAL;
    // the FP64 tile kernels have no 64 x 32 form (a mixed-precision level cut
    // for the FP32 ones)
    if (tiled2d(c) && !c->lay.strip[level] && c->lay.tile_y[level] == chhs::kTileYTall)
        return CHHS_E_INVAL;
    smooth_steps(c, level, nsweeps, nullptr, level == 0 ? CHHS_K_PRE0 : CHHS_K_COARSE);
    if (c->cur[level] != 0) {
        // the single instance's level: make the result copy 0 again
        const LevelDesc<double>& d = c->lay.desc[level];
        const size_t nb = size_t(d.n) * sizeof(double);
        for (int k = 0; k < 3; ++k)
            HIP_TRY(hipMemcpyAsync(d.u[0][k], d.u[1][k], nb, hipMemcpyDeviceToDevice, c->stream));
        c->cur[level] = 0;
    }
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return CHHS_OK;
}

int chhs_restrict(chhs_ctx* c, int32_t level) {
    if (c == nullptr || c->n_inst != 1 || level < 0 || level + 1 >= c->lay.info[0].nlev)
        return CHHS_E_INVAL;
    chhs::launch_restrict_residual(c->dim, batch(c, level, nullptr), c->A[level + 1].dev,
                                   c->A[level + 1].n, c->stream);
    chhs::launch_coarse_rhs(c->dim, batch(c, level, nullptr), c->A[level + 1].dev,
                            c->A[level + 1].n, c->stream);
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return CHHS_OK;
}

int chhs_get_timing(chhs_ctx* c, chhs_timing* out, int32_t reset) {
    if (c == nullptr || out == nullptr) return CHHS_E_INVAL;
    HIP_TRY(hipStreamSynchronize(c->stream));
    resolve_timing(c);
    for (int k = 0; k < CHHS_K_COUNT; ++k) {
        out->ms[k] = c->t_ms[k];
        out->launches[k] = c->t_n[k];
        if (reset) {
            c->t_ms[k] = 0.0;
            c->t_n[k] = 0;
        }
    }
    return CHHS_OK;
}

int chhs_set_timing(chhs_ctx* c, int32_t timing) {
    if (c == nullptr || timing < 0) return CHHS_E_INVAL;
    if (timing == c->opts.timing) return CHHS_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    resolve_timing(c);
    // graphs carry the events of the mask they were captured with
    drop_graphs(c);
    c->opts.timing = timing;
    return CHHS_OK;
}

int chhs_tune_sweeps(chhs_ctx* c, const double* phi_prev, const double* phi_cur, const double* mu,
                     const double* p, int32_t* choice_out) {
    if (c == nullptr || phi_prev == nullptr || phi_cur == nullptr || mu == nullptr || p == nullptr)
        return CHHS_E_INVAL;
    // (nu1, nu2) on the finest level, (nu1_coarse, nu2_coarse) below it
    // (0: the same), prolongation, FP32 cycles per refinement (0: one); the
    // context's own options come first
    struct Cand {
        int nu1, nu2, nu1c, nu2c, prolong, inner;
        bool operator==(const Cand& o) const {
            return nu1 == o.nu1 && nu2 == o.nu2 && nu1c == o.nu1c && nu2c == o.nu2c &&
                   prolong == o.prolong && std::max(1, inner) == std::max(1, o.inner);
        }
    };
    const chhs_opts saved = c->opts;
    const int own_inner = saved.inner_cycles;
    HIP_TRY(hipStreamSynchronize(c->stream));
    resolve_timing(c);
    constexpr int kTuneReps = 3;
    // time to tolerance of one candidate (1e300: it did not converge)
    auto time_of = [&](const Cand& q, double& t) -> int {
        c->opts.nu1 = q.nu1;
        c->opts.nu2 = q.nu2;
        c->opts.nu1_coarse = q.nu1c;
        c->opts.nu2_coarse = q.nu2c;
        c->opts.prolong = q.prolong;
        c->opts.inner_cycles = q.inner;
        drop_graphs(c);
        // the first solve captures the cycle graphs; the best of the next
        // kTuneReps is the candidate's time
        t = 1e300;
        double best = 1e300;
        bool ok = true;
        for (int r = 0; r <= kTuneReps && ok; ++r) {
            const auto t0 = std::chrono::steady_clock::now();
            int rc = setup(c, phi_prev, phi_cur, mu, p, true, false);
            if (rc == CHHS_OK) rc = run_cycles(c, true);
            const auto t1 = std::chrono::steady_clock::now();
            if (rc != CHHS_OK) return rc;
            for (int i = 0; i < c->n_inst; ++i) {
                const double res = hres_of(c, i)[3];
                ok = ok && std::isfinite(res) && res <= c->opts.tol;
            }
            if (r > 0) best = std::min(best, std::chrono::duration<double>(t1 - t0).count());
        }
        if (ok) t = best;
        return CHHS_OK;
    };
    // another candidate replaces the current pick only if it is faster by
    // more than the timing noise between repetitions (2%)
    auto choose = [](const std::vector<double>& times) {
        int pick = times[0] < 1e300 ? 0 : -1;
        for (size_t k = 1; k < times.size(); ++k)
            if (times[k] < 1e300 && (pick < 0 || times[k] < 0.98 * times[pick])) pick = int(k);
        return pick;
    };
    c->opts.timing = 0;
    // the cycle shape first (with the context's own inner cycles) ...
    std::vector<Cand> cands = {{saved.nu1, saved.nu2, saved.nu1_coarse, saved.nu2_coarse,
                                saved.prolong, own_inner}};
    for (const Cand& q : {Cand{2, 2, 0, 0, 0, own_inner}, Cand{1, 1, 0, 0, 0, own_inner},
                          Cand{2, 1, 0, 0, 0, own_inner}, Cand{1, 2, 0, 0, 0, own_inner},
                          Cand{2, 2, 1, 1, 0, own_inner}, Cand{1, 1, 2, 2, 0, own_inner},
                          Cand{2, 2, 3, 3, 0, own_inner}, Cand{2, 2, 0, 0, 1, own_inner},
                          Cand{1, 1, 0, 0, 1, own_inner}, Cand{1, 2, 0, 0, 1, own_inner}})
        if (std::find(cands.begin(), cands.end(), q) == cands.end()) cands.push_back(q);
    std::vector<double> times(cands.size(), 1e300);
    int rc = CHHS_OK;
    for (size_t k = 0; k < cands.size() && rc == CHHS_OK; ++k) rc = time_of(cands[k], times[k]);
    int pick = rc == CHHS_OK ? choose(times) : -1;
    Cand q = pick >= 0 ? cands[pick] : cands[0];
    // ... then, for a mixed-precision context, the FP32 cycles per refinement
    if (rc == CHHS_OK && pick >= 0 && c->mixed) {
        std::vector<Cand> ic = {q};
        for (int inner : {1, 2, 3}) {
            Cand r = q;
            r.inner = inner;
            if (std::find(ic.begin(), ic.end(), r) == ic.end()) ic.push_back(r);
        }
        std::vector<double> ti(ic.size(), 1e300);
        ti[0] = times[pick];
        for (size_t k = 1; k < ic.size() && rc == CHHS_OK; ++k) rc = time_of(ic[k], ti[k]);
        if (rc == CHHS_OK) q = ic[choose(ti)];
    }
    c->opts = saved;
    drop_graphs(c);
    if (rc != CHHS_OK) return rc;
    if (pick < 0) return CHHS_E_NOCONV;
    c->opts.nu1 = q.nu1;
    c->opts.nu2 = q.nu2;
    c->opts.nu1_coarse = q.nu1c;
    c->opts.nu2_coarse = q.nu2c;
    c->opts.prolong = q.prolong;
    c->opts.inner_cycles = q.inner;
    if (choice_out != nullptr) {
        choice_out[0] = q.nu1;
        choice_out[1] = q.nu2;
        choice_out[2] = q.nu1c;
        choice_out[3] = q.nu2c;
        choice_out[4] = q.prolong;
        choice_out[5] = q.inner;
    }
    return CHHS_OK;
}

int chhs_get_opts(chhs_ctx* c, chhs_opts* out) {
    if (c == nullptr || out == nullptr) return CHHS_E_INVAL;
    *out = c->opts;
    return CHHS_OK;
}

void chhs_destroy(chhs_ctx* c) {
    if (c == nullptr) return;
    (void)hipStreamSynchronize(c->stream);
    resolve_timing(c);
    drop_graphs(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (int k = 0; k < 2; ++k)
        if (c->cycle_done[k]) (void)hipEventDestroy(c->cycle_done[k]);
    for (int k = 0; k < 3; ++k)
        if (c->hbuf[k]) (void)hipHostFree(c->hbuf[k]);
    if (c->hlog) (void)hipHostFree(c->hlog);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* chhs_strerror(int code) {
    switch (code) {
        case CHHS_OK: return "success";
        case CHHS_E_INVAL: return "invalid argument (sizes, parameters or options)";
        case CHHS_E_NOMEM: return "workspace smaller than chhs_workspace_bytes";
        case CHHS_E_HIP: return "HIP runtime error";
        case CHHS_E_NOCONV: return "FAS did not reach tol within max_vcycles";
        case CHHS_E_NONFINITE: return "residual norm is not finite";
        case CHHS_E_STATE: return "no step system loaded";
        default: return "unknown error code";
    }
}

}  // extern "C"
