// Host driver and C ABI of libchhs (declared in include/chhs.h).
//
// Owns the multigrid hierarchy carved out of the caller's workspace, the FAS
// V-cycle schedule, the stopping test (one residual-norm readback per cycle)
// and the time-step loop with its state rotation.
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "chhs.h"
#include "chhs_internal.hpp"

using chhs::Level;

struct chhs_ctx {
    chhs_problem prob;
    chhs_opts opts;
    int n_inst = 1;
    hipStream_t stream = nullptr;
    std::vector<Level<double>> lv;     // level 0 = finest
    double* partial = nullptr;         // partial_cap x kPartialStride doubles
    int tail = 0;                      // first level handled by the one-workgroup tail
    size_t tail_lds = 0;               // its LDS bytes
    double* dres = nullptr;            // small device result area (64 doubles)
    double* hres = nullptr;            // pinned host mirror of dres
    bool loaded = false;               // a step system is set up
    // kernel timing (opts.timing): event pairs awaiting resolution, totals
    struct Pending { hipEvent_t a, b; int cls; };
    std::vector<hipEvent_t> ev_pool;
    std::vector<Pending> pending;
    double t_ms[CHHS_K_COUNT] = {};
    int64_t t_n[CHHS_K_COUNT] = {};
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

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
    const double cells = double(p->nx) * p->ny * p->nz;
    return cells < 2147483647.0;
}

bool valid_opts(const chhs_opts* o) {
    if (o == nullptr) return false;
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1) return false;
    if (o->max_vcycles < 1 || o->coarse_sweeps < 1) return false;
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return false;
    if (o->precision != 0) return false;   // FP64 only in this build of the driver
    return true;
}

// Extents of every level: halve all directions while every extent is even and
// at least 4; the coarsest extents must be at most 8 and there must be at least
// two levels.
bool level_extents(const chhs_problem* p, std::vector<int>& ext) {
    int nx = p->nx, ny = p->ny, nz = p->nz;
    ext.clear();
    ext.push_back(nx);
    ext.push_back(ny);
    ext.push_back(nz);
    for (;;) {
        const bool even = nx % 2 == 0 && ny % 2 == 0 && (p->dim == 2 || nz % 2 == 0);
        const bool big = nx >= 4 && ny >= 4 && (p->dim == 2 || nz >= 4);
        if (!even || !big) break;
        nx /= 2;
        ny /= 2;
        if (p->dim == 3) nz /= 2;
        ext.push_back(nx);
        ext.push_back(ny);
        ext.push_back(nz);
    }
    const int nlev = int(ext.size() / 3);
    if (nlev < 2) return false;
    return nx <= 8 && ny <= 8 && nz <= 8;
}

// Blocks whose partial sums the reduction buffer must hold.
int partial_capacity(const chhs_problem* p) {
    int cap = chhs::kMaxPartials;
    if (p->dim == 2) {
        const int t = chhs::tile2d_blocks(p->nx, p->ny);
        if (t > cap) cap = t;
    }
    return cap;
}

// First level of the single-workgroup tail: the finest level whose own and
// coarser levels' 11 fields fit the LDS budget.
int pick_tail(const std::vector<Level<double>>& lv, size_t* bytes) {
    const int nlev = int(lv.size());
    std::vector<int> cells(nlev);
    for (int l = 0; l < nlev; ++l) cells[l] = lv[l].n;
    for (int l = 0; l < nlev; ++l) {
        if (nlev - l > chhs::kMaxTailLevels) continue;
        const size_t b = chhs::tail_lds_bytes(&cells[l], nlev - l, sizeof(double));
        if (b <= chhs::kTailLdsBudget) {
            *bytes = b;
            return l;
        }
    }
    *bytes = chhs::tail_lds_bytes(&cells[nlev - 1], 1, sizeof(double));
    return nlev - 1;
}

// Walks the workspace layout; assigns pointers when base != nullptr.
size_t plan(const chhs_problem* p, char* base, std::vector<Level<double>>* out,
            double** partial, double** dres) {
    std::vector<int> ext;
    if (!level_extents(p, ext)) return 0;
    size_t off = 0;
    auto take = [&](size_t count) -> double* {
        double* ptr = base ? reinterpret_cast<double*>(base + off) : nullptr;
        off += align_up(count * sizeof(double));
        return ptr;
    };
    const int nlev = int(ext.size() / 3);
    double h = p->h;
    for (int l = 0; l < nlev; ++l) {
        Level<double> L{};
        L.nx = ext[3 * l];
        L.ny = ext[3 * l + 1];
        L.nz = ext[3 * l + 2];
        L.n = L.nx * L.ny * L.nz;
        const size_t n = size_t(L.n);
        L.phi = take(n);
        L.mu = take(n);
        L.p = take(n);
        if (l > 0) {
            L.ub0 = take(n);
            L.ub1 = take(n);
            L.ub2 = take(n);
        }
        L.f0 = take(n);
        L.f1 = take(n);
        L.f2 = take(n);
        L.pstar = take(n);
        L.psi = take(n);
        if (p->dim == 2) {
            L.phi_alt = take(n);
            L.mu_alt = take(n);
            L.p_alt = take(n);
        }
        L.h = h;
        L.lam = p->dt / (h * h);
        L.kap = 0.75 * p->eps * p->eps / (h * h);
        L.gamma = p->gamma;
        if (out) out->push_back(L);
        h *= 2.0;
    }
    double* part = take(size_t(partial_capacity(p)) * chhs::kPartialStride);
    double* res = take(64);
    if (partial) *partial = part;
    if (dres) *dres = res;
    return off;
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        if ((expr) != hipSuccess) return CHHS_E_HIP;   \
    } while (0)

int check_launch() { return hipGetLastError() == hipSuccess ? CHHS_OK : CHHS_E_HIP; }

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

// Brackets the launches issued during its lifetime with a pair of events on
// the context stream when timing is enabled.
class TimedScope {
  public:
    TimedScope(chhs_ctx* c, int cls) : c_(c), cls_(cls) {
        if (!c_->opts.timing) return;
        a_ = pooled_event(c_);
        if (a_) (void)hipEventRecord(a_, c_->stream);
    }
    ~TimedScope() {
        if (!c_->opts.timing || a_ == nullptr) return;
        hipEvent_t b = pooled_event(c_);
        if (b == nullptr) return;
        (void)hipEventRecord(b, c_->stream);
        c_->pending.push_back({a_, b, cls_});
    }

  private:
    chhs_ctx* c_;
    int cls_;
    hipEvent_t a_ = nullptr;
};

// Accumulates the elapsed times of completed event pairs (stream synchronised).
void resolve_timing(chhs_ctx* c) {
    for (auto& pe : c->pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            c->t_ms[pe.cls] += ms;
            c->t_n[pe.cls] += 1;
        }
        c->ev_pool.push_back(pe.a);
        c->ev_pool.push_back(pe.b);
    }
    c->pending.clear();
}

// After an out-of-place launch on level l: the written copy becomes current.
void swap_u(chhs_ctx* c, int l) {
    Level<double>& L = c->lv[l];
    std::swap(L.phi, L.phi_alt);
    std::swap(L.mu, L.mu_alt);
    std::swap(L.p, L.p_alt);
}

// Per-cell red-black smoothing (3D levels above the tail, and chhs_smooth on 3D).
void smooth_cells(chhs_ctx* c, int l, int cls) {
    for (int color = 0; color < 2; ++color) {
        TimedScope t(c, cls);
        chhs::launch_smooth(c->prob.dim, c->lv[l], color, c->stream);
    }
}

// nsweeps smoothing steps on level l with the production kernels.
void smooth_steps(chhs_ctx* c, int l, int nsweeps, int cls) {
    if (c->prob.dim == 2) {
        const Level<double>& L = c->lv[l];
        while (nsweeps > 0) {
            const int k = nsweeps >= 2 ? 2 : 1;
            nsweeps -= k;
            {
                TimedScope t(c, cls);
                chhs::launch_tile2d<double>(L, L, l == 0, k, 0, false, nullptr, c->stream);
            }
            swap_u(c, l);
        }
        return;
    }
    for (int s = 0; s < nsweeps; ++s) smooth_cells(c, l, cls);
}

// One V-cycle from level l.  Returns the number of residual-norm partials the
// finest level's last post-smoothing launch produced (0 if none).
int vcycle(chhs_ctx* c, int l) {
    const int dim = c->prob.dim;
    const int nlev = int(c->lv.size());
    const bool l0 = l == 0;
    if (l >= c->tail) {
        TimedScope t(c, l0 ? CHHS_K_PRE0 : CHHS_K_COARSE);
        chhs::launch_tail<double>(dim, &c->lv[l], nlev - l, c->opts.nu1, c->opts.nu2,
                                  c->opts.coarse_sweeps, c->tail_lds, c->stream);
        return 0;
    }
    const Level<double>& L = c->lv[l];
    const Level<double>& C = c->lv[l + 1];
    const int pre_cls = l0 ? CHHS_K_PRE0 : CHHS_K_COARSE;
    const int post_cls = l0 ? CHHS_K_POST0 : CHHS_K_COARSE;
    const int xfer_cls = l0 ? CHHS_K_TRANSFER0 : CHHS_K_COARSE;
    int nb = 0;
    if (dim == 2) {
        int rem = c->opts.nu1;
        if (rem == 0) {
            TimedScope t(c, xfer_cls);
            chhs::launch_restrict_residual(dim, L, C, c->stream);
        } else {
            while (rem > 2) {
                {
                    TimedScope t(c, pre_cls);
                    chhs::launch_tile2d<double>(L, C, l0, 2, 0, false, nullptr, c->stream);
                }
                swap_u(c, l);
                rem -= 2;
            }
            {
                TimedScope t(c, pre_cls);
                chhs::launch_tile2d<double>(L, C, l0, rem, 1, false, nullptr, c->stream);
            }
            swap_u(c, l);
        }
        {
            TimedScope t(c, xfer_cls);
            chhs::launch_coarse_rhs(dim, C, c->stream);
        }
        vcycle(c, l + 1);
        rem = c->opts.nu2;
        if (rem == 0) {
            TimedScope t(c, xfer_cls);
            chhs::launch_prolong(dim, L, C, c->stream);
        } else {
            bool first = true;
            while (rem > 0) {
                const int k = rem >= 2 ? 2 : 1;
                rem -= k;
                const bool norm = l0 && rem == 0;
                {
                    TimedScope t(c, post_cls);
                    nb = chhs::launch_tile2d<double>(L, C, l0, k, norm ? 2 : 0, first,
                                                     norm ? c->partial : nullptr, c->stream);
                }
                swap_u(c, l);
                first = false;
            }
        }
        return l0 && c->opts.nu2 > 0 ? nb : 0;
    }
    for (int s = 0; s < c->opts.nu1; ++s) smooth_cells(c, l, pre_cls);
    {
        TimedScope t(c, xfer_cls);
        chhs::launch_restrict_residual(dim, L, C, c->stream);
        chhs::launch_coarse_rhs(dim, C, c->stream);
    }
    vcycle(c, l + 1);
    {
        TimedScope t(c, xfer_cls);
        chhs::launch_prolong(dim, L, C, c->stream);
    }
    for (int s = 0; s < c->opts.nu2; ++s) smooth_cells(c, l, post_cls);
    return 0;
}

// Residual norms of level 0 into hres[0..3] (||R_phi||, ||R_mu||, ||R_p||, total);
// p is shifted to mean zero on the way (it does not enter N).  nb > 0: the
// partial sums of the current iterate are already in the partial buffer.
int residual_and_normalise(chhs_ctx* c, int nb = 0) {
    const Level<double>& L = c->lv[0];
    {
        TimedScope t(c, CHHS_K_NORM);
        if (nb == 0) nb = chhs::launch_residual_partials(c->prob.dim, L, c->partial, c->stream);
        chhs::launch_reduce_final(c->partial, nb, 4, c->dres, c->stream);
        chhs::launch_shift_p(L, c->dres + 3, c->stream);
    }
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->hres, c->dres, 4 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    resolve_timing(c);
    const double hd = std::pow(L.h, c->prob.dim);
    const double s0 = c->hres[0] * hd, s1 = c->hres[1] * hd, s2 = c->hres[2] * hd;
    c->hres[0] = std::sqrt(s0);
    c->hres[1] = std::sqrt(s1);
    c->hres[2] = std::sqrt(s2);
    c->hres[3] = std::sqrt(s0 + s1 + s2);
    return CHHS_OK;
}

int setup(chhs_ctx* c, const double* phi_prev, const double* phi_cur, const double* mu,
          const double* p) {
    const int dim = c->prob.dim;
    const double q = 0.25 * c->prob.eps * c->prob.eps / (c->prob.h * c->prob.h);
    TimedScope t(c, CHHS_K_SETUP);
    chhs::launch_setup(dim, c->lv[0], phi_prev, phi_cur, mu, p, q, c->stream);
    for (size_t l = 0; l + 1 < c->lv.size(); ++l)
        chhs::launch_restrict_frozen(dim, c->lv[l], c->lv[l + 1], c->stream);
    c->loaded = true;
    return check_launch();
}

// Energies of phi against q (and the flow terms when mu != nullptr) into out[0..9]:
// mass, E_h, F_h, diss_mu, diss_u, max|phi|.
int energies(chhs_ctx* c, const double* phi, const double* q, const double* mu,
             const double* p, const double* pstar, double* out) {
    const chhs_problem& P = c->prob;
    {
        TimedScope t(c, CHHS_K_SETUP);
        const int nb = chhs::launch_energy_partials(P.dim, P.nx, P.ny, P.nz, phi, q, mu, p, pstar,
                                                    P.gamma, c->partial, c->stream);
        chhs::launch_reduce_energy(c->partial, nb, c->dres + 8, c->stream);
    }
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->hres + 8, c->dres + 8, 9 * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    resolve_timing(c);
    const double* v = c->hres + 8;
    const double h = P.h, hd = std::pow(h, P.dim), e2 = P.eps * P.eps, ih2 = 1.0 / (h * h);
    const double E = hd * (0.25 * v[2] - 0.5 * v[1] + 0.5 * e2 * v[3] * ih2);
    out[0] = hd * v[0];
    out[1] = E;
    out[2] = E + hd * (0.25 * v[4] + 0.125 * e2 * v[5] * ih2);
    out[3] = P.dt * hd * v[6] * ih2;
    out[4] = P.gamma > 0.0 ? P.dt / P.gamma * hd * v[7] * ih2 : 0.0;
    out[5] = v[8];
    return CHHS_OK;
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
    o->use_graph = 0;
    o->timing = 0;
}

size_t chhs_workspace_bytes(const chhs_problem* p, int32_t n_inst, const chhs_opts* o) {
    if (n_inst != 1 || !valid_problem(p) || !valid_opts(o)) return 0;
    return plan(p, nullptr, nullptr, nullptr, nullptr);
}

int chhs_init(const chhs_problem* p, int32_t n_inst, const chhs_opts* o, void* workspace_dev,
              size_t ws_bytes, void* hip_stream, chhs_ctx** out) {
    if (out == nullptr) return CHHS_E_INVAL;
    *out = nullptr;
    if (n_inst != 1 || !valid_problem(p) || !valid_opts(o) || workspace_dev == nullptr)
        return CHHS_E_INVAL;
    if (reinterpret_cast<uintptr_t>(workspace_dev) % kAlign != 0) return CHHS_E_INVAL;
    const size_t need = plan(p, nullptr, nullptr, nullptr, nullptr);
    if (need == 0) return CHHS_E_INVAL;
    if (ws_bytes < need) return CHHS_E_NOMEM;
    chhs_ctx* c = new chhs_ctx();
    c->prob = *p;
    c->opts = *o;
    c->n_inst = n_inst;
    c->stream = static_cast<hipStream_t>(hip_stream);
    plan(p, static_cast<char*>(workspace_dev), &c->lv, &c->partial, &c->dres);
    c->tail = pick_tail(c->lv, &c->tail_lds);
    if (chhs::prepare_tail<double>(p->dim, c->tail_lds) != 0) {
        delete c;
        return CHHS_E_HIP;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&c->hres), 64 * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
        delete c;
        return CHHS_E_HIP;
    }
    *out = c;
    return CHHS_OK;
}

int chhs_setup_step(chhs_ctx* c, const double* phi_prev, const double* phi_cur,
                    const double* mu, const double* p) {
    if (c == nullptr || phi_prev == nullptr || phi_cur == nullptr || mu == nullptr ||
        p == nullptr)
        return CHHS_E_INVAL;
    int rc = setup(c, phi_prev, phi_cur, mu, p);
    if (rc) return rc;
    return residual_and_normalise(c);
}

int chhs_fas_vcycle(chhs_ctx* c, double* res_norm_host) {
    if (c == nullptr) return CHHS_E_INVAL;
    if (!c->loaded) return CHHS_E_STATE;
    const int nb = vcycle(c, 0);
    int rc = check_launch();
    if (rc) return rc;
    rc = residual_and_normalise(c, nb);
    if (rc) return rc;
    if (res_norm_host) res_norm_host[0] = c->hres[3];
    return std::isfinite(c->hres[3]) ? CHHS_OK : CHHS_E_NONFINITE;
}

int chhs_residual_norms(chhs_ctx* c, double* out_host) {
    if (c == nullptr || out_host == nullptr) return CHHS_E_INVAL;
    if (!c->loaded) return CHHS_E_STATE;
    int rc = residual_and_normalise(c);
    if (rc) return rc;
    std::memcpy(out_host, c->hres, 4 * sizeof(double));
    return CHHS_OK;
}

int chhs_get_solution(chhs_ctx* c, double* phi, double* mu, double* p) {
    if (c == nullptr) return CHHS_E_INVAL;
    if (!c->loaded) return CHHS_E_STATE;
    const Level<double>& L = c->lv[0];
    const size_t bytes = size_t(L.n) * sizeof(double);
    if (phi) HIP_TRY(hipMemcpyAsync(phi, L.phi, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (mu) HIP_TRY(hipMemcpyAsync(mu, L.mu, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (p) HIP_TRY(hipMemcpyAsync(p, L.p, bytes, hipMemcpyDeviceToDevice, c->stream));
    return CHHS_OK;
}

int chhs_step(chhs_ctx* c, double* phi_prev, double* phi_cur, double* mu, double* p,
              int32_t nsteps, chhs_stats* stats_host) {
    if (c == nullptr || phi_prev == nullptr || phi_cur == nullptr || mu == nullptr ||
        p == nullptr || nsteps < 0)
        return CHHS_E_INVAL;
    chhs_stats st;
    std::memset(&st, 0, sizeof(st));
    const Level<double>& L = c->lv[0];
    const size_t bytes = size_t(L.n) * sizeof(double);
    int rc = CHHS_OK;
    for (int m = 0; m < nsteps; ++m) {
        rc = chhs_setup_step(c, phi_prev, phi_cur, mu, p);
        if (rc) break;
        st.res0 = c->hres[3];
        int cycles = 0;
        while (c->hres[3] > c->opts.tol && cycles < c->opts.max_vcycles) {
            const int nb = vcycle(c, 0);
            rc = residual_and_normalise(c, nb);
            if (rc) break;
            ++cycles;
            if (!std::isfinite(c->hres[3])) break;
        }
        if (rc) break;
        st.vcycles = cycles;
        st.total_vcycles += cycles;
        for (int k = 0; k < 3; ++k) st.res[k] = c->hres[k];
        st.res_norm = c->hres[3];
        if (!std::isfinite(c->hres[3])) {
            rc = CHHS_E_NONFINITE;
            break;
        }
        if (c->hres[3] > c->opts.tol) {
            rc = CHHS_E_NOCONV;
            break;
        }
        if (m == nsteps - 1 && stats_host != nullptr) {
            double e[6];
            rc = energies(c, L.phi, phi_cur, L.mu, L.p, L.pstar, e);
            if (rc) break;
            st.mass = e[0];
            st.E_h = e[1];
            st.F_h = e[2];
            st.diss_mu = e[3];
            st.diss_u = e[4];
            st.max_abs_phi = e[5];
        }
        // rotate: (phi^{m-1}, phi^m) <- (phi^m, phi^{m+1}); mu, p <- this step's
        if (hipMemcpyAsync(phi_prev, phi_cur, bytes, hipMemcpyDeviceToDevice, c->stream) ||
            hipMemcpyAsync(phi_cur, L.phi, bytes, hipMemcpyDeviceToDevice, c->stream) ||
            hipMemcpyAsync(mu, L.mu, bytes, hipMemcpyDeviceToDevice, c->stream) ||
            hipMemcpyAsync(p, L.p, bytes, hipMemcpyDeviceToDevice, c->stream)) {
            rc = CHHS_E_HIP;
            break;
        }
        ++st.steps_done;
    }
    st.status = rc;
    if (stats_host) *stats_host = st;
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == CHHS_OK) rc = CHHS_E_HIP;
    return rc;
}

int chhs_energy_mass(chhs_ctx* c, const double* phi, const double* phi_prev, double* out_host) {
    if (c == nullptr || phi == nullptr || phi_prev == nullptr || out_host == nullptr)
        return CHHS_E_INVAL;
    double e[6];
    int rc = energies(c, phi, phi_prev, nullptr, nullptr, nullptr, e);
    if (rc) return rc;
    out_host[0] = e[0];
    out_host[1] = e[1];
    out_host[2] = e[2];
    return CHHS_OK;
}

int chhs_level_count(chhs_ctx* c, int32_t* levels) {
    if (c == nullptr || levels == nullptr) return CHHS_E_INVAL;
    *levels = int32_t(c->lv.size());
    return CHHS_OK;
}

int chhs_level_shape(chhs_ctx* c, int32_t level, int32_t* nxyz3) {
    if (c == nullptr || nxyz3 == nullptr || level < 0 || level >= int(c->lv.size()))
        return CHHS_E_INVAL;
    nxyz3[0] = c->lv[level].nx;
    nxyz3[1] = c->lv[level].ny;
    nxyz3[2] = c->lv[level].nz;
    return CHHS_OK;
}

int chhs_copy_field(chhs_ctx* c, int32_t level, int32_t field, double* dev, int32_t dir) {
    if (c == nullptr || dev == nullptr || level < 0 || level >= int(c->lv.size()) ||
        field < 0 || field > 7 || (dir != 0 && dir != 1))
        return CHHS_E_INVAL;
    Level<double>& L = c->lv[level];
    double* f[8] = {L.phi, L.mu, L.p, L.f0, L.f1, L.f2, L.pstar, L.psi};
    const size_t bytes = size_t(L.n) * sizeof(double);
    if (dir == 0)
        HIP_TRY(hipMemcpyAsync(dev, f[field], bytes, hipMemcpyDeviceToDevice, c->stream));
    else
        HIP_TRY(hipMemcpyAsync(f[field], dev, bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return CHHS_OK;
}

int chhs_smooth(chhs_ctx* c, int32_t level, int32_t nsweeps) {
    if (c == nullptr || level < 0 || level >= int(c->lv.size()) || nsweeps < 0)
        return CHHS_E_INVAL;
    smooth_steps(c, level, nsweeps, level == 0 ? CHHS_K_PRE0 : CHHS_K_COARSE);
    int rc = check_launch();
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return CHHS_OK;
}

int chhs_restrict(chhs_ctx* c, int32_t level) {
    if (c == nullptr || level < 0 || level + 1 >= int(c->lv.size())) return CHHS_E_INVAL;
    chhs::launch_restrict_residual(c->prob.dim, c->lv[level], c->lv[level + 1], c->stream);
    chhs::launch_coarse_rhs(c->prob.dim, c->lv[level + 1], c->stream);
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

void chhs_destroy(chhs_ctx* c) {
    if (c == nullptr) return;
    if (!c->pending.empty()) {
        (void)hipStreamSynchronize(c->stream);
        resolve_timing(c);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->hres) (void)hipHostFree(c->hres);
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
