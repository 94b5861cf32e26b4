// C ABI of libmg.so (declared in include/mg.h).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "mg_cc.h"
#include "mg_cd.h"
#include "mg_st.h"
#include "mg_solver.h"

using namespace mg;

// Complex-diffusion hierarchy: levels n, n/2, ..., 1 cells per axis; per level
// the iterate and its Jacobi partner (level 0's iterate is the caller's), the
// right-hand side, the diffusivity and the restricted full approximation.
struct CDState {
    int dim = 0, n = 0;
    double tau = 0.0;
    CDConst K{};
    bool jacobi = false;
    int nu1 = 2, nu2 = 2;
    std::vector<int> ln;
    std::vector<void*> u, t, f, g, uh;
    double* part = nullptr;
    double* norm = nullptr;
    double* h_norm = nullptr;  // pinned
    ~CDState() {
        for (size_t l = 0; l < ln.size(); ++l) {
            if (l > 0 && u[l]) (void)hipFree(u[l]);
            for (void* p : {t[l], f[l], g[l], uh[l]})
                if (p) (void)hipFree(p);
        }
        if (part) (void)hipFree(part);
        if (norm) (void)hipFree(norm);
        if (h_norm) (void)hipHostFree(h_norm);
    }
};

namespace {

int dev_status(hipError_t e) {
    if (e == hipSuccess) return MG_OK;
    if (e == hipErrorOutOfMemory) return MG_ENOMEM;
    return MG_EDEVICE;
}

#define CK(x)                                 \
    do {                                      \
        hipError_t e_ = (x);                  \
        if (e_ != hipSuccess) return dev_status(e_); \
    } while (0)

double level_c(int n) {
    const double h = 1.0 / (double)(n - 1);
    return 1.0 / (h * h);
}
double level_wd(int dim, int n, double omega) {
    const double h = 1.0 / (double)(n - 1);
    return (omega * (h * h)) / (2.0 * (double)dim);
}

hipError_t zalloc(void** p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    return hipMemsetAsync(*p, 0, bytes, s);
}

void ffree(void* p) {
    if (p) (void)hipFree(p);
}

// Refinement forms (FP32 or binary16 cycles inside FP64 refinement).
bool is_ir(const mg_params& p) { return p.precision == MG_PREC_FP32_IR || p.precision == MG_PREC_FP16_IR; }
bool is_h16(const mg_params& p) { return p.precision == MG_PREC_FP16_IR; }
// word size of the cycle fields of a refinement form
int ir_elem(const mg_params& p) { return is_h16(p) ? 2 : 4; }

// Build a hierarchy of 'elem'-byte values.  Level 0 u/f are left null when
// caller-owned (own0 = false).  k0: device nodal coefficient of level 0 in the
// same precision (or null).
hipError_t build_levels(Levels& L, int dim, const std::vector<int>& n, int elem, bool own0, const void* k0,
                        hipStream_t s) {
    L.dim = dim;
    L.nlev = (int)n.size();
    L.elem = elem;
    L.n = n;
    L.u.assign(n.size(), nullptr);
    L.t.assign(n.size(), nullptr);
    L.f.assign(n.size(), nullptr);
    L.k.assign(n.size(), nullptr);
    L.own_u.assign(n.size(), 0);
    L.own_f.assign(n.size(), 0);
    for (size_t l = 0; l < n.size(); ++l) {
        const size_t bytes = npts(dim, n[l]) * (size_t)elem;
        if (l > 0 || own0) {
            hipError_t e = zalloc(&L.u[l], bytes, s);
            if (e != hipSuccess) return e;
            e = zalloc(&L.f[l], bytes, s);
            if (e != hipSuccess) return e;
            L.own_u[l] = 1;
            L.own_f[l] = 1;
        }
        if (n[l] > 3) {
            hipError_t e = zalloc(&L.t[l], bytes, s);
            if (e != hipSuccess) return e;
        }
    }
    if (k0) {
        L.k[0] = const_cast<void*>(k0);
        for (size_t l = 1; l < n.size(); ++l) {
            const size_t bytes = npts(dim, n[l]) * (size_t)elem;
            hipError_t e = zalloc(&L.k[l], bytes, s);
            if (e != hipSuccess) return e;
            e = elem == 8 ? launch_inject<double, double>(dim, n[l - 1], (const double*)L.k[l - 1], n[l],
                                                          (double*)L.k[l], s)
                          : launch_inject<float, float>(dim, n[l - 1], (const float*)L.k[l - 1], n[l],
                                                        (float*)L.k[l], s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

void free_levels(Levels& L) {
    for (size_t l = 0; l < L.u.size(); ++l) {
        if (L.own_u[l]) ffree(L.u[l]);
        if (L.own_f[l]) ffree(L.f[l]);
        ffree(L.t[l]);
        if (l > 0 || L.own_k0) ffree(L.k[l]);
    }
    for (void* p : L.fx) ffree(p);
    L.u.clear();
    L.t.clear();
    L.f.clear();
    L.k.clear();
    L.fx.clear();
}

// Face coefficients of every 3D variable-coefficient level with inner nodes
// to sweep (n >= 5), from the level's k in its arithmetic type.
hipError_t build_faces(Levels& L, hipStream_t s) {
    L.fx.assign((size_t)L.nlev, nullptr);
    if (L.dim != 3 || L.k.empty() || !L.k[0]) return hipSuccess;
    for (int l = 0; l < L.nlev; ++l) {
        const int n = L.n[(size_t)l];
        if (n < 5) continue;
        hipError_t e = hipMalloc(&L.fx[(size_t)l], 3 * npts(3, n) * (size_t)L.elem);
        if (e != hipSuccess) return e;
        e = L.elem == 8 ? launch_faces3d<double>((const double*)L.k[(size_t)l], (double*)L.fx[(size_t)l], n, s)
                        : launch_faces3d<float>((const float*)L.k[(size_t)l], (float*)L.fx[(size_t)l], n, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One descriptor per level for a single-instance hierarchy.
hipError_t build_groups(std::vector<Group>& G, const Levels& L, const Problem& P, const int* done, hipStream_t s) {
    G.assign((size_t)L.nlev, Group{});
    for (int l = 0; l < L.nlev; ++l) {
        Group& g = G[(size_t)l];
        g.n = L.n[(size_t)l];
        g.ninst = 1;
        GridDesc d{};
        d.u = L.u[(size_t)l];
        d.t = L.t[(size_t)l];
        d.f = L.f[(size_t)l];
        d.k = L.k[(size_t)l];
        d.fx = (size_t)l < L.fx.size() ? L.fx[(size_t)l] : nullptr;
        d.uc = l + 1 < L.nlev ? L.u[(size_t)l + 1] : nullptr;
        d.fc = l + 1 < L.nlev ? L.f[(size_t)l + 1] : nullptr;
        d.done = done;
        d.n = g.n;
        d.inst = 0;
        d.c = level_c(g.n);
        d.wd = level_wd(P.dim, g.n, P.omega);
        d.omega = P.omega;
        g.h.assign(1, d);
        hipError_t e = hipMalloc((void**)&g.d, sizeof(GridDesc));
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(g.d, g.h.data(), sizeof(GridDesc), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(s);
}

// Tail descriptor of a single-instance hierarchy: its levels from 'first' on.
hipError_t build_tail(TailPlan& T, const std::vector<Group>& G, int first, hipStream_t s) {
    T = TailPlan{};
    if (first < 0) return hipSuccess;
    TailDesc h{};
    h.nlev = (int)G.size() - first;
    for (int j = 0; j < h.nlev; ++j) h.lv[j] = G[(size_t)(first + j)].h[0];
    hipError_t e = hipMalloc((void**)&T.d, sizeof(TailDesc));
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(T.d, &h, sizeof(TailDesc), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    T.first = first;
    T.ninst = 1;
    return hipStreamSynchronize(s);
}

void free_groups(std::vector<Group>& G) {
    for (auto& g : G) ffree(g.d);
    G.clear();
}

// Cell-centred Neumann grids: n = 2^L cells per axis (L >= 1).
bool valid_cc(int dim, int n) { return n >= 2 && (n & (n - 1)) == 0 && n <= (dim == 2 ? 8192 : 512); }

int validate_cc(const mg_params* p) {
    if (!valid_cc(p->dim, p->n)) return MG_EINVAL;
    if (p->smoother != MG_SMOOTH_RBGS && p->smoother != MG_SMOOTH_WJACOBI) return MG_EINVAL;
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu1 > 16 || p->nu2 > 16) return MG_EINVAL;
    if (p->cycle < MG_CYCLE_V || p->cycle > MG_CYCLE_F || p->cg_iters < 0) return MG_EINVAL;
    if (!(p->omega == p->omega) || p->omega > 2.0) return MG_EINVAL;
    if (p->op != MG_OP_LAPLACE || p->precision != MG_PREC_FP64 || p->coarse_n != 0) return MG_ENOTSUP;
    return MG_OK;
}

// Grid spacing: 0 selects the unit domain's h; any other value must be it
// (1/(n-1) on node grids, 1/n on cell-centred grids).
int validate_h(const mg_params* p) {
    if (p->h == 0.0) return MG_OK;
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return MG_EINVAL;
    const double h = p->bc == MG_BC_NEUMANN_CC ? 1.0 / (double)p->n : 1.0 / (double)(p->n - 1);
    return p->h == h ? MG_OK : MG_ENOTSUP;
}

// A constant stencil: 2d+1 finite FP64 coefficients on the host, centre > 0.
int validate_stencil(const mg_params* p) {
    if (!p->stencil) return MG_EINVAL;
    for (int q = 0; q < 2 * p->dim + 1; ++q)
        if (!std::isfinite(p->stencil[q])) return MG_EINVAL;
    if (!(p->stencil[0] > 0.0)) return MG_EINVAL;
    if (p->precision != MG_PREC_FP64 || p->coarse_n > 3) return MG_ENOTSUP;
    return MG_OK;
}

int validate(const mg_params* p) {
    if (!p) return MG_EINVAL;
    if (p->dim != 2 && p->dim != 3) return MG_EINVAL;
    if (p->bc == MG_BC_NEUMANN_CC) {
        const int v = validate_cc(p);
        return v != MG_OK ? v : validate_h(p);
    }
    if (!valid_edge(p->dim, p->n)) return MG_EINVAL;
    if (p->bc != MG_BC_DIRICHLET_ZERO) return MG_ENOTSUP;
    if (p->op != MG_OP_LAPLACE && p->op != MG_OP_VARCOEF_NODAL && p->op != MG_OP_CONST_STENCIL) return MG_ENOTSUP;
    if (p->op == MG_OP_VARCOEF_NODAL && !p->k) return MG_EINVAL;
    {
        const int vh = validate_h(p);
        if (vh != MG_OK) return vh;
    }
    if (p->smoother != MG_SMOOTH_RBGS && p->smoother != MG_SMOOTH_WJACOBI && p->smoother != MG_SMOOTH_RBGS_SYM)
        return MG_EINVAL;
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu1 > 16 || p->nu2 > 16) return MG_EINVAL;
    if (p->cycle < MG_CYCLE_V || p->cycle > MG_CYCLE_F || p->cg_iters < 0) return MG_EINVAL;
    if (p->coarse_n != 0 && (!valid_edge(p->dim, p->coarse_n) || p->coarse_n > p->n)) return MG_EINVAL;
    if (p->coarse_n > tail_max_edge(p->dim, p->precision == MG_PREC_FP64 ? 8 : 4)) return MG_ENOTSUP;
    if (p->precision != MG_PREC_FP64 && p->precision != MG_PREC_FP32_IR && p->precision != MG_PREC_FP16_IR)
        return MG_ENOTSUP;
    if (p->precision == MG_PREC_FP16_IR && p->op != MG_OP_LAPLACE) return MG_ENOTSUP;
    if (!(p->omega == p->omega) || p->omega > 2.0) return MG_EINVAL;
    if (p->op == MG_OP_CONST_STENCIL) return validate_stencil(p);
    return MG_OK;
}

void destroy(mg_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    free_groups(c->G64);
    free_groups(c->G32);
    ffree(c->tail64.d);
    ffree(c->tail32.d);
    free_levels(c->L64);
    free_levels(c->L32);
    for (size_t l = 0; l < c->ccn.size(); ++l) {
        if (l > 0) ffree(c->ccu[l]);
        ffree(c->cct[l]);
        if (l > 0) ffree(c->ccf[l]);
    }
    ffree(c->ccfh);
    ffree(c->cc_work);
    ffree(c->cc_mean);
    delete c->cd;
    for (size_t l = 0; l < c->stn.size(); ++l) {
        if (l > 0) ffree(c->stu[l]);
        ffree(c->stt[l]);
        if (l > 0) ffree(c->stf[l]);
    }
    ffree(c->d_ir);
    ffree(c->d_scl);
    ffree(c->d_pmax);
    ffree(c->d_top);
    ffree(c->u64_scratch);
    ffree(c->k64);
    ffree(c->d_partial);
    ffree(c->d_spart);
    ffree(c->d_norm);
    ffree(c->d_norm0);
    ffree(c->d_ctrl);
    ffree(c->d_hist);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    for (auto e : c->prof_ev) (void)hipEventDestroy(e);
    delete c;
}

// Point the level-0 descriptors at the caller's u and f (only when they change).
int bind(mg_ctx* c, const void* u, const void* f) {
    if (!u || !f) return MG_EINVAL;
    if (u == c->bound_u && f == c->bound_f) return MG_OK;
    c->h_top.u = const_cast<void*>(u);
    c->h_top.f = f;
    CK(hipMemcpyAsync(c->d_top, &c->h_top, sizeof(GridDesc), hipMemcpyHostToDevice, c->stream));
    if (c->p.precision == MG_PREC_FP64) {
        GridDesc& d = c->G64[0].h[0];
        d.u = const_cast<void*>(u);
        d.f = f;
        CK(hipMemcpyAsync(c->G64[0].d, &d, sizeof(GridDesc), hipMemcpyHostToDevice, c->stream));
    } else {
        c->h_ir.u[0] = (double*)const_cast<void*>(u);
        c->h_ir.f = (const double*)f;
        CK(hipMemcpyAsync(c->d_ir, &c->h_ir, sizeof(IRDesc), hipMemcpyHostToDevice, c->stream));
    }
    CK(hipStreamSynchronize(c->stream));  // the host descriptors may change again right away
    c->bound_u = u;
    c->bound_f = f;
    return MG_OK;
}

int* ctl_done(mg_ctx* c) { return c->d_ctrl; }
int* ctl_steps(mg_ctx* c) { return c->d_ctrl + 1; }
int* ctl_status(mg_ctx* c) { return c->d_ctrl + 2; }

// FP64 norm of the bound (u, f) into d_norm (partials + fixed-order finalize).
// With 'step' > 0 and measurement on, the finest-level pass (not its
// finalize) is bracketed by an event pair tagged (step, kernel 1).
bool prof_begin(mg_ctx* c, int step, hipStream_t s) {
    if (step <= 0 || !c->prof_on || c->prof_n + 2 > (int)c->prof_ev.size()) return false;
    return hipEventRecord(c->prof_ev[(size_t)c->prof_n], s) == hipSuccess;
}
void prof_end(mg_ctx* c, int step, int kind, hipStream_t s) {
    if (hipEventRecord(c->prof_ev[(size_t)c->prof_n + 1], s) != hipSuccess) return;
    c->prof_n += 2;
    c->prof_step.push_back(step);
    c->prof_kind.push_back(kind);
}

hipError_t enqueue_norm(mg_ctx* c, hipStream_t s, int step = 0) {
    const bool var = c->prob.var;
    const int nparts = norm_tiles(c->p.dim, c->p.n, c->top.norm);
    const bool timed = prof_begin(c, step, s);
    hipError_t e = launch_norm(c->p.dim, var, c->d_top, 1, c->p.n, 0, c->d_partial, c->pstride, c->top.norm, s);
    if (timed) prof_end(c, step, 1, s);
    if (e != hipSuccess) return e;
    return launch_norm_finalize(c->d_partial, c->pstride, nparts, 0, 1, c->d_norm, s);
}

// FP64 with the fused norm: the first pre-smoothing sweep of the next cycle
// (reads the bound u, writes its ping-pong partner, leaving u as it is) and
// the norm of u's residual that it sums, into d_norm.  With 'step' > 0 and
// measurement on, the sweep is bracketed and tagged (step, kernel 1).
hipError_t enqueue_nrm_sweep(mg_ctx* c, hipStream_t s, int step = 0) {
    const TileCfg cfg = c->tl64[0].smooth_nrm;
    const int nparts = smooth_tiles(c->p.dim, c->prob.smoother, c->p.n, cfg);
    const bool timed = prof_begin(c, step, s);
    hipError_t e = launch_smooth<double>(c->p.dim, c->prob.smoother, c->prob.var, c->G64[0].d, 1, c->p.n, 0,
                                         SWEEP_NORM, cfg, s);
    if (timed) prof_end(c, step, 1, s);
    if (e != hipSuccess) return e;
    return launch_norm_finalize(c->d_spart, nparts, nparts, 0, 1, c->d_norm, s);
}

hipError_t enqueue_ir(mg_ctx* c, int sel, int flags, hipStream_t s, int step = 0) {
    const int nparts = norm_tiles(c->p.dim, c->p.n, c->top.norm);
    const bool timed = prof_begin(c, step, s);
    const bool h16 = is_h16(c->p);
    hipError_t e = h16 ? launch_ir_update_f16(c->p.dim, c->d_ir, 1, c->p.n, sel, flags, c->d_partial, c->pstride,
                                              c->top.norm, s)
                       : launch_ir_update(c->p.dim, c->prob.var, c->d_ir, 1, c->p.n, sel, flags, c->d_partial,
                                          c->pstride, c->top.norm, s);
    if (timed) prof_end(c, step, 1, s);
    if (e != hipSuccess) return e;
    if (h16) return launch_norm_finalize_f16(c->d_partial, c->d_pmax, nparts, c->d_norm, c->d_scl, ctl_done(c), s);
    return launch_norm_finalize(c->d_partial, c->pstride, nparts, 0, 1, c->d_norm, s);
}

// Residual of the bound (u, f) handed to the refinement's first cycle, with
// rho_0 in d_norm.  The binary16 form first measures the residual's largest
// magnitude, then writes the residual with the scale that magnitude gives.
hipError_t enqueue_ir_start(mg_ctx* c, hipStream_t s) {
    if (is_h16(c->p)) {
        hipError_t e = enqueue_ir(c, 0, IR_NO_UPDATE, s);
        if (e != hipSuccess) return e;
    }
    return enqueue_ir(c, 0, IR_NO_UPDATE, s);
}

// K solve steps (cycle + residual norm + stop test), IR steps alternate the
// FP64 ping-pong starting from sel 0 (K even keeps the parity per chunk).
// With 'prof', step0 + i + 1 tags the measured launches of step i.  Refinement
// step i reads the FP64 iterate from ping-pong buffer (par0 + i) & 1.
hipError_t enqueue_steps(mg_ctx* c, int K, double tol, int max_cycles, hipStream_t s, bool prof, int step0 = 0,
                         int par0 = 0) {
    hipEvent_t* pev = prof ? c->prof_ev.data() : nullptr;
    int* pn = prof ? &c->prof_n : nullptr;
    const int pcap = (int)c->prof_ev.size();
    for (int i = 0; i < K; ++i) {
        hipError_t e;
        const int step = prof ? step0 + i + 1 : 0;
        const int n0 = c->prof_n;
        if (c->p.precision == MG_PREC_FP64) {
            // with the fused norm the cycle's first sweep ran at the end of the
            // previous step (or before the first); this step ends with the next one's
            e = vcycle<double>(c->prob, c->G64, false, c->tl64, s, pev, pn, pcap, &c->tail64, c->nrm_fused);
            for (int j = n0; prof && j < c->prof_n; j += 2) c->prof_step.push_back(step), c->prof_kind.push_back(0);
            if (e != hipSuccess) return e;
            e = c->nrm_fused ? enqueue_nrm_sweep(c, s, step) : enqueue_norm(c, s, step);
        } else {
            e = is_h16(c->p) ? vcycle<half_t>(c->prob, c->G32, true, c->tl32, s, pev, pn, pcap, &c->tail32)
                             : vcycle<float>(c->prob, c->G32, true, c->tl32, s, pev, pn, pcap, &c->tail32);
            for (int j = n0; prof && j < c->prof_n; j += 2) c->prof_step.push_back(step), c->prof_kind.push_back(0);
            if (e != hipSuccess) return e;
            e = enqueue_ir(c, (par0 + i) & 1, 0, s, step);
        }
        if (e != hipSuccess) return e;
        e = launch_stop_test(c->d_norm, c->d_norm0, ctl_done(c), ctl_steps(c), ctl_status(c), c->d_hist,
                             c->hist_cap, tol, max_cycles, 1, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int ensure_hist(mg_ctx* c, int cap) {
    if (cap <= c->hist_cap) return MG_OK;
    ffree(c->d_hist);
    c->d_hist = nullptr;
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    c->h_pin = nullptr;
    c->hist_cap = 0;
    CK(hipMalloc((void**)&c->d_hist, sizeof(double) * (size_t)cap));
    CK(hipHostMalloc((void**)&c->h_pin, sizeof(double) * (size_t)(cap + 8), hipHostMallocDefault));
    c->hist_cap = cap;
    // the hist pointer is baked into captured graphs
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    return MG_OK;
}

int run_chunk(mg_ctx* c, int K, double tol, int max_cycles, int step0) {
    const bool use_graph = !c->prof_on && c->use_graphs;
    const int par0 = is_ir(c->p) ? (step0 & 1) : 0;
    if (!use_graph) {
        CK(enqueue_steps(c, K, tol, max_cycles, c->stream, c->prof_on, step0, par0));
        return MG_OK;
    }
    hipGraphExec_t exec = nullptr;
    for (const auto& g : c->graphs)
        if (g.steps == K && g.par == par0 && g.tol == tol && g.max_cycles == max_cycles) exec = g.exec;
    if (!exec) {
        if (c->graphs.size() >= 16) {  // a new tolerance or limit: start over
            for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
            c->graphs.clear();
        }
        if (!c->cap_stream) CK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        CK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_steps(c, K, tol, max_cycles, c->cap_stream, false, 0, par0);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return dev_status(e);
        }
        CK(e2);
        hipError_t e3 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        CK(e3);
        c->graphs.push_back({K, par0, max_cycles, tol, exec});
    }
    CK(hipGraphLaunch(exec, c->stream));
    return MG_OK;
}

// Steps of the next chunk: as many as the contraction of the last step
// predicts are still needed to reach tol (at least one, at most kmax).  hist
// holds the norms of steps 0 .. steps.
int next_chunk(const double* hist, int steps, double tol, int kmax) {
    if (steps < 1) return kmax;
    const double r0 = hist[0], rk = hist[steps], rp = hist[steps - 1];
    if (!(r0 > 0.0) || !(rk > 0.0) || !(rp > 0.0)) return kmax;
    const double rate = rk / rp;
    if (!(rate < 0.9)) return kmax;
    const double need = std::log(tol * r0 / rk) / std::log(rate);
    if (!(need > 0.0)) return 1;
    return std::max(1, std::min(kmax, (int)std::ceil(need - 1e-9)));
}


// ---------------------------------------------------------------------------
// Cell-centred Neumann grids: Algorithm 1 level by level (V, W or F), plain
// kernels; the iterate of level l is in 'cur' (the other buffer of the level
// is the Jacobi partner).  Returns the buffer that holds the result.
// ---------------------------------------------------------------------------
hipError_t cc_smooth_level(mg_ctx* c, int l, double*& cur, double*& other, const double* f, CCConst L) {
    const int dim = c->p.dim;
    hipStream_t s = c->stream;
    if (c->p.smoother == MG_SMOOTH_WJACOBI) {
        hipError_t e = cc_relax(dim, true, cur, other, f, L, 0, s);
        std::swap(cur, other);
        return e;
    }
    hipError_t e = cc_relax(dim, false, cur, cur, f, L, 0, s);
    if (e != hipSuccess) return e;
    return cc_relax(dim, false, cur, cur, f, L, 1, s);
}

hipError_t cc_cycle(mg_ctx* c, int l, int kind, double*& cur, double*& other, const double* f) {
    const int dim = c->p.dim, n = c->ccn[(size_t)l];
    hipStream_t s = c->stream;
    hipError_t e = hipSuccess;
    if (l + 1 == (int)c->ccn.size()) return cc_fill(cur, cc_cells(dim, n), 0.0, s);  // one cell: zero correction
    const CCConst L = cc_const(dim, n, c->p.omega);
    for (int i = 0; i < c->p.nu1 && e == hipSuccess; ++i) e = cc_smooth_level(c, l, cur, other, f, L);
    if (e != hipSuccess) return e;
    double* fc = c->ccf[(size_t)l + 1];
    e = cc_restrict(dim, cur, f, fc, L, s);
    if (e != hipSuccess) return e;
    double* ucur = c->ccu[(size_t)l + 1];
    double* uoth = c->cct[(size_t)l + 1];
    e = cc_fill(ucur, cc_cells(dim, n / 2), 0.0, s);
    if (e != hipSuccess) return e;
    if (kind == MG_CYCLE_V) {
        e = cc_cycle(c, l + 1, MG_CYCLE_V, ucur, uoth, fc);
    } else if (kind == MG_CYCLE_W) {
        e = cc_cycle(c, l + 1, MG_CYCLE_W, ucur, uoth, fc);
        if (e == hipSuccess) e = cc_cycle(c, l + 1, MG_CYCLE_W, ucur, uoth, fc);
    } else {
        e = cc_cycle(c, l + 1, MG_CYCLE_F, ucur, uoth, fc);
        if (e == hipSuccess) e = cc_cycle(c, l + 1, MG_CYCLE_V, ucur, uoth, fc);
    }
    if (e != hipSuccess) return e;
    // the coarse buffers keep their roles for the next cycle
    c->ccu[(size_t)l + 1] = ucur;
    c->cct[(size_t)l + 1] = uoth;
    e = cc_prolong(dim, cur, ucur, n, s);
    for (int i = 0; i < c->p.nu2 && e == hipSuccess; ++i) e = cc_smooth_level(c, l, cur, other, f, L);
    return e;
}

// One cycle on the caller's u (level 0), the result back in u.
hipError_t cc_cycle_top(mg_ctx* c, double* u, const double* f) {
    double* cur = u;
    double* other = c->cct[0];
    hipError_t e = cc_cycle(c, 0, c->p.cycle, cur, other, f);
    if (e == hipSuccess && cur != u)
        e = hipMemcpyAsync(u, cur, cc_cells(c->p.dim, c->p.n) * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    return e;
}

int cc_setup(mg_ctx* c) {
    const int dim = c->p.dim;
    hipStream_t s = c->stream;
    c->cc = true;
    for (int m = c->p.n; m >= 1; m /= 2) c->ccn.push_back(m);
    const size_t L = c->ccn.size();
    c->ccu.assign(L, nullptr);
    c->cct.assign(L, nullptr);
    c->ccf.assign(L, nullptr);
    for (size_t l = 0; l < L; ++l) {
        const size_t bytes = cc_cells(dim, c->ccn[l]) * sizeof(double);
        if (l > 0) CK(zalloc((void**)&c->ccu[l], bytes, s));
        CK(zalloc((void**)&c->cct[l], bytes, s));
        if (l > 0) CK(zalloc((void**)&c->ccf[l], bytes, s));
    }
    CK(zalloc((void**)&c->ccfh, cc_cells(dim, c->p.n) * sizeof(double), s));
    CK(hipMalloc((void**)&c->cc_work, cc_work_doubles(dim, c->p.n) * sizeof(double)));
    CK(hipMalloc((void**)&c->cc_mean, sizeof(double)));
    c->nlev = (int)L;
    c->pstride = cc_norm_parts(dim, c->p.n);
    CK(hipMalloc((void**)&c->d_partial, sizeof(double) * (size_t)c->pstride));
    CK(hipMalloc((void**)&c->d_norm, sizeof(double)));
    CK(hipMalloc((void**)&c->d_norm0, sizeof(double)));
    CK(hipMalloc((void**)&c->d_ctrl, 3 * sizeof(int)));
    CK(launch_fill_int(c->d_ctrl, 0, 3, s));
    int r = ensure_hist(c, 64);
    if (r != MG_OK) return r;
    CK(hipStreamSynchronize(s));
    return MG_OK;
}

int cc_solve(mg_ctx* c, double* u, const double* f, double tol, int max_cycles, int* cycles_done, double* res_hist) {
    const int dim = c->p.dim, n = c->p.n;
    hipStream_t s = c->stream;
    const CCConst L0 = cc_const(dim, n, c->p.omega);
    int r = ensure_hist(c, max_cycles + 1);
    if (r != MG_OK) return r;
    CK(hipMemcpyAsync(c->ccfh, f, cc_cells(dim, n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    CK(cc_remove_mean(dim, n, c->ccfh, c->cc_work, c->cc_mean, s));
    CK(cc_remove_mean(dim, n, u, c->cc_work, c->cc_mean, s));
    CK(launch_fill_int(ctl_done(c), 0, 1, s));
    CK(cc_norm(dim, u, c->ccfh, L0, c->d_partial, c->d_norm, s));
    CK(launch_solve_init(c->d_norm, c->d_norm0, ctl_done(c), ctl_steps(c), ctl_status(c), c->d_hist, c->hist_cap, 1,
                         s));
    int* ctl = (int*)c->h_pin;
    CK(hipMemcpyAsync(ctl, c->d_ctrl, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    int steps = 0;
    // one cycle per round trip: the host keeps the Jacobi buffer roles, so no
    // cycle is queued past the stop test
    while (!ctl[0] && steps < max_cycles) {
        CK(cc_cycle_top(c, u, c->ccfh));
        CK(cc_remove_mean(dim, n, u, c->cc_work, c->cc_mean, s));
        CK(cc_norm(dim, u, c->ccfh, L0, c->d_partial, c->d_norm, s));
        CK(launch_stop_test(c->d_norm, c->d_norm0, ctl_done(c), ctl_steps(c), ctl_status(c), c->d_hist, c->hist_cap,
                            tol, max_cycles, 1, s));
        CK(hipMemcpyAsync(ctl, c->d_ctrl, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        ++steps;
    }
    steps = ctl[1];
    const int status = ctl[2];
    if (res_hist) {
        CK(hipMemcpyAsync(c->h_pin, c->d_hist, sizeof(double) * (size_t)(steps + 1), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        std::memcpy(res_hist, c->h_pin, sizeof(double) * (size_t)(steps + 1));
    }
    if (cycles_done) *cycles_done = steps;
    if (status == 0) return MG_OK;
    if (status == -5) return MG_EDIVERGED;
    return MG_ENOTCONV;
}

// ---------------------------------------------------------------------------
// Constant stencil: Algorithm 1 level by level (V, W or F), plain kernels,
// levels n, (n-1)/2+1, ..., 3; the iterate of level l is in 'cur' (the other
// buffer of the level is the Jacobi partner).
// ---------------------------------------------------------------------------
hipError_t st_smooth_level(mg_ctx* c, double*& cur, double*& other, const double* f, const STConst& L, bool post) {
    const int dim = c->p.dim;
    hipStream_t s = c->stream;
    if (c->p.smoother == MG_SMOOTH_WJACOBI) {
        hipError_t e = st_relax(dim, true, cur, other, f, L, 0, s);
        std::swap(cur, other);
        return e;
    }
    const int first = (post && c->p.smoother == MG_SMOOTH_RBGS_SYM) ? 1 : 0;
    hipError_t e = st_relax(dim, false, cur, cur, f, L, first, s);
    if (e != hipSuccess) return e;
    return st_relax(dim, false, cur, cur, f, L, 1 - first, s);
}

hipError_t st_cycle(mg_ctx* c, int l, int kind, double*& cur, double*& other, const double* f) {
    const int dim = c->p.dim, n = c->stn[(size_t)l];
    hipStream_t s = c->stream;
    const STConst L = st_const(dim, n, c->st_coef, c->p.omega);
    if (l + 1 == (int)c->stn.size()) return st_coarsest(dim, cur, f, L, s);  // n = 3: one unknown
    hipError_t e = hipSuccess;
    for (int i = 0; i < c->p.nu1 && e == hipSuccess; ++i) e = st_smooth_level(c, cur, other, f, L, false);
    if (e != hipSuccess) return e;
    double* fc = c->stf[(size_t)l + 1];
    if ((e = st_restrict(dim, cur, f, fc, L, s)) != hipSuccess) return e;
    double* ucur = c->stu[(size_t)l + 1];
    double* uoth = c->stt[(size_t)l + 1];
    const int nc = c->stn[(size_t)l + 1];
    if ((e = cc_fill(ucur, npts(dim, nc), 0.0, s)) != hipSuccess) return e;  // zero guess
    if (kind == MG_CYCLE_V) {
        e = st_cycle(c, l + 1, MG_CYCLE_V, ucur, uoth, fc);
    } else if (kind == MG_CYCLE_W) {
        e = st_cycle(c, l + 1, MG_CYCLE_W, ucur, uoth, fc);
        if (e == hipSuccess) e = st_cycle(c, l + 1, MG_CYCLE_W, ucur, uoth, fc);
    } else {
        e = st_cycle(c, l + 1, MG_CYCLE_F, ucur, uoth, fc);
        if (e == hipSuccess) e = st_cycle(c, l + 1, MG_CYCLE_V, ucur, uoth, fc);
    }
    if (e != hipSuccess) return e;
    c->stu[(size_t)l + 1] = ucur;
    c->stt[(size_t)l + 1] = uoth;
    e = st_prolong(dim, cur, ucur, n, s);
    for (int i = 0; i < c->p.nu2 && e == hipSuccess; ++i) e = st_smooth_level(c, cur, other, f, L, true);
    return e;
}

hipError_t st_cycle_top(mg_ctx* c, double* u, const double* f) {
    double* cur = u;
    double* other = c->stt[0];
    hipError_t e = st_cycle(c, 0, c->p.cycle, cur, other, f);
    if (e == hipSuccess && cur != u)
        e = hipMemcpyAsync(u, cur, npts(c->p.dim, c->p.n) * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    return e;
}

int st_setup(mg_ctx* c) {
    const int dim = c->p.dim;
    hipStream_t s = c->stream;
    c->st = true;
    for (int q = 0; q < 2 * dim + 1; ++q) c->st_coef[q] = c->p.stencil[q];
    c->p.stencil = nullptr;  // the context keeps its own copy
    for (int m = c->p.n; m >= 3; m = (m - 1) / 2 + 1) {
        c->stn.push_back(m);
        if (m == 3) break;
    }
    const size_t L = c->stn.size();
    c->stu.assign(L, nullptr);
    c->stt.assign(L, nullptr);
    c->stf.assign(L, nullptr);
    for (size_t l = 0; l < L; ++l) {
        const size_t bytes = npts(dim, c->stn[l]) * sizeof(double);
        if (l > 0) CK(zalloc((void**)&c->stu[l], bytes, s));
        CK(zalloc((void**)&c->stt[l], bytes, s));
        if (l > 0) CK(zalloc((void**)&c->stf[l], bytes, s));
    }
    c->nlev = (int)L;
    c->pstride = st_norm_parts(dim, c->p.n);
    CK(hipMalloc((void**)&c->d_partial, sizeof(double) * (size_t)c->pstride));
    CK(hipMalloc((void**)&c->d_norm, sizeof(double)));
    CK(hipMalloc((void**)&c->d_norm0, sizeof(double)));
    CK(hipMalloc((void**)&c->d_ctrl, 3 * sizeof(int)));
    CK(launch_fill_int(c->d_ctrl, 0, 3, s));
    int r = ensure_hist(c, 64);
    if (r != MG_OK) return r;
    CK(hipStreamSynchronize(s));
    return MG_OK;
}

int st_solve(mg_ctx* c, double* u, const double* f, double tol, int max_cycles, int* cycles_done, double* res_hist) {
    const int dim = c->p.dim, n = c->p.n;
    hipStream_t s = c->stream;
    const STConst L0 = st_const(dim, n, c->st_coef, c->p.omega);
    int r = ensure_hist(c, max_cycles + 1);
    if (r != MG_OK) return r;
    CK(launch_fill_int(ctl_done(c), 0, 1, s));
    CK(st_norm(dim, u, f, L0, c->d_partial, c->d_norm, s));
    CK(launch_solve_init(c->d_norm, c->d_norm0, ctl_done(c), ctl_steps(c), ctl_status(c), c->d_hist, c->hist_cap, 1,
                         s));
    int* ctl = (int*)c->h_pin;
    CK(hipMemcpyAsync(ctl, c->d_ctrl, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    int steps = 0;
    while (!ctl[0] && steps < max_cycles) {
        CK(st_cycle_top(c, u, f));
        CK(st_norm(dim, u, f, L0, c->d_partial, c->d_norm, s));
        CK(launch_stop_test(c->d_norm, c->d_norm0, ctl_done(c), ctl_steps(c), ctl_status(c), c->d_hist, c->hist_cap,
                            tol, max_cycles, 1, s));
        CK(hipMemcpyAsync(ctl, c->d_ctrl, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        ++steps;
    }
    steps = ctl[1];
    const int status = ctl[2];
    if (res_hist) {
        CK(hipMemcpyAsync(c->h_pin, c->d_hist, sizeof(double) * (size_t)(steps + 1), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        std::memcpy(res_hist, c->h_pin, sizeof(double) * (size_t)(steps + 1));
    }
    if (cycles_done) *cycles_done = steps;
    if (status == 0) return MG_OK;
    if (status == -5) return MG_EDIVERGED;
    return MG_ENOTCONV;
}

// ---------------------------------------------------------------------------
// Complex diffusion: FAS level by level.
// ---------------------------------------------------------------------------
size_t cd_cells(const CDState& S, int l) {
    const size_t n = (size_t)S.ln[(size_t)l];
    return S.dim == 2 ? n * n : n * n * n;
}

// one sweep (both colours or Jacobi): tiled into the level's other buffer, or
// per cell (small 3D levels), g of the pre-sweep iterate formed in the relaxation
hipError_t cd_sweep_level(CDState& S, int l, void*& cur, void*& other, const void* f, hipStream_t s,
                          const void* uc = nullptr, const void* uh = nullptr) {
    const CDLevel L = cd_level(S.ln[(size_t)l]);
    if (cd_tiled(S.dim, L.n)) {
        const hipError_t e = cd_sweep(S.dim, S.jacobi, cur, other, f, S.K, L, s, uc, uh);
        std::swap(cur, other);
        return e;
    }
    hipError_t e = hipSuccess;
    if (S.jacobi) {
        e = cd_relax(S.dim, true, cur, other, f, S.g[(size_t)l], S.K, L, 0, s);
        std::swap(cur, other);
        return e;
    }
    e = cd_relax(S.dim, false, cur, cur, f, S.g[(size_t)l], S.K, L, 0, s);
    if (e != hipSuccess) return e;
    return cd_relax(S.dim, false, cur, cur, f, S.g[(size_t)l], S.K, L, 1, s);
}

hipError_t cd_fas_level(CDState& S, int l, void*& cur, void*& other, const void* f, hipStream_t s) {
    const size_t N = cd_cells(S, l);
    if (l + 1 == (int)S.ln.size()) return cd_scale(f, cur, N, S.tau, s);  // one cell: N(u) = u / tau
    const CDLevel L = cd_level(S.ln[(size_t)l]), Lc = cd_level(S.ln[(size_t)l + 1]);
    hipError_t e = hipSuccess;
    for (int i = 0; i < S.nu1 && e == hipSuccess; ++i) e = cd_sweep_level(S, l, cur, other, f, s);
    if (e != hipSuccess) return e;
    const size_t c1 = (size_t)l + 1;
    void* ucur = S.u[c1];
    void* uoth = S.t[c1];
    if ((e = cd_restrict(S.dim, cur, f, S.uh[c1], S.f[c1], S.K, L, s)) != hipSuccess) return e;
    if ((e = cd_coarse_rhs(S.dim, S.uh[c1], S.f[c1], ucur, S.K, Lc, s)) != hipSuccess) return e;
    if ((e = cd_fas_level(S, l + 1, ucur, uoth, S.f[c1], s)) != hipSuccess) return e;
    S.u[c1] = ucur;
    S.t[c1] = uoth;
    // tiled levels apply the correction in the first post-smoothing sweep's loads
    const bool fused = S.nu2 >= 1 && cd_sweep_corrects(S.dim, S.jacobi, S.ln[(size_t)l]);
    if (!fused && (e = cd_prolong(S.dim, cur, ucur, S.uh[c1], S.ln[(size_t)l], s)) != hipSuccess) return e;
    for (int i = 0; i < S.nu2 && e == hipSuccess; ++i)
        e = fused && i == 0 ? cd_sweep_level(S, l, cur, other, f, s, ucur, S.uh[c1])
                            : cd_sweep_level(S, l, cur, other, f, s);
    return e;
}

hipError_t cd_fas_top(CDState& S, void* u, const void* f, hipStream_t s) {
    void* cur = u;
    void* other = S.t[0];
    hipError_t e = cd_fas_level(S, 0, cur, other, f, s);
    if (e == hipSuccess && cur != u) e = hipMemcpyAsync(u, cur, cd_cells(S, 0) * 16, hipMemcpyDeviceToDevice, s);
    return e;
}

// ||f - N(u)|| (g of u) to the host
int cd_norm_host(CDState& S, const void* u, const void* f, hipStream_t s, double* out) {
    CK(cd_norm(S.dim, u, f, S.K, cd_level(S.n), S.part, S.norm, s));
    CK(hipMemcpyAsync(S.h_norm, S.norm, sizeof(double), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    *out = S.h_norm[0];
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: for every level large enough to matter, time each candidate
// launch geometry (tile rows x z-chunk) of the smoothing, restriction and
// finest-level norm / refinement kernels on the context's own buffers and
// keep the fastest.  Results are bitwise independent of the geometry, so
// tuning changes time only.  Choices are cached per process.
// ---------------------------------------------------------------------------

// dim, elem, n, family, smoother, var, mode, batch (0: one grid; else bit length of the instance count)
typedef std::tuple<int, int, int, int, int, int, int, int> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, TileCfg> g_tune;

constexpr size_t kTuneMinPoints = 1u << 16;

// Candidate launch geometries.  In 3D, smoothing (family 0) and the norm /
// refinement pass (family 2) also vary the wavefronts per workgroup (8 for
// 16- and 32-row tiles); smoothing also runs one wavefront per tile with 8 or
// 12 rows in registers.
std::vector<TileCfg> tune_candidates(int dim, int planes, bool with_pd, int family, int elem, bool var) {
    std::vector<TileCfg> v;
    const int geo[7][2] = {{8, 4}, {16, 4}, {32, 4}, {16, 8}, {32, 8}, {8, 1}, {12, 1}};
    for (const auto& g : geo) {
        const int by = g[0], wv = g[1];
        if (wv != 4 && (dim == 2 || family == 1 || (family == 2 && wv == 1))) continue;
        if (by > max_tile_rows(dim, elem, var, family, wv)) continue;
        if (dim == 2) {
            v.push_back({by, 1, 1, 4});
            if (family == 2 && !var && by == 16) {  // two nodes per lane, marching chunks of rows
                for (int yc = 8; yc <= 256 && yc <= std::max(8, planes); yc *= 2) {
                    v.push_back({16, yc, 1, 4, 0, 2});
                    if (with_pd) v.push_back({16, yc, 2, 4, 0, 2});
                }
            }
            continue;
        }
        for (int zc = 4; zc <= 256; zc *= 2) {
            if (zc > std::max(4, planes)) break;
            v.push_back({by, zc, 1, wv});
            if (with_pd) v.push_back({by, zc, 2, wv});
            if (family == 2 && !var && by <= 4 * wv) {  // two nodes per lane, at most four rows per thread
                v.push_back({by, zc, 1, wv, 0, 2});
                if (with_pd) v.push_back({by, zc, 2, wv, 0, 2});
            }
        }
    }
    return v;
}

// Time every candidate (after warming the GPU up to its working clocks) in three
// interleaved rounds and keep the fastest by its best round.
template <class Launch>
TileCfg pick_fastest(const std::vector<TileCfg>& cands, TileCfg fallback, Launch&& launch, hipStream_t s) {
    hipEvent_t a = nullptr, b = nullptr;
    if (cands.empty() || hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return fallback;
    std::vector<float> best_ms(cands.size(), 1e30f);
    std::vector<char> ok(cands.size(), 1);
    // warm-up: about 60 ms of the first candidate (the GPU leaves its idle clocks)
    {
        (void)hipEventRecord(a, s);
        (void)launch(cands[0]);
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        const int reps = std::min(600, std::max(2, (int)(60.0f / std::max(ms, 1e-3f))));
        for (int r = 0; r < reps; ++r) (void)launch(cands[0]);
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
    }
    for (int round = 0; round < 3; ++round) {
        for (size_t i = 0; i < cands.size(); ++i) {
            if (!ok[i]) continue;
            if (launch(cands[i]) != hipSuccess) {
                (void)hipGetLastError();
                ok[i] = 0;
                continue;
            }
            (void)hipEventRecord(a, s);
            for (int r = 0; r < 3; ++r) (void)launch(cands[i]);
            (void)hipEventRecord(b, s);
            if (hipEventSynchronize(b) != hipSuccess) {
                ok[i] = 0;
                continue;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, a, b);
            best_ms[i] = std::min(best_ms[i], ms);
        }
    }
    TileCfg best = fallback;
    float bt = 1e30f;
    for (size_t i = 0; i < cands.size(); ++i)
        if (ok[i] && best_ms[i] < bt) {
            bt = best_ms[i];
            best = cands[i];
        }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

// Time of one configuration as pick_fastest measures it (best of three
// rounds of three launches, in ms), or a huge value if it fails.
template <class Launch>
float time_launch(Launch&& launch, TileCfg cfg, hipStream_t s) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return 1e30f;
    float best = 1e30f;
    for (int round = 0; round < 3; ++round) {
        if (launch(cfg) != hipSuccess) {
            (void)hipGetLastError();
            best = 1e30f;
            break;
        }
        (void)hipEventRecord(a, s);
        for (int r = 0; r < 3; ++r) (void)launch(cfg);
        (void)hipEventRecord(b, s);
        if (hipEventSynchronize(b) != hipSuccess) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        best = std::min(best, ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

// Block order of a chosen smoothing geometry: XCD bands or linear, whichever
// times faster.
template <class Launch>
TileCfg pick_order(TileCfg best, Launch&& launch, hipStream_t s) {
    TileCfg lin = best;
    lin.order = 1;
    return pick_fastest(std::vector<TileCfg>{best, lin}, best, launch, s);
}

bool tune_lookup(const TuneKey& k, TileCfg* out) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const TuneKey& k, TileCfg v) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[k] = v;
}

// Launch shapes of the two fused pre-smoothing sweeps from a zero iterate:
// 3D rows 12 / 16 x z-chunks of 8 .. 128 planes, 2D chunks of 16 .. 256 rows
// per wavefront; both block orders.
std::vector<TileCfg> smooth2_candidates(int dim, int n) {
    std::vector<TileCfg> cands;
    const int m = n - 2;
    for (int by : dim == 2 ? std::vector<int>{1} : std::vector<int>{12, 16})
        for (int zc = dim == 2 ? 16 : 8; zc <= (dim == 2 ? 256 : 128) && zc <= std::max(dim == 2 ? 16 : 8, m); zc *= 2)
            for (int order : {0, 1}) {
                TileCfg t{dim == 2 ? 12 : by, zc};
                t.order = order;
                cands.push_back(t);
            }
    return cands;
}

// Tune one hierarchy (levels of 'elem' bytes).  scratch_u / scratch_f stand in
// for caller-owned level-0 arrays.
hipError_t tune_levels(mg_ctx* c, const Levels& L, std::vector<Tiles>& tl, void* scratch_u, void* scratch_f) {
    const int dim = c->p.dim;
    hipStream_t s = c->stream;
    GridDesc* d = nullptr;
    hipError_t e = hipMalloc((void**)&d, sizeof(GridDesc));
    if (e != hipSuccess) return e;
    for (int l = 0; l + 1 < L.nlev; ++l) {
        const int n = L.n[(size_t)l];
        if (npts(dim, n) < kTuneMinPoints) continue;
        GridDesc h{};
        h.u = L.u[(size_t)l] ? L.u[(size_t)l] : scratch_u;
        h.t = L.t[(size_t)l];
        h.f = L.f[(size_t)l] ? L.f[(size_t)l] : scratch_f;
        h.k = L.k[(size_t)l];
        h.fx = (size_t)l < L.fx.size() ? L.fx[(size_t)l] : nullptr;
        h.fc = L.f[(size_t)l + 1];
        h.uc = L.u[(size_t)l + 1];
        h.n = n;
        h.c = level_c(n);
        h.wd = level_wd(dim, n, c->p.omega);
        h.omega = c->p.omega;
        e = hipMemcpyAsync(d, &h, sizeof(GridDesc), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) break;
        const bool var = c->prob.var;
        const int sm = c->prob.smoother;
        TileCfg cfg;
        // the three sweep variants (plain, from a zero iterate, with the fused
        // coarse-grid correction) load different data and are tuned separately
        const int vflags[3] = {0, SWEEP_ZERO_GUESS, SWEEP_PROLONG};
        TileCfg* vcfg[3] = {&tl[(size_t)l].smooth, &tl[(size_t)l].smooth_zg, &tl[(size_t)l].smooth_pro};
        for (int v = 0; v < 3; ++v) {
            const int fl = vflags[v];
            TuneKey ks{dim, L.elem, n, 0, sm, var ? 1 : 0, 10 + v, 0};
            if (!tune_lookup(ks, &cfg)) {
                auto run = [&](TileCfg t) {
                    return L.elem == 8   ? launch_smooth<double>(dim, sm, var, d, 1, n, 0, fl, t, s)
                           : L.elem == 4 ? launch_smooth<float>(dim, sm, var, d, 1, n, 0, fl, t, s)
                                         : launch_smooth<half_t>(dim, sm, var, d, 1, n, 0, fl, t, s);
                };
                cfg = pick_fastest(tune_candidates(dim, n - 2, true, 0, L.elem, var), *vcfg[v], run, s);
                cfg = pick_order(cfg, run, s);
                tune_store(ks, cfg);
            }
            *vcfg[v] = cfg;
        }
        // FP64 finest level: the first pre-smoothing sweep that also sums the
        // incoming iterate's r^2 (LDS tile geometries only)
        if (l == 0 && L.elem == 8 && c->nrm_fused) {
            TuneKey kn{dim, 8, n, 0, sm, var ? 1 : 0, 13, 0};
            if (!tune_lookup(kn, &cfg)) {
                h.npart = c->d_spart;
                e = hipMemcpyAsync(d, &h, sizeof(GridDesc), hipMemcpyHostToDevice, s);
                if (e != hipSuccess) break;
                std::vector<TileCfg> cands;
                for (TileCfg t : tune_candidates(dim, n - 2, true, 0, 8, var))
                    if (t.wv != 1 && smooth_tiles(dim, sm, n, t) <= c->spart_cap) cands.push_back(t);
                auto run = [&](TileCfg t) { return launch_smooth<double>(dim, sm, var, d, 1, n, 0, SWEEP_NORM, t, s); };
                cfg = pick_fastest(cands, tl[(size_t)l].smooth_nrm, run, s);
                cfg = pick_order(cfg, run, s);
                tune_store(kn, cfg);
            }
            tl[(size_t)l].smooth_nrm = cfg;
        }
        TuneKey kr{dim, L.elem, n, 1, 0, var ? 1 : 0, 0, 0};
        if (!tune_lookup(kr, &cfg)) {
            std::vector<TileCfg> cands;
            for (TileCfg t : tune_candidates(dim, (n - 1) / 2 - 1, false, 1, L.elem, var))
                if (t.by >= 8) cands.push_back(t);
            cfg = pick_fastest(cands, tl[(size_t)l].restr, [&](TileCfg t) {
                return L.elem == 8   ? launch_restrict<double>(dim, var, d, 1, n, 0, t, s)
                       : L.elem == 4 ? launch_restrict<float>(dim, var, d, 1, n, 0, t, s)
                                     : launch_restrict<half_t>(dim, var, d, 1, n, 0, t, s);
            }, s);
            tune_store(kr, cfg);
        }
        tl[(size_t)l].restr = cfg;
        // the last pre-smoothing sweep fused with the residual and restriction,
        // kept if it beats the plain sweep and the restriction it replaces
        if (dim == 3 && !var && sm == SM_RBGS && L.elem <= 4 && c->p.nu1 >= 1) {
            TuneKey kf{dim, L.elem, n, 5, sm, 0, 0, 0};
            if (!tune_lookup(kf, &cfg)) {
                std::vector<TileCfg> cands;
                for (int zc : {2, 4, 8, 16})
                    for (int order : {0, 1}) {
                        TileCfg t{16, zc};
                        t.order = order;
                        cands.push_back(t);
                    }
                auto runf = [&](TileCfg t) {
                    return L.elem == 4 ? launch_smooth_restrict3d<float>(d, 1, n, 0, t, s)
                                       : launch_smooth_restrict3d<half_t>(d, 1, n, 0, t, s);
                };
                TileCfg best = pick_fastest(cands, cands[0], runf, s);
                const float t_fused = time_launch(runf, best, s);
                const TileCfg sw = tl[(size_t)l].smooth, rs = tl[(size_t)l].restr;
                const float t_sep =
                    time_launch([&](TileCfg) {
                        if (L.elem == 4) {
                            (void)launch_smooth<float>(dim, sm, false, d, 1, n, 0, 0, sw, s);
                            return launch_restrict<float>(dim, false, d, 1, n, 1, rs, s);
                        }
                        (void)launch_smooth<half_t>(dim, sm, false, d, 1, n, 0, 0, sw, s);
                        return launch_restrict<half_t>(dim, false, d, 1, n, 1, rs, s);
                    }, sw, s);
                cfg = best;
                if (!(t_fused < t_sep)) cfg.zchunk = -best.zchunk;  // declined (depth kept for forcing)
                tune_store(kf, cfg);
            }
            tl[(size_t)l].fused = cfg;
            if (cfg.zchunk < 0) tl[(size_t)l].fused.zchunk = std::getenv("MG_FUSED_RESTRICT") ? -cfg.zchunk : 0;
        }
        // the first two pre-smoothing sweeps from a zero iterate in one launch,
        // kept if it beats the two sweeps it replaces
        if (!var && sm == SM_RBGS && L.elem <= 4 && c->p.nu1 >= 2) {
            TuneKey k2{dim, L.elem, n, 6, sm, 0, 0, 0};
            if (!tune_lookup(k2, &cfg)) {
                const std::vector<TileCfg> cands = smooth2_candidates(dim, n);
                auto run2 = [&](TileCfg t) {
                    if (dim == 2)
                        return L.elem == 4 ? launch_smooth2d_zg2<float>(d, 1, n, 1, t, s)
                                           : launch_smooth2d_zg2<half_t>(d, 1, n, 1, t, s);
                    return L.elem == 4 ? launch_smooth3d_zg2<float>(d, 1, n, 1, t, s)
                                       : launch_smooth3d_zg2<half_t>(d, 1, n, 1, t, s);
                };
                TileCfg best = pick_fastest(cands, cands[0], run2, s);
                const float t_two = time_launch(run2, best, s);
                const TileCfg zg = tl[(size_t)l].smooth_zg, sw = tl[(size_t)l].smooth;
                const float t_sep = time_launch([&](TileCfg) {
                    if (L.elem == 4) {
                        (void)launch_smooth<float>(dim, sm, false, d, 1, n, 0, SWEEP_ZERO_GUESS, zg, s);
                        return launch_smooth<float>(dim, sm, false, d, 1, n, 1, 0, sw, s);
                    }
                    (void)launch_smooth<half_t>(dim, sm, false, d, 1, n, 0, SWEEP_ZERO_GUESS, zg, s);
                    return launch_smooth<half_t>(dim, sm, false, d, 1, n, 1, 0, sw, s);
                }, sw, s);
                cfg = best;
                if (!(t_two < t_sep)) cfg.zchunk = -best.zchunk;  // declined (depth kept for forcing)
                tune_store(k2, cfg);
            }
            tl[(size_t)l].smooth_zg2 = cfg;
            if (cfg.zchunk < 0) tl[(size_t)l].smooth_zg2.zchunk = std::getenv("MG_FUSED_SMOOTH2") ? -cfg.zchunk : 0;
        }
        // 2D: the first two post-smoothing sweeps in one launch, kept if faster
        if (dim == 2 && !var && sm == SM_RBGS && L.elem <= 4 && c->p.nu2 >= 2) {
            TuneKey kp{dim, L.elem, n, 7, sm, 0, 0, 0};
            if (!tune_lookup(kp, &cfg)) {
                const std::vector<TileCfg> cands = smooth2_candidates(dim, n);
                auto runp = [&](TileCfg t) {
                    return L.elem == 4 ? launch_smooth2d_pro2<float>(d, 1, n, 0, t, s)
                                       : launch_smooth2d_pro2<half_t>(d, 1, n, 0, t, s);
                };
                TileCfg best = pick_fastest(cands, cands[0], runp, s);
                const float t_two = time_launch(runp, best, s);
                const TileCfg pr = tl[(size_t)l].smooth_pro, sw = tl[(size_t)l].smooth;
                const float t_sep = time_launch([&](TileCfg) {
                    if (L.elem == 4) {
                        (void)launch_smooth<float>(dim, sm, false, d, 1, n, 0, SWEEP_PROLONG, pr, s);
                        return launch_smooth<float>(dim, sm, false, d, 1, n, 1, 0, sw, s);
                    }
                    (void)launch_smooth<half_t>(dim, sm, false, d, 1, n, 0, SWEEP_PROLONG, pr, s);
                    return launch_smooth<half_t>(dim, sm, false, d, 1, n, 1, 0, sw, s);
                }, sw, s);
                cfg = best;
                if (!(t_two < t_sep)) cfg.zchunk = -best.zchunk;
                tune_store(kp, cfg);
            }
            tl[(size_t)l].smooth_pro2 = cfg;
            if (cfg.zchunk < 0) tl[(size_t)l].smooth_pro2.zchunk = std::getenv("MG_FUSED_POST2") ? -cfg.zchunk : 0;
        }
    }
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(d);
    return e != hipSuccess ? e : e2;
}

}  // namespace

// Batched launches: the three sweep variants and the restriction of one
// absolute level, launched over all 'count' instances of that level as the
// batched V-cycle launches them.  Runs on the instances' own level arrays
// (clear at setup; sweeps and restrictions write inner nodes only).
namespace mg {
hipError_t tune_group(int dim, int smoother, const GridDesc* d, int count, int n, Tiles& t, hipStream_t s) {
    if (count <= 0 || n <= 3 || npts(dim, n) * (size_t)count < kTuneMinPoints) return hipSuccess;
    int bucket = 0;
    for (int c = count; c; c >>= 1) ++bucket;
    TileCfg cfg;
    const int vflags[3] = {0, SWEEP_ZERO_GUESS, SWEEP_PROLONG};
    TileCfg* vcfg[3] = {&t.smooth, &t.smooth_zg, &t.smooth_pro};
    for (int v = 0; v < 3; ++v) {
        const int fl = vflags[v];
        TuneKey ks{dim, 4, n, 0, smoother, 0, 10 + v, bucket};
        if (!tune_lookup(ks, &cfg)) {
            auto run = [&](TileCfg c) { return launch_smooth<float>(dim, smoother, false, d, count, n, 0, fl, c, s); };
            cfg = pick_fastest(tune_candidates(dim, n - 2, true, 0, 4, false), *vcfg[v], run, s);
            cfg = pick_order(cfg, run, s);
            tune_store(ks, cfg);
        }
        *vcfg[v] = cfg;
    }
    TuneKey kr{dim, 4, n, 1, 0, 0, 0, bucket};
    if (!tune_lookup(kr, &cfg)) {
        std::vector<TileCfg> cands;
        for (TileCfg c : tune_candidates(dim, (n - 1) / 2 - 1, false, 1, 4, false))
            if (c.by >= 8) cands.push_back(c);
        cfg = pick_fastest(cands, t.restr, [&](TileCfg c) {
            return launch_restrict<float>(dim, false, d, count, n, 0, c, s);
        }, s);
        tune_store(kr, cfg);
    }
    t.restr = cfg;
    // the two fused pre-smoothing sweeps from a zero iterate, kept if faster
    if (smoother == SM_RBGS) {
        TuneKey k2{dim, 4, n, 6, smoother, 0, 0, bucket};
        if (!tune_lookup(k2, &cfg)) {
            auto run2 = [&](TileCfg c) {
                return dim == 2 ? launch_smooth2d_zg2<float>(d, count, n, 1, c, s)
                                : launch_smooth3d_zg2<float>(d, count, n, 1, c, s);
            };
            const std::vector<TileCfg> cands = smooth2_candidates(dim, n);
            TileCfg best = pick_fastest(cands, cands[0], run2, s);
            const float t_two = time_launch(run2, best, s);
            const TileCfg zg = t.smooth_zg, sw = t.smooth;
            const float t_sep = time_launch([&](TileCfg) {
                (void)launch_smooth<float>(dim, smoother, false, d, count, n, 0, SWEEP_ZERO_GUESS, zg, s);
                return launch_smooth<float>(dim, smoother, false, d, count, n, 1, 0, sw, s);
            }, sw, s);
            cfg = best;
            if (!(t_two < t_sep)) cfg.zchunk = -best.zchunk;
            tune_store(k2, cfg);
        }
        t.smooth_zg2 = cfg;
        if (cfg.zchunk < 0) t.smooth_zg2.zchunk = std::getenv("MG_FUSED_SMOOTH2") ? -cfg.zchunk : 0;
    }
    if (smoother == SM_RBGS && dim == 2) {
        TuneKey kp{dim, 4, n, 7, smoother, 0, 0, bucket};
        if (!tune_lookup(kp, &cfg)) {
            auto runp = [&](TileCfg c) { return launch_smooth2d_pro2<float>(d, count, n, 0, c, s); };
            const std::vector<TileCfg> cands = smooth2_candidates(dim, n);
            TileCfg best = pick_fastest(cands, cands[0], runp, s);
            const float t_two = time_launch(runp, best, s);
            const TileCfg pr = t.smooth_pro, sw = t.smooth;
            const float t_sep = time_launch([&](TileCfg) {
                (void)launch_smooth<float>(dim, smoother, false, d, count, n, 0, SWEEP_PROLONG, pr, s);
                return launch_smooth<float>(dim, smoother, false, d, count, n, 1, 0, sw, s);
            }, sw, s);
            cfg = best;
            if (!(t_two < t_sep)) cfg.zchunk = -best.zchunk;
            tune_store(kp, cfg);
        }
        t.smooth_pro2 = cfg;
        if (cfg.zchunk < 0) t.smooth_pro2.zchunk = std::getenv("MG_FUSED_POST2") ? -cfg.zchunk : 0;
    }
    return hipStreamSynchronize(s);
}
}  // namespace mg

namespace {

hipError_t autotune(mg_ctx* c) {
    const int dim = c->p.dim, n = c->p.n;
    const size_t N = npts(dim, n);
    hipStream_t s = c->stream;
    void* su = nullptr;
    void* sf = nullptr;
    hipError_t e = hipSuccess;
    if (N >= kTuneMinPoints) {
        e = zalloc(&su, N * sizeof(double), s);
        if (e == hipSuccess) e = zalloc(&sf, N * sizeof(double), s);
    }
    if (e == hipSuccess) {
        if (c->p.precision == MG_PREC_FP64) e = tune_levels(c, c->L64, c->tl64, su, sf);
        else e = tune_levels(c, c->L32, c->tl32, nullptr, nullptr);
    }
    // finest-level FP64 norm (FP64 solves) or refinement pass (mixed precision)
    if (e == hipSuccess && N >= kTuneMinPoints) {
        const bool var = c->prob.var;
        const int mode = c->p.precision == MG_PREC_FP64 ? 0 : (is_h16(c->p) ? 2 : 1);
        TuneKey kn{dim, 8, n, 2, 0, var ? 1 : 0, mode, 0};
        TileCfg cfg;
        if (!tune_lookup(kn, &cfg)) {
            std::vector<TileCfg> cands;
            for (TileCfg t : tune_candidates(dim, n - 2, true, 2, 8, var))
                if (mode != 2 || t.xp == 2) cands.push_back(t);  // the binary16 pass has two nodes per lane
            const double* scl = nullptr;
            int maxparts = 1;
            for (TileCfg t : cands) maxparts = std::max(maxparts, norm_tiles(dim, n, t));
            (void)scl;
            double* part = nullptr;
            e = hipMalloc((void**)&part, sizeof(double) * (size_t)maxparts);
            if (e == hipSuccess) {
                if (mode == 0) {
                    GridDesc h = c->h_top;
                    h.u = su;
                    h.f = sf;
                    GridDesc* d = nullptr;
                    e = hipMalloc((void**)&d, sizeof(GridDesc));
                    if (e == hipSuccess) e = hipMemcpyAsync(d, &h, sizeof(GridDesc), hipMemcpyHostToDevice, s);
                    if (e == hipSuccess)
                        cfg = pick_fastest(cands, c->top.norm, [&](TileCfg t) {
                            return launch_norm(dim, var, d, 1, n, 0, part, maxparts, t, s);
                        }, s);
                    (void)hipStreamSynchronize(s);
                    ffree(d);
                } else {
                    IRDesc h = c->h_ir;
                    h.u[0] = (double*)su;
                    h.f = (const double*)sf;
                    h.done = nullptr;
                    double* tscl = nullptr;
                    double* tmax = nullptr;
                    const double scl0[2] = {1.0, 1.0};
                    if (mode == 2) {  // scale state and partial maxima of the binary16 pass
                        e = hipMalloc((void**)&tscl, 2 * sizeof(double));
                        if (e == hipSuccess) e = hipMemcpy(tscl, scl0, sizeof(scl0), hipMemcpyHostToDevice);
                        if (e == hipSuccess) e = hipMalloc((void**)&tmax, sizeof(double) * (size_t)maxparts);
                        h.scl = tscl;
                        h.pmax = tmax;
                    }
                    IRDesc* d = nullptr;
                    if (e == hipSuccess) e = hipMalloc((void**)&d, sizeof(IRDesc));
                    if (e == hipSuccess) e = hipMemcpyAsync(d, &h, sizeof(IRDesc), hipMemcpyHostToDevice, s);
                    if (e == hipSuccess)
                        cfg = pick_fastest(cands, c->top.norm, [&](TileCfg t) {
                            return mode == 2 ? launch_ir_update_f16(dim, d, 1, n, 0, 0, part, maxparts, t, s)
                                             : launch_ir_update(dim, var, d, 1, n, 0, 0, part, maxparts, t, s);
                        }, s);
                    (void)hipStreamSynchronize(s);
                    ffree(d);
                    ffree(tscl);
                    ffree(tmax);
                }
                ffree(part);
                if (e == hipSuccess) tune_store(kn, cfg);
            }
        }
        if (e == hipSuccess) c->top.norm = cfg;
    }
    (void)hipStreamSynchronize(s);
    ffree(su);
    ffree(sf);
    return e;
}

}  // namespace

extern "C" {

const char* mg_strerror(int code) {
    switch (code) {
        case MG_OK: return "ok";
        case MG_ENOTCONV: return "not converged within max_cycles";
        case MG_EINVAL: return "invalid argument";
        case MG_ENOTSUP: return "unsupported combination";
        case MG_ENOMEM: return "out of device memory or budget";
        case MG_EDEVICE: return "HIP runtime error";
        case MG_EDIVERGED: return "diverged (NaN/Inf or residual growth)";
        case MG_EBUSY: return "no capacity for the request now";
        default: return "unknown status";
    }
}

int mg_setup(const mg_params* p, void* stream, mg_ctx** out) {
    if (!out) return MG_EINVAL;
    *out = nullptr;
    int v = validate(p);
    if (v != MG_OK) return v;
    mg_ctx* c = new (std::nothrow) mg_ctx();
    if (!c) return MG_ENOMEM;
    c->p = *p;
    if (c->p.omega <= 0.0) c->p.omega = p->smoother == MG_SMOOTH_WJACOBI ? 0.8 : 1.0;
    c->stream = (hipStream_t)stream;
    if (p->op == MG_OP_CONST_STENCIL) {
        (void)hipGetDevice(&c->device);
        const int r = st_setup(c);
        if (r != MG_OK) {
            destroy(c);
            return r;
        }
        *out = c;
        return MG_OK;
    }
    if (p->bc == MG_BC_NEUMANN_CC) {
        (void)hipGetDevice(&c->device);
        const int r = cc_setup(c);
        if (r != MG_OK) {
            destroy(c);
            return r;
        }
        *out = c;
        return MG_OK;
    }
    c->use_graphs = std::getenv("MG_NO_GRAPHS") == nullptr;
    (void)hipGetDevice(&c->device);
    const int dim = p->dim;
    c->prob = Problem{dim, p->smoother == MG_SMOOTH_WJACOBI ? SM_JACOBI : SM_RBGS, p->nu1, p->nu2, c->p.omega,
                      p->op == MG_OP_VARCOEF_NODAL};
    c->prob.sym = p->smoother == MG_SMOOTH_RBGS_SYM;
    c->prob.cycle = p->cycle;
    c->prob.cg_iters = p->cg_iters;
    const int coarse_n = p->coarse_n > 3 ? p->coarse_n : 3;
    for (int m = p->n;; m = (m - 1) / 2 + 1) {
        c->n.push_back(m);
        if (m <= coarse_n) break;
    }
    c->nlev = (int)c->n.size();
    for (int l = 0; l < c->nlev; ++l) {
        c->tl64.push_back(default_tiles(dim, 8, c->n[(size_t)l], c->prob.smoother));
        c->tl32.push_back(default_tiles(dim, 4, c->n[(size_t)l], c->prob.smoother));
    }
    c->top = c->tl64[0];
    if (is_h16(c->p)) {  // the binary16 refinement pass has two nodes per lane
        c->top.norm.xp = 2;
        if (dim == 2) c->top.norm.zchunk = 32;
        else c->top.norm.by = std::min(c->top.norm.by, 4 * c->top.norm.wv);
    }
    const char* at = std::getenv("MG_AUTOTUNE");
    c->autotune = !(at && at[0] == '0');
    hipStream_t s = c->stream;
    const size_t N = npts(dim, p->n);
    hipError_t e = hipSuccess;
#define SETUP_CK(x)                \
    do {                           \
        e = (x);                   \
        if (e != hipSuccess) {     \
            destroy(c);            \
            return dev_status(e);  \
        }                          \
    } while (0)
    if (c->prob.var) {
        SETUP_CK(hipMalloc((void**)&c->k64, N * sizeof(double)));
        SETUP_CK(hipMemcpyAsync(c->k64, p->k, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    SETUP_CK(hipMalloc((void**)&c->d_ctrl, 3 * sizeof(int)));
    SETUP_CK(launch_fill_int(c->d_ctrl, 0, 3, s));
    if (p->precision == MG_PREC_FP64) {
        SETUP_CK(build_levels(c->L64, dim, c->n, 8, false, c->k64, s));
        SETUP_CK(build_faces(c->L64, s));
        SETUP_CK(build_groups(c->G64, c->L64, c->prob, ctl_done(c), s));
        SETUP_CK(build_tail(c->tail64, c->G64, tail_first_level(dim, 8, c->n, false), s));
    } else {
        SETUP_CK(build_levels(c->L32, dim, c->n, ir_elem(c->p), true, nullptr, s));
        if (c->prob.var) {
            void* k32 = nullptr;
            SETUP_CK(zalloc(&k32, N * sizeof(float), s));
            SETUP_CK((launch_convert<double, float>(N, c->k64, (float*)k32, s)));
            c->L32.k[0] = k32;
            for (int l = 1; l < c->nlev; ++l) {
                SETUP_CK(zalloc(&c->L32.k[(size_t)l], npts(dim, c->n[(size_t)l]) * sizeof(float), s));
                SETUP_CK((launch_inject<float, float>(dim, c->n[(size_t)l - 1],
                                                      (const float*)c->L32.k[(size_t)l - 1], c->n[(size_t)l],
                                                      (float*)c->L32.k[(size_t)l], s)));
            }
            c->L32.own_k0 = true;
        }
        SETUP_CK(build_faces(c->L32, s));
        SETUP_CK(build_groups(c->G32, c->L32, c->prob, ctl_done(c), s));
        SETUP_CK(build_tail(c->tail32, c->G32, tail_first_level(dim, ir_elem(c->p), c->n, true), s));
        SETUP_CK(zalloc((void**)&c->u64_scratch, N * sizeof(double), s));
        c->h_ir = IRDesc{};
        c->h_ir.u[0] = nullptr;
        c->h_ir.u[1] = c->u64_scratch;
        c->h_ir.e = c->L32.u[0];
        c->h_ir.f = nullptr;
        c->h_ir.k = c->k64;
        c->h_ir.r = c->L32.f[0];
        if (is_h16(c->p)) {
            SETUP_CK(zalloc((void**)&c->d_scl, 2 * sizeof(double), s));
            c->h_ir.scl = c->d_scl;
        }
        c->h_ir.done = ctl_done(c);
        c->h_ir.n = p->n;
        c->h_ir.inst = 0;
        c->h_ir.c = level_c(p->n);
        SETUP_CK(hipMalloc((void**)&c->d_ir, sizeof(IRDesc)));
        SETUP_CK(hipMemcpyAsync(c->d_ir, &c->h_ir, sizeof(IRDesc), hipMemcpyHostToDevice, s));
    }
    // FP64 view of the finest level for residual norms
    c->h_top = GridDesc{};
    c->h_top.k = c->k64;
    c->h_top.n = p->n;
    c->h_top.inst = 0;
    c->h_top.c = level_c(p->n);
    c->h_top.wd = level_wd(dim, p->n, c->p.omega);
    c->h_top.omega = c->p.omega;
    SETUP_CK(hipMalloc((void**)&c->d_top, sizeof(GridDesc)));
    SETUP_CK(hipMemcpyAsync(c->d_top, &c->h_top, sizeof(GridDesc), hipMemcpyHostToDevice, s));
    // FP64: each cycle's residual norm from the next cycle's first pre-smoothing sweep
    c->nrm_fused = p->precision == MG_PREC_FP64 && c->nlev >= 2 && p->nu1 >= 1 && c->tail64.first != 0 &&
                   std::getenv("MG_NO_FUSED_NORM") == nullptr;
    if (c->nrm_fused) {
        const int sm = c->prob.smoother;
        int cap = smooth_tiles(dim, sm, p->n, c->tl64[0].smooth_nrm);
        for (TileCfg t : tune_candidates(dim, p->n - 2, true, 0, 8, c->prob.var))
            if (t.wv != 1) cap = std::max(cap, smooth_tiles(dim, sm, p->n, t));
        c->spart_cap = cap;
        SETUP_CK(hipMalloc((void**)&c->d_spart, sizeof(double) * (size_t)cap));
        GridDesc& d0 = c->G64[0].h[0];
        d0.npart = c->d_spart;
        SETUP_CK(hipMemcpyAsync(c->G64[0].d, &d0, sizeof(GridDesc), hipMemcpyHostToDevice, s));
    }
    if (c->autotune) SETUP_CK(autotune(c));
    if (c->nrm_fused && smooth_tiles(dim, c->prob.smoother, p->n, c->tl64[0].smooth_nrm) > c->spart_cap)
        c->nrm_fused = false;
    c->pstride = std::max(1, norm_tiles(dim, p->n, c->top.norm));
    SETUP_CK(hipMalloc((void**)&c->d_partial, sizeof(double) * (size_t)c->pstride));
    if (is_h16(c->p)) {
        SETUP_CK(hipMalloc((void**)&c->d_pmax, sizeof(double) * (size_t)c->pstride));
        c->h_ir.pmax = c->d_pmax;
        SETUP_CK(hipMemcpyAsync(c->d_ir, &c->h_ir, sizeof(IRDesc), hipMemcpyHostToDevice, s));
    }
    SETUP_CK(hipMalloc((void**)&c->d_norm, sizeof(double)));
    SETUP_CK(hipMalloc((void**)&c->d_norm0, sizeof(double)));
    c->prof_ev.resize(512);
    for (auto& ev : c->prof_ev) SETUP_CK(hipEventCreate(&ev));
    int r = ensure_hist(c, 64);
    if (r != MG_OK) {
        destroy(c);
        return r;
    }
    SETUP_CK(hipStreamSynchronize(s));
#undef SETUP_CK
    *out = c;
    return MG_OK;
}

void mg_destroy(mg_ctx* c) {
    if (c && is_batch_handle(c)) destroy_batch_handle(c);
    else destroy(c);
}

int mg_num_levels(const mg_ctx* c) {
    if (!c || is_batch_handle(c)) return MG_EINVAL;
    return c->cd ? (int)c->cd->ln.size() : c->nlev;
}

int mg_tile_config(const mg_ctx* c, int level, int family, int* by, int* zchunk, int* prefetch, int* waves,
                   int* order, int* pairs) {
    if (!c || is_batch_handle(c) || !by || !zchunk || level < 0 || level >= c->nlev || family < 0 || family > 8)
        return MG_EINVAL;
    if (c->cc || c->st || c->cd) return MG_ENOTSUP;  // plain kernels, no tiles
    const std::vector<Tiles>& tl = c->p.precision == MG_PREC_FP64 ? c->tl64 : c->tl32;
    const Tiles& tv = tl[(size_t)level];
    const TileCfg t = family == 0   ? tv.smooth
                      : family == 1 ? tv.restr
                      : family == 2 ? c->top.norm
                      : family == 3 ? tv.smooth_zg
                      : family == 4 ? tv.smooth_pro
                      : family == 5 ? tv.fused
                      : family == 6 ? tv.smooth_nrm
                      : family == 7 ? tv.smooth_zg2
                                    : tv.smooth_pro2;
    if ((family == 2 || family == 6) && level != 0) return MG_EINVAL;
    if (family == 6 && !c->nrm_fused) {  // the norm is a pass of its own
        *by = *zchunk = 0;
        if (prefetch) *prefetch = 0;
        if (waves) *waves = 0;
        if (order) *order = 0;
        if (pairs) *pairs = 0;
        return MG_OK;
    }
    *by = t.by;
    *zchunk = t.zchunk;
    if (prefetch) *prefetch = t.pd;
    if (waves) *waves = t.wv;
    if (order) *order = t.order;
    if (pairs) *pairs = t.xp == 2 ? 1 : 0;
    return MG_OK;
}

int mg_vcycle(mg_ctx* c, double* u, const double* f) {
    if (!c) return MG_EINVAL;
    if (is_batch_handle(c)) return MG_EINVAL;
    if (c->cd) return MG_EINVAL;  // complex-diffusion handles take the mg_cdiff_* calls
    if (c->cc) {
        if (!u || !f) return MG_EINVAL;
        CK(cc_cycle_top(c, u, f));
        return MG_OK;
    }
    if (c->st) {
        if (!u || !f) return MG_EINVAL;
        CK(st_cycle_top(c, u, f));
        return MG_OK;
    }
    int r = bind(c, u, f);
    if (r != MG_OK) return r;
    CK(launch_fill_int(ctl_done(c), 0, 1, c->stream));
    if (c->p.precision == MG_PREC_FP64) {
        CK(vcycle<double>(c->prob, c->G64, false, c->tl64, c->stream, nullptr, nullptr, 0, &c->tail64));
    } else {
        CK(enqueue_ir_start(c, c->stream));
        if (is_h16(c->p)) CK(vcycle<half_t>(c->prob, c->G32, true, c->tl32, c->stream, nullptr, nullptr, 0, &c->tail32));
        else CK(vcycle<float>(c->prob, c->G32, true, c->tl32, c->stream, nullptr, nullptr, 0, &c->tail32));
        CK(enqueue_ir(c, 0, 0, c->stream));
        CK(hipMemcpyAsync(u, c->u64_scratch, npts(c->p.dim, c->p.n) * sizeof(double), hipMemcpyDeviceToDevice,
                          c->stream));
    }
    return MG_OK;
}

int mg_residual_norm(mg_ctx* c, const double* u, const double* f, double* out) {
    if (!c || !out) return MG_EINVAL;
    if (is_batch_handle(c)) return MG_EINVAL;
    if (c->cd) return MG_EINVAL;  // complex-diffusion handles take the mg_cdiff_* calls
    if (c->cc) {
        if (!u || !f) return MG_EINVAL;
        CK(cc_norm(c->p.dim, u, f, cc_const(c->p.dim, c->p.n, c->p.omega), c->d_partial, c->d_norm, c->stream));
        CK(hipMemcpyAsync(c->h_pin, c->d_norm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CK(hipStreamSynchronize(c->stream));
        *out = c->h_pin[0];
        return MG_OK;
    }
    if (c->st) {
        if (!u || !f) return MG_EINVAL;
        CK(st_norm(c->p.dim, u, f, st_const(c->p.dim, c->p.n, c->st_coef, c->p.omega), c->d_partial, c->d_norm,
                   c->stream));
        CK(hipMemcpyAsync(c->h_pin, c->d_norm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CK(hipStreamSynchronize(c->stream));
        *out = c->h_pin[0];
        return MG_OK;
    }
    int r = bind(c, u, f);
    if (r != MG_OK) return r;
    CK(enqueue_norm(c, c->stream));
    CK(hipMemcpyAsync(c->h_pin, c->d_norm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CK(hipStreamSynchronize(c->stream));
    *out = c->h_pin[0];
    return MG_OK;
}

int mg_solve(mg_ctx* c, double* u, const double* f, double tol, int max_cycles, int* cycles_done, double* res_hist) {
    if (!c || max_cycles < 0 || !(tol >= 0.0)) return MG_EINVAL;
    if (is_batch_handle(c)) return MG_EINVAL;
    if (c->cd) return MG_EINVAL;  // complex-diffusion handles take the mg_cdiff_* calls
    if (c->cc) {
        if (!u || !f) return MG_EINVAL;
        return cc_solve(c, u, f, tol, max_cycles, cycles_done, res_hist);
    }
    if (c->st) {
        if (!u || !f) return MG_EINVAL;
        return st_solve(c, u, f, tol, max_cycles, cycles_done, res_hist);
    }
    int r = bind(c, u, f);
    if (r != MG_OK) return r;
    r = ensure_hist(c, max_cycles + 1);
    if (r != MG_OK) return r;
    hipStream_t s = c->stream;
    const bool ir = is_ir(c->p);
    c->prof_n = 0;  // measured launches are tagged per solve
    c->prof_step.clear();
    c->prof_kind.clear();
    // rho_0 (clear the stop flag a previous solve left set first: every kernel honours it)
    CK(launch_fill_int(ctl_done(c), 0, 1, s));
    if (ir) CK(enqueue_ir_start(c, s));
    else if (c->nrm_fused) CK(enqueue_nrm_sweep(c, s));
    else CK(enqueue_norm(c, s));
    CK(launch_solve_init(c->d_norm, c->d_norm0, ctl_done(c), ctl_steps(c), ctl_status(c), c->d_hist, c->hist_cap, 1,
                         s));
    // steps in chunks: the first of kmax steps, later ones sized by
    // next_chunk; kernels of a finished solve exit at once
    const size_t N = npts(c->p.dim, c->p.n);
    const int kmax = N > (size_t)(1 << 20) ? 4 : 10;
    int K = kmax;
    int steps = 0, status = 1, done = 0;
    CK(hipMemcpyAsync(c->h_pin, c->d_ctrl, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    done = ((int*)c->h_pin)[0];
    status = ((int*)c->h_pin)[2];
    int enqueued = 0;
    while (!done && enqueued < max_cycles) {
        const int k = std::min(K, max_cycles - enqueued);
        r = run_chunk(c, k, tol, max_cycles, enqueued);
        if (r != MG_OK) return r;
        enqueued += k;
        CK(hipMemcpyAsync(c->h_pin, c->d_ctrl, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(c->h_pin + 2, c->d_hist, sizeof(double) * (size_t)(enqueued + 1), hipMemcpyDeviceToHost,
                          s));
        CK(hipStreamSynchronize(s));
        done = ((int*)c->h_pin)[0];
        steps = ((int*)c->h_pin)[1];
        status = ((int*)c->h_pin)[2];
        K = next_chunk(c->h_pin + 2, steps, tol, kmax);
    }
    CK(hipMemcpyAsync(c->h_pin, c->d_ctrl, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    steps = ((int*)c->h_pin)[1];
    status = ((int*)c->h_pin)[2];
    if (res_hist) {
        CK(hipMemcpyAsync(c->h_pin, c->d_hist, sizeof(double) * (size_t)(steps + 1), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        std::memcpy(res_hist, c->h_pin, sizeof(double) * (size_t)(steps + 1));
    }
    if (ir && (steps & 1)) {  // the last refinement step wrote the scratch iterate
        CK(hipMemcpyAsync(u, c->u64_scratch, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        CK(hipStreamSynchronize(s));
    }
    if (c->prof_on) {
        // launches of steps past the last one the solve ran found the stop
        // flag set and did no work: they are not counted
        for (size_t j = 0; j < c->prof_step.size() && 2 * j + 1 < (size_t)c->prof_n; ++j) {
            if (c->prof_step[j] > steps) continue;
            float t = 0.f;
            CK(hipEventElapsedTime(&t, c->prof_ev[2 * j], c->prof_ev[2 * j + 1]));
            const int k = c->prof_kind[j] & 1;
            c->prof_launches[k] += 1;
            c->prof_ms[k] += (double)t;
        }
        c->prof_n = 0;
        c->prof_step.clear();
        c->prof_kind.clear();
    }
    if (cycles_done) *cycles_done = steps;
    if (status == 0) return MG_OK;
    if (status == -5) return MG_EDIVERGED;
    return MG_ENOTCONV;
}

int mg_prof_enable(mg_ctx* c, int on) {
    if (!c) return MG_EINVAL;
    if (is_batch_handle(c)) return MG_EINVAL;
    c->prof_on = on != 0;
    c->prof_n = 0;
    c->prof_step.clear();
    c->prof_kind.clear();
    c->prof_launches[0] = c->prof_launches[1] = 0;
    c->prof_ms[0] = c->prof_ms[1] = 0.0;
    return MG_OK;
}

int mg_prof_read_kernel(mg_ctx* c, int kernel, int* launches, double* total_ms) {
    if (!c || (kernel != 0 && kernel != 1)) return MG_EINVAL;
    if (is_batch_handle(c)) return MG_EINVAL;
    if (launches) *launches = c->prof_launches[kernel];
    if (total_ms) *total_ms = c->prof_ms[kernel];
    c->prof_launches[kernel] = 0;
    c->prof_ms[kernel] = 0.0;
    return MG_OK;
}

int mg_prof_read(mg_ctx* c, int* launches, double* total_ms) { return mg_prof_read_kernel(c, 0, launches, total_ms); }

int mg_copy_kernel(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || bytes % 16 != 0) return MG_EINVAL;
    CK(launch_copy_bytes(dst, src, bytes, (hipStream_t)stream));
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Single-level operations
// ---------------------------------------------------------------------------

static TileCfg pick_cfg(int dim, int elem, int n, int smoother, int by, int zchunk, int kind) {
    Tiles t = default_tiles(dim, elem, n, smoother);
    TileCfg c = kind == 0 ? t.smooth : (kind == 1 ? t.restr : t.norm);
    if (by) c.by = by;
    if (zchunk) c.zchunk = zchunk;
    return c;
}

static bool valid_cfg(TileCfg c, int dim, int elem, bool var, int family) {
    if (c.xp != 1 && !(c.xp == 2 && family == 2 && !var && (dim == 2 ? c.wv == 4 : c.by <= 4 * c.wv)))
        return false;
    if (c.wv == 1) {  // 3D sweep, one wavefront per tile
        if (dim != 3 || family != 0 || (c.by != 8 && c.by != 12)) return false;
    } else {
        if (c.by != 8 && c.by != 16 && c.by != 32) return false;
        if (c.wv != 4 && !(c.wv == 8 && dim == 3 && (family == 0 || family == 2) && c.by >= 16)) return false;
    }
    return c.by <= max_tile_rows(dim, elem, var, family, c.wv) && c.zchunk >= 1 && (c.pd == 1 || c.pd == 2);
}

// Temporary device descriptor for a context-free call; the stream is synchronised before release.
static int with_desc(const GridDesc& h, hipStream_t s, GridDesc** d) {
    CK(hipMalloc((void**)d, sizeof(GridDesc)));
    CK(hipMemcpyAsync(*d, &h, sizeof(GridDesc), hipMemcpyHostToDevice, s));
    return MG_OK;
}

static int finish_desc(void* d, hipStream_t s, hipError_t launch) {
    hipError_t e = hipStreamSynchronize(s);
    (void)hipFree(d);
    if (launch != hipSuccess) return dev_status(launch);
    return dev_status(e);
}

// word size of a level-operation dtype (0 FP64, 1 FP32, 2 binary16), 0 if invalid
static int dtype_elem(int dtype) { return dtype == 0 ? 8 : (dtype == 1 ? 4 : (dtype == 2 ? 2 : 0)); }

int mg_level_smooth(int dim, int n, int dtype, int smoother, double omega, const void* k, const void* u_in,
                    const void* f, void* u_out, const void* ec, int zero_guess, int by, int zchunk, int prefetch,
                    int waves, int order, void* stream) {
    const int elem = dtype_elem(dtype);
    if (!valid_edge(dim, n) || n < 5 || !elem) return MG_EINVAL;
    if ((smoother != 0 && smoother != 1 && smoother != 2) || !f || !u_out || (!u_in && !zero_guess)) return MG_EINVAL;
    if (ec && zero_guess) return MG_EINVAL;
    if (elem == 2 && k) return MG_ENOTSUP;
    const int sel = smoother == 2 ? SEL_BLACK_FIRST : 0;
    if (smoother == 2) smoother = SM_RBGS;
    TileCfg cfg = pick_cfg(dim, elem, n, smoother, by, zchunk, 0);
    if (prefetch) cfg.pd = prefetch;
    if (waves) cfg.wv = waves;
    if (order != 0 && order != 1) return MG_EINVAL;
    cfg.order = order;
    if (!valid_cfg(cfg, dim, elem, k != nullptr, 0)) return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    GridDesc h{};
    h.u = const_cast<void*>(u_in);
    h.t = u_out;
    h.f = f;
    h.k = k;
    h.uc = const_cast<void*>(ec);
    h.n = n;
    h.c = level_c(n);
    h.wd = level_wd(dim, n, omega);
    h.omega = omega;
    void* fxt = nullptr;  // face coefficients of a 3D variable-coefficient grid (freed after the sweep)
    if (k && dim == 3) {
        CK(hipMalloc(&fxt, 3 * npts(3, n) * (size_t)elem));
        const hipError_t ef = elem == 8 ? launch_faces3d<double>((const double*)k, (double*)fxt, n, s)
                                        : launch_faces3d<float>((const float*)k, (float*)fxt, n, s);
        if (ef != hipSuccess) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(fxt);
            return dev_status(ef);
        }
        h.fx = fxt;
    }
    GridDesc* d = nullptr;
    int r = with_desc(h, s, &d);
    if (r != MG_OK) {
        (void)hipStreamSynchronize(s);
        if (fxt) (void)hipFree(fxt);
        return r;
    }
    const int flags = (zero_guess ? SWEEP_ZERO_GUESS : 0) | (ec ? SWEEP_PROLONG : 0);
    hipError_t e = elem == 8   ? launch_smooth<double>(dim, smoother, k != nullptr, d, 1, n, sel, flags, cfg, s)
                   : elem == 4 ? launch_smooth<float>(dim, smoother, k != nullptr, d, 1, n, sel, flags, cfg, s)
                               : launch_smooth<half_t>(dim, smoother, false, d, 1, n, sel, flags, cfg, s);
    r = finish_desc(d, s, e);  // synchronises the stream
    if (fxt) (void)hipFree(fxt);
    return r;
}

int mg_level_smooth_restrict(int dim, int n, int dtype, const void* u_in, const void* f, void* u_out, void* fc,
                             int zchunk, int order, void* stream) {
    const int elem = dtype_elem(dtype);
    if (dim != 3 || !valid_edge(dim, n) || n < 5 || (elem != 4 && elem != 2)) return MG_EINVAL;
    if (!u_in || !f || !u_out || !fc || u_in == u_out || zchunk < 1 || (order != 0 && order != 1)) return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    GridDesc h{};
    h.u = const_cast<void*>(u_in);
    h.t = u_out;
    h.f = f;
    h.fc = fc;
    h.n = n;
    h.c = level_c(n);
    h.wd = level_wd(dim, n, 1.0);
    h.omega = 1.0;
    GridDesc* d = nullptr;
    int r = with_desc(h, s, &d);
    if (r != MG_OK) return r;
    TileCfg cfg{16, zchunk};
    cfg.order = order;
    const hipError_t e = elem == 4 ? launch_smooth_restrict3d<float>(d, 1, n, 0, cfg, s)
                                   : launch_smooth_restrict3d<half_t>(d, 1, n, 0, cfg, s);
    return finish_desc(d, s, e);
}

int mg_level_smooth2_zero(int dim, int n, int dtype, const void* f, void* u_out, int by, int zchunk, int order,
                          void* stream) {
    const int elem = dtype_elem(dtype);
    if (!valid_edge(dim, n) || n < 5 || (elem != 4 && elem != 2)) return MG_EINVAL;
    if (!f || !u_out || f == u_out || (dim == 3 && by != 12 && by != 16) || zchunk < 1 || (order != 0 && order != 1))
        return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    GridDesc h{};
    h.u = u_out;  // the second sweep's output (select 1)
    h.f = f;
    h.n = n;
    h.c = level_c(n);
    h.wd = level_wd(dim, n, 1.0);
    h.omega = 1.0;
    GridDesc* d = nullptr;
    int r = with_desc(h, s, &d);
    if (r != MG_OK) return r;
    TileCfg cfg{by, zchunk};
    cfg.order = order;
    hipError_t e;
    if (dim == 2) e = elem == 4 ? launch_smooth2d_zg2<float>(d, 1, n, 1, cfg, s) : launch_smooth2d_zg2<half_t>(d, 1, n, 1, cfg, s);
    else e = elem == 4 ? launch_smooth3d_zg2<float>(d, 1, n, 1, cfg, s) : launch_smooth3d_zg2<half_t>(d, 1, n, 1, cfg, s);
    return finish_desc(d, s, e);
}

int mg_level_smooth2_correct(int dim, int n, int dtype, int smoother, const void* u_in, const void* f,
                             const void* ec, void* u_out, int zchunk, int order, void* stream) {
    const int elem = dtype_elem(dtype);
    if (dim != 2 || !valid_edge(dim, n) || n < 5 || (elem != 4 && elem != 2)) return MG_EINVAL;
    if (!u_in || !f || !ec || !u_out || u_in == u_out || (smoother != 0 && smoother != 2) || zchunk < 1 ||
        (order != 0 && order != 1))
        return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    GridDesc h{};
    h.u = const_cast<void*>(u_in);
    h.t = u_out;
    h.f = f;
    h.uc = const_cast<void*>(ec);
    h.n = n;
    h.c = level_c(n);
    h.wd = level_wd(dim, n, 1.0);
    h.omega = 1.0;
    GridDesc* d = nullptr;
    int r = with_desc(h, s, &d);
    if (r != MG_OK) return r;
    TileCfg cfg{12, zchunk};
    cfg.order = order;
    const int sel = smoother == 2 ? SEL_BLACK_FIRST : 0;
    const hipError_t e = elem == 4 ? launch_smooth2d_pro2<float>(d, 1, n, sel, cfg, s)
                                   : launch_smooth2d_pro2<half_t>(d, 1, n, sel, cfg, s);
    return finish_desc(d, s, e);
}

int mg_level_residual_restrict(int dim, int n, int dtype, const void* k, const void* u, const void* f, void* fc,
                               int by, int zchunk, void* stream) {
    const int elem = dtype_elem(dtype);
    if (!valid_edge(dim, n) || n < 5 || !elem) return MG_EINVAL;
    if (!u || !f || !fc) return MG_EINVAL;
    if (elem == 2 && k) return MG_ENOTSUP;
    const TileCfg cfg = pick_cfg(dim, elem, n, 0, by, zchunk, 1);
    if (!valid_cfg(cfg, dim, elem, k != nullptr, 1)) return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    GridDesc h{};
    h.u = const_cast<void*>(u);
    h.f = f;
    h.k = k;
    h.fc = fc;
    h.n = n;
    h.c = level_c(n);
    GridDesc* d = nullptr;
    int r = with_desc(h, s, &d);
    if (r != MG_OK) return r;
    hipError_t e = elem == 8   ? launch_restrict<double>(dim, k != nullptr, d, 1, n, 0, cfg, s)
                   : elem == 4 ? launch_restrict<float>(dim, k != nullptr, d, 1, n, 0, cfg, s)
                               : launch_restrict<half_t>(dim, false, d, 1, n, 0, cfg, s);
    return finish_desc(d, s, e);
}

int mg_level_prolong_correct(int dim, int n, int dtype, void* u, const void* ec, void* stream) {
    const int elem = dtype_elem(dtype);
    if (!valid_edge(dim, n) || n < 5 || !elem) return MG_EINVAL;
    if (!u || !ec) return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    GridDesc h{};
    h.u = u;
    h.uc = const_cast<void*>(ec);
    h.n = n;
    GridDesc* d = nullptr;
    int r = with_desc(h, s, &d);
    if (r != MG_OK) return r;
    hipError_t e = elem == 8   ? launch_prolong<double>(dim, d, 1, n, 0, s)
                   : elem == 4 ? launch_prolong<float>(dim, d, 1, n, 0, s)
                               : launch_prolong<half_t>(dim, d, 1, n, 0, s);
    return finish_desc(d, s, e);
}

int mg_level_coarsest(int dim, int dtype, const void* k, void* u, const void* f, void* stream) {
    const int elem = dtype_elem(dtype);
    if ((dim != 2 && dim != 3) || !elem || !u || !f) return MG_EINVAL;
    if (elem == 2 && k) return MG_ENOTSUP;
    hipStream_t s = (hipStream_t)stream;
    GridDesc h{};
    h.u = u;
    h.f = f;
    h.k = k;
    h.n = 3;
    h.c = level_c(3);
    GridDesc* d = nullptr;
    int r = with_desc(h, s, &d);
    if (r != MG_OK) return r;
    hipError_t e = elem == 8   ? launch_coarsest<double>(dim, k != nullptr, d, 1, s)
                   : elem == 4 ? launch_coarsest<float>(dim, k != nullptr, d, 1, s)
                               : launch_coarsest<half_t>(dim, false, d, 1, s);
    return finish_desc(d, s, e);
}

int mg_level_coarsest_cg(int dim, int n, int dtype, const void* k, void* u, const void* f, int iters,
                         void* stream) {
    const int elem = dtype_elem(dtype);
    if (!valid_edge(dim, n) || !elem || !u || !f || iters < 0) return MG_EINVAL;
    if (elem == 2 && k) return MG_ENOTSUP;
    if (n > tail_max_edge(dim, elem)) return MG_ENOTSUP;
    hipStream_t s = (hipStream_t)stream;
    GridDesc h{};
    h.u = u;
    h.f = f;
    h.k = k;
    h.n = n;
    h.c = level_c(n);
    GridDesc* d = nullptr;
    int r = with_desc(h, s, &d);
    if (r != MG_OK) return r;
    const int it = iters > 0 ? iters : 4 * (n - 1);
    hipError_t e = elem == 8   ? launch_cg<double>(dim, k != nullptr, d, 1, n, it, s)
                   : elem == 4 ? launch_cg<float>(dim, k != nullptr, d, 1, n, it, s)
                               : launch_cg<half_t>(dim, false, d, 1, n, it, s);
    return finish_desc(d, s, e);
}

int mg_level_ir_update(int dim, int n, const double* k, const double* u_in, const float* e, const double* f,
                       double* u_out, float* r, double* norm_out, int by, int zchunk, int prefetch, int waves,
                       int pairs, void* stream) {
    if (!valid_edge(dim, n) || n < 5) return MG_EINVAL;
    if (!u_in || !e || !f || !u_out || !r || !norm_out || u_in == u_out) return MG_EINVAL;
    TileCfg cfg = pick_cfg(dim, 8, n, 0, by, zchunk, 2);
    if (prefetch) cfg.pd = prefetch;
    if (waves) cfg.wv = waves;
    cfg.xp = pairs ? 2 : 1;
    if (cfg.xp == 2 && dim == 2 && !zchunk) cfg.zchunk = 32;  // rows each wavefront marches
    if (!valid_cfg(cfg, dim, 8, k != nullptr, 2)) return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    IRDesc h{};
    h.u[0] = const_cast<double*>(u_in);
    h.u[1] = u_out;
    h.e = e;
    h.f = f;
    h.k = k;
    h.r = r;
    h.n = n;
    h.c = level_c(n);
    const int nparts = norm_tiles(dim, n, cfg);
    IRDesc* d = nullptr;
    double* part = nullptr;
    double* nrm = nullptr;
    CK(hipMalloc((void**)&d, sizeof(IRDesc)));
    hipError_t err = hipMalloc((void**)&part, sizeof(double) * (size_t)nparts);
    if (err == hipSuccess) err = hipMalloc((void**)&nrm, sizeof(double));
    if (err == hipSuccess) err = hipMemcpyAsync(d, &h, sizeof(IRDesc), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = launch_ir_update(dim, k != nullptr, d, 1, n, 0, 0, part, nparts, cfg, s);
    if (err == hipSuccess) err = launch_norm_finalize(part, nparts, nparts, 0, 1, nrm, s);
    if (err == hipSuccess) err = hipMemcpyAsync(norm_out, nrm, sizeof(double), hipMemcpyDeviceToHost, s);
    hipError_t e2 = hipStreamSynchronize(s);
    ffree(d);
    ffree(part);
    ffree(nrm);
    if (err != hipSuccess) return dev_status(err);
    return dev_status(e2);
}

int mg_level_ir_update_f16(int dim, int n, const double* u_in, const void* e16, double e_scale, double prev_max,
                           const double* f, double* u_out, void* r16, double* norm_out, double* max_out, int by,
                           int zchunk, int prefetch, int waves, void* stream) {
    if (!valid_edge(dim, n) || n < 5) return MG_EINVAL;
    if (!u_in || !f || !r16 || !norm_out || !max_out || (e16 && (!u_out || u_in == u_out))) return MG_EINVAL;
    if (e16 && !(e_scale > 0.0)) return MG_EINVAL;
    TileCfg cfg = pick_cfg(dim, 8, n, 0, by, zchunk, 2);
    if (prefetch) cfg.pd = prefetch;
    if (waves) cfg.wv = waves;
    cfg.xp = 2;
    if (dim == 2 && !zchunk) cfg.zchunk = 32;
    if (dim == 3 && !by) cfg.by = std::min(cfg.by, 4 * cfg.wv);
    if (!valid_cfg(cfg, dim, 8, false, 2)) return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int nparts = norm_tiles(dim, n, cfg);
    IRDesc h{};
    h.u[0] = const_cast<double*>(u_in);
    h.u[1] = e16 ? u_out : const_cast<double*>(u_in);
    h.e = e16;
    h.f = f;
    h.r = r16;
    h.n = n;
    h.c = level_c(n);
    const double hs[2] = {e16 ? e_scale : 1.0, prev_max};
    IRDesc* d = nullptr;
    double* buf = nullptr;  // part[nparts], pmax[nparts], scl[2], norm
    CK(hipMalloc((void**)&d, sizeof(IRDesc)));
    hipError_t err = hipMalloc((void**)&buf, sizeof(double) * (size_t)(2 * nparts + 3));
    double* part = buf;
    double* pmax = buf ? buf + nparts : nullptr;
    double* scl = buf ? buf + 2 * nparts : nullptr;
    double* nrm = buf ? buf + 2 * nparts + 2 : nullptr;
    h.scl = scl;
    h.pmax = pmax;
    double host[2] = {0.0, 0.0};
    if (err == hipSuccess) err = hipMemcpyAsync(scl, hs, sizeof(hs), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipMemcpyAsync(d, &h, sizeof(IRDesc), hipMemcpyHostToDevice, s);
    if (err == hipSuccess)
        err = launch_ir_update_f16(dim, d, 1, n, 0, e16 ? 0 : IR_NO_UPDATE, part, nparts, cfg, s);
    if (err == hipSuccess) err = launch_norm_finalize_f16(part, pmax, nparts, nrm, scl, nullptr, s);
    if (err == hipSuccess) err = hipMemcpyAsync(&host[0], nrm, sizeof(double), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipMemcpyAsync(&host[1], scl + 1, sizeof(double), hipMemcpyDeviceToHost, s);
    hipError_t e2 = hipStreamSynchronize(s);
    ffree(d);
    ffree(buf);
    if (err != hipSuccess) return dev_status(err);
    if (e2 != hipSuccess) return dev_status(e2);
    *norm_out = host[0];
    *max_out = host[1];
    return MG_OK;
}

int mg_cdiff_setup(const mg_cdiff_params* p, void* stream, mg_ctx** out) {
    if (!out) return MG_EINVAL;
    *out = nullptr;
    if (!p || (p->dim != 2 && p->dim != 3) || p->n < 2 || (p->n & (p->n - 1)) ||
        p->n > (p->dim == 2 ? 4096 : 256))
        return MG_EINVAL;
    if (!(p->tau > 0.0) || !(p->theta > 0.0) || !(p->theta < 1.5707963267948966) || !(p->k > 0.0)) return MG_EINVAL;
    if (p->smoother != MG_SMOOTH_RBGS && p->smoother != MG_SMOOTH_WJACOBI) return MG_EINVAL;
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu1 > 16 || p->nu2 > 16 || !(p->omega <= 2.0)) return MG_EINVAL;
    mg_ctx* c = new (std::nothrow) mg_ctx();
    if (!c) return MG_ENOMEM;
    c->stream = (hipStream_t)stream;
    (void)hipGetDevice(&c->device);
    c->p = mg_params{};
    c->p.dim = p->dim;
    c->p.n = p->n;
    c->cd = new (std::nothrow) CDState();
    if (!c->cd) {
        delete c;
        return MG_ENOMEM;
    }
    CDState& S = *c->cd;
    S.dim = p->dim;
    S.n = p->n;
    S.tau = p->tau;
    S.jacobi = p->smoother == MG_SMOOTH_WJACOBI;
    S.nu1 = p->nu1;
    S.nu2 = p->nu2;
    S.K.itau = 1.0 / p->tau;
    S.K.ktheta = p->k * p->theta;
    S.K.ct = std::cos(p->theta);
    S.K.st = std::sin(p->theta);
    S.K.omega = p->omega > 0.0 ? p->omega : (S.jacobi ? 0.8 : 1.0);
    for (int m = p->n; m >= 1; m /= 2) S.ln.push_back(m);
    const size_t L = S.ln.size();
    S.u.assign(L, nullptr);
    S.t.assign(L, nullptr);
    S.f.assign(L, nullptr);
    S.g.assign(L, nullptr);
    S.uh.assign(L, nullptr);
    hipStream_t s = c->stream;
    hipError_t e = hipSuccess;
    for (size_t l = 0; l < L && e == hipSuccess; ++l) {
        const size_t bytes = cd_cells(S, (int)l) * 16;
        if (l > 0) e = zalloc(&S.u[l], bytes, s);
        if (e == hipSuccess) e = zalloc(&S.t[l], bytes, s);
        if (e == hipSuccess) e = zalloc(&S.f[l], bytes, s);
        if (e == hipSuccess) e = zalloc(&S.g[l], bytes, s);
        if (e == hipSuccess && l > 0) e = zalloc(&S.uh[l], bytes, s);
    }
    const int np = cd_norm_parts(S.dim, S.n);
    if (e == hipSuccess) e = hipMalloc((void**)&S.part, sizeof(double) * (size_t)np);
    if (e == hipSuccess) e = hipMalloc((void**)&S.norm, sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&S.h_norm, sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        destroy(c);
        return dev_status(e);
    }
    *out = c;
    return MG_OK;
}

inline bool al16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int mg_cdiff_fas(mg_ctx* c, double* u, const double* f) {
    if (!c || is_batch_handle(c) || !c->cd || !u || !f || !al16(u) || !al16(f)) return MG_EINVAL;
    CK(cd_fas_top(*c->cd, u, f, c->stream));
    return MG_OK;
}

int mg_cdiff_apply(mg_ctx* c, const double* u, double* out) {
    if (!c || is_batch_handle(c) || !c->cd || !u || !out || !al16(u) || !al16(out)) return MG_EINVAL;
    CDState& S = *c->cd;
    CK(cd_compute_g(u, S.g[0], cd_cells(S, 0), S.K, c->stream));
    CK(cd_apply_op(S.dim, u, S.g[0], out, S.K, cd_level(S.n), c->stream));
    return MG_OK;
}

int mg_cdiff_run(mg_ctx* c, double* u, int steps, double tol, int max_cycles, int* cycles, double* res_hist) {
    if (!c || is_batch_handle(c) || !c->cd || !u || !al16(u) || steps < 0 || max_cycles < 0 || !(tol >= 0.0)) return MG_EINVAL;
    CDState& S = *c->cd;
    hipStream_t s = c->stream;
    const size_t N = cd_cells(S, 0);
    void* f0 = S.f[0];
    int status = MG_OK;
    for (int m = 0; m < steps; ++m) {
        CK(cd_scale(u, f0, N, S.K.itau, s));  // right-hand side u^m / tau
        double rho0 = 0.0;
        int r = cd_norm_host(S, u, f0, s, &rho0);
        if (r != MG_OK) return r;
        double* hm = res_hist ? res_hist + (size_t)m * (size_t)(max_cycles + 1) : nullptr;
        if (hm) hm[0] = rho0;
        int it = 0;
        bool done = rho0 == 0.0;
        while (!done && it < max_cycles) {
            CK(cd_fas_top(S, u, f0, s));
            ++it;
            double rho = 0.0;
            r = cd_norm_host(S, u, f0, s, &rho);
            if (r != MG_OK) return r;
            if (hm) hm[it] = rho;
            done = rho <= tol * rho0;
        }
        if (!done) status = MG_ENOTCONV;
        if (cycles) cycles[m] = it;
    }
    return status;
}

int mg_level_st_smooth(int dim, int n, const double* stencil, int smoother, double omega, const double* u_in,
                       const double* f, double* u_out, void* stream) {
    if ((dim != 2 && dim != 3) || !valid_edge(dim, n) || !stencil || !u_in || !f || !u_out) return MG_EINVAL;
    if (smoother != MG_SMOOTH_RBGS && smoother != MG_SMOOTH_WJACOBI && smoother != MG_SMOOTH_RBGS_SYM)
        return MG_EINVAL;
    if (!(stencil[0] > 0.0)) return MG_EINVAL;
    if (omega <= 0.0) omega = smoother == MG_SMOOTH_WJACOBI ? 0.8 : 1.0;
    hipStream_t s = (hipStream_t)stream;
    const STConst L = st_const(dim, n, stencil, omega);
    if (u_out != u_in)
        CK(hipMemcpyAsync(u_out, u_in, npts(dim, n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (smoother == MG_SMOOTH_WJACOBI) {
        if (u_out == u_in) return MG_EINVAL;
        CK(st_relax(dim, true, u_in, u_out, f, L, 0, s));
        return MG_OK;
    }
    const int first = smoother == MG_SMOOTH_RBGS_SYM ? 1 : 0;
    CK(st_relax(dim, false, u_out, u_out, f, L, first, s));
    CK(st_relax(dim, false, u_out, u_out, f, L, 1 - first, s));
    return MG_OK;
}

int mg_level_st_residual_restrict(int dim, int n, const double* stencil, const double* u, const double* f,
                                  double* fc, void* stream) {
    if ((dim != 2 && dim != 3) || !valid_edge(dim, n) || n < 5 || !stencil || !u || !f || !fc) return MG_EINVAL;
    CK(st_restrict(dim, u, f, fc, st_const(dim, n, stencil, 1.0), (hipStream_t)stream));
    return MG_OK;
}

int mg_level_st_coarsest(int dim, const double* stencil, double* u, const double* f, void* stream) {
    if ((dim != 2 && dim != 3) || !stencil || !u || !f || !(stencil[0] > 0.0)) return MG_EINVAL;
    CK(st_coarsest(dim, u, f, st_const(dim, 3, stencil, 1.0), (hipStream_t)stream));
    return MG_OK;
}

int mg_level_cc_smooth(int dim, int n, int smoother, double omega, const double* u_in, const double* f,
                       double* u_out, void* stream) {
    if ((dim != 2 && dim != 3) || !valid_cc(dim, n) || !u_in || !f || !u_out || (smoother != 0 && smoother != 1))
        return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (omega <= 0.0) omega = smoother == 1 ? 0.8 : 1.0;
    const CCConst L = cc_const(dim, n, omega);
    if (smoother == 1) {
        if (u_in == u_out) return MG_EINVAL;
        CK(cc_relax(dim, true, u_in, u_out, f, L, 0, s));
        return MG_OK;
    }
    if (u_in != u_out)
        CK(hipMemcpyAsync(u_out, u_in, cc_cells(dim, n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    CK(cc_relax(dim, false, u_out, u_out, f, L, 0, s));
    CK(cc_relax(dim, false, u_out, u_out, f, L, 1, s));
    return MG_OK;
}

int mg_level_cc_residual_restrict(int dim, int n, const double* u, const double* f, double* fc, void* stream) {
    if ((dim != 2 && dim != 3) || !valid_cc(dim, n) || !u || !f || !fc) return MG_EINVAL;
    CK(cc_restrict(dim, u, f, fc, cc_const(dim, n, 1.0), (hipStream_t)stream));
    return MG_OK;
}

int mg_level_cc_prolong_correct(int dim, int n, double* u, const double* ec, void* stream) {
    if ((dim != 2 && dim != 3) || !valid_cc(dim, n) || !u || !ec) return MG_EINVAL;
    CK(cc_prolong(dim, u, ec, n, (hipStream_t)stream));
    return MG_OK;
}

int mg_level_cc_remove_mean(int dim, int n, double* v, double* mean_out, void* stream) {
    if ((dim != 2 && dim != 3) || !valid_cc(dim, n) || !v || !mean_out) return MG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double* buf = nullptr;
    CK(hipMalloc((void**)&buf, (cc_work_doubles(dim, n) + 1) * sizeof(double)));
    hipError_t e = cc_remove_mean(dim, n, v, buf + 1, buf, s);
    double m = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&m, buf, sizeof(double), hipMemcpyDeviceToHost, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    ffree(buf);
    if (e != hipSuccess) return dev_status(e);
    if (e2 != hipSuccess) return dev_status(e2);
    *mean_out = m;
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free refinement pass.  Its scratch (the launch descriptor, one
// norm partial per workgroup and the finalized norm) lives in a static device
// array of fixed size instead of hipMalloc'd buffers.  Each device holds its
// own copy of the array; its address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to the kernels and
// copies.  Calls on one device share the array.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr size_t kScratchBytes = size_t(1) << 20;  // per device
constexpr size_t kScratchNormOff = 256;            // finalized norm (one double)
constexpr size_t kScratchPartOff = 512;            // norm partials
constexpr int kScratchMaxParts = (int)((kScratchBytes - kScratchPartOff) / sizeof(double));
static_assert(sizeof(mg::IRDesc) <= kScratchNormOff, "descriptor must fit before the norm");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per device).
int scratch_ptr(unsigned char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dev_status(e);
    if (dev < 0 || dev >= kMaxDevices) return MG_EDEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return e != hipSuccess ? dev_status(e) : MG_EDEVICE;
        g_scratch[dev] = (unsigned char*)p;
    }
    *out = g_scratch[dev];
    return MG_OK;
}

}  // namespace

extern "C" {

int mg_level_ir_update_noalloc(int dim, int n, const double* k, const double* u_in, const float* e, const double* f,
                               double* u_out, float* r, double* norm_out, int by, int zchunk, int prefetch,
                               int waves, int pairs, void* stream) {
    if (!valid_edge(dim, n) || n < 5) return MG_EINVAL;
    if (!u_in || !e || !f || !u_out || !r || !norm_out || u_in == u_out) return MG_EINVAL;
    TileCfg cfg = pick_cfg(dim, 8, n, 0, by, zchunk, 2);
    if (prefetch) cfg.pd = prefetch;
    if (waves) cfg.wv = waves;
    cfg.xp = pairs ? 2 : 1;
    if (cfg.xp == 2 && dim == 2 && !zchunk) cfg.zchunk = 32;
    if (!valid_cfg(cfg, dim, 8, k != nullptr, 2)) return MG_EINVAL;
    const int nparts = norm_tiles(dim, n, cfg);
    if (nparts > kScratchMaxParts) return MG_ENOMEM;
    unsigned char* base = nullptr;
    const int rs = scratch_ptr(&base);
    if (rs != MG_OK) return rs;
    hipStream_t s = (hipStream_t)stream;
    IRDesc h{};
    h.u[0] = const_cast<double*>(u_in);
    h.u[1] = u_out;
    h.e = e;
    h.f = f;
    h.k = k;
    h.r = r;
    h.n = n;
    h.c = level_c(n);
    IRDesc* d = (IRDesc*)base;
    double* nrm = (double*)(base + kScratchNormOff);
    double* part = (double*)(base + kScratchPartOff);
    // Every partial the finalize step reads is written by the pass (one per
    // workgroup), so nothing in the array has to start at zero.
    hipError_t err = hipMemcpyAsync(d, &h, sizeof(IRDesc), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = launch_ir_update(dim, k != nullptr, d, 1, n, 0, 0, part, nparts, cfg, s);
    if (err == hipSuccess) err = launch_norm_finalize(part, nparts, nparts, 0, 1, nrm, s);
    if (err == hipSuccess) err = hipMemcpyAsync(norm_out, nrm, sizeof(double), hipMemcpyDeviceToHost, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    if (err != hipSuccess) return dev_status(err);
    return dev_status(e2);
}

}  // extern "C"
