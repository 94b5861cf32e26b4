// Batched and served solves: many independent grids (of uneven sizes) share
// every kernel launch.
//
// Each instance keeps a resident hierarchy: FP32 levels n = 2^a+1, ..., 3 for
// the V-cycle on the correction equation, plus the FP64 partner array of the
// refinement ping-pong.  Grids of different sizes meet on common absolute
// levels (every grid with 2^a+1 >= n_level has a level of exactly that size),
// so one launch per V-cycle step and absolute level covers every active
// instance (blockIdx.y selects the instance), and the descending leg picks up
// an instance at its own finest level.  The FP64 refinement pass runs once per
// distinct finest size.  Each instance has its own device stop flag, step
// counter and ping-pong parity: a converged instance's work is skipped inside
// the kernels while the others continue, and per-instance arithmetic is
// exactly that of a solve of the instance alone.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "mg_sched.h"
#include "mg_solver.h"

namespace mg {
namespace {

double lvl_c(int n) {
    const double h = 1.0 / (double)(n - 1);
    return 1.0 / (h * h);
}
double lvl_wd(int dim, int n, double omega) {
    const double h = 1.0 / (double)(n - 1);
    return (omega * (h * h)) / (2.0 * (double)dim);
}
int log2edge(int n) {
    int a = 0;
    while ((1 << a) + 1 < n) ++a;
    return a;
}

int st(hipError_t e) {
    if (e == hipSuccess) return MG_OK;
    return e == hipErrorOutOfMemory ? MG_ENOMEM : MG_EDEVICE;
}
#define BCK(x)                              \
    do {                                    \
        hipError_t e_ = (x);                \
        if (e_ != hipSuccess) return st(e_); \
    } while (0)

// One resident hierarchy.
struct Inst {
    int dim = 0, n = 0, a = 0;  // finest edge n = 2^a + 1
    int slot = -1;
    long long join_step = 0;     // serving: the step whose launches first include it
    std::vector<void*> e, t, r;  // FP32 levels, 0 = finest
    double* u2 = nullptr;        // FP64 ping-pong partner of u
    double* u64 = nullptr;       // owned FP64 iterate (served requests)
    double* f64 = nullptr;       // owned FP64 rhs (served requests)
    size_t bytes = 0;
    double* u = nullptr;        // bound FP64 iterate
    const double* f = nullptr;  // bound FP64 rhs
};

size_t inst_bytes(int dim, int n, bool own_io) {
    size_t b = 0;
    for (int m = n;; m = (m - 1) / 2 + 1) {
        b += npts(dim, m) * 4 * (m > 3 ? 3 : 2);
        if (m == 3) break;
    }
    b += npts(dim, n) * 8 * (own_io ? 3 : 1);
    return b;
}

void free_inst(Inst& I) {
    for (void* p : I.e) (void)hipFree(p);
    for (void* p : I.t) (void)hipFree(p);
    for (void* p : I.r) (void)hipFree(p);
    if (I.u2) (void)hipFree(I.u2);
    if (I.u64) (void)hipFree(I.u64);
    if (I.f64) (void)hipFree(I.f64);
    I.e.clear();
    I.t.clear();
    I.r.clear();
    I.u2 = I.u64 = I.f64 = nullptr;
}

hipError_t zmalloc(void** p, size_t bytes, hipStream_t s) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    return hipMemsetAsync(*p, 0, bytes, s);
}

hipError_t alloc_inst(Inst& I, int dim, int n, bool own_io, hipStream_t s) {
    I.dim = dim;
    I.n = n;
    I.a = log2edge(n);
    I.bytes = inst_bytes(dim, n, own_io);
    hipError_t e = hipSuccess;
    for (int m = n;; m = (m - 1) / 2 + 1) {
        const size_t b = npts(dim, m) * 4;
        void *pe = nullptr, *pt = nullptr, *pr = nullptr;
        e = zmalloc(&pe, b, s);
        I.e.push_back(pe);
        if (e != hipSuccess) break;
        if (m > 3) {
            e = zmalloc(&pt, b, s);
            I.t.push_back(pt);
            if (e != hipSuccess) break;
        } else {
            I.t.push_back(nullptr);
        }
        e = zmalloc(&pr, b, s);
        I.r.push_back(pr);
        if (e != hipSuccess) break;
        if (m == 3) break;
    }
    const size_t N = npts(dim, n) * 8;
    if (e == hipSuccess) e = zmalloc((void**)&I.u2, N, s);
    if (e == hipSuccess && own_io) e = zmalloc((void**)&I.u64, N, s);
    if (e == hipSuccess && own_io) e = zmalloc((void**)&I.f64, N, s);
    if (e != hipSuccess) free_inst(I);
    return e;
}

struct IRGroup {
    int a, n, cnt;
    IRDesc* d;
};

// Pinned host staging for descriptor uploads in a ring of generations: a
// rebuild writes one generation while the copies of earlier ones may still be
// queued behind running work, so a rebuild rarely waits for the device (only
// when it comes back to a generation whose copies have not run yet).
struct Staging {
    static constexpr int G = 4;
    char* buf[G] = {};
    size_t cap[G] = {};
    hipEvent_t ev[G] = {};
    bool queued[G] = {};
    int g = 0;
    size_t off = 0;
    static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
    hipError_t begin(size_t need) {
        g = (g + 1) % G;
        if (queued[g]) {
            hipError_t e = hipEventSynchronize(ev[g]);
            if (e != hipSuccess) return e;
            queued[g] = false;
        }
        if (!ev[g]) {
            hipError_t e = hipEventCreateWithFlags(&ev[g], hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        if (need > cap[g]) {
            if (buf[g]) (void)hipHostFree(buf[g]);
            buf[g] = nullptr;
            cap[g] = 0;
            hipError_t e = hipHostMalloc((void**)&buf[g], need, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            cap[g] = need;
        }
        off = 0;
        return hipSuccess;
    }
    hipError_t put(void* dst, const void* src, size_t bytes, hipStream_t s) {
        if (bytes == 0) return hipSuccess;
        std::memcpy(buf[g] + off, src, bytes);
        hipError_t e = hipMemcpyAsync(dst, buf[g] + off, bytes, hipMemcpyHostToDevice, s);
        off += round(bytes);
        return e;
    }
    hipError_t end(hipStream_t s) {
        queued[g] = true;
        return hipEventRecord(ev[g], s);
    }
    ~Staging() {
        for (int i = 0; i < G; ++i) {
            if (queued[i]) (void)hipEventSynchronize(ev[i]);
            if (buf[i]) (void)hipHostFree(buf[i]);
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        }
    }
};

// Shared launch machinery for a set of instances of one dimension.
struct Engine {
    int dim = 2;
    Problem prob{};
    hipStream_t s = nullptr;
    int cap = 0;        // instance slots
    int max_a = 1;      // largest finest level accepted
    std::vector<Tiles> tiles;  // by absolute level a (index a)
    int pstride = 1;
    int *d_done = nullptr, *d_steps = nullptr, *d_status = nullptr, *d_par = nullptr, *d_nparts = nullptr;
    int* d_rows = nullptr;
    int* d_newrows = nullptr;
    double *d_norm = nullptr, *d_norm0 = nullptr, *d_partial = nullptr;
    int* h_ctrl = nullptr;  // pinned: done, steps, status (3 * cap)
    double* h_nrm = nullptr;  // pinned: norm, norm0 (2 * cap)
    // serving: control snapshots taken after a step, two in flight
    int* h_snap[2] = {nullptr, nullptr};    // pinned: done, steps, status (3 * cap)
    double* h_snrm[2] = {nullptr, nullptr}; // pinned: norm, norm0 (2 * cap)
    hipEvent_t snap_ev[2] = {nullptr, nullptr};
    long long snap_step[2] = {-1, -1};
    bool snap_pending[2] = {false, false};
    Staging stage;
    GridDesc* d_gd = nullptr;
    size_t gd_cap = 0;
    IRDesc* d_ir = nullptr;
    size_t ir_cap = 0;
    TailDesc* d_tail = nullptr;  // one per member: its levels at or below the tail edge
    size_t tail_cap = 0;
    std::vector<TailDesc> h_tail;
    TailPlan tailplan;
    std::vector<GridDesc> h_gd;
    std::vector<IRDesc> h_ir;
    std::vector<Group> groups;  // finest-first over absolute levels
    std::vector<Tiles> gtiles;  // tiles in group order
    std::vector<IRGroup> irg;   // all members, by finest size
    std::vector<IRGroup> irg_new;
    std::vector<int> h_rows, h_newrows;
    std::vector<Inst*> members;
    std::vector<Inst*> fresh;  // members that still need their initial residual
    struct ChunkGraph {  // captured chunk of K steps for a tolerance and step limit
        int k, max_steps;
        double tol;
        hipGraphExec_t exec;
    };
    std::vector<ChunkGraph> graphs;  // for the current descriptors (cleared by rebuild)
    hipStream_t cap_stream = nullptr;

    ~Engine() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (void* p : {(void*)d_done, (void*)d_steps, (void*)d_status, (void*)d_par, (void*)d_nparts,
                        (void*)d_rows, (void*)d_newrows, (void*)d_norm, (void*)d_norm0, (void*)d_partial,
                        (void*)d_gd, (void*)d_ir, (void*)d_tail})
            if (p) (void)hipFree(p);
        if (h_ctrl) (void)hipHostFree(h_ctrl);
        if (h_nrm) (void)hipHostFree(h_nrm);
        for (int b = 0; b < 2; ++b) {
            if (snap_ev[b]) (void)hipEventDestroy(snap_ev[b]);
            if (h_snap[b]) (void)hipHostFree(h_snap[b]);
            if (h_snrm[b]) (void)hipHostFree(h_snrm[b]);
        }
    }

    int init(int dim_, const Problem& P, hipStream_t s_, int cap_, int max_n) {
        dim = dim_;
        prob = P;
        s = s_;
        cap = cap_;
        max_a = log2edge(max_n);
        tiles.resize((size_t)max_a + 1);
        for (int a = 1; a <= max_a; ++a) {
            tiles[(size_t)a] = default_tiles(dim, 4, (1 << a) + 1, P.smoother);
            // 2D refinement pass (batches are Laplacian): two nodes per lane,
            // each wavefront marching 32 rows (longer chunks leave the smaller
            // grids of a batch too few workgroups)
            if (dim == 2) tiles[(size_t)a].norm = TileCfg{16, 32, 2, 4, 0, 2};
        }
        for (int a = 2; a <= max_a; ++a)
            pstride = std::max(pstride, norm_tiles(dim, (1 << a) + 1, tiles[(size_t)a].norm));
        const size_t ci = sizeof(int) * (size_t)cap;
        BCK(hipMalloc((void**)&d_done, ci));
        BCK(hipMalloc((void**)&d_steps, ci));
        BCK(hipMalloc((void**)&d_status, ci));
        BCK(hipMalloc((void**)&d_par, ci));
        BCK(hipMalloc((void**)&d_nparts, ci));
        BCK(hipMalloc((void**)&d_rows, ci));
        BCK(hipMalloc((void**)&d_newrows, ci));
        BCK(hipMalloc((void**)&d_norm, sizeof(double) * (size_t)cap));
        BCK(hipMalloc((void**)&d_norm0, sizeof(double) * (size_t)cap));
        BCK(hipMalloc((void**)&d_partial, sizeof(double) * (size_t)cap * (size_t)pstride));
        BCK(hipHostMalloc((void**)&h_ctrl, 3 * ci, hipHostMallocDefault));
        BCK(hipHostMalloc((void**)&h_nrm, 2 * sizeof(double) * (size_t)cap, hipHostMallocDefault));
        for (int b = 0; b < 2; ++b) {
            BCK(hipHostMalloc((void**)&h_snap[b], 3 * ci, hipHostMallocDefault));
            BCK(hipHostMalloc((void**)&h_snrm[b], 2 * sizeof(double) * (size_t)cap, hipHostMallocDefault));
            BCK(hipEventCreateWithFlags(&snap_ev[b], hipEventDisableTiming));
        }
        BCK(launch_fill_int(d_done, 1, cap, s));  // empty slots are "done"
        BCK(launch_fill_int(d_steps, 0, cap, s));
        BCK(launch_fill_int(d_status, 0, cap, s));
        BCK(launch_fill_int(d_par, 0, cap, s));
        BCK(launch_fill_int(d_nparts, 0, cap, s));
        return MG_OK;
    }

    GridDesc level_desc(const Inst& I, int a) const {
        const int l = I.a - a;  // level index inside the instance
        GridDesc d{};
        const int n = (1 << a) + 1;
        d.u = I.e[(size_t)l];
        d.t = I.t[(size_t)l];
        d.f = I.r[(size_t)l];
        d.k = nullptr;
        d.uc = a > 1 ? I.e[(size_t)l + 1] : nullptr;
        d.fc = a > 1 ? I.r[(size_t)l + 1] : nullptr;
        d.done = d_done + I.slot;
        d.n = n;
        d.inst = I.slot;
        d.c = lvl_c(n);
        d.wd = lvl_wd(dim, n, prob.omega);
        d.omega = prob.omega;
        return d;
    }

    IRDesc ir_desc(const Inst& I) const {
        IRDesc d{};
        d.u[0] = I.u;
        d.u[1] = I.u2;
        d.e = (const float*)I.e[0];
        d.f = I.f;
        d.k = nullptr;
        d.r = (float*)I.r[0];
        d.done = d_done + I.slot;
        d.par = d_par + I.slot;
        d.n = I.n;
        d.inst = I.slot;
        d.c = lvl_c(I.n);
        return d;
    }

    // Rebuild every descriptor for the current members and upload them.
    int rebuild() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
        std::sort(members.begin(), members.end(), [](const Inst* x, const Inst* y) { return x->slot < y->slot; });
        groups.clear();
        gtiles.clear();
        irg.clear();
        irg_new.clear();
        h_gd.clear();
        h_ir.clear();
        h_tail.clear();
        tailplan = TailPlan{};
        if (members.empty()) return MG_OK;
        int amax = 1;
        for (const Inst* I : members) amax = std::max(amax, I->a);
        std::vector<std::pair<size_t, size_t>> goff;  // (offset, count) into h_gd per absolute level
        for (int a = amax; a >= 1; --a) {
            const size_t off = h_gd.size();
            for (const Inst* I : members)
                if (I->a >= a) h_gd.push_back(level_desc(*I, a));
            goff.push_back({off, h_gd.size() - off});
        }
        // coarse tail: every member's levels with edges up to the tail edge, in
        // one workgroup per member (all batched iterates start at zero)
        const int a_t = std::getenv("MG_NO_TAIL") ? 0 : log2edge(tail_max_edge(dim, 4));
        if (a_t >= 1 && a_t <= kMaxTailLevels) {
            for (const Inst* I : members) {
                TailDesc t{};
                const int top = std::min(I->a, a_t);
                t.nlev = top;
                for (int j = 0; j < top; ++j) t.lv[j] = level_desc(*I, top - j);
                h_tail.push_back(t);
            }
            tailplan.first = amax - std::min(amax, a_t);
            tailplan.ninst = (int)h_tail.size();
        }
        std::vector<std::pair<int, std::pair<size_t, size_t>>> ioff, inew;
        for (int pass = 0; pass < 2; ++pass) {
            const std::vector<Inst*>& list = pass == 0 ? members : fresh;
            for (int a = amax; a >= 1; --a) {
                const size_t off = h_ir.size();
                for (const Inst* I : list)
                    if (I->a == a) h_ir.push_back(ir_desc(*I));
                if (h_ir.size() > off) (pass == 0 ? ioff : inew).push_back({a, {off, h_ir.size() - off}});
            }
        }
        if (h_gd.size() > gd_cap || h_ir.size() > ir_cap || h_tail.size() > tail_cap)
            BCK(hipStreamSynchronize(s));  // old arrays may be in use
        if (h_tail.size() > tail_cap) {
            if (d_tail) (void)hipFree(d_tail);
            tail_cap = std::max(h_tail.size(), 2 * tail_cap);
            BCK(hipMalloc((void**)&d_tail, sizeof(TailDesc) * tail_cap));
        }
        if (h_gd.size() > gd_cap) {
            if (d_gd) (void)hipFree(d_gd);
            gd_cap = std::max(h_gd.size(), 2 * gd_cap);
            BCK(hipMalloc((void**)&d_gd, sizeof(GridDesc) * gd_cap));
        }
        if (h_ir.size() > ir_cap) {
            if (d_ir) (void)hipFree(d_ir);
            ir_cap = std::max(h_ir.size(), 2 * ir_cap);
            BCK(hipMalloc((void**)&d_ir, sizeof(IRDesc) * ir_cap));
        }
        h_rows.clear();
        for (const Inst* I : members) h_rows.push_back(I->slot);
        h_newrows.clear();
        for (const Inst* I : fresh) h_newrows.push_back(I->slot);
        std::vector<int> np((size_t)cap, 0);
        for (const Inst* I : members) np[(size_t)I->slot] = norm_tiles(dim, I->n, tiles[(size_t)I->a].norm);
        // uploads are ordered behind the work already queued on the stream
        BCK(stage.begin(Staging::round(sizeof(TailDesc) * h_tail.size()) +
                        Staging::round(sizeof(GridDesc) * h_gd.size()) + Staging::round(sizeof(IRDesc) * h_ir.size()) +
                        Staging::round(sizeof(int) * h_rows.size()) + Staging::round(sizeof(int) * h_newrows.size()) +
                        Staging::round(sizeof(int) * np.size())));
        if (!h_tail.empty()) {
            BCK(stage.put(d_tail, h_tail.data(), sizeof(TailDesc) * h_tail.size(), s));
            tailplan.d = d_tail;
        }
        BCK(stage.put(d_gd, h_gd.data(), sizeof(GridDesc) * h_gd.size(), s));
        BCK(stage.put(d_ir, h_ir.data(), sizeof(IRDesc) * h_ir.size(), s));
        BCK(stage.put(d_rows, h_rows.data(), sizeof(int) * h_rows.size(), s));
        BCK(stage.put(d_newrows, h_newrows.data(), sizeof(int) * h_newrows.size(), s));
        BCK(stage.put(d_nparts, np.data(), sizeof(int) * np.size(), s));
        BCK(stage.end(s));
        for (size_t g = 0; g < goff.size(); ++g) {
            Group G;
            G.n = (1 << (amax - (int)g)) + 1;
            G.ninst = (int)goff[g].second;
            G.d = d_gd + goff[g].first;
            groups.push_back(G);
            gtiles.push_back(tiles[(size_t)(amax - (int)g)]);
        }
        for (auto& x : ioff) irg.push_back({x.first, (1 << x.first) + 1, (int)x.second.second, d_ir + x.second.first});
        for (auto& x : inew)
            irg_new.push_back({x.first, (1 << x.first) + 1, (int)x.second.second, d_ir + x.second.first});
        return MG_OK;
    }

    // Autotune the FP32 sweeps and restrictions of every level above the
    // coarse tail for the current members (MG_AUTOTUNE=0 keeps the heuristic).
    int tune() {
        const char* at = std::getenv("MG_AUTOTUNE");
        if ((at && at[0] == '0') || members.empty()) return MG_OK;
        int r = rebuild();
        if (r != MG_OK) return r;
        const int amax = (int)groups.size();
        const int stop = tailplan.ninst > 0 ? tailplan.first : amax;
        BCK(launch_fill_int(d_done, 0, cap, s));  // kernels skip instances whose flag is set
        for (int g = 0; g < stop; ++g) {
            const int a = amax - g;
            BCK(tune_group(dim, prob.smoother, groups[(size_t)g].d, groups[(size_t)g].ninst, groups[(size_t)g].n,
                           tiles[(size_t)a], s));
        }
        BCK(launch_fill_int(d_done, 1, cap, s));
        return rebuild();
    }

    // Initial residual (rho_0) of the fresh members; their stop flags open.
    hipError_t start_fresh() {
        if (fresh.empty()) return hipSuccess;
        // open the stop flags of the fresh rows (every kernel honours them)
        hipError_t e0 = launch_set_rows(d_done, 0, d_newrows, (int)h_newrows.size(), s);
        if (e0 != hipSuccess) return e0;
        // the iterate starts in u (parity 0), whatever a previous solve in this slot left
        e0 = launch_set_rows(d_par, 0, d_newrows, (int)h_newrows.size(), s);
        if (e0 != hipSuccess) return e0;
        for (const IRGroup& g : irg_new) {
            hipError_t e = launch_ir_update(dim, false, g.d, g.cnt, g.n, 0, IR_NO_UPDATE, d_partial, pstride,
                                            tiles[(size_t)g.a].norm, s);
            if (e != hipSuccess) return e;
        }
        hipError_t e = launch_norm_finalize_rows(d_partial, pstride, d_nparts, d_newrows, (int)h_newrows.size(),
                                                 d_norm, s);
        if (e != hipSuccess) return e;
        return launch_solve_init_rows(d_norm, d_norm0, d_done, d_steps, d_status, d_par, d_newrows,
                                      (int)h_newrows.size(), s);
    }

    // One refinement step of every member: FP32 V-cycle from e = 0, FP64 pass, stop test.
    hipError_t enqueue_step(double tol, int max_steps, hipStream_t q) {
        if (members.empty()) return hipSuccess;
        hipError_t e = vcycle<float>(prob, groups, true, gtiles, q, nullptr, nullptr, 0, &tailplan);
        if (e != hipSuccess) return e;
        for (const IRGroup& g : irg) {
            e = launch_ir_update(dim, false, g.d, g.cnt, g.n, 0, 0, d_partial, pstride, tiles[(size_t)g.a].norm, q);
            if (e != hipSuccess) return e;
        }
        e = launch_norm_finalize_rows(d_partial, pstride, d_nparts, d_rows, (int)h_rows.size(), d_norm, q);
        if (e != hipSuccess) return e;
        return launch_stop_test(d_norm, d_norm0, d_done, d_steps, d_status, nullptr, 0, tol, max_steps, cap, q,
                                d_par);
    }

    int run_chunk(int K, double tol, int max_steps, bool use_graph) {
        if (!use_graph) {
            for (int i = 0; i < K; ++i) BCK(enqueue_step(tol, max_steps, s));
            return MG_OK;
        }
        hipGraphExec_t graph = nullptr;
        for (const auto& g : graphs)
            if (g.k == K && g.tol == tol && g.max_steps == max_steps) graph = g.exec;
        if (!graph) {
            if (graphs.size() >= 8) {  // a new tolerance or limit: start over
                for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
                graphs.clear();
            }
            if (!cap_stream) BCK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
            BCK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int i = 0; i < K && e == hipSuccess; ++i) e = enqueue_step(tol, max_steps, cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(cap_stream, &g);
            if (e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return st(e);
            }
            BCK(e2);
            hipError_t e3 = hipGraphInstantiate(&graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            BCK(e3);
            graphs.push_back({K, max_steps, tol, graph});
        }
        BCK(hipGraphLaunch(graph, s));
        return MG_OK;
    }

    int read_ctrl(bool norms = false) {
        BCK(hipMemcpyAsync(h_ctrl, d_done, sizeof(int) * (size_t)cap, hipMemcpyDeviceToHost, s));
        BCK(hipMemcpyAsync(h_ctrl + cap, d_steps, sizeof(int) * (size_t)cap, hipMemcpyDeviceToHost, s));
        BCK(hipMemcpyAsync(h_ctrl + 2 * cap, d_status, sizeof(int) * (size_t)cap, hipMemcpyDeviceToHost, s));
        if (norms) {
            BCK(hipMemcpyAsync(h_nrm, d_norm, sizeof(double) * (size_t)cap, hipMemcpyDeviceToHost, s));
            BCK(hipMemcpyAsync(h_nrm + cap, d_norm0, sizeof(double) * (size_t)cap, hipMemcpyDeviceToHost, s));
        }
        BCK(hipStreamSynchronize(s));
        return MG_OK;
    }
    int done(int slot) const { return h_ctrl[slot]; }
    int steps(int slot) const { return h_ctrl[cap + slot]; }
    int status(int slot) const { return h_ctrl[2 * cap + slot]; }

    // Serving: copy the control state after step 'step_no' into snapshot
    // buffer step_no & 1 (the caller has consumed what it held).
    hipError_t snapshot(long long step_no) {
        const int b = (int)(step_no & 1);
        const size_t ci = sizeof(int) * (size_t)cap, cd = sizeof(double) * (size_t)cap;
        hipError_t e = hipMemcpyAsync(h_snap[b], d_done, ci, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h_snap[b] + cap, d_steps, ci, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h_snap[b] + 2 * cap, d_status, ci, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h_snrm[b], d_norm, cd, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h_snrm[b] + cap, d_norm0, cd, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(snap_ev[b], s);
        if (e == hipSuccess) {
            snap_step[b] = step_no;
            snap_pending[b] = true;
        }
        return e;
    }

    // After a finished solve: the iterate is in u2 when an odd number of update passes ran.
    hipError_t copy_back(const Inst& I) {
        if (steps(I.slot) & 1) return hipMemcpyAsync(I.u, I.u2, npts(dim, I.n) * 8, hipMemcpyDeviceToDevice, s);
        return hipSuccess;
    }
};

// ---------------------------------------------------------------------------
// Static batch (mg_batch_*)
// ---------------------------------------------------------------------------

struct Batch {
    int count = 0;
    int dim = 2;
    std::vector<Inst> inst;  // in caller order
    std::unique_ptr<Engine> eng;
    bool use_graphs = true;
    ~Batch() {
        if (eng && eng->s) (void)hipStreamSynchronize(eng->s);
        eng.reset();
        for (Inst& I : inst) free_inst(I);
    }
};

// ---------------------------------------------------------------------------
// Server (mg_server_*)
// ---------------------------------------------------------------------------

struct Request {
    long long id = 0;
    int dim = 2, n = 0;
    double* f_pin = nullptr;   // pinned copy of the rhs (until uploaded)
    std::unique_ptr<double[]> f_heap;  // used instead when too many payloads are queued
    double* u_pin = nullptr;   // pinned result (filled by an asynchronous copy)
    const double* f_dev = nullptr;  // device-fed request: the caller's right-hand side
    double* u_dev = nullptr;        // and the caller's device array for the solution
    hipEvent_t ev = nullptr;   // completes when u_pin holds the result
    hipEvent_t up = nullptr;   // completes when the hierarchy holds u = 0 and f
    Inst* inst = nullptr;
    int cycles = 0, status = 1;
    double rel_res = 0.0;
    bool complete = false;
    std::chrono::steady_clock::time_point t_submit, t_admit, t_done;
};

// Host copy of a request payload or result, split over a few threads for
// large buffers (one thread reaches a fraction of the host's memory bandwidth
// on a copy of tens of MB).  A thread that cannot be started copies nothing:
// its part is copied by the caller.
void host_copy(void* dst, const void* src, size_t bytes) {
    constexpr size_t kPart = size_t(4) << 20;
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>(std::min<size_t>(8, hw), (bytes + kPart - 1) / kPart);
    if (nt <= 1) {
        std::memcpy(dst, src, bytes);
        return;
    }
    const size_t part = (bytes / nt + 4095) & ~size_t(4095);
    auto piece = [dst, src, bytes, part](size_t t) {
        const size_t o = t * part;
        if (o < bytes) std::memcpy((char*)dst + o, (const char*)src + o, std::min(part, bytes - o));
    };
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (size_t t = 1; t < nt; ++t) {
        try {
            th.emplace_back(piece, t);
        } catch (...) {
            piece(t);
        }
    }
    piece(0);
    for (std::thread& x : th) x.join();
}

// Pinned host buffers by size (request payloads and results).
struct PinnedPool {
    std::map<size_t, std::vector<void*>> free;
    void* get(size_t bytes) {
        auto& v = free[bytes];
        if (!v.empty()) {
            void* p = v.back();
            v.pop_back();
            return p;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        return p;
    }
    void put(void* p, size_t bytes) {
        if (p) free[bytes].push_back(p);
    }
    ~PinnedPool() {
        for (auto& kv : free)
            for (void* p : kv.second) (void)hipHostFree(p);
    }
};

// Device side of the serving policy: request hierarchies (FP32 levels plus
// owned FP64 u, f and the refinement partner).
struct InstBackend {
    hipStream_t s = nullptr;  // the copy stream: allocation clears and uploads are ordered on it
    size_t bytes(int dim, int n) const { return inst_bytes(dim, n, true); }
    size_t bytes_of(const Inst* I) const { return I->bytes; }
    int alloc(int dim, int n, Inst** out) {
        Inst* I = new (std::nothrow) Inst();
        if (!I) return MG_ENOMEM;
        hipError_t e = alloc_inst(*I, dim, n, true, s);
        if (e != hipSuccess) {
            delete I;
            return e == hipErrorOutOfMemory ? 1 : st(e);
        }
        *out = I;
        return 0;
    }
    void release(Inst* I) {
        (void)hipStreamSynchronize(s);  // a result copy out of the hierarchy may be in flight
        free_inst(*I);
        delete I;
    }
};

struct Server {
    mg_server_params sp{};
    PinnedPool pinned;
    size_t queued_pinned = 0;  // bytes of queued payloads held in pinned memory
    static constexpr size_t kMaxQueuedPinned = size_t(4) << 30;
    std::vector<Request*> copying;          // results on their way to the host
    // payloads whose upload the compute stream waits for: released once it landed
    struct Upload {
        hipEvent_t ev;
        void* pin;
        size_t bytes;
        std::unique_ptr<double[]> heap;
    };
    std::vector<Upload> uploading;
    std::vector<Request*> staged;  // admitted, upload in flight, not yet in an engine
    long long step_no = 0;         // refinement steps enqueued so far
    hipStream_t s = nullptr;   // compute stream (the caller's)
    hipStream_t cs = nullptr;  // copy stream: uploads and result copies overlap compute
    std::unique_ptr<Engine> eng[2];  // 2D, 3D
    std::map<long long, std::unique_ptr<Request>> reqs;
    Sched<Inst*> sch;                  // queue, slots, pool and budget
    InstBackend backend;
    std::vector<long long> completed;  // not yet returned by poll
    long long next_id = 1;
    double* h_norm = nullptr;

    ~Server() {
        if (s) (void)hipStreamSynchronize(s);
        if (cs) (void)hipStreamSynchronize(cs);
        for (auto& kv : reqs) {
            if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
            if (kv.second->up) (void)hipEventDestroy(kv.second->up);
            if (kv.second->f_pin) pinned.put(kv.second->f_pin, npts(kv.second->dim, kv.second->n) * 8);
            if (kv.second->u_pin) pinned.put(kv.second->u_pin, npts(kv.second->dim, kv.second->n) * 8);
        }
        for (auto& u : uploading) {
            pinned.put(u.pin, u.bytes);
            (void)hipEventDestroy(u.ev);
        }
        for (int d = 0; d < 2; ++d) eng[d].reset();
        sch.drain_pool(backend);
        for (auto& kv : reqs)
            if (kv.second->inst) backend.release(kv.second->inst);
        if (h_norm) (void)hipHostFree(h_norm);
        if (cs) (void)hipStreamDestroy(cs);
    }
};

}  // namespace
}  // namespace mg

using namespace mg;

// Batched / served contexts live behind the same opaque handle type.
struct mg_batch_handle {
    int kind;  // 1 batch, 2 server
    mg::Batch* batch = nullptr;
    mg::Server* server = nullptr;
};

namespace {

mg_batch_handle* as_handle(mg_ctx* c) { return reinterpret_cast<mg_batch_handle*>(c); }

// Handles of batches and servers are told apart from solver contexts by a registry.
std::mutex g_reg_mu;
std::vector<mg_batch_handle*> g_reg;

bool registered(mg_ctx* c) {
    std::lock_guard<std::mutex> g(g_reg_mu);
    return std::find(g_reg.begin(), g_reg.end(), as_handle(c)) != g_reg.end();
}

void reg_add(mg_batch_handle* h) {
    std::lock_guard<std::mutex> g(g_reg_mu);
    g_reg.push_back(h);
}

void reg_remove(mg_batch_handle* h) {
    std::lock_guard<std::mutex> g(g_reg_mu);
    g_reg.erase(std::remove(g_reg.begin(), g_reg.end(), h), g_reg.end());
}

bool same_solver(const mg_params& a, const mg_params& b) {
    return a.dim == b.dim && a.smoother == b.smoother && a.nu1 == b.nu1 && a.nu2 == b.nu2 && a.omega == b.omega &&
           a.precision == b.precision && a.op == b.op && a.bc == b.bc && a.cycle == b.cycle &&
           a.coarse_n == b.coarse_n;
}

int server_admit(Server& S);
int server_join(Server& S);
int server_consume(Server& S, int d, long long upto, bool wait);
void server_collect(Server& S);

}  // namespace

namespace mg {
bool is_batch_handle(const mg_ctx* c) { return registered(const_cast<mg_ctx*>(c)); }
void destroy_batch_handle(mg_ctx* c) {
    mg_batch_handle* h = as_handle(c);
    reg_remove(h);
    delete h->batch;
    delete h->server;
    delete h;
}
}  // namespace mg

extern "C" {

int mg_batch_setup(int count, const mg_params* each, void* stream, mg_ctx** out) {
    if (!out) return MG_EINVAL;
    *out = nullptr;
    if (count <= 0 || !each) return MG_EINVAL;
    const mg_params& p0 = each[0];
    if (p0.dim != 2 && p0.dim != 3) return MG_EINVAL;
    if (p0.precision != MG_PREC_FP32_IR || p0.op != MG_OP_LAPLACE || p0.bc != MG_BC_DIRICHLET_ZERO) return MG_ENOTSUP;
    if (p0.smoother != MG_SMOOTH_RBGS && p0.smoother != MG_SMOOTH_WJACOBI) return MG_EINVAL;
    if (p0.nu1 < 0 || p0.nu2 < 0 || p0.nu1 > 16 || p0.nu2 > 16) return MG_EINVAL;
    if (p0.cycle != MG_CYCLE_V || p0.coarse_n > 3) return MG_ENOTSUP;  // batches run V-cycles down to n = 3
    int max_n = 3;
    for (int i = 0; i < count; ++i) {
        mg_params q = each[i];
        if (q.omega <= 0.0) q.omega = p0.omega;
        mg_params q0 = p0;
        if (q0.omega <= 0.0) q0.omega = q.omega;
        if (!same_solver(q, q0) || !valid_edge(q.dim, q.n) || q.n < 5) return MG_EINVAL;
        max_n = std::max(max_n, q.n);
    }
    double omega = p0.omega > 0.0 ? p0.omega : (p0.smoother == MG_SMOOTH_RBGS ? 1.0 : 0.8);
    hipStream_t s = (hipStream_t)stream;
    auto* B = new (std::nothrow) Batch();
    if (!B) return MG_ENOMEM;
    B->count = count;
    B->dim = p0.dim;
    B->use_graphs = std::getenv("MG_NO_GRAPHS") == nullptr;
    B->inst.resize((size_t)count);
    B->eng.reset(new Engine());
    Problem P{p0.dim, p0.smoother, p0.nu1, p0.nu2, omega, false};
    int r = B->eng->init(p0.dim, P, s, count, max_n);
    for (int i = 0; r == MG_OK && i < count; ++i) {
        r = st(alloc_inst(B->inst[(size_t)i], p0.dim, each[i].n, false, s));
        B->inst[(size_t)i].slot = i;
    }
    if (r != MG_OK) {
        delete B;
        return r;
    }
    for (Inst& I : B->inst) B->eng->members.push_back(&I);
    r = B->eng->tune();
    if (r != MG_OK) {
        delete B;
        return r;
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        delete B;
        return MG_EDEVICE;
    }
    auto* h = new mg_batch_handle{1, B, nullptr};
    reg_add(h);
    *out = reinterpret_cast<mg_ctx*>(h);
    return MG_OK;
}

int mg_batch_solve(mg_ctx* ctx, double* const* u, const double* const* f, double tol, int max_cycles,
                   int* cycles_done, int* status) {
    if (!ctx || !registered(ctx) || !u || !f || max_cycles < 0 || !(tol >= 0.0)) return MG_EINVAL;
    mg_batch_handle* h = as_handle(ctx);
    if (h->kind != 1) return MG_EINVAL;
    Batch& B = *h->batch;
    Engine& E = *B.eng;
    for (int i = 0; i < B.count; ++i)
        if (!u[i] || !f[i]) return MG_EINVAL;
    bool changed = false;
    for (int i = 0; i < B.count; ++i) {
        Inst& I = B.inst[(size_t)i];
        if (I.u != u[i] || I.f != f[i]) changed = true;
        I.u = u[i];
        I.f = f[i];
    }
    E.fresh = E.members;
    if (changed || E.groups.empty() || E.h_newrows.size() != E.fresh.size()) {
        int r = E.rebuild();
        if (r != MG_OK) return r;
    }
    BCK(E.start_fresh());
    int enq = 0;
    // chunks of steps: the first of kmax, later ones as many as the slowest
    // unfinished instance's last chunk predicts it still needs
    const int kmax = 4;
    int K = kmax;
    int r = E.read_ctrl(true);
    if (r != MG_OK) return r;
    std::vector<double> prev(B.inst.size());
    for (size_t i = 0; i < B.inst.size(); ++i) prev[i] = E.h_nrm[B.inst[i].slot];
    auto all_done = [&]() {
        for (int i = 0; i < B.count; ++i)
            if (!E.done(B.inst[(size_t)i].slot)) return false;
        return true;
    };
    while (!all_done() && enq < max_cycles) {
        const int k = std::min(K, max_cycles - enq);
        r = E.run_chunk(k, tol, max_cycles, B.use_graphs);
        if (r != MG_OK) return r;
        enq += k;
        r = E.read_ctrl(true);
        if (r != MG_OK) return r;
        int need = 1;
        for (size_t i = 0; i < B.inst.size(); ++i) {
            const int sl = B.inst[i].slot;
            const double cur = E.h_nrm[sl], r0 = E.h_nrm[E.cap + sl];
            if (!E.done(sl)) {
                int ni = kmax;
                if (cur > 0.0 && prev[i] > 0.0 && r0 > 0.0) {
                    const double rate = std::pow(cur / prev[i], 1.0 / k);
                    if (rate < 0.9) ni = (int)std::ceil(std::log(tol * r0 / cur) / std::log(rate) - 1e-9);
                }
                need = std::max(need, std::min(kmax, std::max(1, ni)));
            }
            prev[i] = cur;
        }
        K = need;
    }
    int worst = MG_OK;
    for (int i = 0; i < B.count; ++i) {
        Inst& I = B.inst[(size_t)i];
        BCK(E.copy_back(I));
        const int stt = E.status(I.slot);
        if (cycles_done) cycles_done[i] = E.steps(I.slot);
        int code = stt == 0 ? MG_OK : (stt == -5 ? MG_EDIVERGED : MG_ENOTCONV);
        if (status) status[i] = code;
        if (code == MG_EDIVERGED) worst = MG_EDIVERGED;
        else if (code == MG_ENOTCONV && worst == MG_OK) worst = MG_ENOTCONV;
    }
    BCK(hipStreamSynchronize(E.s));
    return worst;
}

int mg_server_create(const mg_server_params* sp, void* stream, mg_ctx** out) {
    if (!out) return MG_EINVAL;
    *out = nullptr;
    if (!sp || sp->max_slots <= 0 || sp->hbm_budget_bytes == 0 || !(sp->tol >= 0.0) || sp->max_cycles <= 0)
        return MG_EINVAL;
    if (sp->smoother != MG_SMOOTH_RBGS && sp->smoother != MG_SMOOTH_WJACOBI) return MG_EINVAL;
    if (!valid_edge(2, sp->max_n2d) || !valid_edge(3, sp->max_n3d)) return MG_EINVAL;
    auto* S = new (std::nothrow) Server();
    if (!S) return MG_ENOMEM;
    S->sp = *sp;
    if (S->sp.omega <= 0.0) S->sp.omega = sp->smoother == MG_SMOOTH_RBGS ? 1.0 : 0.8;
    if (S->sp.nu1 == 0 && S->sp.nu2 == 0) S->sp.nu1 = S->sp.nu2 = 2;
    S->s = (hipStream_t)stream;
    if (hipStreamCreateWithFlags(&S->cs, hipStreamNonBlocking) != hipSuccess) {
        S->cs = nullptr;
        delete S;
        return MG_EDEVICE;
    }
    S->backend.s = S->cs;
    S->sch.init(sp->hbm_budget_bytes, sp->max_slots);
    int r = MG_OK;
    for (int d = 0; d < 2 && r == MG_OK; ++d) {
        S->eng[d].reset(new Engine());
        Problem P{2 + d, S->sp.smoother, S->sp.nu1, S->sp.nu2, S->sp.omega, false};
        r = S->eng[d]->init(2 + d, P, S->s, sp->max_slots, d == 0 ? sp->max_n2d : sp->max_n3d);
    }
    if (r == MG_OK && hipStreamSynchronize(S->s) != hipSuccess) r = MG_EDEVICE;
    if (r != MG_OK) {
        delete S;
        return r;
    }
    auto* h = new mg_batch_handle{2, nullptr, S};
    reg_add(h);
    *out = reinterpret_cast<mg_ctx*>(h);
    return MG_OK;
}

int mg_server_submit(mg_ctx* ctx, int dim, int n, const double* f_host, long long* req_id) {
    if (!ctx || !registered(ctx) || !f_host || !req_id) return MG_EINVAL;
    mg_batch_handle* h = as_handle(ctx);
    if (h->kind != 2) return MG_EINVAL;
    Server& S = *h->server;
    if (!valid_edge(dim, n) || n < 5) return MG_EINVAL;
    if (n > (dim == 2 ? S.sp.max_n2d : S.sp.max_n3d)) return MG_EINVAL;
    if (inst_bytes(dim, n, true) > S.sp.hbm_budget_bytes) return MG_ENOMEM;
    auto R = std::make_unique<Request>();
    R->id = S.next_id++;
    R->dim = dim;
    R->n = n;
    const size_t bytes = npts(dim, n) * sizeof(double);
    if (S.queued_pinned + bytes <= Server::kMaxQueuedPinned) R->f_pin = (double*)S.pinned.get(bytes);
    if (R->f_pin) {
        host_copy(R->f_pin, f_host, bytes);
        S.queued_pinned += bytes;
    } else {
        R->f_heap.reset(new (std::nothrow) double[npts(dim, n)]);
        if (!R->f_heap) return MG_ENOMEM;
        host_copy(R->f_heap.get(), f_host, bytes);
    }
    R->t_submit = std::chrono::steady_clock::now();
    *req_id = R->id;
    S.sch.submit(R->id);
    S.reqs[R->id] = std::move(R);
    return MG_OK;
}

int mg_server_submit_device(mg_ctx* ctx, int dim, int n, const double* f_dev, double* u_dev, long long* req_id) {
    if (!ctx || !registered(ctx) || !f_dev || !u_dev || !req_id) return MG_EINVAL;
    mg_batch_handle* h = as_handle(ctx);
    if (h->kind != 2) return MG_EINVAL;
    Server& S = *h->server;
    if (!valid_edge(dim, n) || n < 5) return MG_EINVAL;
    if (n > (dim == 2 ? S.sp.max_n2d : S.sp.max_n3d)) return MG_EINVAL;
    if (inst_bytes(dim, n, true) > S.sp.hbm_budget_bytes) return MG_ENOMEM;
    auto R = std::make_unique<Request>();
    R->id = S.next_id++;
    R->dim = dim;
    R->n = n;
    R->f_dev = f_dev;
    R->u_dev = u_dev;
    R->t_submit = std::chrono::steady_clock::now();
    *req_id = R->id;
    S.sch.submit(R->id);
    S.reqs[R->id] = std::move(R);
    return MG_OK;
}

int mg_server_step(mg_ctx* ctx, int* n_active, int* n_queued) {
    if (!ctx || !registered(ctx)) return MG_EINVAL;
    mg_batch_handle* h = as_handle(ctx);
    if (h->kind != 2) return MG_EINVAL;
    Server& S = *h->server;
    // Pipelined: the step enqueued here runs while the host completes the
    // previous one, so the device is not idle during admission and retirement.
    int r = server_admit(S);
    for (int d = 0; d < 2 && r == MG_OK; ++d) r = server_consume(S, d, S.step_no - 1, false);  // landed ones
    if (r == MG_OK) r = server_join(S);
    if (r != MG_OK) return r;
    const long long k = S.step_no++;
    for (int d = 0; d < 2; ++d) {
        Engine& E = *S.eng[d];
        if (E.members.empty()) continue;
        BCK(E.start_fresh());
        E.fresh.clear();
        BCK(E.enqueue_step(S.sp.tol, S.sp.max_cycles, S.s));
        BCK(E.snapshot(k));
    }
    for (int d = 0; d < 2; ++d) {
        r = server_consume(S, d, k - 1, true);  // at most step k stays in flight
        if (r != MG_OK) return r;
    }
    server_collect(S);
    if (n_active) *n_active = S.sch.active;
    if (n_queued) *n_queued = (int)S.sch.queue.size();
    return MG_OK;
}

int mg_server_poll(mg_ctx* ctx, long long* done_ids, int cap, int* ndone) {
    if (!ctx || !registered(ctx) || !ndone || (cap > 0 && !done_ids)) return MG_EINVAL;
    mg_batch_handle* h = as_handle(ctx);
    if (h->kind != 2) return MG_EINVAL;
    Server& S = *h->server;
    server_collect(S);
    const int k = std::min<int>(cap, (int)S.completed.size());
    for (int i = 0; i < k; ++i) done_ids[i] = S.completed[(size_t)i];
    S.completed.erase(S.completed.begin(), S.completed.begin() + k);
    *ndone = k;
    return MG_OK;
}

int mg_server_fetch(mg_ctx* ctx, long long req_id, double* u_host, int* cycles, double* final_rel_res,
                    double* latency_s) {
    if (!ctx || !registered(ctx)) return MG_EINVAL;
    mg_batch_handle* h = as_handle(ctx);
    if (h->kind != 2) return MG_EINVAL;
    Server& S = *h->server;
    auto it = S.reqs.find(req_id);
    if (it == S.reqs.end()) return MG_EINVAL;
    Request& R = *it->second;
    if (!R.complete) return MG_EBUSY;
    const size_t bytes = npts(R.dim, R.n) * sizeof(double);
    if (R.u_dev && u_host) return MG_EINVAL;  // a device-fed request's solution is in its u_dev
    if (u_host) host_copy(u_host, R.u_pin, bytes);
    if (R.u_pin) S.pinned.put(R.u_pin, bytes);
    R.u_pin = nullptr;
    if (R.ev) (void)hipEventDestroy(R.ev);
    R.ev = nullptr;
    if (cycles) *cycles = R.cycles;
    if (final_rel_res) *final_rel_res = R.rel_res;
    if (latency_s) *latency_s = std::chrono::duration<double>(R.t_done - R.t_submit).count();
    const int stt = R.status;
    S.reqs.erase(it);
    return stt == 0 ? MG_OK : (stt == -5 ? MG_EDIVERGED : MG_ENOTCONV);
}

int mg_server_info(mg_ctx* ctx, size_t* used_bytes, int* active, int* queued) {
    if (!ctx || !registered(ctx)) return MG_EINVAL;
    mg_batch_handle* h = as_handle(ctx);
    if (h->kind != 2) return MG_EINVAL;
    Server& S = *h->server;
    if (used_bytes) *used_bytes = S.sch.used;
    if (active) *active = S.sch.active;
    if (queued) *queued = (int)S.sch.queue.size();
    return MG_OK;
}

}  // extern "C"

namespace {

// Admit queued requests in arrival order while a slot and the HBM budget
// allow: take a hierarchy of the right size from the pool (or allocate one,
// first releasing pooled hierarchies of other sizes if the budget requires),
// and start clearing u and uploading f on the copy stream.  A request that
// does not fit now stays first in the queue (no overtaking, so no starvation).
int server_admit(Server& S) {
    while (!S.sch.queue.empty()) {
        Request& R = *S.reqs[S.sch.queue.front()];
        int slot = -1;
        Inst* I = nullptr;
        const int a = S.sch.admit_head(S.backend, R.dim, R.n, &slot, &I);
        if (a < 0) return a;
        if (a == 0) break;  // the head waits for a slot or for memory
        I->slot = slot;
        I->u = I->u64;
        I->f = I->f64;
        R.inst = I;
        R.t_admit = std::chrono::steady_clock::now();
        S.staged.push_back(&R);
        const size_t N = npts(R.dim, R.n);
        // ordered after the result copy of the hierarchy's previous request (same stream)
        BCK(hipMemsetAsync(I->u64, 0, N * sizeof(double), S.cs));
        if (R.f_dev) {
            BCK(hipMemcpyAsync(I->f64, R.f_dev, N * sizeof(double), hipMemcpyDeviceToDevice, S.cs));
        } else if (R.f_pin) {
            BCK(hipMemcpyAsync(I->f64, R.f_pin, N * sizeof(double), hipMemcpyHostToDevice, S.cs));
        } else {
            BCK(hipMemcpyAsync(I->f64, R.f_heap.get(), N * sizeof(double), hipMemcpyHostToDevice, S.cs));
        }
        if (!R.up) BCK(hipEventCreateWithFlags(&R.up, hipEventDisableTiming));
        BCK(hipEventRecord(R.up, S.cs));
    }
    return MG_OK;
}

// Admitted requests join their engine once their upload has landed, so the
// upload overlaps the other requests' refinement steps.  An engine with no
// other work takes the request at once and its stream waits for the upload
// on the device.
int server_join(Server& S) {
    bool any[2] = {false, false};
    std::vector<Request*> still;
    for (Request* R : S.staged) {
        const int d = R->dim - 2;
        Engine& E = *S.eng[d];
        const hipError_t q = hipEventQuery(R->up);
        if (q != hipSuccess && q != hipErrorNotReady) return st(q);
        const size_t bytes = npts(R->dim, R->n) * sizeof(double);
        if (q == hipSuccess) {
            if (R->f_pin) S.pinned.put(R->f_pin, bytes);
            R->f_heap.reset();
        } else if (E.members.empty() && !any[d]) {
            BCK(hipStreamWaitEvent(S.s, R->up, 0));
            S.uploading.push_back({R->up, R->f_pin, bytes, std::move(R->f_heap)});  // takes the event
            R->up = nullptr;
        } else {
            still.push_back(R);
            continue;
        }
        if (R->f_pin) S.queued_pinned -= bytes;
        R->f_pin = nullptr;
        R->inst->join_step = S.step_no;
        E.members.push_back(R->inst);
        E.fresh.push_back(R->inst);
        any[d] = true;
    }
    S.staged.swap(still);
    std::vector<Server::Upload> pend;
    for (auto& u : S.uploading) {
        const hipError_t q = hipEventQuery(u.ev);
        if (q == hipSuccess) {
            S.pinned.put(u.pin, u.bytes);
            (void)hipEventDestroy(u.ev);
        } else if (q == hipErrorNotReady) {
            pend.push_back(std::move(u));
        }
        else return st(q);
    }
    S.uploading.swap(pend);
    for (int d = 0; d < 2; ++d)
        if (any[d]) {
            int r = S.eng[d]->rebuild();
            if (r != MG_OK) return r;
        }
    return MG_OK;
}

// Complete the requests that a control snapshot shows finished: copy u to the
// host on the copy stream, return the hierarchy to the pool and free the slot.
// Snapshots of steps up to 'upto' are taken in step order; with 'wait' false
// only those that have already landed.  A snapshot speaks only for members
// that were in its step (later joiners may hold a reused slot).
int server_consume(Server& S, int d, long long upto, bool wait) {
    Engine& E = *S.eng[d];
    for (;;) {
        int b = -1;
        for (int i = 0; i < 2; ++i)
            if (E.snap_pending[i] && E.snap_step[i] <= upto && (b < 0 || E.snap_step[i] < E.snap_step[b])) b = i;
        if (b < 0) return MG_OK;
        if (wait) {
            BCK(hipEventSynchronize(E.snap_ev[b]));
        } else {
            const hipError_t q = hipEventQuery(E.snap_ev[b]);
            if (q == hipErrorNotReady) return MG_OK;
            BCK(q);
        }
        E.snap_pending[b] = false;
        const long long j = E.snap_step[b];
        const int* c = E.h_snap[b];
        const double* nr = E.h_snrm[b];
        std::vector<Inst*> keep;
        std::vector<Request*> out;
        for (Inst* I : E.members) {
            if (I->join_step > j || !c[I->slot]) {
                keep.push_back(I);
                continue;
            }
            Request* R = nullptr;
            for (auto& kv : S.reqs)
                if (kv.second->inst == I) R = kv.second.get();
            if (!R) return MG_EDEVICE;
            const int steps = c[E.cap + I->slot];
            const size_t bytes = npts(I->dim, I->n) * sizeof(double);
            const double* src = (steps & 1) ? I->u2 : I->u64;  // later steps skip the finished slot
            if (R->u_dev) {
                BCK(hipMemcpyAsync(R->u_dev, src, bytes, hipMemcpyDeviceToDevice, S.cs));
            } else {
                R->u_pin = (double*)S.pinned.get(bytes);
                if (!R->u_pin) return MG_ENOMEM;
                BCK(hipMemcpyAsync(R->u_pin, src, bytes, hipMemcpyDeviceToHost, S.cs));
            }
            const double n0 = nr[E.cap + I->slot];
            R->rel_res = n0 > 0.0 ? nr[I->slot] / n0 : 0.0;
            R->cycles = steps;
            R->status = c[2 * E.cap + I->slot];
            R->inst = nullptr;
            // the hierarchy may be reused at once: its next clear and upload are
            // ordered after the copy on the copy stream
            S.sch.retire(I->dim, I->slot, I->n, I);
            out.push_back(R);
        }
        if (out.empty()) continue;
        for (Request* R : out) {
            BCK(hipEventCreateWithFlags(&R->ev, hipEventDisableTiming));
            BCK(hipEventRecord(R->ev, S.cs));
            S.copying.push_back(R);
        }
        E.members = keep;
        const int r = E.rebuild();
        if (r != MG_OK) return r;
    }
}

// Requests whose result copy has landed become complete.
void server_collect(Server& S) {
    std::vector<Request*> still;
    for (Request* R : S.copying) {
        if (hipEventQuery(R->ev) == hipSuccess) {
            R->complete = true;
            R->t_done = std::chrono::steady_clock::now();
            S.completed.push_back(R->id);
        } else {
            still.push_back(R);
        }
    }
    S.copying.swap(still);
}

}  // namespace
