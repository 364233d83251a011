// Batched form: many independent PFC simulations (own n, L, eps, dt) advanced
// together.  Every phase of a multigrid cycle is ONE launch over all
// instances that take part in it (levels aligned from the finest), over a
// work-list of tiles of every instance's part of the phase: one tile per
// workgroup, or persistent (the resident workgroups walk the list).
// Instances whose residual met the tolerance are masked by a device flag, so
// each instance runs exactly the cycle sequence of the single-instance
// driver.  One cycle (stop test + V or F cycle) is captured once as a
// hipGraph and replayed until no instance is active.  Schedule, tile size
// and workgroup size of every phase kind are chosen by an autotuner whose
// choices can be cached in a JSON file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "runtime_internal.h"

using namespace pfc;

struct pfc_batch {
    int count = 0;
    pfc_config cfg{};  // shared cycle parameters (from cfgs[0])
    hipStream_t user_stream = nullptr, stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<pfc_handle *> inst;
    std::vector<double *> prev, cur, nxt, mu, om;  // natural-layout state per instance
    int maxdepth = 0;
    std::vector<std::vector<BSeg>> h_all, h_mid, h_bot;  // per depth (host copies)
    std::vector<BSeg *> d_all, d_mid, d_bot;              // device copies
    BSeg *d_norm = nullptr;
    int n_norm = 0;
    unsigned norm_blocks = 0;
    unsigned long long *partial = nullptr;
    BState st{};
    int **d_valid = nullptr;
    int *h_num = nullptr;   // pinned: the instances' active flags
    int *h_stats = nullptr; // pinned: cycles, status per instance
    double *h_res = nullptr;  // pinned: res0, res per instance
    // per phase kind (smooth, residual + coarsening, tau, interpolation,
    // coarse error): threads per workgroup, tile shape (see kShapes; default
    // 256 items of one plane), schedule (persistent or one tile per
    // workgroup) and, when persistent, the resident workgroups at that size
    int threads[5] = {256, 256, 256, 256, 256};
    int shape[5] = {2, 2, 2, 2, 2};
    bool persist[5] = {false, false, false, false, false};
    unsigned slots[5] = {0, 0, 0, 0, 0};
    // the finest depth's interpolation as column tiles (every instance's
    // finest size a multiple of kBPX), 1 << ptile_zi coarse planes per tile
    bool ptile = false;
    int ptile_zi = 2;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_ready = false;
    std::vector<void *> allocs;
    std::string err;
    ~pfc_batch();
};

pfc_batch::~pfc_batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto *h : inst) pfc_destroy(h);
    for (void *p : allocs) (void)hipFree(p);
    if (h_num) (void)hipHostFree(h_num);
    if (h_stats) (void)hipHostFree(h_stats);
    if (h_res) (void)hipHostFree(h_res);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
}

namespace {
thread_local std::string g_batch_error;

template <typename T>
bool balloc(pfc_batch *B, T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return false;
    B->allocs.push_back(q);
    *p = (T *)q;
    return true;
}

// Tiles of shape `shape` in a launch of `kind` over the list v.
unsigned seg_tiles(const BSeg &g, int kind, int shape) {
    const unsigned W = (unsigned)kTileMin << (shape % kWOpts), Z = 1u << (shape / kWOpts);
    unsigned Q, NPL;
    bseg_planes_host(g, kind, Q, NPL);
    return ((Q + W - 1) / W) * ((NPL + Z - 1) / Z);
}

unsigned ptile_tiles(const std::vector<BSeg> &v, int zi) {
    unsigned b = 0;
    for (const auto &g : v) b += batch_ptile_count(g, zi);
    return b;
}

bool ptile_fits_all(const std::vector<BSeg> &v) {
    return !v.empty() && std::all_of(v.begin(), v.end(), [](const BSeg &g) { return batch_ptile_fits(g); });
}

unsigned tiles_of(const std::vector<BSeg> &v, int kind, int shape) {
    unsigned b = 0;
    for (const auto &g : v) b += seg_tiles(g, kind, shape);
    return b;
}

void phase(pfc_batch *B, int kind, const std::vector<BSeg> &h, BSeg *d, int arg0, int arg1) {
    launch_batch(B->stream, kind, d, (int)h.size(), tiles_of(h, kind, B->shape[kind]), B->shape[kind],
                 B->threads[kind], B->persist[kind] ? B->slots[kind] : 0u, arg0, arg1);
}

BSeg make_seg(pfc_handle *h, int l, int i, const int *active) {
    BSeg g{};
    const Level &A = h->lev[l];
    g.op = op_of(h, l);
    g.u = A.u;
    g.f = A.f;
    // in a time step the finest level's first source component is phi^k (the
    // source kernel writes that copy as well): the phases read it from phk
    if (l == 0) g.f.a = A.phk;
    g.ubar = A.ubar;
    g.phk = A.phk;
    if (l + 1 < h->nlev) {
        const Level &C = h->lev[l + 1];
        g.lay_c = C.lay;
        g.uc = C.u;
        g.fc = C.f;
        g.ubarc = C.ubar;
    } else {
        g.lay_c = A.lay;
    }
    g.lap1 = h->lap1;
    g.lap3 = h->lap3;
    g.minv = h->minv64;
    g.valid = h->valid64;
    g.iters = h->d_iters;
    g.active = active;
    g.inst = i;
    return g;
}

pfc_status bfail(pfc_batch *B, pfc_status s, const std::string &m) {
    if (B)
        B->err = m;
    else
        g_batch_error = m;
    return s;
}

// One cycle of every active instance, aligned by depth from the finest level.
// tau: the levels at depth d still hold I r in f and I u in ubar (the middle
// levels' first pre-sweep, the coarsest levels' solve launch forms the tau
// correction).
void bcycle(pfc_batch *B, int d, bool fcycle, bool tau = false) {
    const hipStream_t s = B->stream;
    if (!B->h_bot[d].empty())
        launch_batch_coarse(s, B->d_bot[d], (int)B->h_bot[d].size(), tau ? 1 : 0);
    if (B->h_mid[d].empty()) return;
    const auto &mid = B->h_mid[d];
    const int picard = B->cfg.lin == PFC_LIN_PICARD;
    // the finest levels' f.a is their phi^k (make_seg): loaded once there
    const int pk1 = d == 0 ? 2 : 0;
    auto sweep = [&](int flags) {
        for (int c = 0; c < 2; ++c) phase(B, BK_SMOOTH, mid, B->d_mid[d], c, picard | pk1 | flags);
    };
    for (int q = 0; q < B->cfg.nu1; ++q) sweep(q == 0 && tau ? 4 : 0);
    phase(B, BK_RR, mid, B->d_mid[d], 0, 0);
    // with pre-sweeps the next depth's levels form the tau correction
    // themselves: the middle ones in their first sweep, the coarsest ones in
    // their solve's launch
    const bool tau_sweep = B->cfg.nu1 >= 1;
    if (!tau_sweep) phase(B, BK_TAU, B->h_all[d + 1], B->d_all[d + 1], 0, 0);
    bcycle(B, d + 1, fcycle, tau_sweep);
    if (fcycle) bcycle(B, d + 1, false);
    if (d == 0 && B->ptile) {  // forms the coarse error itself
        launch_batch_ptile(s, B->d_mid[0], (int)mid.size(), ptile_tiles(mid, B->ptile_zi),
                           B->ptile_zi, B->cfg.nu2 >= 1 ? 1 : 0);
    } else {
        phase(B, BK_ERR, mid, B->d_mid[d], 0, 0);
        phase(B, BK_PROLONG, mid, B->d_mid[d], B->cfg.nu2 >= 1 ? 1 : 0, 0);
    }
    for (int q = 0; q < B->cfg.nu2; ++q) sweep(0);
}

void record_cycle(pfc_batch *B) {
    launch_batch_norm(B->stream, B->d_norm, B->n_norm, B->norm_blocks, B->partial, B->st, B->cfg.tol,
                      B->cfg.max_cycles);
    bcycle(B, 0, B->cfg.cycle == PFC_CYCLE_F);
}

pfc_status capture(pfc_batch *B) {
    if (B->exec) {
        (void)hipGraphExecDestroy(B->exec);
        B->exec = nullptr;
    }
    if (B->graph) {
        (void)hipGraphDestroy(B->graph);
        B->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(B, PFC_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    record_cycle(B);
    e = hipStreamEndCapture(B->stream, &B->graph);
    if (e != hipSuccess) return bfail(B, PFC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bfail(B, PFC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    B->graph_ready = true;
    return PFC_OK;
}

pfc_status run_step(pfc_batch *B, pfc_step_info *infos_step) {
    const hipStream_t s = B->stream;
    for (int i = 0; i < B->count; ++i) step_begin(B->inst[i], B->prev[i], B->cur[i], B->mu[i], B->om[i]);
    launch_batch_reset(s, B->st, B->count, B->d_valid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(B, PFC_ERR_HIP, hipGetErrorString(e));
    if (!B->graph_ready) {
        const pfc_status stc = capture(B);
        if (stc != PFC_OK) return stc;
    }
    for (int guard = 0; guard <= B->cfg.max_cycles + 2; ++guard) {
        e = hipGraphLaunch(B->exec, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(B->h_num, B->st.active, B->count * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return bfail(B, PFC_ERR_HIP, std::string("batched cycle: ") + hipGetErrorString(e));
        if (std::none_of(B->h_num, B->h_num + B->count, [](int a) { return a != 0; })) break;
    }
    for (int i = 0; i < B->count; ++i) step_end(B->inst[i], B->nxt[i], B->mu[i], B->om[i]);
    const size_t n = (size_t)B->count;
    e = hipMemcpyAsync(B->h_stats, B->st.cycles, n * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B->h_stats + n, B->st.status, n * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B->h_res, B->st.res0, n * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(B->h_res + n, B->st.res, n * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bfail(B, PFC_ERR_HIP, std::string("batched step: ") + hipGetErrorString(e));
    pfc_status worst = PFC_OK;
    for (int i = 0; i < B->count; ++i) {
        if (infos_step) {
            infos_step[i].cycles = B->h_stats[i];
            infos_step[i].status = B->h_stats[n + i];
            infos_step[i].res0 = B->h_res[i];
            infos_step[i].res_final = B->h_res[n + i];
        }
        if (B->h_stats[n + i] != PFC_OK && worst == PFC_OK) worst = B->h_stats[n + i];
        std::swap(B->prev[i], B->nxt[i]);   // nxt <- old prev (spare)
        std::swap(B->prev[i], B->cur[i]);   // prev <- old cur, cur <- new phi
    }
    return worst;
}

std::string device_name() {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    return std::string(p.gcnArchName);
}

std::map<std::string, int> read_cache(const char *path) {
    std::map<std::string, int> m;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        const size_t a = line.find('"'), b = line.find('"', a + 1), c = line.find(':', b);
        if (a == std::string::npos || b == std::string::npos || c == std::string::npos) continue;
        m[line.substr(a + 1, b - a - 1)] = std::atoi(line.c_str() + c + 1);
    }
    return m;
}

void write_cache(const char *path, const std::map<std::string, int> &m) {
    std::ofstream out(path);
    out << "{\n";
    size_t k = 0;
    for (const auto &kv : m) out << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
    out << "}\n";
}

}  // namespace

extern "C" {

pfc_status pfc_batch_create(int32_t count, const pfc_config *cfgs, void *stream, pfc_batch **out) {
    if (!out) return bfail(nullptr, PFC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > 4096 || !cfgs) return bfail(nullptr, PFC_ERR_INVALID_ARG, "count must be in 1..4096");
    for (int i = 0; i < count; ++i) {
        const std::string why = validate_config(&cfgs[i]);
        if (!why.empty()) return bfail(nullptr, PFC_ERR_INVALID_ARG, "instance " + std::to_string(i) + ": " + why);
        if (cfgs[i].precision != PFC_FP64) return bfail(nullptr, PFC_ERR_INVALID_ARG, "the batched form is FP64");
        if (cfgs[i].mobility != PFC_MOBILITY_ONE)
            return bfail(nullptr, PFC_ERR_INVALID_ARG, "the batched form has constant mobility");
        if (cfgs[i].scheme != PFC_SCHEME_CS2)
            return bfail(nullptr, PFC_ERR_INVALID_ARG, "the batched form runs scheme (1.10)");
        if (cfgs[i].nu1 != cfgs[0].nu1 || cfgs[i].nu2 != cfgs[0].nu2 || cfgs[i].cycle != cfgs[0].cycle ||
            cfgs[i].lin != cfgs[0].lin || cfgs[i].tol != cfgs[0].tol || cfgs[i].max_cycles != cfgs[0].max_cycles)
            return bfail(nullptr, PFC_ERR_INVALID_ARG, "nu1, nu2, cycle, lin, tol, max_cycles must agree");
    }
    pfc_batch *B = new pfc_batch();
    B->count = count;
    B->cfg = cfgs[0];
    B->user_stream = (hipStream_t)stream;
    if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming) != hipSuccess) {
        delete B;
        return bfail(nullptr, PFC_ERR_HIP, "stream/event creation failed");
    }
    bool ok = true;
    std::vector<int> nlev(count);
    for (int i = 0; i < count && ok; ++i) {
        pfc_handle *h = nullptr;
        const pfc_status st = pfc_create(&cfgs[i], B->stream, &h);
        if (st != PFC_OK) {
            const std::string msg = pfc_last_error(nullptr);
            delete B;
            return bfail(nullptr, st, "instance " + std::to_string(i) + ": " + msg);
        }
        B->inst.push_back(h);
        nlev[i] = h->nlev;
        B->maxdepth = std::max(B->maxdepth, h->nlev);
        const size_t P = h->lev[0].P;
        double *p0, *p1, *p2, *p3, *p4;
        ok = balloc(B, &p0, P) && balloc(B, &p1, P) && balloc(B, &p2, P) && balloc(B, &p3, P) && balloc(B, &p4, P);
        if (!ok) break;
        ok = hipMemset(p0, 0, P * 8) == hipSuccess && hipMemset(p1, 0, P * 8) == hipSuccess &&
             hipMemset(p2, 0, P * 8) == hipSuccess && hipMemset(p3, 0, P * 8) == hipSuccess &&
             hipMemset(p4, 0, P * 8) == hipSuccess;
        B->prev.push_back(p0);
        B->cur.push_back(p1);
        B->nxt.push_back(p2);
        B->mu.push_back(p3);
        B->om.push_back(p4);
    }
    const size_t n = (size_t)count;
    ok = ok && balloc(B, &B->st.active, n) && balloc(B, &B->st.cycles, n) && balloc(B, &B->st.status, n) &&
         balloc(B, &B->st.res0, n) && balloc(B, &B->st.res, n) &&
         balloc(B, &B->d_valid, n);
    unsigned *nf = nullptr, *nbk = nullptr;
    ok = ok && balloc(B, &nf, n) && balloc(B, &nbk, n);
    if (!ok) {
        delete B;
        return bfail(nullptr, PFC_ERR_OOM, "device allocation failed");
    }
    B->st.norm_first = nf;
    B->st.norm_blocks = nbk;
    // segment lists by depth
    B->h_all.resize(B->maxdepth);
    B->h_mid.resize(B->maxdepth);
    B->h_bot.resize(B->maxdepth);
    for (int i = 0; i < count; ++i)
        for (int l = 0; l < nlev[i]; ++l) {
            const BSeg g = make_seg(B->inst[i], l, i, B->st.active + i);
            B->h_all[l].push_back(g);
            (l + 1 < nlev[i] ? B->h_mid[l] : B->h_bot[l]).push_back(g);
        }
    auto upload = [&](const std::vector<BSeg> &v, BSeg **d) -> bool {
        if (v.empty()) {
            *d = nullptr;
            return true;
        }
        std::vector<BSeg> w = v;  // with this list's first tiles
        for (int kind = 0; kind < BK_KINDS; ++kind)
            for (int sh = 0; sh < kShapes; ++sh) {
                unsigned acc = 0;
                for (auto &g : w) {
                    g.first[kind][sh] = acc;
                    acc += seg_tiles(g, kind, sh);
                }
            }
        for (int zi = 0; zi < kZOpts; ++zi) {
            unsigned acc = 0;
            for (auto &g : w) {
                g.ptf[zi] = acc;
                acc += batch_ptile_count(g, zi);
            }
        }
        return balloc(B, d, w.size()) &&
               hipMemcpy(*d, w.data(), w.size() * sizeof(BSeg), hipMemcpyHostToDevice) == hipSuccess;
    };
    B->d_all.resize(B->maxdepth);
    B->d_mid.resize(B->maxdepth);
    B->d_bot.resize(B->maxdepth);
    for (int d = 0; d < B->maxdepth && ok; ++d)
        ok = upload(B->h_all[d], &B->d_all[d]) && upload(B->h_mid[d], &B->d_mid[d]) &&
             upload(B->h_bot[d], &B->d_bot[d]);
    // stop test over the finest levels
    B->ptile = B->maxdepth > 1 && ptile_fits_all(B->h_mid[0]);
    B->d_norm = B->d_all.empty() ? nullptr : B->d_all[0];
    B->n_norm = count;
    std::vector<unsigned> first(n), nblk(n);
    unsigned acc = 0;
    for (int s = 0; s < count; ++s) {
        first[s] = acc;
        nblk[s] = seg_tiles(B->h_all[0][s], BK_NORM, kNormShape);
        acc += nblk[s];
    }
    B->norm_blocks = acc;
    std::vector<int *> valids(n);
    for (int i = 0; i < count; ++i) valids[i] = B->inst[i]->valid64;
    ok = ok && balloc(B, &B->partial, acc + 16) &&
         hipMemcpy(nf, first.data(), n * sizeof(unsigned), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(nbk, nblk.data(), n * sizeof(unsigned), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(B->d_valid, valids.data(), n * sizeof(int *), hipMemcpyHostToDevice) == hipSuccess &&
         hipHostMalloc((void **)&B->h_num, n * sizeof(int), 0) == hipSuccess &&
         hipHostMalloc((void **)&B->h_stats, 2 * n * sizeof(int), 0) == hipSuccess &&
         hipHostMalloc((void **)&B->h_res, 2 * n * sizeof(double), 0) == hipSuccess;
    if (!ok) {
        delete B;
        return bfail(nullptr, PFC_ERR_OOM, "allocation of batch tables failed");
    }
    *out = B;
    return PFC_OK;
}

pfc_status pfc_batch_destroy(pfc_batch *b) {
    if (!b) return PFC_ERR_INVALID_ARG;
    delete b;
    return PFC_OK;
}

static pfc_status check_inst(pfc_batch *b, int32_t i) {
    if (!b) return PFC_ERR_INVALID_ARG;
    if (i < 0 || i >= b->count) return bfail(b, PFC_ERR_INVALID_ARG, "instance index out of range");
    return PFC_OK;
}

pfc_status pfc_batch_set_state(pfc_batch *b, int32_t i, const double *phi_prev, const double *phi_cur,
                               const double *mu, const double *omega) {
    const pfc_status s = check_inst(b, i);
    if (s != PFC_OK) return s;
    if (!phi_prev || !phi_cur || !mu || !omega) return bfail(b, PFC_ERR_INVALID_ARG, "NULL pointer");
    const size_t bytes = b->inst[i]->lev[0].P * sizeof(double);
    (void)hipEventRecord(b->ev_in, b->user_stream);
    (void)hipStreamWaitEvent(b->stream, b->ev_in, 0);
    hipError_t e = hipMemcpyAsync(b->prev[i], phi_prev, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->cur[i], phi_cur, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->mu[i], mu, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->om[i], omega, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, PFC_ERR_HIP, hipGetErrorString(e));
    return PFC_OK;
}

pfc_status pfc_batch_get_state(pfc_batch *b, int32_t i, double *phi_prev, double *phi_cur, double *mu,
                               double *omega) {
    const pfc_status s = check_inst(b, i);
    if (s != PFC_OK) return s;
    const size_t bytes = b->inst[i]->lev[0].P * sizeof(double);
    hipError_t e = hipSuccess;
    if (phi_prev) e = hipMemcpyAsync(phi_prev, b->prev[i], bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess && phi_cur) e = hipMemcpyAsync(phi_cur, b->cur[i], bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess && mu) e = hipMemcpyAsync(mu, b->mu[i], bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess && omega) e = hipMemcpyAsync(omega, b->om[i], bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, PFC_ERR_HIP, hipGetErrorString(e));
    return PFC_OK;
}

pfc_status pfc_batch_run(pfc_batch *b, int32_t steps, pfc_step_info *infos) {
    if (!b || steps < 0) return PFC_ERR_INVALID_ARG;
    (void)hipEventRecord(b->ev_in, b->user_stream);
    (void)hipStreamWaitEvent(b->stream, b->ev_in, 0);
    pfc_status worst = PFC_OK;
    std::vector<pfc_step_info> one((size_t)b->count);
    for (int s = 0; s < steps; ++s) {
        const pfc_status st = run_step(b, one.data());
        if (st == PFC_ERR_HIP) return st;
        if (infos)
            for (int i = 0; i < b->count; ++i) infos[(size_t)i * steps + s] = one[i];
        if (st != PFC_OK && worst == PFC_OK) worst = st;
    }
    (void)hipEventRecord(b->ev_out, b->stream);
    (void)hipStreamWaitEvent(b->user_stream, b->ev_out, 0);
    if (worst != PFC_OK) bfail(b, worst, pfc_status_string(worst));
    return worst;
}

pfc_status pfc_batch_autotune(pfc_batch *b, const char *cache_path, int32_t *chosen) {
    if (!b) return PFC_ERR_INVALID_ARG;
    std::vector<int> sizes;
    for (auto *h : b->inst) sizes.push_back(h->lev[0].n);
    std::sort(sizes.begin(), sizes.end());
    std::ostringstream sig;
    sig << device_name() << "|" << sizes.size() << ":";
    for (size_t i = 0; i < sizes.size(); ++i) sig << (i ? "," : "") << sizes[i];
    static const char *kind_name[5] = {"smooth", "resid_restrict", "tau", "prolong", "coarse_err"};
    std::map<std::string, int> cache;
    if (cache_path) cache = read_cache(cache_path);
    bool changed = false;
    int dev = 0;
    (void)hipGetDevice(&dev);
    // make the working buffers hold a sane state to time on
    for (int i = 0; i < b->count; ++i) step_begin(b->inst[i], b->prev[i], b->cur[i], b->mu[i], b->om[i]);
    launch_batch_reset(b->stream, b->st, b->count, b->d_valid);
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    // a choice is stored as persistent * 100000 + threads * 100 + shape
    auto decode = [](int code, bool &ps, int &th, int &sh) {
        ps = code / 100000 != 0;
        th = (code % 100000) / 100;
        sh = code % 100;
        return (th == 64 || th == 128 || th == 256 || th == 512) && sh < kShapes &&
               (kTileMin << (sh % kWOpts)) >= th;
    };
    auto apply = [&](int kind, bool ps, int th, int sh) {
        b->persist[kind] = ps;
        b->threads[kind] = th;
        b->shape[kind] = sh;
        b->slots[kind] = ps ? (unsigned)batch_phase_slots(kind, th, dev) : 0u;
    };
    for (int kind = 0; kind < 5; ++kind) {
        const std::string key = sig.str() + "|" + kind_name[kind];
        auto it = cache.find(key);
        bool ps;
        int th, sh;
        if (it != cache.end() && decode(it->second, ps, th, sh)) {
            apply(kind, ps, th, sh);
            continue;
        }
        const int d = kind == BK_TAU ? 1 : 0;
        if (d >= b->maxdepth || b->h_mid[0].empty()) continue;
        const auto &segs = kind == BK_TAU ? b->h_all[1] : b->h_mid[0];
        BSeg *dsegs = kind == BK_TAU ? b->d_all[1] : b->d_mid[0];
        float best = 1e30f;
        int best_code = 256 * 100 + 2;
        // the interpolation is timed in the form the cycle runs
        const int pflag = b->cfg.nu2 >= 1 ? 1 : 0;
        for (int persistent = 0; persistent < 2; ++persistent)
            for (int thr : {64, 128, 256}) {
                const unsigned sl = persistent ? (unsigned)batch_phase_slots(kind, thr, dev) : 0u;
                if (persistent && sl == 0) continue;
                for (int sp = 0; sp < kShapes; ++sp) {
                    if ((kTileMin << (sp % kWOpts)) < thr) continue;
                    if (kind == BK_ERR && sp >= kWOpts) continue;  // one plane: Z is moot
                    const unsigned nt = tiles_of(segs, kind, sp);
                    auto run = [&](int rep) {
                        launch_batch(b->stream, kind, dsegs, (int)segs.size(), nt, sp, thr, sl,
                                     kind == BK_PROLONG ? pflag : rep & 1, 0);
                    };
                    for (int rep = 0; rep < 2; ++rep) run(rep);
                    (void)hipEventRecord(t0, b->stream);
                    for (int rep = 0; rep < 6; ++rep) run(rep);
                    (void)hipEventRecord(t1, b->stream);
                    if (hipEventSynchronize(t1) != hipSuccess) break;
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, t0, t1);
                    if (ms < best) {
                        best = ms;
                        best_code = persistent * 100000 + thr * 100 + sp;
                    }
                }
            }
        decode(best_code, ps, th, sh);
        apply(kind, ps, th, sh);
        cache[key] = best_code;
        changed = true;
    }
    // the finest depth's interpolation: the tuned coarse-error pass and
    // interpolation phase, or the column tiles (no coarse-error pass) with
    // 1, 2, 4 or 8 coarse planes per tile; stored as 99 or zi
    if (b->maxdepth > 1 && ptile_fits_all(b->h_mid[0])) {
        const std::string key = sig.str() + "|prolong_tile";
        auto it = cache.find(key);
        if (it != cache.end() && (it->second == 99 || (it->second >= 0 && it->second < kZOpts))) {
            b->ptile = it->second != 99;
            if (b->ptile) b->ptile_zi = it->second;
        } else {
            const auto &segs = b->h_mid[0];
            const int nseg = (int)segs.size(), pflag = b->cfg.nu2 >= 1 ? 1 : 0;
            float best = 1e30f;
            int best_code = 99;
            for (int code = -1; code < kZOpts; ++code) {
                auto run = [&]() {
                    if (code < 0) {
                        launch_batch(b->stream, BK_ERR, b->d_mid[0], nseg,
                                     tiles_of(segs, BK_ERR, b->shape[BK_ERR]), b->shape[BK_ERR],
                                     b->threads[BK_ERR], b->persist[BK_ERR] ? b->slots[BK_ERR] : 0u,
                                     0, 0);
                        launch_batch(b->stream, BK_PROLONG, b->d_mid[0], nseg,
                                     tiles_of(segs, BK_PROLONG, b->shape[BK_PROLONG]),
                                     b->shape[BK_PROLONG], b->threads[BK_PROLONG],
                                     b->persist[BK_PROLONG] ? b->slots[BK_PROLONG] : 0u, pflag, 0);
                    } else {
                        launch_batch_ptile(b->stream, b->d_mid[0], nseg, ptile_tiles(segs, code),
                                           code, pflag);
                    }
                };
                for (int rep = 0; rep < 2; ++rep) run();
                (void)hipEventRecord(t0, b->stream);
                for (int rep = 0; rep < 6; ++rep) run();
                (void)hipEventRecord(t1, b->stream);
                if (hipEventSynchronize(t1) != hipSuccess) break;
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, t0, t1);
                if (ms < best) {
                    best = ms;
                    best_code = code < 0 ? 99 : code;
                }
            }
            b->ptile = best_code != 99;
            if (b->ptile) b->ptile_zi = best_code;
            cache[key] = best_code;
            changed = true;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, PFC_ERR_HIP, hipGetErrorString(e));
    if (cache_path && changed) write_cache(cache_path, cache);
    b->graph_ready = false;  // recapture with the chosen tiles
    if (chosen)
        for (int k = 0; k < 5; ++k) {
            chosen[4 * k] = b->persist[k] ? 1 : 0;
            chosen[4 * k + 1] = b->threads[k];
            chosen[4 * k + 2] = kTileMin << (b->shape[k] % kWOpts);
            chosen[4 * k + 3] = 1 << (b->shape[k] / kWOpts);
            if (k == BK_PROLONG && b->ptile) {  // column tiles: 64 x-pairs of a plane, 2^zi coarse planes
                chosen[4 * k] = 0;
                chosen[4 * k + 1] = 4 * kBPX;
                chosen[4 * k + 2] = 4 * kBPX;
                chosen[4 * k + 3] = 1 << b->ptile_zi;
            }
        }
    return PFC_OK;
}

const char *pfc_batch_last_error(const pfc_batch *b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

}  // extern "C"

extern "C" pfc_status pfc_batch_init_state(pfc_batch *b, int32_t i, const double *phi0) {
    const pfc_status s = check_inst(b, i);
    if (s != PFC_OK) return s;
    if (!phi0) return bfail(b, PFC_ERR_INVALID_ARG, "NULL pointer");
    const size_t bytes = b->inst[i]->lev[0].P * sizeof(double);
    (void)hipEventRecord(b->ev_in, b->user_stream);
    (void)hipStreamWaitEvent(b->stream, b->ev_in, 0);
    hipError_t e = hipMemcpyAsync(b->prev[i], phi0, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b->cur[i], phi0, bytes, hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return bfail(b, PFC_ERR_HIP, hipGetErrorString(e));
    const pfc_status st = pfc_init_guess(b->inst[i], b->cur[i], b->mu[i], b->om[i]);
    if (st != PFC_OK) return bfail(b, st, pfc_last_error(b->inst[i]));
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, PFC_ERR_HIP, hipGetErrorString(e));
    return PFC_OK;
}
