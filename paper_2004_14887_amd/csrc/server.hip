// Serving runtime: continuous batching of many refined-mesh simulations of
// one (lattice, equilibrium order, storage) class on one GPU.
//
// Requests carry a configuration, initial fields and a step count.  A tick
// retires finished simulations (their probe series come back through pinned
// memory), admits queued ones while a slot and a first-fit block of the
// workspace arena are free (a simulation's footprint is exactly its
// dclbm_workspace_bytes), and replays one hipGraph that advances every
// resident simulation by steps_per_tick coarse steps.  The graph holds one
// persistent launch per level substep of the deepest admitted mesh (the
// "phases", in the depth-first order of the sub-cycling of Sec. 3.5) plus a
// tail launch for probes and step counts; the launches read device tables, so
// admission and retirement change tables, never the graph.  Each workgroup of
// a phase runs one workgroup of the single-simulation launch of one resident
// simulation, with that simulation's own arguments, so a result does not
// depend on what else is resident.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/dclbm.h"
#include "engine.hpp"

namespace dclbm {
namespace {

// First-fit allocator over [0, cap) in 256-byte granules, coalescing on free.
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> size
    size_t cap = 0;
    void reset(size_t c)
    {
        free_.clear();
        cap = c;
        if (c) free_[0] = c;
    }
    bool alloc(size_t n, size_t* off)
    {
        n = (size_t)round_up((int64_t)n, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n, o2 = it->first + n;
            free_.erase(it);
            if (rest) free_[o2] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (size_t)round_up((int64_t)n, 256);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const
    {
        size_t s = 0;
        for (auto& kv : free_) s += kv.second;
        return s;
    }
    size_t largest() const
    {
        size_t s = 0;
        for (auto& kv : free_) s = std::max(s, kv.second);
        return s;
    }
};

// Page-locked host buffers in power-of-two size classes, reused, freed with
// the server.  Initial fields wait in them between submission and admission,
// so that their upload is a true asynchronous copy.
struct PinnedPool {
    std::mutex mu;
    std::map<size_t, std::vector<void*>> free_;
    std::vector<void*> all;
    static size_t cls(size_t n)
    {
        size_t c = 1 << 16;
        while (c < n) c <<= 1;
        return c;
    }
    void* get(size_t n)
    {
        const size_t c = cls(n);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto& v = free_[c];
            if (!v.empty()) {
                void* p = v.back();
                v.pop_back();
                return p;
            }
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) return nullptr;
        std::lock_guard<std::mutex> lk(mu);
        all.push_back(p);
        return p;
    }
    void put(void* p, size_t n)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu);
        free_[cls(n)].push_back(p);
    }
    ~PinnedPool()
    {
        for (void* p : all) (void)hipHostFree(p);
    }
};

struct Request {
    uint64_t id = 0;
    int64_t steps = 0;
    std::unique_ptr<Sim> sim;
    double* fields = nullptr;                  // pinned: per level rho [n] then u [D][n]
    size_t fields_bytes = 0;
    std::vector<size_t> field_off;             // per level, in doubles
    size_t bytes = 0, off = 0;
    int state = DCLBM_REQ_QUEUED;
    int slot = -1;
    int64_t launched = 0;
    bool finishing = false;
    hipEvent_t done = nullptr;
    std::vector<double> probes;
    int n_probes = 0;
    int status = DCLBM_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t updates_per_step = 0;
    int bypassed = 0;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct Server {
    dclbm_server_config cfg{};
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int M = 0, NPH = 0, K = 1, G = 0, Gt = 0, depth = 2;
    int D = 2, Q = 9;
    std::vector<std::pair<int, int>> phases;   // (level, substep)
    // device tables
    SlotDev* d_slots = nullptr;
    LevelArgs* d_args = nullptr;   // [M][3][NPH]
    ProbeArgs* d_probe = nullptr;  // [M][2]
    int* d_ptab = nullptr;         // NPH phase tables + the tail list
    double* d_stage = nullptr;
    char* arena_base = nullptr;
    Arena arena;
    size_t ptab_ints = 0, res_stride = 0;
    // pinned host mirrors
    SlotDev* h_slots = nullptr;
    LevelArgs* h_args = nullptr;
    ProbeArgs* h_probe = nullptr;
    static constexpr int kTabs = 8;  // table upload buffers in rotation (more than ticks in flight)
    int* h_ptab[kTabs] = {};
    hipEvent_t ptab_ev[kTabs] = {};
    int ptab_cur = 0;
    char* h_res = nullptr;
    std::unique_ptr<Engine> eng;
    // one tick graph per grid size (powers of two); a tick replays the
    // smallest one covering the largest phase: a workgroup per tile measured
    // faster than fewer workgroups looping over the tiles
    std::vector<int> gsize;
    std::vector<hipGraph_t> graph;
    std::vector<hipGraphExec_t> gexec;
    int need = 0;         // largest phase of the current tables, in workgroups
    int last_grid = 0;
    std::mutex tick_mu;   // one tick at a time; the throttle waits under it only
    std::mutex mu;        // requests, queue, slots: held only for non-blocking work
    PinnedPool pinned;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> slot_req;
    uint64_t next_id = 1;
    bool dirty = false;
    std::deque<hipEvent_t> inflight;
    std::vector<hipEvent_t> pool;
    Clock::time_point origin;
    int64_t ticks = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - origin).count(); }

    hipEvent_t take_event()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }
};

namespace {

void dfs_phases(int l, int sub, int maxL, std::vector<std::pair<int, int>>& out)
{
    out.push_back({l, sub});
    if (l + 1 < maxL) {
        dfs_phases(l + 1, 1, maxL, out);
        dfs_phases(l + 1, 2, maxL, out);
    }
}

struct Layout {
    size_t slots, args, probe, ptab, stage, arena, total;
};

dclbm_status check_server_config(const dclbm_server_config* c)
{
    if (!c) return fail(DCLBM_ERR_INVALID, "null server configuration");
    if (c->abi_version != DCLBM_ABI_VERSION) return fail(DCLBM_ERR_INVALID, "abi_version %d != %d", c->abi_version, DCLBM_ABI_VERSION);
    if (c->lattice != DCLBM_D2Q9 && c->lattice != DCLBM_D3Q19) return fail(DCLBM_ERR_INVALID, "unknown lattice");
    if (c->precision < 0 || c->precision > 2) return fail(DCLBM_ERR_INVALID, "unknown precision");
    if (c->eq_order != 2 && c->eq_order != 3) return fail(DCLBM_ERR_INVALID, "eq_order must be 2 or 3");
    if (c->max_levels < 1 || c->max_levels > DCLBM_MAX_LEVELS) return fail(DCLBM_ERR_INVALID, "max_levels out of range");
    if (c->max_slots < 1 || c->max_slots > 1024) return fail(DCLBM_ERR_INVALID, "max_slots must be in [1, 1024]");
    if (c->steps_per_tick < 1 || c->steps_per_tick > 64) return fail(DCLBM_ERR_INVALID, "steps_per_tick must be in [1, 64]");
    if (c->max_probes < 0 || c->max_probes > 32) return fail(DCLBM_ERR_INVALID, "max_probes must be in [0, 32]");
    if (c->max_probe_steps < 1) return fail(DCLBM_ERR_INVALID, "max_probe_steps must be positive");
    if (c->max_level_nodes < 1) return fail(DCLBM_ERR_INVALID, "max_level_nodes must be positive");
    if (c->grid < 0 || c->grid % 8) return fail(DCLBM_ERR_INVALID, "grid must be 0 or a positive multiple of 8");
    return DCLBM_OK;
}

Layout layout(const dclbm_server_config& c, size_t bytes)
{
    const int M = c.max_slots;
    std::vector<std::pair<int, int>> ph;
    dfs_phases(0, 0, c.max_levels, ph);
    const size_t NPH = ph.size();
    const int D = c.lattice == DCLBM_D2Q9 ? 2 : 3;
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off = (size_t)round_up((int64_t)(off + std::max<size_t>(n, 1)), 256);
        return o;
    };
    L.slots = take(sizeof(SlotDev) * M);
    L.args = take(sizeof(LevelArgs) * M * 3 * NPH);
    L.probe = take(sizeof(ProbeArgs) * M * 2);
    L.ptab = take(sizeof(int) * ((NPH * (3 + 2 * (size_t)M)) + 1 + M));
    L.stage = take(sizeof(double) * (1 + D) * (size_t)c.max_level_nodes);
    L.arena = off;
    L.total = bytes;
    return L;
}

// Fill the pinned phase table from the resident set and enqueue its upload.
dclbm_status upload_tables(Server& sv)
{
    const int cur = sv.ptab_cur;
    // the copy from this buffer was enqueued kTabs uploads (so at least as
    // many ticks) ago, beyond the ticks allowed in flight: already complete
    HIPCHECK(hipEventSynchronize(sv.ptab_ev[cur]));
    int* t = sv.h_ptab[cur];
    const int M = sv.M, stride = 3 + 2 * M;
    std::vector<int> live;
    for (int k = 0; k < M; ++k) {
        const uint64_t id = sv.slot_req[k];
        if (!id) continue;
        const Request& r = *sv.reqs[id];
        if (r.state == DCLBM_REQ_RUNNING && !r.finishing) live.push_back(k);
    }
    for (int p = 0; p < sv.NPH; ++p) {
        int* pt = t + (size_t)p * stride;
        int n = 0, total = 0;
        for (int k : live) {
            const LevelArgs& a = sv.h_args[((size_t)k * 3 + 1) * sv.NPH + p];
            const Request& r = *sv.reqs[sv.slot_req[k]];
            if (sv.phases[p].first >= (int)r.sim->lv.size()) continue;
            const int na = a.nb_probe + a.nb_cap + 8 * a.seg_groups;
            pt[2 + n] = k;
            pt[2 + M + n] = total;
            total += (int)round_up(na, 8) + multi_groups(sv.D, a.tm.per);
            ++n;
        }
        pt[2 + M + n] = total;
        pt[0] = n;
        pt[1] = total;
    }
    int* tl = t + (size_t)sv.NPH * stride;
    tl[0] = (int)live.size();
    for (size_t i = 0; i < live.size(); ++i) tl[1 + i] = live[i];
    HIPCHECK(hipMemcpyAsync(sv.d_ptab, t, sv.ptab_ints * sizeof(int), hipMemcpyHostToDevice, sv.stream));
    HIPCHECK(hipEventRecord(sv.ptab_ev[cur], sv.stream));
    sv.ptab_cur = (cur + 1) % Server::kTabs;
    int need = 0;
    for (int p = 0; p < sv.NPH; ++p) need = std::max(need, t[(size_t)p * stride + 1]);
    sv.need = need;
    sv.dirty = false;
    return DCLBM_OK;
}

// Set the host state of a simulation for one of the three argument variants.
void set_variant(Sim& s, int var)
{
    for (size_t l = 0; l < s.lv.size(); ++l) {
        s.lv[l].parity = (l == 0 && var == 2) ? 1 : 0;
        s.lv[l].captures = var == 0 ? 0 : 2;
    }
}

dclbm_status admit(Server& sv, Request& r, int k, size_t off)
{
    Sim& s = *r.sim;
    dclbm_status st = sim_attach(s, sv.arena_base + off, r.bytes, sv.stream);
    if (st != DCLBM_OK) return st;
    for (size_t l = 0; l < s.lv.size(); ++l) {
        const size_t n = (size_t)s.lv[l].n_dense();
        HIPCHECK(hipMemcpyAsync(sv.d_stage, r.fields + r.field_off[l], (size_t)(1 + s.D) * n * sizeof(double),
                                hipMemcpyHostToDevice, sv.stream));
        s.eng->init(s, (int)l, sv.d_stage, sv.d_stage + n);
        if (s.lv[l].has_child) s.eng->ring_init(s, (int)l);
    }
    HIPCHECK(hipGetLastError());
    // argument tables of the three variants, mapped onto the server's phases
    LevelArgs* ha = sv.h_args + (size_t)k * 3 * sv.NPH;
    ProbeArgs* hp = sv.h_probe + (size_t)k * 2;
    memset(ha, 0, sizeof(LevelArgs) * 3 * sv.NPH);
    std::vector<StepRecord> rec;
    for (int var = 0; var < 3; ++var) {
        set_variant(s, var);
        ProbeArgs pa;
        record_coarse_step(s, rec, pa);
        if (var >= 1) hp[var - 1] = pa;
        size_t next = 0;
        for (int p = 0; p < sv.NPH; ++p) {
            if (sv.phases[p].first >= (int)s.lv.size()) continue;
            if (next >= rec.size() || rec[next].level != sv.phases[p].first || rec[next].substep != sv.phases[p].second)
                return fail(DCLBM_ERR_INVALID, "internal: phase order mismatch");
            ha[(size_t)var * sv.NPH + p] = rec[next].args;
            ha[(size_t)var * sv.NPH + p].nb_probe = 0;   // the tail launch samples the probes
            ha[(size_t)var * sv.NPH + p].seg_every = 0;  // virtual workgroups: segments first
            ++next;
        }
    }
    set_variant(s, 0);
    SlotDev& sd = sv.h_slots[k];
    sd.step = 0;
    sd.target = r.steps;
    sd.args = sv.d_args + (size_t)k * 3 * sv.NPH;
    sd.probe = sv.d_probe + (size_t)k * 2;
    sd.series = s.d_series;
    sd.counter = s.d_counter;
    HIPCHECK(hipMemcpyAsync(sv.d_args + (size_t)k * 3 * sv.NPH, ha, sizeof(LevelArgs) * 3 * sv.NPH,
                            hipMemcpyHostToDevice, sv.stream));
    HIPCHECK(hipMemcpyAsync(sv.d_probe + (size_t)k * 2, hp, sizeof(ProbeArgs) * 2, hipMemcpyHostToDevice, sv.stream));
    HIPCHECK(hipMemcpyAsync(sv.d_slots + k, &sd, sizeof(SlotDev), hipMemcpyHostToDevice, sv.stream));
    r.off = off;
    r.slot = k;
    r.state = DCLBM_REQ_RUNNING;
    r.t_admit = sv.now();
    sv.slot_req[k] = r.id;
    sv.dirty = true;
    return DCLBM_OK;
}

dclbm_status retire(Server& sv)
{
    for (int k = 0; k < sv.M; ++k) {
        const uint64_t id = sv.slot_req[k];
        if (!id) continue;
        Request& r = *sv.reqs[id];
        if (!r.finishing) continue;
        const hipError_t q = hipEventQuery(r.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return fail(DCLBM_ERR_HIP, "hipEventQuery: %s", hipGetErrorString(q));
        const char* res = sv.h_res + (size_t)k * sv.res_stride;
        const size_t nser = (size_t)r.steps * r.n_probes;
        r.probes.assign((const double*)res, (const double*)res + nser);
        int flags[2];
        memcpy(flags, res + (size_t)sv.cfg.max_probe_steps * std::max(1, sv.cfg.max_probes) * sizeof(double), sizeof(flags));
        r.status = (flags[0] & 2) ? DCLBM_ERR_UNSTABLE : (flags[0] & 1) ? DCLBM_ERR_NEWTON : DCLBM_OK;
        r.state = r.status == DCLBM_OK ? DCLBM_REQ_DONE : DCLBM_REQ_FAILED;
        r.t_done = sv.now();
        sv.arena.release(r.off, r.bytes);
        sv.slot_req[k] = 0;
        sv.pool.push_back(r.done);
        r.done = nullptr;
        r.sim.reset();
        sv.pinned.put(r.fields, r.fields_bytes);
        r.fields = nullptr;
    }
    return DCLBM_OK;
}

dclbm_status tick_locked(Server& sv)
{
    dclbm_status st = retire(sv);
    if (st != DCLBM_OK) return st;
    // admission: arrival order; later requests may pass one that does not fit
    // yet, until it has been passed 2 M times
    for (auto it = sv.queue.begin(); it != sv.queue.end();) {
        int k = -1;
        for (int j = 0; j < sv.M; ++j)
            if (!sv.slot_req[j]) {
                k = j;
                break;
            }
        if (k < 0) break;
        Request& r = *sv.reqs[*it];
        size_t off = 0;
        if (!sv.arena.alloc(r.bytes, &off)) {
            if (++r.bypassed > 2 * sv.M) break;
            ++it;
            continue;
        }
        st = admit(sv, r, k, off);
        if (st != DCLBM_OK) {
            sv.arena.release(off, r.bytes);
            sv.slot_req[k] = 0;
            r.state = DCLBM_REQ_FAILED;
            r.status = st;
            r.t_done = sv.now();
            sv.queue.erase(it);
            return st;
        }
        it = sv.queue.erase(it);
    }
    if (sv.dirty) {
        st = upload_tables(sv);
        if (st != DCLBM_OK) return st;
    }
    bool any = false;
    for (int k = 0; k < sv.M && !any; ++k)
        if (sv.slot_req[k] && !sv.reqs[sv.slot_req[k]]->finishing) any = true;
    if (!any) return DCLBM_OK;
    size_t gi = 0;
    while (gi + 1 < sv.gexec.size() && sv.gsize[gi] < sv.need) ++gi;
    HIPCHECK(hipGraphLaunch(sv.gexec[gi], sv.stream));
    sv.last_grid = sv.gsize[gi];
    ++sv.ticks;
    for (int k = 0; k < sv.M; ++k) {
        const uint64_t id = sv.slot_req[k];
        if (!id) continue;
        Request& r = *sv.reqs[id];
        if (r.finishing) continue;
        r.launched = std::min<int64_t>(r.steps, r.launched + sv.K);
        if (r.launched < r.steps) continue;
        // the last step is on the stream: bring the probe series and flags back
        char* res = sv.h_res + (size_t)k * sv.res_stride;
        const Sim& s = *r.sim;
        if (r.n_probes > 0)
            HIPCHECK(hipMemcpyAsync(res, s.d_series, (size_t)r.steps * r.n_probes * sizeof(double),
                                    hipMemcpyDeviceToHost, sv.stream));
        HIPCHECK(hipMemcpyAsync(res + (size_t)sv.cfg.max_probe_steps * std::max(1, sv.cfg.max_probes) * sizeof(double),
                                s.d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost, sv.stream));
        r.done = sv.take_event();
        if (!r.done) return fail(DCLBM_ERR_HIP, "hipEventCreate failed");
        HIPCHECK(hipEventRecord(r.done, sv.stream));
        r.finishing = true;
        sv.dirty = true;
    }
    hipEvent_t e = sv.take_event();
    if (!e) return fail(DCLBM_ERR_HIP, "hipEventCreate failed");
    HIPCHECK(hipEventRecord(e, sv.stream));
    sv.inflight.push_back(e);
    return DCLBM_OK;
}

void counts(Server& sv, int32_t* running, int32_t* queued)
{
    int nr = 0;
    for (int k = 0; k < sv.M; ++k)
        if (sv.slot_req[k]) ++nr;
    if (running) *running = nr;
    if (queued) *queued = (int32_t)sv.queue.size();
}

}  // namespace
}  // namespace dclbm

using namespace dclbm;

struct dclbm_server {
    Server s;
};

extern "C" {

dclbm_status dclbm_server_workspace_bytes(const dclbm_server_config* cfg, size_t arena_bytes, size_t* total)
{
    dclbm_status st = check_server_config(cfg);
    if (st != DCLBM_OK) return st;
    if (!total) return fail(DCLBM_ERR_INVALID, "null argument");
    const Layout L = layout(*cfg, 0);
    *total = L.arena + (size_t)round_up((int64_t)arena_bytes, 256);
    return DCLBM_OK;
}

dclbm_status dclbm_server_create(const dclbm_server_config* cfg, void* d_workspace, size_t bytes, void* stream,
                                 dclbm_server** out)
{
    dclbm_status st = check_server_config(cfg);
    if (st != DCLBM_OK) return st;
    if (!out) return fail(DCLBM_ERR_INVALID, "null argument");
    *out = nullptr;
    if (!stream) return fail(DCLBM_ERR_INVALID, "the server needs a non-default stream (its step is a graph)");
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) return fail(DCLBM_ERR_INVALID, "workspace must be 256-byte aligned");
    const Layout L = layout(*cfg, bytes);
    if (bytes <= L.arena) return fail(DCLBM_ERR_NOMEM, "workspace %zu bytes leaves no arena (tables need %zu)", bytes, L.arena);
    std::unique_ptr<dclbm_server> h(new dclbm_server());
    Server& sv = h->s;
    sv.cfg = *cfg;
    sv.stream = (hipStream_t)stream;
    sv.ws = (char*)d_workspace;
    sv.ws_bytes = bytes;
    sv.M = cfg->max_slots;
    dfs_phases(0, 0, cfg->max_levels, sv.phases);
    sv.NPH = (int)sv.phases.size();
    sv.K = cfg->steps_per_tick;
    sv.depth = cfg->max_inflight > 0 ? std::min(cfg->max_inflight, Server::kTabs - 2) : 2;
    sv.D = cfg->lattice == DCLBM_D2Q9 ? 2 : 3;
    sv.Q = cfg->lattice == DCLBM_D2Q9 ? 9 : 19;
    sv.d_slots = (SlotDev*)(sv.ws + L.slots);
    sv.d_args = (LevelArgs*)(sv.ws + L.args);
    sv.d_probe = (ProbeArgs*)(sv.ws + L.probe);
    sv.d_ptab = (int*)(sv.ws + L.ptab);
    sv.d_stage = (double*)(sv.ws + L.stage);
    sv.arena_base = sv.ws + L.arena;
    sv.arena.reset(bytes - L.arena);
    sv.ptab_ints = (size_t)sv.NPH * (3 + 2 * (size_t)sv.M) + 1 + sv.M;
    sv.res_stride = (size_t)round_up((int64_t)((size_t)cfg->max_probe_steps * std::max(1, cfg->max_probes) * sizeof(double) + 64), 256);
    sv.slot_req.assign(sv.M, 0);
    sv.eng.reset(make_engine(sv.D, cfg->eq_order, cfg->precision));
    // grids of the phase launches: a configured size, else powers of two
    // from 2048 to 262144 workgroups (beyond that a launch loops)
    if (cfg->grid > 0) {
        sv.gsize.push_back(cfg->grid);
    } else {
        for (int g = 2048; g <= (1 << 18); g *= 2) sv.gsize.push_back(g);
    }
    sv.G = sv.gsize.back();
    sv.Gt = std::min(sv.M, 256);
    HIPCHECK(hipHostMalloc((void**)&sv.h_slots, sizeof(SlotDev) * sv.M, hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void**)&sv.h_args, sizeof(LevelArgs) * sv.M * 3 * sv.NPH, hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void**)&sv.h_probe, sizeof(ProbeArgs) * sv.M * 2, hipHostMallocDefault));
    for (int b = 0; b < Server::kTabs; ++b) {
        HIPCHECK(hipHostMalloc((void**)&sv.h_ptab[b], sv.ptab_ints * sizeof(int), hipHostMallocDefault));
        memset(sv.h_ptab[b], 0, sv.ptab_ints * sizeof(int));
        HIPCHECK(hipEventCreateWithFlags(&sv.ptab_ev[b], hipEventDisableTiming));
        HIPCHECK(hipEventRecord(sv.ptab_ev[b], sv.stream));
    }
    HIPCHECK(hipHostMalloc((void**)&sv.h_res, sv.res_stride * sv.M, hipHostMallocDefault));
    memset(sv.h_slots, 0, sizeof(SlotDev) * sv.M);
    // empty tables on the device, then the graph of one tick
    HIPCHECK(hipMemcpyAsync(sv.d_ptab, sv.h_ptab[0], sv.ptab_ints * sizeof(int), hipMemcpyHostToDevice, sv.stream));
    HIPCHECK(hipMemcpyAsync(sv.d_slots, sv.h_slots, sizeof(SlotDev) * sv.M, hipMemcpyHostToDevice, sv.stream));
    HIPCHECK(hipStreamSynchronize(sv.stream));
    for (int G : sv.gsize) {
        HIPCHECK(hipStreamBeginCapture(sv.stream, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < sv.K; ++k) {
            for (int p = 0; p < sv.NPH; ++p) {
                MultiArgs m{sv.d_slots, sv.d_ptab, sv.M, sv.NPH, p};
                sv.eng->launch_multi(sv.stream, m, (unsigned)G);
            }
            MultiArgs m{sv.d_slots, sv.d_ptab, sv.M, sv.NPH, sv.NPH};
            sv.eng->launch_tail(sv.stream, m, (unsigned)sv.Gt);
        }
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(sv.stream, &g);
        if (ce != hipSuccess) return fail(DCLBM_ERR_HIP, "graph capture: %s", hipGetErrorString(ce));
        sv.graph.push_back(g);
        hipGraphExec_t ge = nullptr;
        HIPCHECK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        sv.gexec.push_back(ge);
    }
    sv.origin = Clock::now();
    *out = h.release();
    return DCLBM_OK;
}

dclbm_status dclbm_server_destroy(dclbm_server* h)
{
    if (!h) return DCLBM_OK;
    Server& sv = h->s;
    if (sv.stream) (void)hipStreamSynchronize(sv.stream);
    for (hipGraphExec_t e : sv.gexec) (void)hipGraphExecDestroy(e);
    for (hipGraph_t g : sv.graph) (void)hipGraphDestroy(g);
    for (auto& kv : sv.reqs)
        if (kv.second->done) (void)hipEventDestroy(kv.second->done);
    for (hipEvent_t e : sv.inflight) (void)hipEventDestroy(e);
    for (hipEvent_t e : sv.pool) (void)hipEventDestroy(e);
    for (int b = 0; b < Server::kTabs; ++b) {
        if (sv.ptab_ev[b]) (void)hipEventDestroy(sv.ptab_ev[b]);
        if (sv.h_ptab[b]) (void)hipHostFree(sv.h_ptab[b]);
    }
    if (sv.h_slots) (void)hipHostFree(sv.h_slots);
    if (sv.h_args) (void)hipHostFree(sv.h_args);
    if (sv.h_probe) (void)hipHostFree(sv.h_probe);
    if (sv.h_res) (void)hipHostFree(sv.h_res);
    delete h;
    return DCLBM_OK;
}

dclbm_status dclbm_server_submit(dclbm_server* h, const dclbm_config* cfg, int64_t steps, const double* const* h_rho,
                                 const double* const* h_u, uint64_t* id)
{
    if (!h || !cfg || !h_rho || !h_u || !id) return fail(DCLBM_ERR_INVALID, "null argument");
    Server& sv = h->s;
    const double t_arrival = sv.now();
    const dclbm_server_config& c = sv.cfg;
    if (cfg->lattice != c.lattice || cfg->precision != c.precision || cfg->eq_order != c.eq_order)
        return fail(DCLBM_ERR_INVALID, "request class (lattice, precision, eq_order) differs from the server's");
    if (cfg->n_levels > c.max_levels) return fail(DCLBM_ERR_INVALID, "request has %d levels, server admits %d", cfg->n_levels, c.max_levels);
    if (cfg->n_probes > c.max_probes) return fail(DCLBM_ERR_INVALID, "request has %d probes, server keeps %d", cfg->n_probes, c.max_probes);
    if (cfg->collision != DCLBM_BGK) return fail(DCLBM_ERR_INVALID, "the serving launches run the BGK collision only");
    if (cfg->sponge_cells > 0 && cfg->sponge_sigma > 0.0)
        return fail(DCLBM_ERR_INVALID, "the serving launches have no absorbing layer");
    if (cfg->h_region) return fail(DCLBM_ERR_INVALID, "the serving launches take box-shaped refined levels only");
    if (steps < 1 || steps > c.max_probe_steps) return fail(DCLBM_ERR_INVALID, "steps must be in [1, %lld]", (long long)c.max_probe_steps);
    std::unique_ptr<Request> r(new Request());
    r->steps = steps;
    r->sim.reset(new Sim());
    Sim& s = *r->sim;
    s.cfg = *cfg;
    s.cfg.probe_capacity = steps;
    dclbm_status st = build_geometry(s);
    if (st != DCLBM_OK) return st;
    s.cfg.h_probe_xyz = nullptr;
    for (auto& L : s.lv)
        if (L.n_dense() > c.max_level_nodes)
            return fail(DCLBM_ERR_INVALID, "a level has %lld nodes, server stages %lld", (long long)L.n_dense(), (long long)c.max_level_nodes);
    r->bytes = s.need_bytes;
    if (r->bytes > sv.arena.cap) return fail(DCLBM_ERR_NOMEM, "request needs %zu bytes, arena holds %zu", r->bytes, sv.arena.cap);
    r->n_probes = cfg->n_probes;
    size_t nd = 0;
    for (size_t l = 0; l < s.lv.size(); ++l) {
        if (!h_rho[l] || !h_u[l]) return fail(DCLBM_ERR_INVALID, "null field of level %zu", l);
        r->field_off.push_back(nd);
        nd += (size_t)(1 + s.D) * (size_t)s.lv[l].n_dense();
        r->updates_per_step += s.lv[l].n_active << l;
    }
    r->fields_bytes = nd * sizeof(double);
    r->fields = (double*)sv.pinned.get(r->fields_bytes);
    if (!r->fields) return fail(DCLBM_ERR_HIP, "hipHostMalloc of %zu bytes failed", r->fields_bytes);
    for (size_t l = 0; l < s.lv.size(); ++l) {
        const size_t n = (size_t)s.lv[l].n_dense();
        memcpy(r->fields + r->field_off[l], h_rho[l], n * sizeof(double));
        memcpy(r->fields + r->field_off[l] + n, h_u[l], (size_t)s.D * n * sizeof(double));
    }
    std::lock_guard<std::mutex> lk(sv.mu);
    r->id = sv.next_id++;
    r->t_submit = t_arrival;
    *id = r->id;
    sv.queue.push_back(r->id);
    sv.reqs[r->id] = std::move(r);
    return DCLBM_OK;
}

dclbm_status dclbm_server_tick(dclbm_server* h, int32_t* n_running, int32_t* n_queued)
{
    if (!h) return fail(DCLBM_ERR_INVALID, "null server");
    Server& sv = h->s;
    std::lock_guard<std::mutex> tk(sv.tick_mu);
    // bound the ticks queued on the stream, without holding the request lock
    // (a submitting thread must not wait for the GPU)
    while ((int)sv.inflight.size() >= sv.depth) {
        HIPCHECK(hipEventSynchronize(sv.inflight.front()));
        sv.pool.push_back(sv.inflight.front());
        sv.inflight.pop_front();
    }
    std::lock_guard<std::mutex> lk(sv.mu);
    dclbm_status st = tick_locked(sv);
    counts(sv, n_running, n_queued);
    return st;
}

dclbm_status dclbm_server_poll(dclbm_server* h, uint64_t id, int32_t* state)
{
    if (!h || !state) return fail(DCLBM_ERR_INVALID, "null argument");
    Server& sv = h->s;
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.reqs.find(id);
    if (it == sv.reqs.end()) return fail(DCLBM_ERR_INVALID, "unknown request %llu", (unsigned long long)id);
    *state = it->second->state;
    return DCLBM_OK;
}

dclbm_status dclbm_server_result(dclbm_server* h, uint64_t id, double* h_probes, int64_t* n_steps,
                                 dclbm_request_info* info)
{
    if (!h) return fail(DCLBM_ERR_INVALID, "null server");
    Server& sv = h->s;
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.reqs.find(id);
    if (it == sv.reqs.end()) return fail(DCLBM_ERR_INVALID, "unknown request %llu", (unsigned long long)id);
    const Request& r = *it->second;
    if (info) {
        info->t_submit = r.t_submit;
        info->t_admit = r.t_admit;
        info->t_done = r.t_done;
        info->steps = r.steps;
        info->updates = r.updates_per_step * r.steps;
        info->workspace_bytes = (int64_t)r.bytes;
        info->slot = r.slot;
        info->state = r.state;
        info->status = r.status;
        info->n_probes = r.n_probes;
    }
    if (r.state != DCLBM_REQ_DONE && r.state != DCLBM_REQ_FAILED) {
        if (n_steps) *n_steps = 0;
        return DCLBM_ERR_BUSY;
    }
    if (n_steps) *n_steps = r.state == DCLBM_REQ_DONE ? r.steps : 0;
    if (h_probes && r.state == DCLBM_REQ_DONE) memcpy(h_probes, r.probes.data(), r.probes.size() * sizeof(double));
    return (dclbm_status)r.status;
}

dclbm_status dclbm_server_release(dclbm_server* h, uint64_t id)
{
    if (!h) return fail(DCLBM_ERR_INVALID, "null server");
    Server& sv = h->s;
    std::lock_guard<std::mutex> lk(sv.mu);
    auto it = sv.reqs.find(id);
    if (it == sv.reqs.end()) return fail(DCLBM_ERR_INVALID, "unknown request %llu", (unsigned long long)id);
    if (it->second->state != DCLBM_REQ_DONE && it->second->state != DCLBM_REQ_FAILED)
        return fail(DCLBM_ERR_BUSY, "request %llu has not finished", (unsigned long long)id);
    sv.reqs.erase(it);
    return DCLBM_OK;
}

dclbm_status dclbm_server_stats(dclbm_server* h, dclbm_server_info* out)
{
    if (!h || !out) return fail(DCLBM_ERR_INVALID, "null argument");
    Server& sv = h->s;
    std::lock_guard<std::mutex> lk(sv.mu);
    counts(sv, &out->running, &out->queued);
    out->ticks = sv.ticks;
    out->arena_bytes = (int64_t)sv.arena.cap;
    out->arena_free = (int64_t)sv.arena.free_bytes();
    out->arena_largest_free = (int64_t)sv.arena.largest();
    out->grid = sv.last_grid;
    out->n_phases = sv.NPH;
    return DCLBM_OK;
}

}  // extern "C"
