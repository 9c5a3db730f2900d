// Host-side state of one simulation and the type-erased engine that launches
// its kernels; shared by the single-simulation C ABI and the serving runtime.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dclbm.h"
#include "kernels.hpp"

namespace dclbm {

extern thread_local std::string g_err;
dclbm_status fail(dclbm_status s, const char* fmt, ...);

#define HIPCHECK(expr)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(DCLBM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct HostLevel {
    int nx = 1, ny = 1, nz = 1, nxb = 1;
    int xsh = 6;                // row blocks of 2^xsh nodes
    int64_t elems = 0;          // storage elements per buffer (Q per node slot, 64-node row blocks)
    int periodic = 0, boundary = 0, has_child = 0;
    int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
    int plo[3] = {0, 0, 0};
    double ur[3] = {0.0, 0.0, 0.0};   // reference velocity of the carried variable (shifted forms)
    float k1[19] = {}, k2[19] = {};   // per-direction constants of the shifted equilibrium
    int xface = 0;                    // x-face nodes live in xf[2] (3-D refined levels)
    int64_t xf_elems = 0;
    double tau = 0.0;
    int64_t n_active = 0;
    // interface with the parent (level >= 1)
    std::vector<int4> tf_meta, ie_meta;   // co-located (x,y,z,Gamma=R mask), hanging (x,y,z,missing mask)
    std::vector<int> tfmap;               // co-located index at fine coords (2a,2b,2c), -1 elsewhere
    int mx = 1, my = 1, mz = 1;
    std::vector<int4> seg_info;           // (tf_off, tf_cnt, ie_off, ie_cnt)
    std::vector<int> seg_tf, seg_ie, seg_sten;
    std::vector<int4> seg_tfm;   // tf_meta of each seg_tf entry (segment order)
    std::vector<int> ie_tf;               // [16][n_ie] co-located indices of each hanging node's stencil
    // interface with the child (coarse co-located nodes, child's order)
    std::vector<int4> tfc_meta;
    // workspace offsets
    int64_t off_f[2] = {0, 0}, off_xf[2] = {0, 0}, off_tf = 0, off_ie = 0, off_X = 0, off_tfc = 0, off_H = 0, off_seg_info = 0,
            off_seg_tf = 0, off_seg_ie = 0, off_seg_sten = 0, off_seg_tfm = 0;
    int64_t off_M = 0, off_Mring = 0, off_ie_tf = 0;   // H-RR
    // refined region of level-0 cells (level 1 and its parent): node classes
    std::vector<uint8_t> cls;
    int64_t off_cls = 0;
    uint8_t* d_cls = nullptr;
    // device pointers
    void* f[2] = {nullptr, nullptr};
    void* xf[2] = {nullptr, nullptr};
    int64_t off_xn[2] = {0, 0};
    void* xn[2] = {nullptr, nullptr};   // BGK: second copies of what the x faces pull from the next planes
    int4 *d_tf = nullptr, *d_ie = nullptr, *d_tfc = nullptr, *d_seg_info = nullptr;
    int *d_seg_tf = nullptr, *d_seg_ie = nullptr, *d_seg_sten = nullptr;
    int4* d_seg_tfm = nullptr;
    void *X = nullptr, *H = nullptr;
    // H-RR: (drho, du) of every node [4][n]; its post-streaming values at the
    // coarse times t-dt, t, t+dt [3][4][n] (level with a child); gradients of
    // the co-located nodes [18][n_tf]; hanging-node stencils [16][n_ie]
    void *d_M = nullptr, *d_Mring = nullptr;
    int* d_ie_tf = nullptr;
    int parity = 0;
    int64_t captures = 0;

    LevelDev dev() const
    {
        LevelDev g;
        g.nx = nx;
        g.ny = ny;
        g.nz = nz;
        g.nxb = nxb;
        g.xsh = xsh;
        g.periodic = periodic;
        g.boundary = boundary;
        g.has_child = has_child;
        for (int a = 0; a < 3; ++a) {
            g.clo[a] = clo[a];
            g.chi[a] = chi[a];
            g.ur[a] = ur[a];
        }
        for (int i = 0; i < 19; ++i) {
            g.k1[i] = k1[i];
            g.k2[i] = k2[i];
        }
        g.xface = xface;
        g.xf[0] = xf[0];
        g.xf[1] = xf[1];
        g.xn[0] = xn[0];
        g.xn[1] = xn[1];
        g.cls = d_cls;
        return g;
    }
    int64_t n_dense() const { return (int64_t)nx * ny * nz; }
    // Bulk tiles: 64 x 4 nodes, covering the nodes that can be bulk nodes
    // (a refined level's own boundary is all interface, so its last x tile
    // or row group may hold none: a 257-node row needs 4 tiles, not 5)
    TileMap tiles() const
    {
        TileMap m;
        m.tx = ((boundary ? nx - 2 : nx - 1) >> 6) + 1;
        m.ty = ((boundary ? ny - 2 : ny - 1) >> 2) + 1;
        m.nrows = m.ty * nz;
        m.per = m.tx * ((m.nrows + 7) / 8);
        m.blk = 1;
        return m;
    }
    int64_t elem0(int Q, int x, int y, int z) const
    {
        return (((int64_t)z * ny + y) * nxb + (x >> xsh)) * ((int64_t)Q << xsh) + (x & ((1 << xsh) - 1));
    }
};

struct Sim;

// Type-erased launcher set for one (lattice, equilibrium order, storage form).
struct Engine {
    virtual ~Engine() {}
    virtual void level_step(Sim& s, int l, int substep, int first) = 0;
    // H-RR on a refined mesh: a level substep opens (macroscopic fields,
    // interface completion) before its child's substeps and closes
    // (gradients, collision of every node) after them
    virtual void hrr_open(Sim& s, int l, int substep, int first) = 0;
    virtual void hrr_close(Sim& s, int l, int substep, int first) = 0;
    // the three slots of level l's macroscopic-field ring from its initial fields
    virtual void hrr_ring_init(Sim& s, int l, const double* rho, const double* u) = 0;
    // the absorbing layer on level 0's current state
    virtual void sponge(Sim& s) = 0;
    virtual void probe(Sim& s) = 0;
    virtual void init(Sim& s, int l, const double* rho, const double* u) = 0;
    virtual void ring_init(Sim& s, int l) = 0;
    virtual void fill_nan(Sim& s) = 0;
    virtual void read(Sim& s, int l, double* f, double* rho, double* u) = 0;
    virtual void read_shared(Sim& s, int l, double* out) = 0;
    virtual void balance(Sim& s, int l, double* partial, int nblocks) = 0;
    // serving: one phase of the resident simulations, and the step tail
    virtual void launch_multi(hipStream_t st, const MultiArgs& m, unsigned grid) = 0;
    virtual void launch_tail(hipStream_t st, const MultiArgs& m, unsigned grid) = 0;
    // graph construction: the kernel node(s) of one recorded level substep,
    // each depending on `deps`; on return `deps` holds the new node(s)
    virtual hipError_t add_nodes(Sim& s, hipGraph_t g, const struct StepRecord& r, std::vector<hipGraphNode_t>& deps) = 0;
};

struct ProbeLoc {
    int level;
    int64_t off;   // element of direction 0 in the main buffer
    int x, y, z;   // node in level coordinates
};

struct Sim {
    dclbm_config cfg;
    int D = 2, Q = 9, P = 0, EQ = 2;
    size_t tsize = 8, rsize = 8;   // storage and arithmetic element sizes
    std::vector<HostLevel> lv;
    std::vector<ProbeLoc> probes;
    std::vector<int32_t> probe_xyz;
    hipStream_t stream = nullptr;
    // second stream and fork/join events of the split 3-D FP16 level substeps
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0, need_bytes = 0;
    int64_t off_series = 0, off_counter = 0, off_flags = 0, off_partial = 0, off_bal = 0, off_probe_args = 0;
    int64_t off_psum = 0;
    double* d_series = nullptr;
    int64_t* d_counter = nullptr;     // [0] steps sampled by the probes, [1] coarse steps started,
                                      // [2, 3] the window of the running sums, [4] steps summed
    double* d_psum = nullptr;         // running sums of the probes [3][n_probes]
    ProbeArgs* d_probe_args = nullptr; // [2] by level-0 parity
    std::vector<ProbeArgs> h_probe_args;
    int* d_flags = nullptr;
    double* d_partial = nullptr;
    double* d_bal = nullptr;
    int partial_blocks = 1024;
    int hrr = 0;                      // H-RR collision
    int sponge_w = 0;                 // absorbing layer on level 0: width in cells (0: none)
    double sponge_sigma = 0.0;
    int device = -1;                  // device current at creation
    double* d_scratch = nullptr;      // that device's static scratch array (dclbm_balance_static)
    std::unique_ptr<Engine> eng;
    int split_mode = -1;              // 3-D FP16 split substeps: -1 by weight, 0 never, 1 wherever segments exist
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    int64_t steps_done = 0;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[DCLBM_MAX_LEVELS];
    double tms[DCLBM_MAX_LEVELS] = {0, 0, 0, 0};
    int64_t tlaunch[DCLBM_MAX_LEVELS] = {0, 0, 0, 0};
    double newton_tol = 1e-12;
    int newton_maxit = 20;
    // first failed HIP call of the launch sequence of a step (event records
    // and waits of the split substeps, timing events); checked after the
    // eager launches or the capture of every coarse step
    hipError_t launch_err = hipSuccess;
    void note(hipError_t e)
    {
        if (launch_err == hipSuccess && e != hipSuccess) launch_err = e;
    }

    template <typename T>
    T* at(int64_t off) const
    {
        return reinterpret_cast<T*>(ws + off);
    }

    ~Sim()
    {
        if (side) {
            (void)hipStreamSynchronize(side);
            (void)hipStreamDestroy(side);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
    }
};

template <typename V>
inline hipError_t upload(Sim& s, void* dst, const std::vector<V>& v)
{
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, s.stream);
}


// Geometry, classification, interface tables and workspace layout of a
// configuration (host only, no device calls).
dclbm_status build_geometry(Sim& s);
// Point the simulation at its workspace, upload its tables, create its
// engine, fill the state with NaN and clear its counters; enqueued on the
// stream, no synchronisation.
dclbm_status sim_attach(Sim& s, void* d_workspace, size_t bytes, hipStream_t stream);
// Arguments of one level substep from the current host state, and its grid.
LevelArgs level_args(const Sim& s, int l, int substep, int first, unsigned* grid);
// Probe arguments for the current host state (after a coarse step).
ProbeArgs probe_args(const Sim& s);
// The level substeps of one coarse step in launch order (level, substep,
// arguments, grid) from the current host state, and the probe arguments of
// the state after it.  Advances the host state like a launched step.
struct StepRecord {
    int level, substep;
    LevelArgs args;
    unsigned grid;
};
void record_coarse_step(Sim& s, std::vector<StepRecord>& out, ProbeArgs& probe_after);
Engine* make_engine(int D, int EQ, int P);

}  // namespace dclbm
