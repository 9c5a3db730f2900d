// Host driver and C ABI of the direct-coupling refined LBM library (gfx950).
//
// A simulation is a periodic coarse level and up to three nested refined
// boxes.  The host classifies the interface nodes once (co-located nodes with
// their (Gamma, gamma) couples of Sec. 3.4, hanging nodes with their missing
// directions), cuts each refined level's interface into segments (tiles of
// the interface line or face, with the co-located halo their 4-point stencils
// need), carves the caller's workspace, and drives the recursive sub-cycling
// of Sec. 3.5: each level makes two substeps per step of its parent
// (Sec. 3.1, acoustic scaling).  A level substep is one kernel launch; after
// the first coarse step each coarse step is replayed as one hipGraph (two
// graphs, one per A/B parity of level 0).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dclbm.h"
#include "engine.hpp"

namespace dclbm {

thread_local std::string g_err;

dclbm_status fail(dclbm_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

// ------------------------------------------------------------------ static scratch
// Block partial sums of dclbm_balance_static, for callers that cannot
// allocate: every level's kBalanceBlocks partials (5 doubles each), then the
// per-level totals.  Each GPU holds its own copy of the array (about 160 KB)
// until the process ends; host code uses the address that
// hipGetSymbolAddress returned for the current device, never the array's
// name.  Calls on one GPU share the array: calls that overlap on one GPU
// race.
constexpr int kBalanceBlocks = 1024;   // partial blocks per level (the same as dclbm_balance)
constexpr int64_t kScratchDoubles = (int64_t)DCLBM_MAX_LEVELS * kBalanceBlocks * 5 + DCLBM_MAX_LEVELS * 5;
__device__ __align__(256) double scratch[kScratchDoubles];

static std::mutex g_scratch_mu;
static std::map<int, double*> g_scratch_ptr;   // device -> device address of its scratch array

// Device address of the current device's scratch array, resolved once per
// device (at dclbm_create, with the simulation's device current).
static dclbm_status scratch_address(int device, double** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return DCLBM_OK;
    }
    double* p = nullptr;
    HIPCHECK(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(DCLBM_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = p;
    *out = p;
    return DCLBM_OK;
}

// Sum of the per-level totals (level order, from zero, as dclbm_balance sums
// them on the host) into the caller's five doubles.
static __global__ __launch_bounds__(64) void k_balance_levels(const double* __restrict__ totals, int n_levels,
                                                              double* __restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= 5) return;
    double v = 0.0;
    for (int l = 0; l < n_levels; ++l) v += totals[5 * l + k];
    out[k] = v;
}

// ------------------------------------------------------------------ launch arguments
// 3-D: one group of 8 segment workgroups after every kSegEvery3D groups of
// bulk workgroups (fewer where the bulk is small), so that the segments of a
// refined level's faces spread over the front third of its launch.
static constexpr int kSegEvery3D = 32;

LevelArgs level_args(const Sim& s, int l, int substep, int first, unsigned* grid)
{
    const HostLevel& L = s.lv[l];
    LevelArgs a;
    memset(&a, 0, sizeof(a));
    a.g = L.dev();
    a.src = L.f[L.parity];
    a.par = L.parity;
    a.dst = L.f[L.parity ^ 1];
    a.keep = 1.0 - 1.0 / L.tau;
    a.tm = L.tiles();
    a.flags = s.d_flags;
    if (L.has_child) {
        a.n_cap = (int)L.tfc_meta.size();
        a.nb_cap = (a.n_cap + kBlock - 1) / kBlock;
        a.cap_meta = L.d_tfc;
        a.H_own = L.H;
    }
    if (l > 0) {
        const HostLevel& Pn = s.lv[l - 1];
        a.nb_seg = (int)L.seg_info.size();
        a.seg_info = L.d_seg_info;
        a.seg_tf = L.d_seg_tf;
        a.seg_tfm = L.d_seg_tfm;
        a.seg_ie = L.d_seg_ie;
        a.seg_sten = L.d_seg_sten;
        a.n_ie = (int)L.ie_meta.size();
        a.tf_meta = L.d_tf;
        a.ie_meta = L.d_ie;
        a.n_tf = (int)L.tf_meta.size();
        a.H_parent = Pn.H;
        a.X = L.X;
        a.substep = substep;
        a.first = first;
        a.maxit = s.newton_maxit;
        a.Rfac = L.tau / (2.0 * Pn.tau);
        a.tol = s.newton_tol;
        a.gp = Pn.dev();
        a.dst_parent = Pn.f[Pn.parity ^ 1];
        a.tfc_meta = Pn.d_tfc;
        a.keep_parent = 1.0 - 1.0 / Pn.tau;
    }
    // Segment workgroups go ahead of the bulk: their latency-bound work then
    // overlaps the bulk tiles, and none of it lands in the launch's tail (in
    // 2-D all first; in 3-D interleaved over the front, see seg_every below).
    a.seg_groups = (a.nb_seg + 7) / 8;
    if (l == 0) {
        a.nb_probe = 1;
        a.probe = s.d_probe_args + L.parity;
        a.series = s.d_series;
        a.counter = s.d_counter;
        a.psums = s.d_psum;
    }
    // the tiles per bulk workgroup of the kernel this launch uses (with or
    // without the segment role; a split substep sizes its bulk kernel itself)
    const int nbg = bulk_groups(a.tm.per, bulk_k(s.D, s.P, a.nb_seg > 0)) / 8;
    if (s.D == 3 && a.seg_groups > 0) a.seg_every = std::min(kSegEvery3D, nbg / a.seg_groups);
    *grid = (unsigned)(a.nb_probe + a.nb_cap + 8 * a.seg_groups + 8 * nbg);
    return a;
}

ProbeArgs probe_args(const Sim& s)
{
    ProbeArgs a;
    memset(&a, 0, sizeof(a));
    a.n = (int)s.probes.size();
    a.capacity = s.cfg.probe_capacity;
    for (int p = 0; p < a.n; ++p) {
        const ProbeLoc& pl = s.probes[p];
        const HostLevel& L = s.lv[pl.level];
        if (L.xface && (pl.x == 0 || pl.x == L.nx - 1)) {
            a.buf[p] = L.xf[L.parity];
            a.off[p] = ((int64_t)(pl.x == 0 ? 0 : 1) * s.Q * L.nz + pl.z) * L.ny + pl.y;
            a.stride[p] = (int64_t)L.nz * L.ny;
        } else {
            a.buf[p] = L.f[L.parity];
            a.off[p] = pl.off;
            a.stride[p] = (int64_t)1 << L.xsh;
        }
    }
    return a;
}

// ------------------------------------------------------------------ engines
// One factory per (lattice, equilibrium order, storage form) class, each
// compiled from engine_inst.hip in its own translation unit.
#define DCLBM_DECLARE(D, EQ)                \
    Engine* make_engine_d##D##EQ##_0();     \
    Engine* make_engine_d##D##EQ##_1();     \
    Engine* make_engine_d##D##EQ##_2();
DCLBM_DECLARE(2, 2)
DCLBM_DECLARE(2, 3)
DCLBM_DECLARE(3, 2)
DCLBM_DECLARE(3, 3)
#undef DCLBM_DECLARE

Engine* make_engine(int D, int EQ, int P)
{
    static Engine* (*const table[2][2][3])() = {
        {{make_engine_d22_0, make_engine_d22_1, make_engine_d22_2},
         {make_engine_d23_0, make_engine_d23_1, make_engine_d23_2}},
        {{make_engine_d32_0, make_engine_d32_1, make_engine_d32_2},
         {make_engine_d33_0, make_engine_d33_1, make_engine_d33_2}}};
    return table[D == 3][EQ == 3][P]();
}

// ------------------------------------------------------------------ geometry
static const int kCx2[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
static const int kCy2[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};

static void dirs(int D, int i, int c[3])
{
    if (D == 2) {
        c[0] = kCx2[i];
        c[1] = kCy2[i];
        c[2] = 0;
    } else {
        c[0] = Lat<3>::cx[i];
        c[1] = Lat<3>::cy[i];
        c[2] = Lat<3>::cz[i];
    }
}

// Stencil positions of a hanging node along axis a (odd coordinate k, line 0..N).
static void stencil_positions(int k, int N, int pos[4])
{
    if (k == 1) {
        pos[0] = 0; pos[1] = 2; pos[2] = 4; pos[3] = 6;
    } else if (k == N - 1) {
        pos[0] = N; pos[1] = N - 2; pos[2] = N - 4; pos[3] = N - 6;
    } else {
        pos[0] = k - 3; pos[1] = k - 1; pos[2] = k + 1; pos[3] = k + 3;
    }
}

// Points and weight type of hanging node k on a refined region's boundary
// (2-D, one odd coordinate), along its odd axis, from the co-located nodes
// present on that line: k-3, k-1, k+1, k+3 if all are (type 1), else k-1,
// k+1, k+3, k+5 or k+1, k-1, k-3, k-5 (type 2), else k-1, k+1 (type 3, the
// last two points repeat k-1 with zero weight).  On a box face this gives
// the box line's stencils.  Returns the type, 0 if none fits.
static int region_stencil(const HostLevel& L, const int k[3], int pos[4])
{
    const int a = (k[0] & 1) ? 0 : 1;
    auto tf = [&](int o) {
        int q[2] = {k[0], k[1]};
        q[a] += o;
        return q[0] >= 0 && q[1] >= 0 && q[0] < L.nx && q[1] < L.ny &&
               L.cls[(size_t)q[1] * L.nx + q[0]] == kClsTf;
    };
    if (tf(-3) && tf(-1) && tf(1) && tf(3)) {
        pos[0] = k[a] - 3; pos[1] = k[a] - 1; pos[2] = k[a] + 1; pos[3] = k[a] + 3;
        return 1;
    }
    for (int sg = 1; sg >= -1; sg -= 2)
        if (tf(-sg) && tf(sg) && tf(3 * sg) && tf(5 * sg)) {
            pos[0] = k[a] - sg; pos[1] = k[a] + sg; pos[2] = k[a] + 3 * sg; pos[3] = k[a] + 5 * sg;
            return 2;
        }
    if (tf(-1) && tf(1)) {
        pos[0] = k[a] - 1; pos[1] = k[a] + 1; pos[2] = k[a] - 1; pos[3] = k[a] - 1;
        return 3;
    }
    return 0;
}

// Segment of a boundary node: the face it is assigned to (the first axis on
// which it sits on the box boundary, and the side) and its tile within that
// face: 256 positions along the line in 2-D, 16 x 16 in 3-D.
static std::tuple<int, int, int> segment_key(int D, const int k[3], const int n[3])
{
    int face = -1;
    for (int a = 0; a < D && face < 0; ++a) {
        if (k[a] == 0) face = 2 * a;
        else if (k[a] == n[a] - 1) face = 2 * a + 1;
    }
    // tiles of 256 positions on a 2-D interface line; 32 x 20 positions on a
    // 3-D face, the longer side along the face's faster storage axis (160
    // own co-located nodes plus an 87-node stencil halo fit one workgroup)
    const int ax = face / 2;
    int t[2] = {0, 0}, no = 0;
    const int T[2] = {D == 2 ? 256 : 32, D == 2 ? 16 : 20};
    for (int a = 0; a < D; ++a)
        if (a != ax) {
            t[no] = k[a] / T[no];
            ++no;
        }
    return std::make_tuple(face, t[0], t[1]);
}

static dclbm_status build_segments(Sim& s, int l)
{
    const int D = s.D;
    HostLevel& L = s.lv[l];
    const int n[3] = {L.nx, L.ny, L.nz};
    const bool region = !L.cls.empty();
    // a region's interface is grouped by 64 x 8 tiles of the level
    auto key = [&](const int k[3]) {
        return region ? std::make_tuple(7, k[1] / 8, k[0] / 64) : segment_key(D, k, n);
    };
    struct Seg {
        std::vector<int> own, ie;
    };
    std::map<std::tuple<int, int, int>, Seg> segs;
    for (size_t t = 0; t < L.tf_meta.size(); ++t) {
        const int k[3] = {L.tf_meta[t].x, L.tf_meta[t].y, L.tf_meta[t].z};
        segs[key(k)].own.push_back((int)t);
    }
    for (size_t e = 0; e < L.ie_meta.size(); ++e) {
        const int k[3] = {L.ie_meta[e].x, L.ie_meta[e].y, L.ie_meta[e].z};
        segs[key(k)].ie.push_back((int)e);
    }
    const size_t nie = L.ie_meta.size();
    L.seg_info.clear();
    L.seg_tf.clear();
    L.seg_tfm.clear();
    L.seg_ie.clear();
    L.seg_sten.assign(16 * nie, 0);
    L.ie_tf.assign(16 * nie, 0);
    const int TFM = D == 2 ? SegLimits<2>::TF : SegLimits<3>::TF;
    for (auto& kv : segs) {
        Seg& sg = kv.second;
        std::map<int, int> local;   // co-located index -> local slot
        std::vector<int> list;
        for (int t : sg.own) {
            local[t] = (int)list.size();
            list.push_back(t | (1 << 30));
        }
        const int ie_off = (int)L.seg_ie.size();
        for (int e : sg.ie) {
            const int4& m = L.ie_meta[e];
            const int k[3] = {m.x, m.y, m.z};
            int pos[3][4], odd[2] = {-1, -1}, no = 0;
            for (int a = 0; a < 3; ++a) {
                pos[a][0] = pos[a][1] = pos[a][2] = pos[a][3] = k[a];
                if (a < D && (k[a] & 1)) {
                    if (region) {
                        if (!region_stencil(L, k, pos[a]))
                            return fail(DCLBM_ERR_INVALID, "level %d hanging node (%d,%d): no co-located nodes on its line",
                                        l, k[0], k[1]);
                    } else {
                        if (n[a] - 1 < 6)
                            return fail(DCLBM_ERR_INVALID, "level %d box too small for the 4-point stencil", l);
                        stencil_positions(k[a], n[a] - 1, pos[a]);
                    }
                    odd[no++] = a;
                }
            }
            if (no < 1 || no > 2) return fail(DCLBM_ERR_INVALID, "level %d: hanging node with %d odd coordinates", l, no);
            const int nq = no == 2 ? 16 : 4;
            const size_t slot = L.seg_ie.size();
            for (int q = 0; q < nq; ++q) {
                int c[3] = {k[0], k[1], k[2]};
                c[odd[0]] = pos[odd[0]][q & 3];
                if (no == 2) c[odd[1]] = pos[odd[1]][q >> 2];
                if ((c[0] | c[1] | c[2]) & 1) return fail(DCLBM_ERR_INVALID, "stencil off the co-located lattice");
                const size_t key = ((size_t)(c[2] / 2) * L.my + c[1] / 2) * L.mx + c[0] / 2;
                if (key >= L.tfmap.size() || L.tfmap[key] < 0)
                    return fail(DCLBM_ERR_INVALID, "level %d hanging node (%d,%d,%d): stencil node is not co-located", l,
                                m.x, m.y, m.z);
                const int t = L.tfmap[key];
                auto it = local.find(t);
                int li;
                if (it == local.end()) {
                    li = (int)list.size();
                    local[t] = li;
                    list.push_back(t);
                } else {
                    li = it->second;
                }
                L.seg_sten[(size_t)q * nie + slot] = li;
                L.ie_tf[(size_t)q * nie + e] = t;
            }
            L.seg_ie.push_back(e);
        }
        if ((int)list.size() > TFM || (int)list.size() > kBlock || (int)sg.ie.size() > SegLimits<3>::IE)
            return fail(DCLBM_ERR_INVALID, "level %d: interface segment too large (%zu co-located, %zu hanging)", l,
                        list.size(), sg.ie.size());
        L.seg_info.push_back(make_int4((int)L.seg_tf.size(), (int)list.size(), ie_off, (int)sg.ie.size()));
        L.seg_tf.insert(L.seg_tf.end(), list.begin(), list.end());
        for (int e : list) L.seg_tfm.push_back(L.tf_meta[e & 0x3fffffff]);
    }
    // the stencil table is indexed by position in seg_ie, which is the IE order of the segments
    return DCLBM_OK;
}

// Width of a level's row blocks (log2): 64 nodes, one wavefront, the width
// the bulk role takes as a compile-time constant.  Blocks of 128 and 256
// nodes (longer contiguous runs per direction) measured no faster on the
// 256^3 D3Q19 levels, and waste memory on odd extents.
static int row_block_shift(int D, const HostLevel& L)
{
    (void)D;
    (void)L;
    return kRowShift;
}

dclbm_status build_geometry(Sim& s)
{
    const dclbm_config& c = s.cfg;
    if (c.abi_version != DCLBM_ABI_VERSION) return fail(DCLBM_ERR_INVALID, "abi_version %d != %d", c.abi_version, DCLBM_ABI_VERSION);
    if (c.lattice != DCLBM_D2Q9 && c.lattice != DCLBM_D3Q19) return fail(DCLBM_ERR_INVALID, "unknown lattice %d", c.lattice);
    if (c.precision < 0 || c.precision > 2) return fail(DCLBM_ERR_INVALID, "unknown precision %d", c.precision);
    if (c.coupling != 1 && c.coupling != 2) return fail(DCLBM_ERR_INVALID, "coupling must be 1 (DC1) or 2 (DC2)");
    if (c.eq_order != 2 && c.eq_order != 3) return fail(DCLBM_ERR_INVALID, "eq_order must be 2 or 3");
    if (c.n_levels < 1 || c.n_levels > DCLBM_MAX_LEVELS) return fail(DCLBM_ERR_INVALID, "n_levels out of range");
    if (!(c.tau0 > 0.5)) return fail(DCLBM_ERR_INVALID, "tau0 must exceed 1/2");
    if (c.n_probes < 0 || c.n_probes > kMaxProbes)
        return fail(DCLBM_ERR_INVALID, "n_probes must be in [0, %d]", kMaxProbes);
    if (c.n_probes > 0 && (!c.h_probe_xyz || c.probe_capacity < 1))
        return fail(DCLBM_ERR_INVALID, "probes need coordinates and a capacity");
    if (c.collision != DCLBM_BGK && c.collision != DCLBM_HRR) return fail(DCLBM_ERR_INVALID, "unknown collision model %d", c.collision);
    if (c.collision == DCLBM_HRR) {
        if (!(c.hrr_sigma >= 0.0 && c.hrr_sigma <= 1.0)) return fail(DCLBM_ERR_INVALID, "hrr_sigma must be in [0, 1]");
    }
    s.hrr = c.collision == DCLBM_HRR ? 1 : 0;
    if (c.sponge_cells < 0 || !(c.sponge_sigma >= 0.0 && c.sponge_sigma <= 1.0))
        return fail(DCLBM_ERR_INVALID, "sponge_cells must be >= 0 and sponge_sigma in [0, 1]");
    s.sponge_w = c.sponge_sigma > 0.0 ? c.sponge_cells : 0;
    s.sponge_sigma = c.sponge_sigma;
    s.D = c.lattice == DCLBM_D2Q9 ? 2 : 3;
    s.Q = s.D == 2 ? 9 : 19;
    s.P = c.precision;
    s.EQ = c.eq_order;
    s.tsize = s.P == 0 ? 8 : (s.P == 1 ? 4 : 2);
    s.rsize = s.P == 0 ? 8 : 4;
    s.newton_maxit = c.newton_max_iter > 0 ? c.newton_max_iter : 20;
    s.newton_tol = c.newton_tol > 0 ? c.newton_tol : (s.P == 0 ? 1e-12 : 2e-6);
    const int D = s.D, Q = s.Q;
    double ur2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(c.u_ref[a])) return fail(DCLBM_ERR_INVALID, "u_ref must be finite");
        if (a < D) ur2 += c.u_ref[a] * c.u_ref[a];
    }
    if (ur2 >= 1.0 / 3.0) return fail(DCLBM_ERR_INVALID, "|u_ref| must be below the sound speed");
    s.lv.assign(c.n_levels, HostLevel());
    for (auto& L : s.lv) {
        for (int a = 0; a < 3; ++a) L.ur[a] = (s.P == 0 || a >= D) ? 0.0 : c.u_ref[a];
        // w_i (1 + B_i(ur)) (with the H3 terms when eq_order = 3) and
        // 3 + 9 xi_i.ur of the equilibrium in the carried variable
        const double uu = L.ur[0] * L.ur[0] + L.ur[1] * L.ur[1] + L.ur[2] * L.ur[2];
        for (int i = 0; i < Q; ++i) {
            int xi[3];
            dirs(D, i, xi);
            const double cr = xi[0] * L.ur[0] + xi[1] * L.ur[1] + xi[2] * L.ur[2];
            const double w = D == 2 ? Lat<2>::w[i] : Lat<3>::w[i];
            double b3 = 0.0;
            if (c.eq_order == 3)
                for (int a = 0; a < D; ++a)
                    for (int g = 0; g < D; ++g)
                        if (a != g) b3 += (xi[a] * xi[a] * xi[g] - xi[g] / 3.0) * L.ur[a] * L.ur[a] * L.ur[g];
            L.k1[i] = (float)(w * (1.0 + 3.0 * cr + 4.5 * cr * cr - 1.5 * uu + 13.5 * b3));
            L.k2[i] = (float)(3.0 + 9.0 * cr);
        }
    }
    double tau = c.tau0;
    for (int l = 0; l < c.n_levels; ++l) {
        HostLevel& L = s.lv[l];
        int n[3] = {1, 1, 1};
        if (l == 0) {
            for (int a = 0; a < D; ++a) {
                n[a] = c.n0[a];
                if (n[a] < 8) return fail(DCLBM_ERR_INVALID, "level-0 extent must be at least 8");
                if (2 * s.sponge_w >= n[a]) return fail(DCLBM_ERR_INVALID, "absorbing layer wider than half the domain");
                if (n[a] > (1 << 20)) return fail(DCLBM_ERR_INVALID, "level-0 extent too large");
            }
            L.periodic = 1;
        } else {
            HostLevel& Pn = s.lv[l - 1];
            int pn[3] = {Pn.nx, Pn.ny, Pn.nz};
            for (int a = 0; a < D; ++a) {
                const int lo = c.box_lo[l - 1][a], hi = c.box_hi[l - 1][a];
                if (hi - lo < 3) return fail(DCLBM_ERR_INVALID, "level %d box side below 3 parent cells", l);
                if (lo < 2 || hi > pn[a] - 1 - 2)
                    return fail(DCLBM_ERR_INVALID, "level %d box needs a margin of 2 parent cells", l);
                n[a] = 2 * (hi - lo) + 1;
                L.plo[a] = lo;
                Pn.clo[a] = lo;
                Pn.chi[a] = hi;
            }
            Pn.has_child = 1;
            L.boundary = 1;
            if (l == 1 && s.sponge_w > 0)
                for (int a = 0; a < D; ++a)
                    if (Pn.clo[a] < s.sponge_w || Pn.chi[a] > pn[a] - 1 - s.sponge_w)
                        return fail(DCLBM_ERR_INVALID, "the level-1 box reaches into the absorbing layer");
        }
        L.nx = n[0];
        L.ny = n[1];
        L.nz = n[2];
        L.tau = tau;
        tau = 2.0 * tau - 0.5;
    }
    // a refined region of level-0 cells: node classes of level 0 and level 1
    // (a level-0 node is a hole when its four cells are refined, co-located
    // when some are; a level-1 node is active when any of its parent cells is
    // refined, on the interface when not all are; cells outside the box are
    // not refined)
    if (c.h_region) {
        if (D != 2 || c.n_levels != 2) return fail(DCLBM_ERR_INVALID, "refined regions need D2Q9 and two levels");
        HostLevel& L0 = s.lv[0];
        HostLevel& L1 = s.lv[1];
        const int cw = L0.chi[0] - L0.clo[0], ch = L0.chi[1] - L0.clo[1];
        auto refined = [&](int cx, int cy) {
            return cx >= 0 && cy >= 0 && cx < cw && cy < ch && c.h_region[(size_t)cy * cw + cx] != 0;
        };
        L0.cls.assign((size_t)L0.nx * L0.ny, kClsBulk);
        for (int y = L0.clo[1]; y <= L0.chi[1]; ++y)
            for (int x = L0.clo[0]; x <= L0.chi[0]; ++x) {
                int r = 0;
                for (int dy = -1; dy <= 0; ++dy)
                    for (int dx = -1; dx <= 0; ++dx) r += refined(x - L0.clo[0] + dx, y - L0.clo[1] + dy) ? 1 : 0;
                L0.cls[(size_t)y * L0.nx + x] = r == 4 ? kClsHole : (r > 0 ? kClsTfc : kClsBulk);
            }
        L1.cls.assign((size_t)L1.nx * L1.ny, kClsHole);
        int64_t active = 0;
        for (int y = 0; y < L1.ny; ++y)
            for (int x = 0; x < L1.nx; ++x) {
                int tot = 0, r = 0;
                for (int cy = (y - 1) >> 1; cy <= (y >> 1); ++cy)
                    for (int cx = (x - 1) >> 1; cx <= (x >> 1); ++cx) {
                        ++tot;
                        r += refined(cx, cy) ? 1 : 0;
                    }
                uint8_t k = kClsHole;
                if (r > 0) k = r < tot ? ((x & 1) || (y & 1) ? kClsIe : kClsTf) : kClsBulk;
                L1.cls[(size_t)y * L1.nx + x] = k;
                active += k != kClsHole;
            }
        if (active == 0) return fail(DCLBM_ERR_INVALID, "the refined region is empty");
    }
    // storage layout per level: row blocks of 2^xsh nodes, Q directions per block
    for (int l = 0; l < c.n_levels; ++l) {
        HostLevel& L = s.lv[l];
        L.xsh = row_block_shift(D, L);
        // a 3-D refined level keeps its x = nx - 1 face in the face buffer
        // (x = 0 keeps an unused slot in block 0), so its rows need only
        // the blocks of x < nx - 1: a 257-node row takes 4 blocks, the
        // pitch of a 256-node row (with a fifth block the launches fetched
        // 12-22% more than the algorithmic bytes and ran 4-5% slower)
        const int stored = D == 3 && L.boundary ? L.nx - 1 : L.nx;
        L.nxb = (stored + (1 << L.xsh) - 1) >> L.xsh;
        L.elems = ((int64_t)L.nz * L.ny * L.nxb * Q) << L.xsh;
        int64_t hole = 0;
        if (!L.cls.empty()) {
            for (uint8_t k : L.cls) hole += k == kClsHole;
        } else if (L.has_child) {
            hole = 1;
            for (int a = 0; a < D; ++a) hole *= (L.chi[a] - L.clo[a] - 1);
        }
        L.n_active = L.n_dense() - hole;
    }
    // interface classification, level by level
    for (int l = 1; l < c.n_levels; ++l) {
        HostLevel& L = s.lv[l];
        HostLevel& Pn = s.lv[l - 1];
        const int n[3] = {L.nx, L.ny, L.nz};
        L.mx = L.nx / 2 + 1;
        L.my = L.ny / 2 + 1;
        L.mz = D == 3 ? L.nz / 2 + 1 : 1;
        L.tfmap.assign((size_t)L.mx * L.my * L.mz, -1);
        const uint32_t all = (1u << Q) - 1u;
        for (int z = 0; z < L.nz; ++z)
            for (int y = 0; y < L.ny; ++y)
                for (int x = 0; x < L.nx; ++x) {
                    const int k[3] = {x, y, z};
                    const bool region = !L.cls.empty();
                    bool bnd = false, even = true;
                    for (int a = 0; a < D; ++a) {
                        if (k[a] == 0 || k[a] == n[a] - 1) bnd = true;
                        if (k[a] & 1) even = false;
                    }
                    if (region) {
                        const uint8_t cl = L.cls[(size_t)y * L.nx + x];
                        bnd = cl == kClsTf || cl == kClsIe;
                    }
                    if (!bnd) continue;
                    uint32_t Kf = 0, Kc = 0;
                    for (int i = 0; i < Q; ++i) {
                        int cv[3];
                        dirs(D, i, cv);
                        bool fin = true, hole = true;
                        int sf3[3] = {0, 0, 0}, sc3[3] = {0, 0, 0};
                        for (int a = 0; a < D; ++a) {
                            const int sf = k[a] - cv[a];
                            sf3[a] = sf;
                            if (sf < 0 || sf > n[a] - 1) fin = false;
                            if (even) {
                                const int sc = L.plo[a] + k[a] / 2 - cv[a];
                                sc3[a] = sc;
                                if (!(sc > Pn.clo[a] && sc < Pn.chi[a])) hole = false;
                            }
                        }
                        if (region) {
                            // present sources from the classes: a fine source exists when it is
                            // an active node; a coarse one when it is not a hole
                            if (fin) fin = L.cls[(size_t)sf3[1] * L.nx + sf3[0]] != kClsHole;
                            if (even) hole = Pn.cls[(size_t)sc3[1] * Pn.nx + sc3[0]] == kClsHole;
                        }
                        if (fin) Kf |= 1u << i;
                        if (even && !hole) Kc |= 1u << i;
                    }
                    if (even) {
                        // Table choice_Gamma_fine: DC1 takes M^f from the coarse grid, DC2 P and M^f
                        const uint32_t P_ = Kf & Kc, Mf = all & ~Kf;
                        const uint32_t gR = c.coupling == 1 ? Mf : (P_ | Mf);
                        if ((gR & ~Kc) || ((all & ~gR) & ~Kf))
                            return fail(DCLBM_ERR_INVALID, "level %d node (%d,%d,%d): no valid couples", l, x, y, z);
                        L.tfmap[((size_t)(z / 2) * L.my + y / 2) * L.mx + x / 2] = (int)L.tf_meta.size();
                        L.tf_meta.push_back(make_int4(x, y, z, (int)gR));
                        int p[3] = {0, 0, 0};
                        for (int a = 0; a < D; ++a) p[a] = L.plo[a] + k[a] / 2;
                        Pn.tfc_meta.push_back(make_int4(p[0], p[1], p[2], (int)Kc));
                    } else {
                        int wtype = 0;
                        if (region) {
                            int pos[4];
                            wtype = region_stencil(L, k, pos);
                            if (!wtype)
                                return fail(DCLBM_ERR_INVALID, "level %d hanging node (%d,%d): no co-located nodes on its line",
                                            l, x, y);
                        }
                        L.ie_meta.push_back(make_int4(x, y, z, (int)((all & ~Kf) | ((uint32_t)wtype << 24))));
                    }
                }
        // Renumber co-located and hanging nodes in segment order, so that one
        // segment's ring entries, shared states and metadata are contiguous
        // (its gathers then touch few cache lines), then build the final tables.
        dclbm_status st = build_segments(s, l);
        if (st != DCLBM_OK) return st;
        {
            std::vector<int> tf_order, ie_order = L.seg_ie;
            for (size_t g = 0; g < L.seg_info.size(); ++g) {
                const int4 info = L.seg_info[g];
                for (int j = 0; j < info.y; ++j) {
                    const int e = L.seg_tf[info.x + j];
                    if ((e >> 30) & 1) tf_order.push_back(e & 0x3fffffff);
                }
            }
            if (tf_order.size() != L.tf_meta.size() || ie_order.size() != L.ie_meta.size())
                return fail(DCLBM_ERR_INVALID, "level %d: segment ownership does not cover the interface", l);
            // the parent's co-located list was appended in this level's order, at its end
            const size_t base = Pn.tfc_meta.size() - L.tf_meta.size();
            std::vector<int4> tf2, tfc2, ie2;
            for (int t : tf_order) {
                tf2.push_back(L.tf_meta[t]);
                tfc2.push_back(Pn.tfc_meta[base + t]);
            }
            for (int e : ie_order) ie2.push_back(L.ie_meta[e]);
            L.tf_meta = tf2;
            L.ie_meta = ie2;
            std::copy(tfc2.begin(), tfc2.end(), Pn.tfc_meta.begin() + base);
            std::fill(L.tfmap.begin(), L.tfmap.end(), -1);
            for (size_t t = 0; t < L.tf_meta.size(); ++t) {
                const int4& m = L.tf_meta[t];
                L.tfmap[((size_t)(m.z / 2) * L.my + m.y / 2) * L.mx + m.x / 2] = (int)t;
            }
            st = build_segments(s, l);
            if (st != DCLBM_OK) return st;
            // the segment role reads hanging node q0 of its segment list as
            // ie_meta[q0] (one dependent load fewer): the renumbering makes
            // that list the identity
            for (size_t q = 0; q < L.seg_ie.size(); ++q)
                if (L.seg_ie[q] != (int)q) return fail(DCLBM_ERR_INVALID, "level %d: hanging nodes out of segment order", l);
        }
    }
    // probes: finest level whose closed box contains the point
    s.probes.clear();
    s.probe_xyz.assign(3 * (size_t)c.n_probes, 0);
    const int Lm = c.n_levels - 1;
    for (int p = 0; p < c.n_probes; ++p) {
        int64_t fine[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) {
            const int v = c.h_probe_xyz[3 * p + a];
            s.probe_xyz[3 * p + a] = v;
            if (v < 0 || v >= (a == 0 ? s.lv[0].nx : (a == 1 ? s.lv[0].ny : s.lv[0].nz)))
                return fail(DCLBM_ERR_INVALID, "probe %d outside the domain", p);
            fine[a] = (int64_t)v << Lm;   // in units of the finest spacing
        }
        int64_t org[3] = {0, 0, 0};
        ProbeLoc best{0, 0, 0, 0, 0};
        for (int l = 0; l <= Lm; ++l) {
            if (l > 0)
                for (int a = 0; a < D; ++a) org[a] += (int64_t)s.lv[l].plo[a] << (Lm - l + 1);
            const int sh = Lm - l;
            const int n[3] = {s.lv[l].nx, s.lv[l].ny, s.lv[l].nz};
            int k[3] = {0, 0, 0};
            bool inside = true;
            for (int a = 0; a < D; ++a) {
                const int64_t d = fine[a] - org[a];
                if (d < 0 || (d >> sh) > n[a] - 1 || (d & ((1LL << sh) - 1))) inside = false;
                else k[a] = (int)(d >> sh);
            }
            // a refined region holds the point only where it has a node
            if (inside && !s.lv[l].cls.empty() && s.lv[l].cls[((size_t)k[2] * n[1] + k[1]) * n[0] + k[0]] == kClsHole)
                inside = false;
            if (inside) best = ProbeLoc{l, s.lv[l].elem0(Q, k[0], k[1], k[2]), k[0], k[1], k[2]};
        }
        s.probes.push_back(best);
    }
    // workspace layout
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off = round_up(off + std::max<int64_t>(bytes, 1), 256);
        return o;
    };
    for (auto& L : s.lv) {
        for (int b = 0; b < 2; ++b) L.off_f[b] = take(L.elems * (int64_t)s.tsize);
        if (D == 3 && L.boundary) {
            // the two x faces in their own y-fastest buffers, [2][Q][nz][ny]
            L.xface = 1;
            L.xf_elems = 2 * (int64_t)Q * L.nz * L.ny;
            for (int b = 0; b < 2; ++b) L.off_xf[b] = take(L.xf_elems * (int64_t)s.tsize);
            // with BGK in FP32 and FP64, the directions the faces pull from
            // the next planes once more, in the same layout (256^3 level 1:
            // 508 -> 497 us FP32, 1001 -> 986 us FP64; FP16 lost 2%, and
            // H-RR keeps the row blocks)
            if (!s.hrr && s.P != DCLBM_FP32_FP16)
                for (int b = 0; b < 2; ++b) L.off_xn[b] = take(L.xf_elems * (int64_t)s.tsize);
        }
        if (!L.tf_meta.empty()) {
            L.off_tf = take((int64_t)L.tf_meta.size() * 16);
            L.off_X = take((int64_t)L.tf_meta.size() * 4 * (int64_t)s.rsize);
            L.off_seg_info = take((int64_t)L.seg_info.size() * 16);
            L.off_seg_tf = take((int64_t)L.seg_tf.size() * 4);
            L.off_seg_tfm = take((int64_t)L.seg_tfm.size() * 16);
        }
        if (!L.ie_meta.empty()) {
            L.off_ie = take((int64_t)L.ie_meta.size() * 16);
            L.off_seg_ie = take((int64_t)L.seg_ie.size() * 4);
            L.off_seg_sten = take((int64_t)L.seg_sten.size() * 4);
        }
        if (!L.tfc_meta.empty()) {
            L.off_tfc = take((int64_t)L.tfc_meta.size() * 16);
            L.off_H = take((int64_t)L.tfc_meta.size() * 3 * Q * (int64_t)s.rsize);
        }
    }
    s.off_series = take(std::max<int64_t>(1, c.probe_capacity) * std::max(1, c.n_probes) * 8);
    s.off_counter = take(40);
    s.off_psum = take(3 * (int64_t)std::max(1, c.n_probes) * 8);
    s.off_probe_args = take(2 * (int64_t)sizeof(ProbeArgs));
    s.off_flags = take(8);
    s.off_partial = take((int64_t)DCLBM_MAX_LEVELS * s.partial_blocks * 5 * 8);
    s.off_bal = take(DCLBM_MAX_LEVELS * 5 * 8);
    if (s.hrr)
        for (size_t l = 0; l < s.lv.size(); ++l) {
            HostLevel& L = s.lv[l];
            L.off_M = take(4 * L.n_dense() * (int64_t)s.rsize);
            if (L.has_child) L.off_Mring = take(3 * 4 * L.n_dense() * (int64_t)s.rsize);
            if (!L.ie_meta.empty()) L.off_ie_tf = take((int64_t)L.ie_tf.size() * 4);
        }
    for (auto& L : s.lv)
        if (!L.cls.empty()) L.off_cls = take((int64_t)L.cls.size());
    s.need_bytes = (size_t)off;
    return DCLBM_OK;
}

// The running probe sums restart: zero sums, no shift yet (NaN).
static void clear_probe_sums(Sim& s)
{
    const int64_t n = std::max(1, s.cfg.n_probes);
    hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(64), 0, s.stream, s.d_psum, 2 * n, 0.0);
    hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(64), 0, s.stream, s.d_psum + 2 * n, n, __builtin_nan(""));
}

dclbm_status sim_attach(Sim& s, void* d_workspace, size_t bytes, hipStream_t stream)
{
    if (bytes < s.need_bytes) return fail(DCLBM_ERR_NOMEM, "workspace %zu bytes, need %zu", bytes, s.need_bytes);
    s.ws = (char*)d_workspace;
    s.ws_bytes = bytes;
    s.stream = stream;
    for (auto& L : s.lv) {
        for (int b = 0; b < 2; ++b) {
            L.f[b] = s.ws + L.off_f[b];
            L.xf[b] = L.xface ? s.ws + L.off_xf[b] : nullptr;
            L.xn[b] = L.off_xn[b] > 0 ? s.ws + L.off_xn[b] : nullptr;   // laid out only where used
        }
        if (!L.tf_meta.empty()) {
            L.d_tf = s.at<int4>(L.off_tf);
            L.X = s.ws + L.off_X;
            L.d_seg_info = s.at<int4>(L.off_seg_info);
            L.d_seg_tf = s.at<int>(L.off_seg_tf);
            L.d_seg_tfm = s.at<int4>(L.off_seg_tfm);
            HIPCHECK(upload(s, L.d_tf, L.tf_meta));
            HIPCHECK(upload(s, L.d_seg_info, L.seg_info));
            HIPCHECK(upload(s, L.d_seg_tf, L.seg_tf));
            HIPCHECK(upload(s, L.d_seg_tfm, L.seg_tfm));
        }
        if (!L.ie_meta.empty()) {
            L.d_ie = s.at<int4>(L.off_ie);
            L.d_seg_ie = s.at<int>(L.off_seg_ie);
            L.d_seg_sten = s.at<int>(L.off_seg_sten);
            HIPCHECK(upload(s, L.d_ie, L.ie_meta));
            HIPCHECK(upload(s, L.d_seg_ie, L.seg_ie));
            HIPCHECK(upload(s, L.d_seg_sten, L.seg_sten));
        }
        if (!L.tfc_meta.empty()) {
            L.d_tfc = s.at<int4>(L.off_tfc);
            L.H = s.ws + L.off_H;
            HIPCHECK(upload(s, L.d_tfc, L.tfc_meta));
        }
    }
    s.d_series = s.at<double>(s.off_series);
    s.d_counter = s.at<int64_t>(s.off_counter);
    s.d_psum = s.at<double>(s.off_psum);
    s.d_probe_args = s.at<ProbeArgs>(s.off_probe_args);
    {
        // probe buffers for either parity of level 0 (finer levels start every
        // coarse step at parity 0)
        const int p0 = s.lv[0].parity;
        s.h_probe_args.resize(2);
        for (int par = 0; par < 2; ++par) {
            s.lv[0].parity = par;
            s.h_probe_args[par] = probe_args(s);
        }
        s.lv[0].parity = p0;
        HIPCHECK(upload(s, s.d_probe_args, s.h_probe_args));
    }
    s.d_flags = s.at<int>(s.off_flags);
    if (s.hrr)
        for (auto& L : s.lv) {
            L.d_M = s.ws + L.off_M;
            L.d_Mring = L.has_child ? (void*)(s.ws + L.off_Mring) : nullptr;
            L.d_ie_tf = L.ie_meta.empty() ? nullptr : s.at<int>(L.off_ie_tf);
            if (L.d_ie_tf) HIPCHECK(upload(s, L.d_ie_tf, L.ie_tf));
        }
    for (auto& L : s.lv)
        if (!L.cls.empty()) {
            L.d_cls = (uint8_t*)(s.ws + L.off_cls);
            HIPCHECK(upload(s, L.d_cls, L.cls));
        }
    s.d_partial = s.at<double>(s.off_partial);
    s.d_bal = s.at<double>(s.off_bal);
    s.eng.reset(make_engine(s.D, s.EQ, s.P));
    s.eng->fill_nan(s);
    hipLaunchKernelGGL((k_fill<int64_t>), dim3(1), dim3(64), 0, s.stream, s.d_counter, (int64_t)5, (int64_t)0);
    clear_probe_sums(s);
    hipLaunchKernelGGL((k_fill<int>), dim3(1), dim3(64), 0, s.stream, s.d_flags, (int64_t)2, 0);
    HIPCHECK(hipGetLastError());
    return DCLBM_OK;
}

// ------------------------------------------------------------------ stepping
// One step of level l (substep 1 or 2 of its parent's step) is one launch:
// its bulk nodes, its coarse history capture (if it has a child) and its
// interface segments (if it has a parent; at substep 2 they also restrict
// into the parent).  Then its two child substeps follow.
template <class Fn>
static void walk(Sim& s, int l, int substep, Fn&& fn)
{
    HostLevel& L = s.lv[l];
    const int first = (l > 0 && s.lv[l - 1].captures <= 1) ? 1 : 0;
    fn(l, substep, first);
    if (L.has_child) {
        L.captures++;
        walk(s, l + 1, 1, fn);
        walk(s, l + 1, 2, fn);
    }
    L.parity ^= 1;
}

static void advance(Sim& s, int l, int substep)
{
    walk(s, l, substep, [&](int lv, int sub, int first) { s.eng->level_step(s, lv, sub, first); });
}

// H-RR on a refined mesh (Sec. 3.5): a level opens its substep (streaming,
// macroscopic fields, interface completion), runs its child's two substeps
// (the synchronous one restricting into its coarse co-located nodes), and
// only then closes it (gradients, collision of all its nodes).
static void advance_hrr(Sim& s, int l, int substep)
{
    HostLevel& L = s.lv[l];
    const int first = (l > 0 && s.lv[l - 1].captures <= 1) ? 1 : 0;
    s.eng->hrr_open(s, l, substep, first);
    if (L.has_child) {
        L.captures++;
        advance_hrr(s, l + 1, 1);
        advance_hrr(s, l + 1, 2);
    }
    s.eng->hrr_close(s, l, substep, first);
    L.parity ^= 1;
}

void record_coarse_step(Sim& s, std::vector<StepRecord>& out, ProbeArgs& probe_after)
{
    out.clear();
    walk(s, 0, 0, [&](int lv, int sub, int first) {
        StepRecord r;
        r.level = lv;
        r.substep = sub;
        r.args = level_args(s, lv, sub, first, &r.grid);
        out.push_back(r);
    });
    probe_after = probe_args(s);
}

// Host-side state change of one coarse step, without launching anything.
static void advance_state(Sim& s)
{
    for (size_t l = 0; l < s.lv.size(); ++l) {
        if (s.lv[l].has_child) s.lv[l].captures += (int64_t)1 << l;
    }
    s.lv[0].parity ^= 1;
}

// The probes of a step are sampled by the next step's level-0 launch, or by
// the flush before they are read.
static void one_coarse_step(Sim& s)
{
    if (s.hrr && s.lv.size() > 1)
        advance_hrr(s, 0, 0);
    else
        advance(s, 0, 0);
}

// The first HIP error of a step's launch sequence, if any, as a status.
static dclbm_status launch_status(Sim& s, const char* what)
{
    const hipError_t e = s.launch_err;
    s.launch_err = hipSuccess;
    if (e != hipSuccess) return fail(DCLBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return DCLBM_OK;
}

static dclbm_status coarse_step_eager(Sim& s)
{
    one_coarse_step(s);
    if (s.sponge_w > 0) s.eng->sponge(s);
    HIPCHECK(hipGetLastError());
    return launch_status(s, "level substep launch");
}

static bool all_first_steps_done(const Sim& s)
{
    for (size_t l = 0; l + 1 < s.lv.size(); ++l)
        if (s.lv[l].captures < 2) return false;
    return true;
}

static dclbm_status coarse_step(Sim& s)
{
    if (s.timing || s.stream == nullptr || !all_first_steps_done(s) || (s.hrr && s.lv.size() > 1) || s.sponge_w > 0)
        return coarse_step_eager(s);
    const int par = s.lv[0].parity;
    if (!s.gexec[par]) {
        // the coarse step's launches, recorded from the host state (which
        // this advances like a launched step), as an explicit graph
        std::vector<StepRecord> recs;
        ProbeArgs pa;
        record_coarse_step(s, recs, pa);
        hipGraph_t g = nullptr;
        HIPCHECK(hipGraphCreate(&g, 0));
        std::vector<hipGraphNode_t> deps;
        for (const StepRecord& r : recs) {
            const hipError_t e = s.eng->add_nodes(s, g, r, deps);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return fail(DCLBM_ERR_HIP, "graph node of level %d: %s", r.level, hipGetErrorString(e));
            }
        }
        s.graph[par] = g;
        HIPCHECK(hipGraphInstantiate(&s.gexec[par], g, nullptr, nullptr, 0));
        HIPCHECK(hipGraphLaunch(s.gexec[par], s.stream));   // recording advanced the host state already
        return DCLBM_OK;
    }
    HIPCHECK(hipGraphLaunch(s.gexec[par], s.stream));
    advance_state(s);
    return DCLBM_OK;
}

}  // namespace dclbm

using namespace dclbm;

struct dclbm_sim {
    Sim s;
};

static dclbm_status check_level_impl(const dclbm_sim* sim, int32_t level)
{
    if (!sim) return fail(DCLBM_ERR_INVALID, "null simulation");
    if (level < 0 || level >= (int)sim->s.lv.size()) return fail(DCLBM_ERR_INVALID, "level %d out of range", level);
    return DCLBM_OK;
}

// ------------------------------------------------------------------ checkpoints
// A checkpoint is a 256-byte header followed by the state regions, each at a
// 256-byte aligned offset, in the order state_regions lists them.
// "DCLPKT02": the row pitch of 3-D refined levels changed from "01"
static constexpr uint64_t kCkptMagic = 0x3330544b504c4344ull;   // "DCLPKT03"
static constexpr int64_t kCkptHeader = 256;

struct CkptHeader {
    uint64_t magic, fingerprint, bytes;
    int64_t steps_done;
    int64_t captures[DCLBM_MAX_LEVELS];
    int32_t parity[DCLBM_MAX_LEVELS];
    int32_t n_levels, reserved;
};
static_assert(sizeof(CkptHeader) <= (size_t)kCkptHeader, "checkpoint header exceeds its slot");

// 64-bit FNV-1a over the configuration fields that fix the layout and the
// arithmetic of a simulation.
struct Fnv1a {
    uint64_t h = 14695981039346656037ull;
    template <typename V>
    void add(const V& v)
    {
        const unsigned char* p = reinterpret_cast<const unsigned char*>(&v);
        for (size_t k = 0; k < sizeof(V); ++k) {
            h ^= p[k];
            h *= 1099511628211ull;
        }
    }
};

static uint64_t config_fingerprint(const Sim& s)
{
    const dclbm_config& c = s.cfg;
    Fnv1a f;
    f.add(c.lattice);
    f.add(c.precision);
    f.add(c.coupling);
    f.add(c.eq_order);
    f.add(c.n_levels);
    for (int a = 0; a < s.D; ++a) f.add(c.n0[a]);
    for (int k = 0; k + 1 < c.n_levels; ++k)
        for (int a = 0; a < s.D; ++a) {
            f.add(c.box_lo[k][a]);
            f.add(c.box_hi[k][a]);
        }
    f.add(c.tau0);
    f.add(c.probe_capacity);
    f.add(s.newton_maxit);
    f.add(s.newton_tol);
    for (int a = 0; a < s.D; ++a) f.add(c.u_ref[a]);
    f.add(c.collision);
    if (c.collision == DCLBM_HRR) {
        f.add(c.hrr_sigma);
        f.add(c.hrr_psi);
    }
    f.add(s.sponge_w);
    if (s.sponge_w > 0) f.add(c.sponge_sigma);
    for (const auto& L : s.lv)
        for (uint8_t k : L.cls) f.add((int32_t)k);
    f.add((uint64_t)s.need_bytes);
    f.add((uint64_t)s.probe_xyz.size());
    for (int32_t v : s.probe_xyz) f.add(v);
    return f.h;
}

// The device state carried from one coarse step to the next, for the
// current parities: (pointer, bytes) in checkpoint order.
template <class Fn>
static void state_regions(const Sim& s, Fn&& fn)
{
    for (const HostLevel& L : s.lv) {
        fn(L.f[L.parity], L.elems * (int64_t)s.tsize);
        if (L.xface) fn(L.xf[L.parity], L.xf_elems * (int64_t)s.tsize);
        if (L.xn[0]) fn(L.xn[L.parity], L.xf_elems * (int64_t)s.tsize);
        if (!L.tf_meta.empty()) fn(L.X, (int64_t)L.tf_meta.size() * 4 * (int64_t)s.rsize);
        if (!L.tfc_meta.empty()) fn(L.H, (int64_t)L.tfc_meta.size() * 3 * s.Q * (int64_t)s.rsize);
        if (L.d_Mring) fn(L.d_Mring, 3 * 4 * L.n_dense() * (int64_t)s.rsize);
    }
    fn((void*)s.d_series, std::max<int64_t>(1, s.cfg.probe_capacity) * std::max(1, s.cfg.n_probes) * 8);
    fn((void*)s.d_counter, (int64_t)40);
    fn((void*)s.d_psum, 3 * (int64_t)std::max(1, s.cfg.n_probes) * 8);
    fn((void*)s.d_flags, (int64_t)8);
}

static int64_t checkpoint_size(const Sim& s)
{
    int64_t n = kCkptHeader;
    state_regions(s, [&](void*, int64_t b) { n += round_up(b, 256); });
    return n;
}

// Copies every state region between the simulation and a checkpoint body
// (to_blob: simulation -> checkpoint), enqueued on the stream.
static hipError_t copy_regions(const Sim& s, char* body, bool to_blob)
{
    hipError_t e = hipSuccess;
    state_regions(s, [&](void* p, int64_t b) {
        if (e == hipSuccess)
            e = to_blob ? hipMemcpyAsync(body, p, (size_t)b, hipMemcpyDeviceToDevice, s.stream)
                        : hipMemcpyAsync(p, body, (size_t)b, hipMemcpyDeviceToDevice, s.stream);
        body += round_up(b, 256);
    });
    return e;
}

extern "C" {

const char* dclbm_last_error(void) { return g_err.c_str(); }

dclbm_status dclbm_lattice_table(int32_t lattice, int32_t* q, int32_t* h_xi, double* h_w)
{
    if (lattice != DCLBM_D2Q9 && lattice != DCLBM_D3Q19) return fail(DCLBM_ERR_INVALID, "unknown lattice");
    const int D = lattice == DCLBM_D2Q9 ? 2 : 3, Q = D == 2 ? 9 : 19;
    if (q) *q = Q;
    for (int i = 0; i < Q; ++i) {
        int c[3];
        dirs(D, i, c);
        if (h_xi)
            for (int a = 0; a < 3; ++a) h_xi[3 * i + a] = c[a];
        if (h_w) h_w[i] = D == 2 ? Lat<2>::w[i] : Lat<3>::w[i];
    }
    return DCLBM_OK;
}

dclbm_status dclbm_workspace_bytes(const dclbm_config* cfg, size_t* bytes)
{
    if (!cfg || !bytes) return fail(DCLBM_ERR_INVALID, "null argument");
    Sim s;
    s.cfg = *cfg;
    dclbm_status st = build_geometry(s);
    if (st != DCLBM_OK) return st;
    *bytes = s.need_bytes;
    return DCLBM_OK;
}

dclbm_status dclbm_create(const dclbm_config* cfg, void* d_workspace, size_t bytes, void* stream, dclbm_sim** out)
{
    if (!cfg || !out) return fail(DCLBM_ERR_INVALID, "null argument");
    *out = nullptr;
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) return fail(DCLBM_ERR_INVALID, "workspace must be 256-byte aligned");
    std::unique_ptr<dclbm_sim> h(new dclbm_sim());
    Sim& s = h->s;
    s.cfg = *cfg;
    s.cfg.h_probe_xyz = nullptr;
    {
        Sim tmp;
        tmp.cfg = *cfg;
        dclbm_status st = build_geometry(tmp);
        if (st != DCLBM_OK) return st;
        s.lv = std::move(tmp.lv);
        s.probes = std::move(tmp.probes);
        s.probe_xyz = std::move(tmp.probe_xyz);
        s.D = tmp.D;
        s.Q = tmp.Q;
        s.P = tmp.P;
        s.EQ = tmp.EQ;
        s.tsize = tmp.tsize;
        s.rsize = tmp.rsize;
        s.newton_maxit = tmp.newton_maxit;
        s.newton_tol = tmp.newton_tol;
        s.need_bytes = tmp.need_bytes;
        s.off_series = tmp.off_series;
        s.off_counter = tmp.off_counter;
        s.off_psum = tmp.off_psum;
        s.off_probe_args = tmp.off_probe_args;
        s.off_flags = tmp.off_flags;
        s.off_partial = tmp.off_partial;
        s.off_bal = tmp.off_bal;
        s.hrr = tmp.hrr;
        s.sponge_w = tmp.sponge_w;
        s.sponge_sigma = tmp.sponge_sigma;
    }
    dclbm_status st = sim_attach(s, d_workspace, bytes, (hipStream_t)stream);
    if (st != DCLBM_OK) return st;
    HIPCHECK(hipGetDevice(&s.device));
    st = scratch_address(s.device, &s.d_scratch);
    if (st != DCLBM_OK) return st;
    if (s.D == 3 && s.P == 2) {
        // side stream (default priority) for the interface half of split substeps
        HIPCHECK(hipStreamCreateWithFlags(&s.side, hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&s.ev_fork, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&s.ev_join, hipEventDisableTiming));
    }
    HIPCHECK(hipStreamSynchronize(s.stream));
    *out = h.release();
    return DCLBM_OK;
}

dclbm_status dclbm_destroy(dclbm_sim* sim)
{
    if (!sim) return DCLBM_OK;
    Sim& s = sim->s;
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    for (int p = 0; p < 2; ++p) {
        if (s.gexec[p]) (void)hipGraphExecDestroy(s.gexec[p]);
        if (s.graph[p]) (void)hipGraphDestroy(s.graph[p]);
    }
    for (int l = 0; l < DCLBM_MAX_LEVELS; ++l) {
        for (auto& e : s.tev[l]) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
    delete sim;   // releases the side stream and its events
    return DCLBM_OK;
}

dclbm_status dclbm_level_shape(const dclbm_sim* sim, int32_t level, int32_t dims[3], int64_t* n_active)
{
    dclbm_status st = check_level_impl(sim, level);
    if (st != DCLBM_OK) return st;
    const HostLevel& L = sim->s.lv[level];
    if (dims) {
        dims[0] = L.nx;
        dims[1] = L.ny;
        dims[2] = L.nz;
    }
    if (n_active) *n_active = L.n_active;
    return DCLBM_OK;
}

dclbm_status dclbm_updates_per_step(const dclbm_sim* sim, int64_t* updates)
{
    if (!sim || !updates) return fail(DCLBM_ERR_INVALID, "null argument");
    int64_t u = 0;
    for (size_t l = 0; l < sim->s.lv.size(); ++l) u += sim->s.lv[l].n_active << l;
    *updates = u;
    return DCLBM_OK;
}

dclbm_status dclbm_init_equilibrium(dclbm_sim* sim, int32_t level, const double* d_rho, const double* d_u)
{
    dclbm_status st = check_level_impl(sim, level);
    if (st != DCLBM_OK) return st;
    if (!d_rho || !d_u) return fail(DCLBM_ERR_INVALID, "null field");
    Sim& s = sim->s;
    s.eng->init(s, level, d_rho, d_u);
    if (s.lv[level].has_child) s.eng->ring_init(s, level);
    if (s.hrr && s.lv[level].has_child) s.eng->hrr_ring_init(s, level, d_rho, d_u);
    s.lv[level].captures = 0;
    HIPCHECK(hipGetLastError());
    return DCLBM_OK;
}

dclbm_status dclbm_step(dclbm_sim* sim, int32_t n)
{
    if (!sim || n < 0) return fail(DCLBM_ERR_INVALID, "bad argument");
    for (int32_t k = 0; k < n; ++k) {
        dclbm_status st = coarse_step(sim->s);
        if (st != DCLBM_OK) return st;
        sim->s.steps_done++;
    }
    return DCLBM_OK;
}

static dclbm_status read_flags(Sim& s)
{
    int flags[2] = {0, 0};
    HIPCHECK(hipMemcpyAsync(flags, s.d_flags, sizeof(int), hipMemcpyDeviceToHost, s.stream));
    HIPCHECK(hipStreamSynchronize(s.stream));
    // an instability is reported first: it also stops Newton from converging
    if (flags[0] & 2) return fail(DCLBM_ERR_UNSTABLE, "non-finite or non-positive density found");
    if (flags[0] & 1) return fail(DCLBM_ERR_NEWTON, "Newton did not converge at a co-located node");
    return DCLBM_OK;
}

dclbm_status dclbm_check(dclbm_sim* sim)
{
    if (!sim) return fail(DCLBM_ERR_INVALID, "null simulation");
    return read_flags(sim->s);
}

dclbm_status dclbm_read_populations(const dclbm_sim* sim, int32_t level, double* d_out)
{
    dclbm_status st = check_level_impl(sim, level);
    if (st != DCLBM_OK) return st;
    Sim& s = const_cast<Sim&>(sim->s);
    s.eng->read(s, level, d_out, nullptr, nullptr);
    HIPCHECK(hipGetLastError());
    return DCLBM_OK;
}

dclbm_status dclbm_read_macros(const dclbm_sim* sim, int32_t level, double* d_rho, double* d_u)
{
    dclbm_status st = check_level_impl(sim, level);
    if (st != DCLBM_OK) return st;
    Sim& s = const_cast<Sim&>(sim->s);
    s.eng->read(s, level, nullptr, d_rho, d_u);
    HIPCHECK(hipGetLastError());
    return DCLBM_OK;
}

dclbm_status dclbm_velocity_divergence(const dclbm_sim* sim, int32_t level, const double* d_u, double* d_div)
{
    dclbm_status st = check_level_impl(sim, level);
    if (st != DCLBM_OK) return st;
    if (!d_u || !d_div) return fail(DCLBM_ERR_INVALID, "null field pointer");
    const Sim& s = sim->s;
    const HostLevel& L = s.lv[level];
    const int64_t n = L.n_dense();
    const dim3 grid((unsigned)((n + 255) / 256));
    if (s.D == 2)
        hipLaunchKernelGGL((k_divergence<2>), grid, dim3(256), 0, s.stream, L.dev(), d_u, d_div);
    else
        hipLaunchKernelGGL((k_divergence<3>), grid, dim3(256), 0, s.stream, L.dev(), d_u, d_div);
    HIPCHECK(hipGetLastError());
    return DCLBM_OK;
}

dclbm_status dclbm_read_shared(const dclbm_sim* sim, int32_t level, double* d_out)
{
    dclbm_status st = check_level_impl(sim, level);
    if (st != DCLBM_OK) return st;
    Sim& s = const_cast<Sim&>(sim->s);
    s.eng->read_shared(s, level, d_out);
    HIPCHECK(hipGetLastError());
    return DCLBM_OK;
}

dclbm_status dclbm_read_probes(const dclbm_sim* sim, double* d_out, int64_t* n_steps)
{
    if (!sim || !n_steps) return fail(DCLBM_ERR_INVALID, "null argument");
    Sim& s = const_cast<Sim&>(sim->s);
    s.eng->probe(s);
    HIPCHECK(hipGetLastError());
    int64_t cnt = 0;
    HIPCHECK(hipMemcpyAsync(&cnt, s.d_counter, 8, hipMemcpyDeviceToHost, s.stream));
    HIPCHECK(hipStreamSynchronize(s.stream));
    const int64_t stored = std::min<int64_t>(cnt, s.cfg.probe_capacity);
    *n_steps = stored;
    if (d_out && stored > 0 && !s.probes.empty())
        HIPCHECK(hipMemcpyAsync(d_out, s.d_series, (size_t)stored * s.probes.size() * 8, hipMemcpyDeviceToDevice,
                                s.stream));
    HIPCHECK(hipStreamSynchronize(s.stream));
    return DCLBM_OK;
}

dclbm_status dclbm_set_probe_window(dclbm_sim* sim, int64_t start, int64_t stop)
{
    if (!sim) return fail(DCLBM_ERR_INVALID, "null argument");
    if (start < 0 || stop < start) return fail(DCLBM_ERR_INVALID, "probe window needs 0 <= start <= stop");
    Sim& s = sim->s;
    // stream-ordered, so the window applies from the steps enqueued after
    // this call; the sums restart from zero
    hipLaunchKernelGGL((k_fill<int64_t>), dim3(1), dim3(64), 0, s.stream, s.d_counter + 2, (int64_t)1, start);
    hipLaunchKernelGGL((k_fill<int64_t>), dim3(1), dim3(64), 0, s.stream, s.d_counter + 3, (int64_t)1, stop);
    hipLaunchKernelGGL((k_fill<int64_t>), dim3(1), dim3(64), 0, s.stream, s.d_counter + 4, (int64_t)1, (int64_t)0);
    clear_probe_sums(s);
    HIPCHECK(hipGetLastError());
    return DCLBM_OK;
}

dclbm_status dclbm_read_probe_sums(const dclbm_sim* sim, double* d_out, int64_t* n_summed)
{
    if (!sim || !n_summed) return fail(DCLBM_ERR_INVALID, "null argument");
    Sim& s = const_cast<Sim&>(sim->s);
    s.eng->probe(s);
    HIPCHECK(hipGetLastError());
    int64_t c = 0;
    HIPCHECK(hipMemcpyAsync(&c, s.d_counter + 4, 8, hipMemcpyDeviceToHost, s.stream));
    HIPCHECK(hipStreamSynchronize(s.stream));
    *n_summed = c;
    if (d_out && !s.probes.empty())
        HIPCHECK(hipMemcpyAsync(d_out, s.d_psum, 3 * s.probes.size() * 8, hipMemcpyDeviceToDevice, s.stream));
    HIPCHECK(hipStreamSynchronize(s.stream));
    return DCLBM_OK;
}

dclbm_status dclbm_balance(dclbm_sim* sim, double h_out[5])
{
    if (!sim || !h_out) return fail(DCLBM_ERR_INVALID, "null argument");
    Sim& s = sim->s;
    double res[DCLBM_MAX_LEVELS][5];
    for (size_t l = 0; l < s.lv.size(); ++l) {
        double* part = s.d_partial + (int64_t)l * s.partial_blocks * 5;
        s.eng->balance(s, (int)l, part, s.partial_blocks);
        hipLaunchKernelGGL(k_balance_final, dim3(1), dim3(64), 0, s.stream, part, s.partial_blocks, s.d_bal + 5 * l);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(res, s.d_bal, sizeof(double) * 5 * s.lv.size(), hipMemcpyDeviceToHost, s.stream));
    HIPCHECK(hipStreamSynchronize(s.stream));
    for (int k = 0; k < 5; ++k) {
        h_out[k] = 0.0;
        for (size_t l = 0; l < s.lv.size(); ++l) h_out[k] += res[l][k];
    }
    return read_flags(s);
}

dclbm_status dclbm_balance_static(dclbm_sim* sim, double* d_out)
{
    if (!sim || !d_out) return fail(DCLBM_ERR_INVALID, "null argument");
    Sim& s = sim->s;
    const int L = (int)s.lv.size();
    if (s.partial_blocks != kBalanceBlocks || (int64_t)L * kBalanceBlocks * 5 + (int64_t)L * 5 > kScratchDoubles)
        return fail(DCLBM_ERR_INVALID, "balance of %d levels x %d blocks exceeds the static scratch (%d levels x %d)",
                    L, s.partial_blocks, DCLBM_MAX_LEVELS, kBalanceBlocks);
    if (!s.d_scratch) return fail(DCLBM_ERR_HIP, "static scratch not resolved for this simulation's device");
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    if (dev != s.device)
        return fail(DCLBM_ERR_INVALID, "device %d is current, the simulation lives on device %d", dev, s.device);
    double* part = s.d_scratch;
    double* totals = s.d_scratch + (int64_t)DCLBM_MAX_LEVELS * kBalanceBlocks * 5;
    for (int l = 0; l < L; ++l) {
        double* pl = part + (int64_t)l * kBalanceBlocks * 5;
        s.eng->balance(s, l, pl, kBalanceBlocks);
        hipLaunchKernelGGL(k_balance_final, dim3(1), dim3(64), 0, s.stream, pl, kBalanceBlocks, totals + 5 * l);
    }
    hipLaunchKernelGGL(k_balance_levels, dim3(1), dim3(64), 0, s.stream, totals, L, d_out);
    HIPCHECK(hipGetLastError());
    return DCLBM_OK;
}

dclbm_status dclbm_checkpoint_bytes(const dclbm_sim* sim, size_t* bytes)
{
    if (!sim || !bytes) return fail(DCLBM_ERR_INVALID, "null argument");
    *bytes = (size_t)checkpoint_size(sim->s);
    return DCLBM_OK;
}

dclbm_status dclbm_save(dclbm_sim* sim, void* d_blob, size_t bytes)
{
    if (!sim || !d_blob) return fail(DCLBM_ERR_INVALID, "null argument");
    if ((uintptr_t)d_blob & 255) return fail(DCLBM_ERR_INVALID, "checkpoint buffer must be 256-byte aligned");
    Sim& s = sim->s;
    const int64_t need = checkpoint_size(s);
    if ((int64_t)bytes < need)
        return fail(DCLBM_ERR_INVALID, "checkpoint buffer %zu bytes, need %lld", bytes, (long long)need);
    s.eng->probe(s);   // the last step's probes, if still pending, go into the saved series
    HIPCHECK(hipGetLastError());
    HIPCHECK(copy_regions(s, (char*)d_blob + kCkptHeader, true));
    CkptHeader h;
    memset(&h, 0, sizeof(h));
    h.magic = kCkptMagic;
    h.fingerprint = config_fingerprint(s);
    h.bytes = (uint64_t)need;
    h.steps_done = s.steps_done;
    h.n_levels = (int32_t)s.lv.size();
    for (size_t l = 0; l < s.lv.size(); ++l) {
        h.captures[l] = s.lv[l].captures;
        h.parity[l] = s.lv[l].parity;
    }
    HIPCHECK(hipMemcpyAsync(d_blob, &h, sizeof(h), hipMemcpyHostToDevice, s.stream));
    HIPCHECK(hipStreamSynchronize(s.stream));
    return DCLBM_OK;
}

dclbm_status dclbm_load(dclbm_sim* sim, const void* d_blob, size_t bytes)
{
    if (!sim || !d_blob) return fail(DCLBM_ERR_INVALID, "null argument");
    if ((uintptr_t)d_blob & 255) return fail(DCLBM_ERR_INVALID, "checkpoint buffer must be 256-byte aligned");
    if (bytes < (size_t)kCkptHeader) return fail(DCLBM_ERR_INVALID, "not a checkpoint: %zu bytes", bytes);
    Sim& s = sim->s;
    CkptHeader h;
    HIPCHECK(hipMemcpyAsync(&h, d_blob, sizeof(h), hipMemcpyDeviceToHost, s.stream));
    HIPCHECK(hipStreamSynchronize(s.stream));
    if (h.magic != kCkptMagic) return fail(DCLBM_ERR_INVALID, "not a checkpoint");
    if (h.fingerprint != config_fingerprint(s) || h.n_levels != (int32_t)s.lv.size())
        return fail(DCLBM_ERR_INVALID, "checkpoint written for another configuration");
    const int64_t need = checkpoint_size(s);
    if ((int64_t)h.bytes != need || (int64_t)bytes < need)
        return fail(DCLBM_ERR_INVALID, "checkpoint of %llu bytes in a %zu-byte buffer, expected %lld",
                    (unsigned long long)h.bytes, bytes, (long long)need);
    if (h.steps_done < 0) return fail(DCLBM_ERR_INVALID, "corrupt checkpoint header");
    for (size_t l = 0; l < s.lv.size(); ++l)
        if ((h.parity[l] & ~1) || h.captures[l] < 0) return fail(DCLBM_ERR_INVALID, "corrupt checkpoint header");
    // host state first: the regions are those of the saved parities
    for (size_t l = 0; l < s.lv.size(); ++l) {
        s.lv[l].parity = h.parity[l];
        s.lv[l].captures = h.captures[l];
    }
    s.steps_done = h.steps_done;
    HIPCHECK(copy_regions(s, (char*)d_blob + kCkptHeader, false));
    HIPCHECK(hipStreamSynchronize(s.stream));
    return DCLBM_OK;
}

dclbm_status dclbm_copy_calibration(void* d_dst, const void* d_src, size_t bytes, void* stream, int32_t repeats,
                                    double* ms_per_copy)
{
    if (!d_dst || !d_src || bytes < 16 || (bytes & 15) || ((uintptr_t)d_dst & 15) || ((uintptr_t)d_src & 15) ||
        repeats < 1)
        return fail(DCLBM_ERR_INVALID, "copy calibration needs 16-byte aligned buffers, a multiple of 16 bytes");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = (int64_t)(bytes / 16);
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 1 << 20);
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, st, (const uint4*)d_src, (uint4*)d_dst, n);
    HIPCHECK(hipEventRecord(e0, st));
    for (int r = 0; r < repeats; ++r)
        hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, st, (const uint4*)d_src, (uint4*)d_dst, n);
    HIPCHECK(hipEventRecord(e1, st));
    HIPCHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ms_per_copy) *ms_per_copy = ms / repeats;
    return DCLBM_OK;
}

dclbm_status dclbm_interface_bytes(const dclbm_sim* sim, int32_t level, double* bytes_per_launch)
{
    dclbm_status st = check_level_impl(sim, level);
    if (st != DCLBM_OK) return st;
    if (!bytes_per_launch) return fail(DCLBM_ERR_INVALID, "null argument");
    const Sim& s = sim->s;
    const HostLevel& L = s.lv[level];
    const double ts = (double)s.tsize, rs = (double)s.rsize;
    double b = 0.0;
    // coarse co-located nodes of this level: the ring shift of every known
    // direction (one pull, two ring reads, three ring writes)
    for (const int4& m : L.tfc_meta) b += __builtin_popcount((unsigned)m.w) * (ts + 5.0 * rs);
    if (level > 0) {
        for (const int4& m : L.tf_meta) {
            // Gamma = R directions come from the parent's ring (three values at
            // the asynchronous substep, one at the synchronous) instead of a
            // pull; X is written
            b += __builtin_popcount((unsigned)m.w) * (2.0 * rs - ts) + 4.0 * rs;
        }
        // restriction into the parent's co-located nodes, every other launch
        b += 0.5 * (double)L.tf_meta.size() * s.Q * ts;
    }
    *bytes_per_launch = b;
    return DCLBM_OK;
}

dclbm_status dclbm_set_split(dclbm_sim* sim, int32_t mode)
{
    if (!sim) return fail(DCLBM_ERR_INVALID, "null simulation");
    if (mode < -1 || mode > 1) return fail(DCLBM_ERR_INVALID, "split mode %d is not -1, 0 or 1", mode);
    Sim& s = sim->s;
    if (mode == s.split_mode) return DCLBM_OK;
    // the coarse-step graphs hold the launches of the old choice
    if (s.stream) HIPCHECK(hipStreamSynchronize(s.stream));
    for (int p = 0; p < 2; ++p) {
        if (s.gexec[p]) HIPCHECK(hipGraphExecDestroy(s.gexec[p]));
        if (s.graph[p]) HIPCHECK(hipGraphDestroy(s.graph[p]));
        s.gexec[p] = nullptr;
        s.graph[p] = nullptr;
    }
    s.split_mode = mode;
    return DCLBM_OK;
}

dclbm_status dclbm_set_timing(dclbm_sim* sim, int32_t on)
{
    if (!sim) return fail(DCLBM_ERR_INVALID, "null simulation");
    sim->s.timing = on != 0;
    return DCLBM_OK;
}

dclbm_status dclbm_bulk_time(dclbm_sim* sim, int32_t level, double* ms, int64_t* launches, int64_t* nodes_per_launch)
{
    dclbm_status st = check_level_impl(sim, level);
    if (st != DCLBM_OK) return st;
    Sim& s = sim->s;
    HIPCHECK(hipStreamSynchronize(s.stream));
    for (auto& e : s.tev[level]) {
        float t = 0.f;
        HIPCHECK(hipEventElapsedTime(&t, e.first, e.second));
        s.tms[level] += t;
        s.tlaunch[level] += 1;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    s.tev[level].clear();
    if (ms) *ms = s.tms[level];
    if (launches) *launches = s.tlaunch[level];
    if (nodes_per_launch) *nodes_per_launch = s.lv[level].n_active - (int64_t)s.lv[level].tfc_meta.size();
    return DCLBM_OK;
}

}  // extern "C"
