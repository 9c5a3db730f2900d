// HIP kernels (gfx950) of the direct-coupling refined LBM step.
//
// Layout.  Each level keeps two population buffers (A/B).  A buffer is a
// sequence of row blocks of B = 2^xsh nodes (B >= 64, per level); inside a
// block the Q directions follow each other, B contiguous values each:
//     element(i, x, y, z) = ((z*ny + y)*nxb + x/B)*Q*B + i*B + x%B
// A wavefront (64 lanes, one per node of a 64-node piece of a row block)
// reads every direction as one coalesced 64-element run, and all Q
// directions of one row block sit in one contiguous span, which keeps the
// pull stream's 3^D neighbouring row blocks in few DRAM pages and
// translation entries.
//
// One launch per level substep (k_level) runs these kinds of workgroups:
//   probe     (level 0 only) samples the probes of the previous coarse step;
//   capture   coarse co-located nodes store their streamed populations in a
//             3-deep history ring (the input of Eq.(TempInt));
//   segment   one tile of the fine interface line/face: Newton for the shared
//             state X of every co-located node the tile's hanging nodes need
//             (Eq.(system_fi), Eq.(updated_macro)), rebuild of each Gamma=R
//             direction (Eq.(rescff)) into LDS, collision of the tile's own
//             co-located nodes with X, and at synchronous substeps the
//             restriction of Eq.(rescfc) with the coarse collision of the
//             co-located coarse node; then the hanging nodes take their
//             missing directions by 4-point 1-D interpolation from LDS and
//             collide.  Halo co-located nodes are recomputed, not exchanged;
//   bulk      fused pull-stream + BGK of every other node (Eq.(LBMequation),
//             Eq.(LBMscheme_reg) with BGK), 64 x 4 node tiles, whole tile
//             rows per XCD, rows interleaved over the 8 XCDs.
// The serving kernels (k_level_multi, k_server_tail) run the same workgroups
// for many resident simulations from device work tables.  Plus
// initialisation, conversion, probe and balance kernels.
#pragma once
#include <type_traits>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace dclbm {

// ---------------------------------------------------------------- storage forms
// P = 0: FP64, carried value s = f.
// P = 1: FP32 arithmetic, stored s = f - w (deviation from rest).
// P = 2: FP32 arithmetic, stored FP16(256 (f - w)).
// Storage forms: load / store of the carried variable.  The bulk streams
// with nontemporal stores; interface nodes, whose stores on some faces cover
// a few bytes of each cache line, store through the cache (store_wb) so that
// partial lines can merge before they are written back.
template <int P>
struct Form;
template <>
struct Form<0> {
    using T = double;
    using R = double;
    static constexpr double rho0 = 0.0;
    static constexpr bool shifted = false;
    __device__ static __forceinline__ R load(const T* p) { return *p; }
    __device__ static __forceinline__ void store(T* p, R v) { __builtin_nontemporal_store(v, p); }
    __device__ static __forceinline__ void store_wb(T* p, R v) { *p = v; }
    __device__ static __forceinline__ T nan() { return __builtin_nan(""); }
};
template <>
struct Form<1> {
    using T = float;
    using R = float;
    static constexpr double rho0 = 1.0;
    static constexpr bool shifted = true;
    __device__ static __forceinline__ R load(const T* p) { return *p; }
    __device__ static __forceinline__ void store(T* p, R v) { __builtin_nontemporal_store(v, p); }
    __device__ static __forceinline__ void store_wb(T* p, R v) { *p = v; }
    __device__ static __forceinline__ T nan() { return __builtin_nanf(""); }
};
template <>
struct Form<2> {
    using T = __half;
    using R = float;
    static constexpr double rho0 = 1.0;
    static constexpr bool shifted = true;
    static constexpr float scale = 256.0f;
    __device__ static __forceinline__ R load(const T* p)
    {
        const unsigned short b = *reinterpret_cast<const unsigned short*>(p);
        return __half2float(__ushort_as_half(b)) * (1.0f / scale);
    }
    __device__ static __forceinline__ void store(T* p, R v)
    {
        const unsigned short b = __half_as_ushort(__float2half_rn(v * scale));
        __builtin_nontemporal_store(b, reinterpret_cast<unsigned short*>(p));
    }
    __device__ static __forceinline__ void store_wb(T* p, R v)
    {
        *reinterpret_cast<unsigned short*>(p) = __half_as_ushort(__float2half_rn(v * scale));
    }
    __device__ static __forceinline__ T nan() { return __ushort_as_half((unsigned short)0x7e00); }
};

// ---------------------------------------------------------------- level geometry
// Row blocks hold 2^kRowShift nodes (one wavefront of 64) on every level.
constexpr int kRowShift = 6;

struct LevelDev {
    int nx, ny, nz;
    int nxb;           // row blocks per row
    int xsh;           // a row block holds 2^xsh nodes (>= 64)
    int periodic;      // level 0
    int boundary;      // own box faces are interfaces (level >= 1)
    int has_child;
    int clo[3], chi[3];// child box, closed, in this level's node coordinates
    double ur[3];      // reference velocity of the carried variable (shifted forms; 0 for FP64)
    // per direction, for the shifted equilibrium (host-computed from ur, the
    // same for every node): w_i (1 + B_i(ur)) (H3 terms included when the
    // equilibrium has them) and 3 + 9 xi_i.ur
    float k1[19], k2[19];
    // 3-D refined levels: the x-face nodes (x = 0 and nx - 1) live in their
    // own y-fastest buffers xf[parity], [2][Q][nz][ny] (face x = 0 first), so
    // that the interface tiles of those faces read and write whole lines
    int xface;
    void* xf[2];
    // 3-D refined levels with BGK: the directions that the x-face nodes pull
    // from the planes next to them (x = 1 with xi_x = -1, x = nx - 2 with
    // xi_x = +1), kept a second time in y-fastest buffers laid out like xf;
    // null: the faces pull from the row blocks (one cache line per lane)
    void* xn[2];
    // a level shaped by a refined region of level-0 cells (and its parent):
    // one class byte per node, x fastest (kClsBulk, kClsHole for holes and for
    // refined-level nodes outside the region, kClsTfc, kClsTf, kClsIe); null
    // for box levels, whose classes follow from the box
    const uint8_t* cls;
};

constexpr uint8_t kClsBulk = 0, kClsHole = 1, kClsTfc = 2, kClsTf = 3, kClsIe = 4;

template <typename R>
__device__ __forceinline__ Ref<R> ref_of(const LevelDev& g)
{
    Ref<R> r;
    r.ur[0] = R(g.ur[0]);
    r.ur[1] = R(g.ur[1]);
    r.ur[2] = R(g.ur[2]);
    return r;
}

// E_i = f0_i(1, ur) in FP64: the population the shifted forms subtract.
template <int DIM, int EQ>
__device__ __forceinline__ double ref_pop(int i, const LevelDev& g)
{
    const double uu = g.ur[0] * g.ur[0] + g.ur[1] * g.ur[1] + g.ur[2] * g.ur[2];
    return Lat<DIM>::w[i] * (1.0 + eq_bracket<DIM, EQ, double>(i, g.ur, uu));
}

// BGK of a bulk node in a shifted form with the second-order equilibrium,
// from the per-direction constants of LevelDev: s0_i = drho k1_i + w_i rho
// (dc (k2_i + 4.5 dc) - 1.5 q), dc = xi_i.du (the expansion of eq_s with
// B_i(ur) and xi_i.ur precomputed; only drho, du and q vary per node).
template <int DIM, typename R>
__device__ __forceinline__ void bgk_shift2(R s[], const LevelDev& g, R drho, const R du[3], R keep)
{
    R q = R(0);
#pragma unroll
    for (int a = 0; a < DIM; ++a) q += du[a] * (R(2) * R(g.ur[a]) + du[a]);
    const R rho = R(1) + drho;
    const R q15 = R(1.5) * q;
#pragma unroll
    for (int i = 0; i < Lat<DIM>::Q; ++i) {
        R dc = R(0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (cdir<DIM>(i, a) > 0) dc += du[a];
            if (cdir<DIM>(i, a) < 0) dc -= du[a];
        }
        const R e = drho * R(g.k1[i]) + R(Lat<DIM>::w[i]) * rho * (dc * (R(g.k2[i]) + R(4.5) * dc) - q15);
        s[i] = e + keep * (s[i] - e);
    }
}

// Equilibrium and gradient for Newton in a shifted form with the
// second-order equilibrium, from the same per-direction constants:
//   s0_i = drho k1_i + w_i rho (dc (k2_i + 4.5 dc) - 1.5 q),
//   d s0_i / d drho = k1_i + w_i (dc (k2_i + 4.5 dc) - 1.5 q),
//   d s0_i / d du_b = w_i rho (xi_ib (k2_i + 9 dc) - 3 u_b),  dc = xi_i.du.
template <int DIM, typename R>
struct EqGradShift2 {
    const LevelDev& g;
    __device__ __forceinline__ void operator()(int i, const Mac<R>& m, R& e, R gr[4]) const
    {
        R dc = R(0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) dc += R(cdir<DIM>(i, a)) * m.du[a];
        const R wi = R(Lat<DIM>::w[i]), k1 = R(g.k1[i]), k2 = R(g.k2[i]);
        const R rho = R(1) + m.drho;
        const R D = dc * (k2 + R(4.5) * dc) - R(1.5) * m.q;
        e = m.drho * k1 + wi * rho * D;
        gr[0] = k1 + wi * D;
        const R t = k2 + R(9) * dc;
#pragma unroll
        for (int b = 0; b < DIM; ++b) gr[1 + b] = wi * rho * (R(cdir<DIM>(i, b)) * t - R(3) * m.u[b]);
        if (DIM == 2) gr[3] = R(0);
    }
};

// All Q equilibria of a node in the carried variable, with the node-level
// products formed once:
//   shifted: s0_i = drho k1_i + w_i rho (dc (k2_i + 4.5 dc) - 1.5 q
//                   [+ 13.5 sum_{a!=g} h_{i,ag} (du_a (2 ur_a + du_a) u_g + ur_a^2 du_g)])
//   FP64:    f0_i = w_i rho (1 + cu (3 + 4.5 cu) - 1.5 u.u [+ 13.5 sum_{a!=g} h_{i,ag} u_a^2 u_g])
// with dc = xi_i.du, cu = xi_i.u, h_{i,ag} = xi_a^2 xi_g - xi_g/3 (the H3
// terms of Eq.(fEq_herm) when EQ = 3); the same values as eq_s.
template <int DIM, int EQ, bool SH, typename R>
__device__ __forceinline__ void eq_all(const LevelDev& g, const Ref<R>& rf, const Mac<R>& m, R out[])
{
    constexpr int Q = Lat<DIM>::Q;
    const R rho = (SH ? R(1) : R(0)) + m.drho;
    R T[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            T[a][c] = (EQ == 3 && a != c && a < DIM && c < DIM)
                          ? (SH ? m.du[a] * (R(2) * rf.ur[a] + m.du[a]) * m.u[c] + rf.ur[a] * rf.ur[a] * m.du[c]
                                : m.u[a] * m.u[a] * m.u[c])
                          : R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        R dc = R(0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (cdir<DIM>(i, a) > 0) dc += m.du[a];
            if (cdir<DIM>(i, a) < 0) dc -= m.du[a];
        }
        R b = SH ? dc * (R(g.k2[i]) + R(4.5) * dc) - R(1.5) * m.q : dc * (R(3) + R(4.5) * dc) - R(1.5) * m.uu;
        if constexpr (EQ == 3) {
            R t = R(0);
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    if (a == c || cdir<DIM>(i, c) == 0) continue;
                    const R h = (cdir<DIM>(i, a) != 0 ? R(1) : R(0)) - R(1) / R(3);
                    if (cdir<DIM>(i, c) > 0) t += h * T[a][c];
                    else t -= h * T[a][c];
                }
            b += R(13.5) * t;
        }
        out[i] = SH ? m.drho * R(g.k1[i]) + R(Lat<DIM>::w[i]) * rho * b : R(Lat<DIM>::w[i]) * rho * (R(1) + b);
    }
}

// Reciprocal: in FP32 the hardware estimate refined by one Newton step
// (r + r (1 - x r), two FMAs; the bare 1-ulp estimate biases u step after
// step), exact division in FP64.
template <typename R>
__device__ __forceinline__ R recip(R x)
{
    if constexpr (sizeof(R) == 4) {
        const float r = __builtin_amdgcn_rcpf(x);
        return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
    } else {
        return R(1) / x;
    }
}

// Element index of direction i at node (x, y, z).
template <int DIM>
__device__ __forceinline__ int64_t eoff(const LevelDev& g, int i, int x, int y, int z)
{
    return (((int64_t)z * g.ny + y) * g.nxb + (x >> g.xsh)) * ((int64_t)Lat<DIM>::Q << g.xsh) +
           ((int64_t)i << g.xsh) + (x & ((1 << g.xsh) - 1));
}

template <int DIM>
__device__ __forceinline__ bool on_xface(const LevelDev& g, int x)
{
    return DIM == 3 && g.xface && (x == 0 || x == g.nx - 1);
}

// Element index of direction i at x-face node (x, y, z) in the face buffer.
template <int DIM>
__device__ __forceinline__ int64_t xfoff(const LevelDev& g, int x, int i, int y, int z)
{
    return (((int64_t)(x == 0 ? 0 : 1) * Lat<DIM>::Q + i) * g.nz + z) * g.ny + y;
}

// Direction i of node (x, y, z) is one that an x-face node pulls from the
// plane next to it (and so is kept in xn as well).
template <int DIM>
__device__ __forceinline__ bool on_xnext(const LevelDev& g, int x, int i)
{
    return DIM == 3 && g.xn[0] != nullptr &&
           ((x == 1 && cdir<DIM>(i, 0) == -1) || (x == g.nx - 2 && cdir<DIM>(i, 0) == 1));
}

// Its element in xn[par] (side 0 for x = 1, side 1 for x = nx - 2).
template <int DIM>
__device__ __forceinline__ int64_t xnoff(const LevelDev& g, int x, int i, int y, int z)
{
    return xfoff<DIM>(g, x == 1 ? 0 : g.nx - 1, i, y, z);
}

// Direction i of node (x, y, z) in the state of parity par (base = f[par]).
template <int DIM, typename T>
__device__ __forceinline__ T* node_elem(const LevelDev& g, T* base, int par, int i, int x, int y, int z)
{
    if (on_xface<DIM>(g, x)) return reinterpret_cast<T*>(g.xf[par]) + xfoff<DIM>(g, x, i, y, z);
    return base + eoff<DIM>(g, i, x, y, z);
}

// Pull-stream source of direction i: node (x, y, z) - xi_i, periodic on level 0.
template <int DIM>
__device__ __forceinline__ int64_t src_off(const LevelDev& g, int x, int y, int z, int i)
{
    int sx = x - cdir<DIM>(i, 0), sy = y - cdir<DIM>(i, 1), sz = z - cdir<DIM>(i, 2);
    if (g.periodic) {
        sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
        sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
        if (DIM == 3) sz = sz < 0 ? sz + g.nz : (sz >= g.nz ? sz - g.nz : sz);
    }
    return eoff<DIM>(g, i, sx, sy, sz);
}

// The same source as an element pointer of the state of parity par.
template <int DIM, typename T>
__device__ __forceinline__ const T* pull_elem(const LevelDev& g, const T* src, int par, int x, int y, int z, int i)
{
    int sx = x - cdir<DIM>(i, 0), sy = y - cdir<DIM>(i, 1), sz = z - cdir<DIM>(i, 2);
    if (g.periodic) {
        sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
        sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
        if (DIM == 3) sz = sz < 0 ? sz + g.nz : (sz >= g.nz ? sz - g.nz : sz);
    }
    if (on_xnext<DIM>(g, sx, i)) return reinterpret_cast<const T*>(g.xn[par]) + xnoff<DIM>(g, sx, i, sy, sz);
    return node_elem<DIM>(g, const_cast<T*>(src), par, i, sx, sy, sz);
}

// Store of direction i of node (x, y, z) into the state of parity par
// through the cache, with its second copy where an x face pulls it.
template <int DIM, int P>
__device__ __forceinline__ void store_node_wb(const LevelDev& g, typename Form<P>::T* base, int par, int i, int x,
                                              int y, int z, typename Form<P>::R v)
{
    using T = typename Form<P>::T;
    Form<P>::store_wb(node_elem<DIM>(g, base, par, i, x, y, z), v);
    if (on_xnext<DIM>(g, x, i)) Form<P>::store_wb(reinterpret_cast<T*>(g.xn[par]) + xnoff<DIM>(g, x, i, y, z), v);
}

// A box level's interface nodes and holes (from its box and its child's).
template <int DIM>
__device__ __forceinline__ bool is_interface_or_hole_box(const LevelDev& g, int x, int y, int z)
{
    if (g.boundary &&
        (x == 0 || x == g.nx - 1 || y == 0 || y == g.ny - 1 || (DIM == 3 && (z == 0 || z == g.nz - 1))))
        return true;
    if (g.has_child && x >= g.clo[0] && x <= g.chi[0] && y >= g.clo[1] && y <= g.chi[1] &&
        (DIM == 2 || (z >= g.clo[2] && z <= g.chi[2])))
        return true;
    return false;
}

// Any level: a refined region's class bytes, else the box.
template <int DIM>
__device__ __forceinline__ bool is_interface_or_hole(const LevelDev& g, int x, int y, int z)
{
    if (g.cls) return g.cls[((int64_t)z * g.ny + y) * g.nx + x] != kClsBulk;
    return is_interface_or_hole_box<DIM>(g, x, y, z);
}

template <int DIM>
__device__ __forceinline__ bool is_hole(const LevelDev& g, int x, int y, int z)
{
    if (g.cls) return g.cls[((int64_t)z * g.ny + y) * g.nx + x] == kClsHole;
    return g.has_child && x > g.clo[0] && x < g.chi[0] && y > g.clo[1] && y < g.chi[1] &&
           (DIM == 2 || (z > g.clo[2] && z < g.chi[2]));
}

// Weights of a hanging node's stencil on a refined region's boundary, by the
// type the host stored in bits 24-26 of its metadata: 1 centred (-1, 9, 9,
// -1)/16, 2 one-sided (5, 15, -5, 1)/16 (the host orders the points away
// from the step), 3 linear (1/2, 1/2) on a run of one parent cell.
__device__ __forceinline__ void typed_weights(int type, float w[4])
{
    if (type == 1) {
        w[0] = -1.f / 16; w[1] = 9.f / 16; w[2] = 9.f / 16; w[3] = -1.f / 16;
    } else if (type == 2) {
        w[0] = 5.f / 16; w[1] = 15.f / 16; w[2] = -5.f / 16; w[3] = 1.f / 16;
    } else {
        w[0] = 0.5f; w[1] = 0.5f; w[2] = 0.f; w[3] = 0.f;
    }
}

// 4-point stencil along one axis for odd position k on a line 0..N:
// centred (-1,9,9,-1)/16 at k-3..k+3, one-sided (5,15,-5,1)/16 at line ends
// (nodes 0,2,4,6 or N,N-2,N-4,N-6).
__device__ __forceinline__ void line_weights(int k, int N, float w[4])
{
    if (k == 1 || k == N - 1) {
        w[0] = 5.f / 16; w[1] = 15.f / 16; w[2] = -5.f / 16; w[3] = 1.f / 16;
    } else {
        w[0] = -1.f / 16; w[1] = 9.f / 16; w[2] = 9.f / 16; w[3] = -1.f / 16;
    }
}

// ---------------------------------------------------------------- the level-substep kernel
// Every role runs in workgroups of kBlock threads.  A segment holds at most
// TF co-located nodes in LDS (own + halo, one per thread) and IE hanging
// nodes (two passes of the workgroup).
constexpr int kBlock = 256;
template <int DIM>
struct SegLimits {
    static constexpr int TF = DIM == 2 ? 136 : 256;
    static constexpr int IE = 2 * kBlock;
};

// Bulk tiles are 64 x 4 nodes.  A tile row is the tx tiles sharing one
// (4-row group, z).  Workgroups are dealt round-robin to the 8 XCDs, so
// workgroup b = 8 m + c runs on XCD c; it takes tile m % tx of tile row
// c + 8 (m / tx).  Each XCD walks whole tile rows (x neighbours, whose
// shifted pulls share cache lines, stay in one L2) and the rows of all XCDs
// interleave over the domain (holes do not leave some XCDs idle).
struct TileMap {
    int tx, ty;      // tiles per tile row, 4-row groups per plane
    int nrows;       // tile rows: ty * nz
    int per;         // tiles per XCD: tx * ceil(nrows / 8)
    int blk;         // tile rows dealt to an XCD at a time (1: row by row)
};

// Tile row of XCD c's rr-th row: rows are dealt to the 8 XCDs in turns of
// tm.blk consecutive rows (blk = 1 interleaves single rows over the XCDs).
__device__ __forceinline__ int tile_row(const TileMap& tm, int c, int rr)
{
    return tm.blk == 1 ? c + 8 * rr : c * tm.blk + rr % tm.blk + 8 * tm.blk * (rr / tm.blk);
}

// Bulk workgroups of a level with k tiles per workgroup (bulk_k).
__host__ __device__ constexpr int bulk_groups(int per, int k) { return 8 * ((per + k - 1) / k); }

// Probes of one simulation: at most one per lane of a wave (the probe
// launch is one wave, the probe workgroup of a level launch samples with its
// first kMaxProbes threads).
constexpr int kMaxProbes = 64;

struct ProbeArgs {
    int n;
    int64_t capacity;
    const void* buf[kMaxProbes];   // storage buffer holding the probe's node
    int64_t off[kMaxProbes];       // element offset of direction 0 of that node
    int64_t stride[kMaxProbes];    // element distance between directions (the row-block width, or nz * ny in a face buffer)
};

struct LevelArgs {
    LevelDev g;
    const void* src;      // f[par]
    void* dst;            // f[par ^ 1]
    int par;
    double keep;          // 1 - 1/tau_l
    TileMap tm;
    int nb_cap, nb_seg;   // workgroups of the capture and segment roles
    int seg_groups;       // ceil(nb_seg / 8): segment workgroups are padded to a multiple of 8
    int seg_every;        // 0: the segment groups precede the bulk; else one segment group follows
                          // every seg_every bulk groups (seg_groups * seg_every <= bulk groups)
    // capture (level has a child): coarse co-located nodes of this level
    const int4* cap_meta; // (x, y, z, K^c mask)
    int n_cap;
    void* H_own;          // this level's ring [3][Q][n_cap]
    // segments (level has a parent)
    const int4* seg_info; // (tf_off, tf_cnt, ie_off, ie_cnt)
    const int* seg_tf;    // co-located index | owned << 30
    const int4* seg_tfm;  // the co-located node's metadata, per seg_tf entry
    const int* seg_ie;    // hanging-node index (the identity: hanging nodes are numbered in segment order)
    const int* seg_sten;  // [16][n_ie] local stencil indices into the segment's co-located list
    int n_ie;
    const int4* tf_meta;  // (x, y, z, Gamma=R mask)
    const int4* ie_meta;  // (x, y, z, missing mask)
    int n_tf;
    const void* H_parent; // parent's ring [3][Q][n_tf]
    void* X;              // [4][n_tf] shared state (drho, u) of co-located nodes
    int substep;          // 1 asynchronous, 2 synchronous
    int first;            // parent made a single step: linear time interpolation
    int maxit;
    double Rfac;          // tau_l / (2 tau_{l-1}), Eq.(fneqResc)
    double tol;
    int* flags;           // bit 0: Newton failure, bit 1: non-finite or non-positive density (every level)
    // restriction into the parent at synchronous substeps
    LevelDev gp;
    void* dst_parent;
    const int4* tfc_meta; // parent coordinates of each co-located node (same order)
    double keep_parent;
    // level 0 of a single simulation: one extra workgroup samples the probes
    // of the previous coarse step (this launch only reads level 0's state and
    // does not touch the finer levels), so a step needs no probe launch
    int nb_probe;           // 0 or 1
    const ProbeArgs* probe; // the probe buffers of the state this launch starts from
    double* series;
    int64_t* counter;       // [0] steps sampled, [1] coarse steps started, [2, 3] the sums' window, [4] steps summed
    double* psums;          // running sums of the probes, [3][n]
    // H-RR on refined meshes: the interface role stores completed
    // pre-collision populations and their macroscopic state instead of
    // colliding (the level collides after its child's substeps)
    void* M;                // this level's (drho, du) [4][n]
    void* M_parent;         // the parent's, for its co-located nodes at the synchronous substep
};

// A non-finite or non-positive density (a run that has become unstable)
// latches flag bit 2.  The test costs a compare per node, so every step
// checks every node; a wave holding such a node sets the flag from one lane,
// and only if it is not set yet (a diverged state is NaN everywhere: one
// atomic per lane would serialise the whole launch on one address).
__device__ __forceinline__ void flag_unstable_if(bool bad_lane, int* flags)
{
    const unsigned long long bad = __ballot(bad_lane);
    if (bad != 0ull && __lane_id() == (unsigned)(__ffsll((unsigned long long)bad) - 1)) {
        if (!(__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2)) atomicOr(flags, 2);
    }
}

template <typename R>
__device__ __forceinline__ void flag_unstable(R rho, int* flags)
{
    flag_unstable_if(!(rho > R(0) && rho < R(1e30)), flags);
}

template <int DIM, int P>
__device__ __forceinline__ void role_capture(const LevelArgs& a, int b)
{
    using F = Form<P>;
    using T = typename F::T;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    const int t = b * kBlock + threadIdx.x;
    if (t >= a.n_cap) return;
    const int4 m = a.cap_meta[t];
    const T* src = (const T*)a.src;
    R* H = (R*)a.H_own;
    const int64_t n = a.n_cap, slot = (int64_t)Q * n;
    // loads of a chunk of directions before its stores (the ring slots do not
    // alias, but the compiler cannot know it); chunks bound the registers held
    constexpr int CH = 7;
#pragma unroll
    for (int i0 = 0; i0 < Q; i0 += CH) {
        R v[CH], h1[CH], h2[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = i0 + c;
            const bool k = i < Q && ((m.w >> i) & 1);
            v[c] = k ? F::load(src + src_off<DIM>(a.g, m.x, m.y, m.z, i)) : R(0);
            h1[c] = k ? H[slot + i * n + t] : R(0);
            h2[c] = k ? H[2 * slot + i * n + t] : R(0);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = i0 + c;
            if (i >= Q || !((m.w >> i) & 1)) continue;
            H[i * n + t] = h1[c];
            H[slot + i * n + t] = h2[c];
            H[2 * slot + i * n + t] = v[c];
        }
    }
}

template <int DIM>
__device__ __forceinline__ int64_t dense_index(const LevelDev& g, int x, int y, int z)
{
    return ((int64_t)z * g.ny + y) * g.nx + x;
}

// (drho, du) of node d into a [4][n] array (in 2-D the third velocity
// component is neither written nor read)
template <int DIM, typename R>
__device__ __forceinline__ void put_mac(void* Mv, int64_t n, int64_t d, R drho, const R du[3])
{
    R* M = (R*)Mv;
    M[d] = drho;
    M[n + d] = du[0];
    M[2 * n + d] = du[1];
    if (DIM == 3) M[3 * n + d] = du[2];
}

// HRR: the H-RR refined-mesh mode (no collision; see LevelArgs::M).
template <int DIM, int EQ, int P, bool ROLLED, bool HRR = false, bool RG = false>
__device__ __forceinline__ void role_segment(const LevelArgs& a, int sgi, typename Form<P>::R* lds,
                                             std::bool_constant<ROLLED> = {})
{
    using F = Form<P>;
    using T = typename F::T;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    constexpr int TFM = SegLimits<DIM>::TF;
    const int4 info = a.seg_info[sgi];
    const T* src = (const T*)a.src;
    T* dst = (T*)a.dst;
    constexpr bool SH = F::shifted;
    const Ref<R> rf = ref_of<R>(a.g);
    const int j = threadIdx.x;
    // ---- phase 1: co-located nodes (own and halo).  Column j of the LDS
    // tile holds the node's h (fine value where Gamma = 1, time-interpolated
    // coarse value where Gamma = R), then its completed populations.  Only
    // thread j touches column j before the barrier, so the column is plain
    // LDS: a volatile column went through flat accesses, each waited for,
    // which serialised the Q loads of the node behind one another.
    if (j < info.y) {
        // index and metadata in one round trip (not index, then metadata)
        const int e = a.seg_tf[info.x + j];
        const int4 m = a.seg_tfm[info.x + j];
        const int t = e & 0x3fffffff;
        const bool owned = (e >> 30) & 1;
        const uint32_t gR = (uint32_t)m.w;
        const R* H = (const R*)a.H_parent;
        const int64_t n = a.n_tf, slot = (int64_t)Q * n;
        R* col = lds + j;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            R v;
            if ((gR >> i) & 1u) {
                const R Hm = H[i * n + t], H0 = H[slot + i * n + t], Hp = H[2 * slot + i * n + t];
                if (a.substep == 2)
                    v = Hp;
                else if (a.first)
                    v = R(0.5) * H0 + R(0.5) * Hp;
                else
                    v = R(-0.125) * Hm + R(0.75) * H0 + R(0.375) * Hp;
            } else {
                v = F::load(pull_elem<DIM>(a.g, src, a.par, m.x, m.y, m.z, i));
            }
            col[i * TFM] = v;
        }
        auto hv = [&](int i) -> R { return col[i * TFM]; };
        R drho, du[3];
        int it;
        // the constants table is only used where the Newton loop is unrolled:
        // a loop-counter index into the serving kernel's register copy of the
        // arguments would put that copy in scratch
        if constexpr (SH && EQ == 2 && !ROLLED)
            it = newton_v<DIM, EQ, SH, R, decltype(hv), EqGradShift2<DIM, R>, ROLLED>(
                hv, gR, R(a.Rfac), rf, R(a.tol), a.maxit, drho, du, EqGradShift2<DIM, R>{a.g});
        else
            it = newton_v<DIM, EQ, SH, R, decltype(hv), EqGrad<DIM, EQ, SH, R>, ROLLED>(
                hv, gR, R(a.Rfac), rf, R(a.tol), a.maxit, drho, du, EqGrad<DIM, EQ, SH, R>{rf});
        if (it < 0) {
            R jj[3] = {R(0), R(0), R(0)};
            drho = R(0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const R v = hv(i);
                drho += v;
                jj[0] += R(cdir<DIM>(i, 0)) * v;
                jj[1] += R(cdir<DIM>(i, 1)) * v;
                jj[2] += R(cdir<DIM>(i, 2)) * v;
            }
            velocity<DIM, SH, R>(rf, drho, jj, du);
            // non-convergence on finite inputs is a Newton failure (bit 1);
            // non-finite inputs are an instability (bit 2)
            if (owned) {
                const R rho = (SH ? R(1) : R(0)) + drho;
                atomicOr(a.flags, (rho > R(0) && rho < R(1e30)) ? 1 : 2);
            }
        }
        const Mac<R> mx = make_mac<DIM, SH, R>(rf, drho, du);
        auto eq0 = [&](int i) -> R {
            if constexpr (SH && EQ == 2) {
                R e, gr[4];
                EqGradShift2<DIM, R>{a.g}(i, mx, e, gr);
                return e;
            } else {
                return eq_s<DIM, EQ, SH, R>(i, rf, mx);
            }
        };
        // Eq.(rescff) on every coarse-coupled direction
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if ((gR >> i) & 1u) {
                const R e0 = eq0(i);
                col[i * TFM] = e0 + R(a.Rfac) * (col[i * TFM] - e0);
            }
        }
        if (owned) {
            R* X = (R*)a.X;
            X[t] = drho;
            X[n + t] = mx.du[0];
            X[2 * n + t] = mx.du[1];
            X[3 * n + t] = mx.du[2];
            if (a.substep == 2) {
                // Eq.(rescfc): every coarse population from the completed fine
                // ones, then the coarse collision with X (H-RR: the coarse
                // level collides them later, from these values and X)
                const int4 pm = a.tfc_meta[t];
                const R invR = R(1.0 / a.Rfac), keepp = R(a.keep_parent);
                T* dp = (T*)a.dst_parent;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const R e0 = eq0(i);
                    const R c = e0 + invR * (col[i * TFM] - e0);
                    F::store_wb(dp + eoff<DIM>(a.gp, i, pm.x, pm.y, pm.z), HRR ? c : e0 + keepp * (c - e0));
                }
                if constexpr (HRR)
                    put_mac<DIM, R>(a.M_parent, (int64_t)a.gp.nx * a.gp.ny * a.gp.nz,
                               dense_index<DIM>(a.gp, pm.x, pm.y, pm.z), mx.drho, mx.du);
            }
            const R keep = R(a.keep);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const R e0 = eq0(i);
                store_node_wb<DIM, P>(a.g, dst, a.par ^ 1, i, m.x, m.y, m.z,
                                      HRR ? R(col[i * TFM]) : e0 + keep * (col[i * TFM] - e0));
            }
            if constexpr (HRR)
                put_mac<DIM, R>(a.M, (int64_t)a.g.nx * a.g.ny * a.g.nz, dense_index<DIM>(a.g, m.x, m.y, m.z), mx.drho,
                           mx.du);
        }
    }
    __syncthreads();
    // ---- phase 2: hanging nodes
    for (int je = j; je < info.w; je += kBlock) {
        const int q0 = info.z + je;
        const int4 m = a.ie_meta[q0];   // hanging nodes are numbered in segment order
        const int k[3] = {m.x, m.y, m.z};
        const int N[3] = {a.g.nx - 1, a.g.ny - 1, a.g.nz - 1};
        // odd axes in increasing order carry the stencil; the first one is fastest
        // (picked with compile-time indices only, so nothing lands in scratch)
        int ka = 0, Na = 0, kb = 0, Nb = 0, no = 0;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            if (k[ax] & 1) {
                if (no == 0) {
                    ka = k[ax];
                    Na = N[ax];
                } else {
                    kb = k[ax];
                    Nb = N[ax];
                }
                ++no;
            }
        }
        float w0[4], w1[4] = {1.f, 0.f, 0.f, 0.f};
        // a refined region's hanging nodes carry their stencil's weight type
        // (compiled only into the region kernels: in the box kernels the
        // extra branch spilled registers)
        const int wtype = RG ? (m.w >> 24) & 7 : 0;
        if (RG && wtype)
            typed_weights(wtype, w0);
        else
            line_weights(ka, Na, w0);
        if (no == 2) line_weights(kb, Nb, w1);
        const int ns = no == 2 ? 16 : 4;
        const uint32_t miss = (uint32_t)m.w & 0xffffffu;
        R s[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            s[i] = ((miss >> i) & 1u) ? R(0) : F::load(pull_elem<DIM>(a.g, src, a.par, m.x, m.y, m.z, i));
#pragma unroll
        for (int q = 0; q < (DIM == 2 ? 4 : 16); ++q) {
            if (q < ns) {
                const int idx = a.seg_sten[(int64_t)q * a.n_ie + q0];
                const R wq = R(w0[q & 3]) * R(w1[q >> 2]);
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if ((miss >> i) & 1u) s[i] += wq * lds[i * TFM + idx];
            }
        }
        R drho, jj[3], du[3];
        moments<DIM, R>(s, drho, jj);
        flag_unstable((SH ? R(1) : R(0)) + drho, a.flags);
        velocity<DIM, SH, R>(rf, drho, jj, du);
        if constexpr (HRR)
            put_mac<DIM, R>(a.M, (int64_t)a.g.nx * a.g.ny * a.g.nz, dense_index<DIM>(a.g, m.x, m.y, m.z), drho, du);
        else
            bgk<DIM, EQ, SH, R>(s, rf, make_mac<DIM, SH, R>(rf, drho, du), R(a.keep));
#pragma unroll
        for (int i = 0; i < Q; ++i) store_node_wb<DIM, P>(a.g, dst, a.par ^ 1, i, m.x, m.y, m.z, s[i]);
    }
}

// Bulk tile bb (64 x 4 nodes), first half: the node's pull-stream loads.
// Returns false for lanes without a bulk node (beyond the level, interface
// nodes, holes), which load nothing.
template <int DIM, int P>
__device__ __forceinline__ bool bulk_load(const LevelArgs& a, int bb, typename Form<P>::R s[], int64_t& e0,
                                          int* xyz = nullptr)
{
    using F = Form<P>;
    using T = typename F::T;
    constexpr int Q = Lat<DIM>::Q;
    const TileMap& tm = a.tm;
    const int m = bb >> 3;
    const int rr = m / tm.tx;
    const int row = tile_row(tm, bb & 7, rr);
    if (row >= tm.nrows) return false;
    const int z = row / tm.ty;
    const int ty = row - z * tm.ty;
    const int x = (m - rr * tm.tx) * 64 + (threadIdx.x & 63);
    const int y = ty * 4 + (threadIdx.x >> 6);
    if (xyz) {
        xyz[0] = x;
        xyz[1] = y;
        xyz[2] = z;
    }
    const LevelDev& g = a.g;
    if (x >= g.nx || y >= g.ny) return false;
    if (is_interface_or_hole<DIM>(g, x, y, z)) return false;
    const T* src = (const T*)a.src;
    // pull sources: the node's element plus per-axis neighbour deltas (the
    // x blocks and the periodic wrap of level 0 resolved once per node), so
    // each direction costs one add
    const int xsh = g.xsh, xm1 = (1 << xsh) - 1;
    const int64_t BX = (int64_t)1 << xsh;
    const int64_t XQ = (int64_t)Q << xsh;
    const int64_t rowe = (int64_t)g.nxb * XQ, plane = rowe * g.ny;
    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1, zm = z - 1, zp = z + 1;
    if (g.periodic) {
        xm = xm < 0 ? xm + g.nx : xm;
        xp = xp >= g.nx ? xp - g.nx : xp;
        ym = ym < 0 ? ym + g.ny : ym;
        yp = yp >= g.ny ? yp - g.ny : yp;
        if (DIM == 3) {
            zm = zm < 0 ? zm + g.nz : zm;
            zp = zp >= g.nz ? zp - g.nz : zp;
        }
    }
    const int64_t ex = (int64_t)(x >> xsh) * XQ + (x & xm1);
    // index c + 1 for xi component c: the source is at coordinate - c
    const int64_t dx[3] = {(int64_t)(xp >> xsh) * XQ + (xp & xm1) - ex, 0, (int64_t)(xm >> xsh) * XQ + (xm & xm1) - ex};
    const int64_t dy[3] = {(int64_t)(yp - y) * rowe, 0, (int64_t)(ym - y) * rowe};
    const int64_t dz[3] = {(int64_t)(zp - z) * plane, 0, (int64_t)(zm - z) * plane};
    e0 = (int64_t)z * plane + (int64_t)y * rowe + ex;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        s[i] = F::load(src + (e0 + dx[cdir<DIM>(i, 0) + 1] + dy[cdir<DIM>(i, 1) + 1] +
                              (DIM == 3 ? dz[cdir<DIM>(i, 2) + 1] : 0) + i * BX));
    if constexpr (DIM == 3) {
        // next to an x face the +x (x = 1) or -x (x = nx - 2) directions
        // come from the face buffer
        if (g.xface && (x == 1 || x == g.nx - 2)) {
            const int c = x == 1 ? 1 : -1;
            const int fx = x == 1 ? 0 : g.nx - 1;
            const T* xs = reinterpret_cast<const T*>(g.xf[a.par]);
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (cdir<DIM>(i, 0) == c)
                    s[i] = F::load(xs + xfoff<DIM>(g, fx, i, y - cdir<DIM>(i, 1), z - cdir<DIM>(i, 2)));
        }
    }
    return true;
}

// BGK collision of one bulk node in place (moments, reference velocity
// split, equilibrium); returns its density.
template <int DIM, int EQ, int P>
__device__ __forceinline__ typename Form<P>::R bulk_collide(const LevelArgs& a, typename Form<P>::R s[])
{
    using F = Form<P>;
    using R = typename F::R;
    const LevelDev& g = a.g;
    constexpr bool SH = F::shifted;
    const Ref<R> rf = ref_of<R>(g);
    R drho, j[3], du[3];
    moments<DIM, R>(s, drho, j);
    const R rho = (SH ? R(1) : R(0)) + drho;
    const R inv = recip<R>(rho);
#pragma unroll
    for (int c = 0; c < 3; ++c) du[c] = c < DIM ? (SH ? j[c] - drho * rf.ur[c] : j[c]) * inv : R(0);
    if constexpr (SH && EQ == 2)
        bgk_shift2<DIM, R>(s, g, drho, du, R(a.keep));
    else
        bgk<DIM, EQ, SH, R>(s, rf, make_mac<DIM, SH, R>(rf, drho, du), R(a.keep));
    return rho;
}

// Second half: moments, BGK collision and the store of the node's element e0.
template <int DIM, int EQ, int P>
__device__ __forceinline__ void bulk_update(const LevelArgs& a, int64_t e0, typename Form<P>::R s[])
{
    using F = Form<P>;
    using T = typename F::T;
    constexpr int Q = Lat<DIM>::Q;
    const int64_t BX = (int64_t)1 << a.g.xsh;
    flag_unstable(bulk_collide<DIM, EQ, P>(a, s), a.flags);
    T* d = (T*)a.dst + e0;
#pragma unroll
    for (int i = 0; i < Q; ++i) F::store(d + i * BX, s[i]);
}

// Raw buffer access through a descriptor (base, size in bytes).  An offset
// at or past the size loads 0 and stores nothing, without a memory access:
// lanes without a node pass such an offset instead of branching around the
// access.
template <int BYTES>
struct Buf;
template <>
struct Buf<2> {
    __device__ static __forceinline__ unsigned short ld(__amdgpu_buffer_rsrc_t r, uint32_t o)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, o, 0, 0);
    }
    __device__ static __forceinline__ void st_nt(__amdgpu_buffer_rsrc_t r, uint32_t o, unsigned short v)
    {
        __builtin_amdgcn_raw_buffer_store_b16(v, r, o, 0, 2);
    }
};
template <>
struct Buf<4> {
    __device__ static __forceinline__ uint32_t ld(__amdgpu_buffer_rsrc_t r, uint32_t o)
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0);
    }
    __device__ static __forceinline__ void st_nt(__amdgpu_buffer_rsrc_t r, uint32_t o, uint32_t v)
    {
        __builtin_amdgcn_raw_buffer_store_b32(v, r, o, 0, 2);
    }
};
template <>
struct Buf<8> {
    using V2 = uint32_t __attribute__((ext_vector_type(2)));
    __device__ static __forceinline__ V2 ld(__amdgpu_buffer_rsrc_t r, uint32_t o)
    {
        return __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0);
    }
    __device__ static __forceinline__ void st_nt(__amdgpu_buffer_rsrc_t r, uint32_t o, V2 v)
    {
        __builtin_amdgcn_raw_buffer_store_b64(v, r, o, 0, 2);
    }
};

// Carried value <-> raw storage bits of each form.
template <int P>
using RawOf = std::conditional_t<P == 0, Buf<8>::V2, std::conditional_t<P == 1, uint32_t, unsigned short>>;
template <int P>
__device__ __forceinline__ typename Form<P>::R from_bits(RawOf<P> b)
{
    if constexpr (P == 0) return __builtin_bit_cast(double, b);
    else if constexpr (P == 1) return __builtin_bit_cast(float, b);
    else return __half2float(__ushort_as_half(b)) * (1.0f / Form<2>::scale);
}
template <int P>
__device__ __forceinline__ RawOf<P> to_bits(typename Form<P>::R v)
{
    if constexpr (P == 0) return __builtin_bit_cast(Buf<8>::V2, v);
    else if constexpr (P == 1) return __builtin_bit_cast(uint32_t, v);
    else return __half_as_ushort(__float2half_rn(v * Form<2>::scale));
}

// Fused pull-stream + BGK of bulk tile bb (64 x 4 nodes, one row of 64
// nodes per wave), in parts so that a workgroup can fetch several tiles
// before it collides the first.  The row of a wave is the same for all its
// lanes, so the 3^(D-1) source rows are buffer descriptors in scalar
// registers; a lane forms the byte offsets of its three x sources (x - 1,
// x, x + 1, wrapped on level 0) and each direction adds a constant that the
// load takes as its immediate offset.  No 64-bit address arithmetic per
// direction, and no branch around a load or store: a lane without a bulk
// node passes offsets past the row, for which the hardware loads 0 and
// stores nothing.  The values are those of bulk_load / bulk_update.
template <int DIM, int P>
struct BulkTile {
    typename Form<P>::R s[Lat<DIM>::Q];
    __amdgpu_buffer_rsrc_t rs[DIM == 3 ? 9 : 3];   // source rows (y - cy, z - cz) at (cy + 1) + 3 (cz + 1)
    __amdgpu_buffer_rsrc_t rd;                       // destination row
    int ox[3];                                       // byte offsets of x + 1, x, x - 1 (past the row: none)
    int x, y, z;
    bool v;                                          // the lane holds a bulk node
    bool any;                                        // the wave holds one
};

// Where tile bb's wave reads and writes; tile_ok false makes it a tile
// without nodes.
// RG: the level (or its child) is a refined region, whose node classes are
// read from its class bytes.  Box levels keep the box test: the class read
// in the tile's locate step raised the 2-D kernels' register demand enough
// to spill part of the tile state to scratch.
template <int DIM, int P, bool RG = false>
__device__ __forceinline__ void bulk_locate(const LevelArgs& a, int bb, BulkTile<DIM, P>& t, bool tile_ok = true)
{
    using T = typename Form<P>::T;
    constexpr int Q = Lat<DIM>::Q;
    const TileMap& tm = a.tm;
    const LevelDev& g = a.g;
    const int m = bb >> 3;
    const int rr = m / tm.tx;
    const int row = tile_row(tm, bb & 7, rr);
    const bool in = tile_ok && row < tm.nrows;
    const int z = in ? row / tm.ty : 0;
    const int y = __builtin_amdgcn_readfirstlane(in ? (row - z * tm.ty) * 4 + (int)(threadIdx.x >> 6) : 0);
    const int x = (m - rr * tm.tx) * 64 + (int)(threadIdx.x & 63);
    t.x = x;
    t.y = y;
    t.z = z;
    if constexpr (RG)
        t.v = in && y < g.ny && x < g.nx && !is_interface_or_hole<DIM>(g, x, y, z);
    else
        t.v = in && y < g.ny && x < g.nx && !is_interface_or_hole_box<DIM>(g, x, y, z);
    t.any = __ballot(t.v) != 0ull;
    // 64-node row blocks (the level's xsh): a compile-time width, so that
    // each direction's offset is an immediate of the access
    constexpr int xsh = kRowShift, xm1 = (1 << xsh) - 1;
    const int64_t XQ = (int64_t)Q << xsh;
    const int64_t rowe = (int64_t)g.nxb * XQ;                 // elements per row
    const int rbytes = (int)(rowe * (int64_t)sizeof(T));
    const int none = rbytes;                                  // past the row
    // a wave with a bulk node lies inside a refined level; level 0 wraps
    // (the rows of a wave without one are never accessed)
    int ys[3] = {y + 1, y, y - 1}, zs[3] = {z + 1, z, z - 1}; // source of xi = c at index c + 1
    int xs[3] = {x + 1, x, x - 1};
    if (g.periodic) {
#pragma unroll
        for (int k = 0; k < 3; k += 2) {
            ys[k] = ys[k] < 0 ? ys[k] + g.ny : (ys[k] >= g.ny ? ys[k] - g.ny : ys[k]);
            zs[k] = zs[k] < 0 ? zs[k] + g.nz : (zs[k] >= g.nz ? zs[k] - g.nz : zs[k]);
            xs[k] = xs[k] < 0 ? xs[k] + g.nx : (xs[k] >= g.nx ? xs[k] - g.nx : xs[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) t.ox[k] = t.v ? ((xs[k] >> xsh) * (int)XQ + (xs[k] & xm1)) * (int)sizeof(T) : none;
    auto rsrc = [&](const void* base, int yy, int zz) {
        return __builtin_amdgcn_make_buffer_rsrc(
            (void*)((const T*)base + ((int64_t)(DIM == 3 ? zz : 0) * g.ny + yy) * rowe), (short)0, rbytes, 0x00020000);
    };
#pragma unroll
    for (int cz = 0; cz < (DIM == 3 ? 3 : 1); ++cz)
#pragma unroll
        for (int cy = 0; cy < 3; ++cy) t.rs[cy + 3 * cz] = rsrc(a.src, ys[cy], zs[DIM == 3 ? cz : 1]);
    t.rd = rsrc(a.dst, ys[1], zs[1]);
}

// The tile's pull-stream loads.
template <int DIM, int P>
__device__ __forceinline__ void bulk_pull(const LevelArgs& a, BulkTile<DIM, P>& t)
{
    using F = Form<P>;
    using T = typename F::T;
    using B = Buf<sizeof(T)>;
    constexpr int Q = Lat<DIM>::Q;
    const LevelDev& g = a.g;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cdir<DIM>(i, 0), cy = cdir<DIM>(i, 1), cz = DIM == 3 ? cdir<DIM>(i, 2) : 0;
        // none + the direction's constant stays past the row (a row is far
        // below 2^31 bytes), so it needs no select; signed, the add cannot
        // wrap and folds into the immediate offset
        t.s[i] = from_bits<P>(B::ld(t.rs[(cy + 1) + 3 * (cz + 1) * (DIM == 3)],
                                    (uint32_t)(t.ox[cx + 1] + i * ((int)sizeof(T) << kRowShift))));
    }
    if constexpr (DIM == 3) {
        // next to an x face the +x (x = 1) or -x (x = nx - 2) directions
        // come from the face buffer; one arm per face, so that each arm's
        // direction set is fixed and its loads issue as one batch
        if (g.xface) {
            const T* xfb = reinterpret_cast<const T*>(g.xf[a.par]);
            if (t.v && t.x == 1) {
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if (cdir<DIM>(i, 0) == 1)
                        t.s[i] = F::load(xfb + xfoff<DIM>(g, 0, i, t.y - cdir<DIM>(i, 1), t.z - cdir<DIM>(i, 2)));
            } else if (t.v && t.x == g.nx - 2) {
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if (cdir<DIM>(i, 0) == -1)
                        t.s[i] =
                            F::load(xfb + xfoff<DIM>(g, g.nx - 1, i, t.y - cdir<DIM>(i, 1), t.z - cdir<DIM>(i, 2)));
            }
        }
    }
}

// Collision and stores of the tile.  The stores are issued by every wave
// (a wave without a bulk node stores nothing: offsets past the row), so
// that the memory counter is the same on both paths and a following tile's
// loads are waited for alone.
template <int DIM, int EQ, int P>
__device__ __forceinline__ void bulk_finish(const LevelArgs& a, BulkTile<DIM, P>& t)
{
    using F = Form<P>;
    using T = typename F::T;
    using R = typename F::R;
    using B = Buf<sizeof(T)>;
    constexpr int Q = Lat<DIM>::Q;
    if (t.any) {                                              // whole wave
        const R rho = bulk_collide<DIM, EQ, P>(a, t.s);
        flag_unstable_if(t.v && !(rho > R(0) && rho < R(1e30)), a.flags);
    }
#pragma unroll
    for (int i = 0; i < Q; ++i)
        B::st_nt(t.rd, (uint32_t)(t.ox[1] + i * ((int)sizeof(T) << kRowShift)), to_bits<P>(t.s[i]));
    if constexpr (DIM == 3) {
        // the planes next to the x faces: the directions the faces pull,
        // a second time into xn
        const LevelDev& g = a.g;
        if (g.xn[0] && t.v && (t.x == 1 || t.x == g.nx - 2)) {
            T* xb = reinterpret_cast<T*>(g.xn[a.par ^ 1]);
            const int c = t.x == 1 ? -1 : 1;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (cdir<DIM>(i, 0) == c) F::store_wb(xb + xnoff<DIM>(g, t.x, i, t.y, t.z), t.s[i]);
        }
    }
}

template <int DIM, int EQ, int P, bool RG = false>
__device__ __forceinline__ void role_bulk(const LevelArgs& a, int bb)
{
    BulkTile<DIM, P> t;
    bulk_locate<DIM, P, RG>(a, bb, t);
    if (!t.any) return;                                       // whole wave
    bulk_pull<DIM, P>(a, t);
    bulk_finish<DIM, EQ, P>(a, t);
}

// Bulk workgroup b of a launch: bulk_k tiles, fetched together, then
// collided and stored in turn (twice the bytes in flight per wave for the
// same per-node work).  Two tiles pay only with FP16 storage, whose 2-byte
// loads keep the fewest bytes in flight: in every 2-D kernel, and in the 3-D
// kernel that carries the segment role (seg), whose registers hold it at 4
// waves per SIMD (256^3 level 1: 331 -> 310 us); the 3-D FP16 kernels
// without it run at 8 waves, where a second tile cost 2-7% (the 512^3
// 4-level mesh).  Workgroup b = 8 q + c (on XCD c) takes the tiles
// 8 (q k + j) + c, j < k, so each XCD still walks whole tile rows.
__host__ __device__ constexpr int bulk_k(int dim, int p, bool seg = false)
{
    return p == 2 && (dim == 2 || seg) ? 2 : 1;
}

template <int DIM, int EQ, int P, bool RG = false, int K = bulk_k(DIM, P)>
__device__ __forceinline__ void role_bulk_group(const LevelArgs& a, int b)
{
    if constexpr (K == 1) {
        role_bulk<DIM, EQ, P, RG>(a, b);
    } else {
        const int c = b & 7, q = b >> 3;
        BulkTile<DIM, P> t[K];
        bool any = false;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int m = q * K + j;   // past the level's tiles: a tile without nodes
            bulk_locate<DIM, P, RG>(a, 8 * m + c, t[j], m < a.tm.per);
            any = any || t[j].any;
        }
        if (!any) return;                                     // whole wave
#pragma unroll
        for (int j = 0; j < K; ++j) bulk_pull<DIM, P>(a, t[j]);
#pragma unroll
        for (int j = 0; j < K; ++j) bulk_finish<DIM, EQ, P>(a, t[j]);
    }
}

// p' = (rho - 1)/3 in FP64 of every probe (thread p), appended to the series
// at row *counter while the series has room; thread 0 then advances the
// counter.  One workgroup.
// sums (null: none kept): when the step lies in the window [counter[2],
// counter[3]), the running sums of the probes take it, whatever the
// series' capacity: the FP64 sums from which the sound pressure level of
// Sec. 4.2 follows for runs of any length.  They are kept about the
// window's first sample K (shifted data, so that a mean far above the
// fluctuations does not cancel them): sums[2n + p] = K (NaN until the first
// sample), sums[p] += d and sums[n + p] += d^2 (the product rounded on its
// own) with d = p' - K; counter[4] counts the steps taken.
template <int DIM, int P>
__device__ __forceinline__ void probe_sample(const ProbeArgs& a, double* series, int64_t* counter, double* sums)
{
    using F = Form<P>;
    constexpr int Q = Lat<DIM>::Q;
    const int64_t step = *counter;
    const int p = threadIdx.x;
    const bool keep = step < a.capacity;
    const bool add = sums && step >= counter[2] && step < counter[3];
    if (p < a.n && (keep || add)) {
        const typename F::T* b = reinterpret_cast<const typename F::T*>(a.buf[p]) + a.off[p];
        double r = F::rho0;
        for (int i = 0; i < Q; ++i) r += (double)F::load(b + i * a.stride[p]);
        const double pp = (r - 1.0) / 3.0;
        if (keep) series[step * a.n + p] = pp;
        if (add) {
            // the square is rounded before the add (no fused multiply-add),
            // so the sums are those of a plain sequential loop
#pragma clang fp contract(off)
            double K = sums[2 * a.n + p];
            if (K != K) sums[2 * a.n + p] = K = pp;
            const double d = pp - K;
            sums[p] += d;
            sums[a.n + p] += d * d;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *counter = step + 1;
        if (add) counter[4] += 1;
    }
}

// Probes of a finished coarse step not sampled yet (counter[0] < counter[1]).
template <int DIM, int P>
__device__ __forceinline__ void probe_pending(const ProbeArgs& pa, double* series, int64_t* counter, double* sums)
{
    const int64_t done = counter[0], started = counter[1];
    if (done < started) probe_sample<DIM, P>(pa, series, counter, sums);
}

// Workgroup b of a level substep.  Grid order: the probe workgroup (level 0
// of a single simulation), the capture workgroups, the interface segments
// (padded to a multiple of 8), then the bulk tiles.  Segment work is
// latency-bound (Newton, gathers) and bulk work bandwidth-bound: placed
// ahead of the bulk, the segments overlap the bulk tiles and stay out of the
// launch's tail.  In 2-D they all go first (spreading them over the grid, or
// placing them after the bulk rows they touch, measured slower).  A 3-D face
// has so many segments that, all first, they hold most of the chip's wave
// slots while they run and starve the bulk; there seg_every interleaves
// them, one group of 8 after every seg_every groups of 8 bulk workgroups, over
// the front of the grid.  Groups of 8 keep bulk workgroup b' on XCD b' % 8 up
// to a fixed rotation, as TileMap assumes.  Every thread of the workgroup
// calls this with the same arguments (the segment role synchronises).
// Returns true when the workgroup used the LDS (segment role).
// ROLLED keeps the Newton loop over directions rolled.  That caps the
// register demand the segment role imposes on the whole kernel: 3-D FP32
// 108 VGPRs, 4 waves/SIMD; 2-D FP16 70 VGPRs, 7 waves/SIMD (unrolled, 91
// and 5).  2-D FP32/FP64 keep the unrolled loop.
template <int DIM, int EQ, int P, bool ROLLED = (DIM == 3 || P == 2), bool SEG = true, bool RG = false>
__device__ __forceinline__ bool level_block(const LevelArgs& a, int b, typename Form<P>::R* lds)
{
    if (b < a.nb_probe) {
        // sample the previous step, then count this one as started
        const int64_t started = a.counter[1];
        probe_pending<DIM, P>(*a.probe, a.series, a.counter, a.psums);
        __syncthreads();
        if (threadIdx.x == 0) a.counter[1] = started + 1;
        return false;
    }
    b -= a.nb_probe;
    if (b < a.nb_cap) {
        role_capture<DIM, P>(a, b);
        return false;
    }
    const int b2 = b - a.nb_cap;
    // the segment workgroup sb, or (sb < 0) the bulk workgroup bb; one call
    // site per role (a second one put the kernel's arguments in scratch)
    int sb = -1, bb = b2 - 8 * a.seg_groups;
    if (a.seg_every > 0) {
        const int G = b2 >> 3, r = b2 & 7, per = a.seg_every + 1;
        const int k = G / per, q = G - k * per;
        if (k < a.seg_groups) {
            if (q == 0)
                sb = 8 * k + r;
            else
                bb = 8 * (k * a.seg_every + q - 1) + r;
        } else {
            bb = 8 * (a.seg_groups * a.seg_every + G - a.seg_groups * per) + r;
        }
    } else if (bb < 0) {
        sb = b2;
    }
    if (sb >= 0) {
        if constexpr (SEG) {
            if (sb < a.nb_seg) {
                role_segment<DIM, EQ, P, ROLLED, false, RG>(a, sb, lds);
                return true;
            }
        }
        return false;
    }
    role_bulk_group<DIM, EQ, P, RG, bulk_k(DIM, P, SEG)>(a, bb);
    return false;
}

template <int DIM, int EQ, int P, bool RG = false>
__global__ __launch_bounds__(kBlock) void k_level(LevelArgs a)
{
    using R = typename Form<P>::R;
    __shared__ R lds[Lat<DIM>::Q * SegLimits<DIM>::TF];
    level_block<DIM, EQ, P, (DIM == 3 || P == 2), true, RG>(a, blockIdx.x, lds);
}

// The same level substep as two kernels that run side by side (3-D, FP16
// storage, levels whose bulk far outweighs their faces): the bulk tiles
// alone, which then run at the occupancy of their own register demand, and
// the probe, capture and interface-segment workgroups.  The two write
// disjoint nodes and read only the source buffers, so neither waits for the
// other.
template <int DIM, int EQ, int P>
__global__ __launch_bounds__(kBlock) void k_bulk(LevelArgs a)
{
    role_bulk_group<DIM, EQ, P>(a, blockIdx.x);
}

template <int DIM, int EQ, int P>
__global__ __launch_bounds__(kBlock) void k_iface(LevelArgs a)
{
    using R = typename Form<P>::R;
    __shared__ R lds[Lat<DIM>::Q * SegLimits<DIM>::TF];
    level_block<DIM, EQ, P>(a, blockIdx.x, lds);   // the grid ends before the bulk tiles (seg_every 0)
}

// Level 0 has no parent interface, so its launch has no segment workgroups:
// compiled without the segment role, the kernel needs only the bulk's
// registers and runs at a higher occupancy (used for FP16 storage).
template <int DIM, int EQ, int P, bool RG = false>
__global__ __launch_bounds__(kBlock) void k_level_top(LevelArgs a)
{
    level_block<DIM, EQ, P, true, false, RG>(a, blockIdx.x, nullptr);
}

// ---------------------------------------------------------------- H-RR collision
// The hybrid recursive regularised collision of Sec. 2 needs the velocity
// and third-order moment gradients of the post-streaming state, so a level
// substep takes two launches: k_hrr_macros pulls and writes each bulk node's
// (drho, du) into M and, on a refined level, completes the co-located and
// hanging nodes (role_segment in its H-RR mode) and writes their populations
// and M without colliding; after the child's substeps k_hrr_collide pulls
// the bulk again, reads M at each node and its 2 D axis neighbours (centred
// differences, Eq.(a1FD_scheme), Eq.(PSI_FD)) and collides every node:
//   psi_i   = -w_i/(2c^4) H2_i:(div Psi)          (App. A; the sign that
//             cancels the lattice's missing third-order moments Psi)
//   a1      = sigma sum_i H2_i (f_i - f0_i + psi_i/2) + (1 - sigma) a1FD
//   a1FD_ab = -tau rho c^2 (d_b u_a + d_a u_b)
//   f*_i    = f0_i + (1 - 1/tau) w_i [H2_i:a1/(2c^4)
//             + sum_{a!=b} H3_{i,aab} (2 u_a a1_ab + u_b a1_aa)/(2c^6)] + psi_i/2
// with Psi = rho u_a^3 on aaa and, in D3Q19, rho u_b u_g^2/2 on aab (g the
// remaining axis) and rho u_x u_y u_z on xyz.  Gradients by node class
// (Sec. 3.3, Sec. 3.5): bulk and coarse co-located nodes use the level's
// stencil (a neighbour in the hole takes the child node co-located with
// it); fine co-located nodes the coarse stencil of +-2 fine cells, whose
// points outside the level are parent nodes (time-interpolated at the
// asynchronous substep), so that the difference over 4 fine cells is the
// S^c/2, psi^c/2 of Eq.(PijResc), Eq.(PSIResc); hanging nodes interpolate
// the co-located nodes' gradients with their populations' weights.
struct HrrArgs {
    LevelArgs a;          // the level substep: source, destination, tiles, probes, captures, segments, flags
    void* M;              // [4][n] (drho, du) of every node, arithmetic type, x fastest
    double tau, sigma;
    int psi;              // cubic Mach correction on
    // refined meshes (null / 0 on a single level)
    void* Mring;              // this level's post-streaming (drho, du) at three coarse times, [3][4][n],
                              // written only at the nodes next to the child's box (the ones its
                              // co-located nodes' stencils reach)
    int ring_new;             // physical slot of Mring that this substep's values go to
    const void* M_child;      // the child's M (gradients of this level's coarse co-located nodes)
    int cn[3];                // the child's extents
    const void* Mring_parent; // the parent's ring (gradients of this level's co-located nodes)
    int pslot[3];             // physical slots of the parent's values at t - dt, t, t + dt
    int plo[3];               // this level's box origin in the parent's node coordinates
    const int* ie_tf;         // [16][n_ie] co-located indices of each hanging node's stencil
    int nb_bulk;              // bulk workgroups of either launch
};

// Psi_abg of Eq.(Psi) at one node, for the index pattern (a, b, g).
template <int DIM, typename R>
__device__ __forceinline__ R hrr_Psi(int a, int b, int g, R rho, const R u[3])
{
    if (a == b && b == g) return rho * u[a] * u[a] * u[a];
    if (DIM == 2) return R(0);
    if (a != b && b != g && a != g) return rho * u[0] * u[1] * u[2];
    const int dbl = a == b ? a : (a == g ? a : b);
    const int sgl = a == b ? g : (a == g ? b : a);
    const int third = 3 - dbl - sgl;
    return R(0.5) * rho * u[sgl] * u[third] * u[third];
}

// (rho, u) of the carried (drho, du) at a [4][n] array's entry d.
template <int DIM, bool SH, typename R>
__device__ __forceinline__ void rho_u_at(const R* M, int64_t n, int64_t d, const Ref<R>& rf, R& rho, R u[3])
{
    rho = (SH ? R(1) : R(0)) + M[d];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = (k < DIM ? M[(1 + k) * n + d] : R(0)) + (SH ? rf.ur[k] : R(0));
}

// Centred differences along axis c from the two stencil points (index 0 at
// -h, 1 at +h): inv2h = 1 / (2 h).
template <int DIM, typename R>
__device__ __forceinline__ void hrr_axis(int c, R inv2h, const R rn[2], const R un[2][3], int psi, R gradu[3][3],
                                         R dPsi[3][3])
{
    // d_c u_a (du differences equal u differences)
#pragma unroll
    for (int k = 0; k < DIM; ++k) gradu[k][c] = inv2h * (un[1][k] - un[0][k]);
    if (psi) {
#pragma unroll
        for (int p = 0; p < DIM; ++p)
#pragma unroll
            for (int q = p; q < DIM; ++q)
                dPsi[p][q] += inv2h * (hrr_Psi<DIM, R>(p, q, c, rn[1], un[1]) - hrr_Psi<DIM, R>(p, q, c, rn[0], un[0]));
    }
}

template <typename R>
__device__ __forceinline__ void zero33(R a[3][3])
{
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) a[r][c] = R(0);
}

// The H-RR collision of one node in place: s holds its (completed)
// pre-collision populations, mc its macroscopic state, gradu its velocity
// gradients d_c u_a, dPsi the upper triangle of sum_g d_g Psi_abg.
template <int DIM, int EQ, int P>
__device__ __forceinline__ void hrr_collide_node(const LevelDev& g, const Ref<typename Form<P>::R>& rf,
                                                 const Mac<typename Form<P>::R>& mc, typename Form<P>::R s[],
                                                 typename Form<P>::R gradu[3][3], typename Form<P>::R dPsi[3][3],
                                                 double keepd, double taud, double sigd, int psi_on)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    constexpr bool SH = F::shifted;
    const R rho = (SH ? R(1) : R(0)) + mc.drho;
#pragma unroll
    for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < p; ++q) dPsi[p][q] = dPsi[q][p];
    // The Hermite contractions use only the non-zero lattice components
    // (compile-time), H2_{i,pq} = xi_p xi_q - c^2 delta_pq:
    //   sum_i H2_{i,pq} x_i = sum_{xi_p xi_q != 0} xi_p xi_q x_i - c^2 delta_pq sum_i x_i
    //   H2_i : A            = sum_{xi_p, xi_q != 0} xi_p xi_q A_pq - c^2 tr A
    constexpr R c2 = R(1) / R(3);
    const R keep = R(keepd), tau = R(taud), sig = R(sigd);
    R trP = R(0);
#pragma unroll
    for (int p = 0; p < DIM; ++p) trP += dPsi[p][p];
    R f0[Q], psi[Q];
    eq_all<DIM, EQ, SH, R>(g, rf, mc, f0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        R t = -c2 * trP;
#pragma unroll
        for (int p = 0; p < DIM; ++p)
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                const int cc = cdir<DIM>(i, p) * cdir<DIM>(i, q);
                if (cc == 1) t += dPsi[p][q];
                if (cc == -1) t -= dPsi[p][q];
            }
        psi[i] = psi_on ? -R(Lat<DIM>::w[i]) * R(4.5) * t : R(0);   // w_i / (2 c^4) = 4.5 w_i
    }
    // second moments of x_i = s_i - f0_i + psi_i / 2
    R m0 = R(0), m2[3][3];
    zero33(m2);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R xv = s[i] - f0[i] + R(0.5) * psi[i];
        m0 += xv;
#pragma unroll
        for (int p = 0; p < DIM; ++p)
#pragma unroll
            for (int q = p; q < DIM; ++q) {
                const int cc = cdir<DIM>(i, p) * cdir<DIM>(i, q);
                if (cc == 1) m2[p][q] += xv;
                if (cc == -1) m2[p][q] -= xv;
            }
    }
    R a1[3][3];
#pragma unroll
    for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = p; q < DIM; ++q) {
            const R pr = m2[p][q] - (p == q ? c2 * m0 : R(0));
            const R fd = -tau * rho * c2 * (gradu[p][q] + gradu[q][p]);
            a1[p][q] = sig * pr + (R(1) - sig) * fd;
            a1[q][p] = a1[p][q];
        }
    R tr1 = R(0);
#pragma unroll
    for (int p = 0; p < DIM; ++p) tr1 += a1[p][p];
    // a_1^(3)_ppq = 2 u_p a1_pq + u_q a1_pp (Eq.(a13RR)), p != q
    R A3[3][3];
#pragma unroll
    for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) A3[p][q] = p == q ? R(0) : R(2) * mc.u[p] * a1[p][q] + mc.u[q] * a1[p][p];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        R t2 = -c2 * tr1, t3 = R(0);
#pragma unroll
        for (int p = 0; p < DIM; ++p)
#pragma unroll
            for (int q = 0; q < DIM; ++q) {
                const int cc = cdir<DIM>(i, p) * cdir<DIM>(i, q);
                if (cc == 1) t2 += a1[p][q];
                if (cc == -1) t2 -= a1[p][q];
                // H3_{i,ppq} = (xi_p^2 - c^2) xi_q, p != q
                if (p != q && cdir<DIM>(i, q) != 0) {
                    const R h3 = (cdir<DIM>(i, p) != 0 ? R(1) - c2 : -c2);
                    if (cdir<DIM>(i, q) > 0) t3 += h3 * A3[p][q];
                    else t3 -= h3 * A3[p][q];
                }
            }
        const R f1 = R(Lat<DIM>::w[i]) * (R(4.5) * t2 + R(13.5) * t3);   // 1/(2c^4), 1/(2c^6)
        s[i] = f0[i] + keep * f1 + R(0.5) * psi[i];
    }
}

// Workgroups of an H-RR macroscopic launch: the probe (level 0), the coarse
// capture (levels with a child), the interface segments (refined levels:
// completion of the co-located and hanging nodes without collision), then
// the bulk tiles, each bulk node writing its post-streaming (drho, du) into
// M and, next to the child's box, into the newest slot of the level's ring.
// The segments go ahead of the bulk, so that their latency-bound work
// overlaps it (one launch measured 13% faster per coarse step than the
// segments in a launch of their own beside it on a second stream); in 3-D
// they are interleaved over the front of the bulk in groups of 8, as in the
// BGK launch (LevelArgs::seg_every).
// SEG: the level has segments (without them the kernel holds no LDS and
// needs fewer registers); RG: they lie on a refined region's boundary.
template <int DIM, int EQ, int P, bool SEG, bool RG = false>
__global__ __launch_bounds__(kBlock) void k_hrr_macros(HrrArgs h)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    __shared__ R lds[SEG ? Q * SegLimits<DIM>::TF : 1];
    const LevelArgs& a = h.a;
    int b = blockIdx.x;
    if (b < a.nb_probe) {
        // the previous coarse step's probes, from the state this step reads
        const int64_t started = a.counter[1];
        probe_pending<DIM, P>(*a.probe, a.series, a.counter, a.psums);
        __syncthreads();
        if (threadIdx.x == 0) a.counter[1] = started + 1;
        return;
    }
    b -= a.nb_probe;
    if (b < a.nb_cap) {
        role_capture<DIM, P>(a, b);
        return;
    }
    b -= a.nb_cap;
    if constexpr (SEG) {
        // the segment workgroup sb, or (sb < 0) the bulk workgroup b
        int sb = -1;
        if (a.seg_every > 0) {
            const int G = b >> 3, r = b & 7, per = a.seg_every + 1;
            const int k = G / per, q = G - k * per;
            if (k < a.seg_groups) {
                if (q == 0)
                    sb = 8 * k + r;
                else
                    b = 8 * (k * a.seg_every + q - 1) + r;
            } else {
                b = 8 * (a.seg_groups * a.seg_every + G - a.seg_groups * per) + r;
            }
        } else if (b < a.nb_seg) {
            sb = b;
        } else {
            b -= a.nb_seg;
        }
        if (sb >= 0) {
            if (sb < a.nb_seg) role_segment<DIM, EQ, P, true, true, RG>(a, sb, lds);
            return;
        }
    }
    R s[Q];
    int64_t e0 = 0;
    int xyz[3];
    if (!bulk_load<DIM, P>(a, b, s, e0, xyz)) return;
    const LevelDev& g = a.g;
    const int x = xyz[0], y = xyz[1], z = xyz[2];
    constexpr bool SH = F::shifted;
    const Ref<R> rf = ref_of<R>(g);
    R drho, j[3], du[3];
    moments<DIM, R>(s, drho, j);
    flag_unstable((SH ? R(1) : R(0)) + drho, a.flags);
    velocity<DIM, SH, R>(rf, drho, j, du);
    const int64_t n = (int64_t)g.nx * g.ny * g.nz, d = dense_index<DIM>(g, x, y, z);
    put_mac<DIM, R>(h.M, n, d, drho, du);
    // a bulk node within one node of the child's box (the box itself holds
    // no bulk nodes)
    if (h.Mring && x >= g.clo[0] - 1 && x <= g.chi[0] + 1 && y >= g.clo[1] - 1 && y <= g.chi[1] + 1 &&
        (DIM == 2 || (z >= g.clo[2] - 1 && z <= g.chi[2] + 1)))
        put_mac<DIM, R>((R*)h.Mring + (int64_t)h.ring_new * 4 * n, n, d, drho, du);
}

// Gradients of co-located node t of a refined level on the coarse stencil:
// the points +-2 fine cells along each axis inside the level are its own
// nodes, those outside are parent nodes, whose ring is read with the weights
// of Eq.(TempInt) at the asynchronous substep (linear while the parent has
// one capture) and at t + dt^c at the synchronous one.
template <int DIM, bool SH, typename R>
__device__ __forceinline__ void tf_gradients(const HrrArgs& h, int t, const Ref<R>& rf, R gradu[3][3], R dPsi[3][3])
{
    const LevelArgs& a = h.a;
    const int4 m = a.tf_meta[t];
    const LevelDev& g = a.g;
    const LevelDev& gp = a.gp;
    const R* M = (const R*)h.M;
    const R* Rp = (const R*)h.Mring_parent;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz, np = (int64_t)gp.nx * gp.ny * gp.nz;
    const R* Hm = Rp + (int64_t)h.pslot[0] * 4 * np;
    const R* H0 = Rp + (int64_t)h.pslot[1] * 4 * np;
    const R* Hp = Rp + (int64_t)h.pslot[2] * 4 * np;
    const int k[3] = {m.x, m.y, m.z}, n3[3] = {g.nx, g.ny, g.nz};
    zero33(gradu);
    zero33(dPsi);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        R rn[2], un[2][3];
#pragma unroll
        for (int sg = 0; sg < 2; ++sg) {
            int q3[3] = {k[0], k[1], k[2]};
            q3[c] += sg ? 2 : -2;
            // a point that is not a node of this level (beyond it, or missing
            // from a refined region) is a bulk node of the parent
            if (q3[c] >= 0 && q3[c] < n3[c] && !is_hole<DIM>(g, q3[0], q3[1], q3[2])) {
                rho_u_at<DIM, SH, R>(M, n, dense_index<DIM>(g, q3[0], q3[1], q3[2]), rf, rn[sg], un[sg]);
            } else {
                int P3[3] = {0, 0, 0};
#pragma unroll
                for (int e = 0; e < DIM; ++e) P3[e] = h.plo[e] + k[e] / 2;
                P3[c] += sg ? 1 : -1;
                const int64_t dp = dense_index<DIM>(gp, P3[0], P3[1], P3[2]);
                R v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const R vm = Hm[e * np + dp], v0 = H0[e * np + dp], vp = Hp[e * np + dp];
                    v[e] = a.substep == 2 ? vp
                                          : (a.first ? R(0.5) * v0 + R(0.5) * vp
                                                     : R(-0.125) * vm + R(0.75) * v0 + R(0.375) * vp);
                }
                rn[sg] = (SH ? R(1) : R(0)) + v[0];
#pragma unroll
                for (int e = 0; e < 3; ++e) un[sg][e] = (e < DIM ? v[1 + e] : R(0)) + (SH ? rf.ur[e] : R(0));
            }
        }
        hrr_axis<DIM, R>(c, R(0.25), rn, un, h.psi, gradu, dPsi);
    }
}

// Macroscopic state of a node from M.
template <int DIM, bool SH, typename R>
__device__ __forceinline__ Mac<R> mac_at(const R* M, int64_t n, int64_t d, const Ref<R>& rf)
{
    R du[3] = {M[n + d], M[2 * n + d], DIM == 3 ? M[3 * n + d] : R(0)};
    return make_mac<DIM, SH, R>(rf, M[d], du);
}

// Workgroups of an H-RR collide launch: on a refined level its co-located
// nodes and its hanging nodes, on a level with a child its coarse co-located
// nodes (these read their completed populations back from the destination;
// they come first, so that their longer dependent chains of loads overlap
// the bulk), then the bulk tiles (pulled again).
template <int DIM, int EQ, int P>
__global__ __launch_bounds__(kBlock) void k_hrr_collide(HrrArgs h)
{
    using F = Form<P>;
    using T = typename F::T;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    constexpr bool SH = F::shifted;
    const LevelArgs& a = h.a;
    const LevelDev& g = a.g;
    const Ref<R> rf = ref_of<R>(g);
    const R* M = (const R*)h.M;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int n3[3] = {g.nx, g.ny, g.nz};
    int b = blockIdx.x;
    R s[Q], gradu[3][3], dPsi[3][3];
    zero33(gradu);
    zero33(dPsi);
    const int ntf = a.tf_meta ? a.n_tf : 0, nie = a.ie_meta ? a.n_ie : 0, ncap = a.cap_meta ? a.n_cap : 0;
    const int gtf = (ntf + kBlock - 1) / kBlock, gie = (nie + kBlock - 1) / kBlock;
    const int gif = gtf + gie + (ncap + kBlock - 1) / kBlock;
    if (b >= gif) {
        b -= gif;
        int64_t e0 = 0;
        int xyz[3];
        if (!bulk_load<DIM, P>(a, b, s, e0, xyz)) return;
        // this node's macroscopic state (as written by k_hrr_macros from the same pulls)
        const int64_t d0 = dense_index<DIM>(g, xyz[0], xyz[1], xyz[2]);
        const Mac<R> mc = mac_at<DIM, SH, R>(M, n, d0, rf);
        // neighbours -e_c (0) and +e_c (1) along each axis, periodic on level 0
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            R un[2][3], rn[2];
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                int q3[3] = {xyz[0], xyz[1], xyz[2]};
                q3[c] += sg ? 1 : -1;
                q3[c] = q3[c] < 0 ? q3[c] + n3[c] : (q3[c] >= n3[c] ? q3[c] - n3[c] : q3[c]);
                rho_u_at<DIM, SH, R>(M, n, dense_index<DIM>(g, q3[0], q3[1], q3[2]), rf, rn[sg], un[sg]);
            }
            hrr_axis<DIM, R>(c, R(0.5), rn, un, h.psi, gradu, dPsi);
        }
        hrr_collide_node<DIM, EQ, P>(g, rf, mc, s, gradu, dPsi, a.keep, h.tau, h.sigma, h.psi);
        T* dst = (T*)a.dst + e0;
        const int64_t BX = (int64_t)1 << g.xsh;
#pragma unroll
        for (int i = 0; i < Q; ++i) F::store(dst + i * BX, s[i]);
        return;
    }
    T* dst = (T*)a.dst;
    int4 m;
    if (b < gtf) {
        // co-located nodes: the coarse stencil
        const int t = b * kBlock + threadIdx.x;
        if (t >= ntf) return;
        m = a.tf_meta[t];
        tf_gradients<DIM, SH, R>(h, t, rf, gradu, dPsi);
    } else if (b < gtf + gie) {
        // hanging nodes: the co-located nodes' gradients with the weights of
        // their populations' 4-point stencils (the first odd axis fastest)
        const int q0 = (b - gtf) * kBlock + threadIdx.x;
        if (q0 >= nie) return;
        m = a.ie_meta[q0];
        const int k[3] = {m.x, m.y, m.z};
        const int N[3] = {g.nx - 1, g.ny - 1, g.nz - 1};
        int ka = 0, Na = 0, kb = 0, Nb = 0, no = 0;
#pragma unroll
        for (int ax = 0; ax < DIM; ++ax) {
            if (k[ax] & 1) {
                if (no == 0) {
                    ka = k[ax];
                    Na = N[ax];
                } else {
                    kb = k[ax];
                    Nb = N[ax];
                }
                ++no;
            }
        }
        float w0[4], w1[4] = {1.f, 0.f, 0.f, 0.f};
        const int wtype = (m.w >> 24) & 7;
        if (wtype)
            typed_weights(wtype, w0);
        else
            line_weights(ka, Na, w0);
        if (no == 2) line_weights(kb, Nb, w1);
        const int ns = no == 2 ? 16 : 4;
        for (int qq = 0; qq < ns; ++qq) {
            const int t = h.ie_tf[(int64_t)qq * nie + q0];
            const R wq = R(w0[qq & 3]) * R(w1[qq >> 2]);
            R gu[3][3], gp[3][3];
            tf_gradients<DIM, SH, R>(h, t, rf, gu, gp);
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    gradu[p][q] += wq * gu[p][q];
                    dPsi[p][q] += wq * gp[p][q];
                }
        }
    } else {
        // coarse co-located nodes: the level's stencil, a neighbour in the
        // hole taken from the child node co-located with it
        const int t = (b - gtf - gie) * kBlock + threadIdx.x;
        if (t >= ncap) return;
        m = a.cap_meta[t];
        const R* Mc = (const R*)h.M_child;
        const int64_t nc = (int64_t)h.cn[0] * h.cn[1] * h.cn[2];
        const int k[3] = {m.x, m.y, m.z};
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            R un[2][3], rn[2];
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                int q3[3] = {k[0], k[1], k[2]};
                q3[c] += sg ? 1 : -1;
                q3[c] = q3[c] < 0 ? q3[c] + n3[c] : (q3[c] >= n3[c] ? q3[c] - n3[c] : q3[c]);
                if (is_hole<DIM>(g, q3[0], q3[1], q3[2])) {
                    const int cx = 2 * (q3[0] - g.clo[0]), cy = 2 * (q3[1] - g.clo[1]),
                              cz = DIM == 3 ? 2 * (q3[2] - g.clo[2]) : 0;
                    rho_u_at<DIM, SH, R>(Mc, nc, ((int64_t)cz * h.cn[1] + cy) * h.cn[0] + cx, rf, rn[sg], un[sg]);
                } else {
                    rho_u_at<DIM, SH, R>(M, n, dense_index<DIM>(g, q3[0], q3[1], q3[2]), rf, rn[sg], un[sg]);
                }
            }
            hrr_axis<DIM, R>(c, R(0.5), rn, un, h.psi, gradu, dPsi);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) s[i] = F::load(node_elem<DIM>(g, dst, a.par ^ 1, i, m.x, m.y, m.z));
    const Mac<R> mc = mac_at<DIM, SH, R>(M, n, dense_index<DIM>(g, m.x, m.y, m.z), rf);
    hrr_collide_node<DIM, EQ, P>(g, rf, mc, s, gradu, dPsi, a.keep, h.tau, h.sigma, h.psi);
#pragma unroll
    for (int i = 0; i < Q; ++i) F::store_wb(node_elem<DIM>(g, dst, a.par ^ 1, i, m.x, m.y, m.z), s[i]);
}

// The three slots of an H-RR level's macroscopic-field ring from its initial
// fields (dense FP64 rho [n], u [D][n]), in the carried variables.
template <int DIM, int P>
__global__ __launch_bounds__(256) void k_hrr_ring_init(LevelDev g, void* Mring, const double* __restrict__ rho,
                                                       const double* __restrict__ u)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr bool SH = F::shifted;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    R v[4];
    v[0] = R(SH ? rho[d] - 1.0 : rho[d]);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[1 + k] = k < DIM ? R(u[k * n + d] - (SH ? g.ur[k] : 0.0)) : R(0);
    R* Rg = (R*)Mring;
#pragma unroll
    for (int slot = 0; slot < 3; ++slot)
#pragma unroll
        for (int c = 0; c < 4; ++c) Rg[(4 * slot + c) * n + d] = v[c];
}

// Absorbing layer on level 0 (one thread per node; nodes outside the layer
// return at once): f_i <- f_i - s(x) (f0_i(rho, u) - f0_i(1, u_t)) on the
// state of parity par, with s(x) = sigma ((W - e) / W)^2 and e the node's
// distance in cells to the domain's outermost nodes.
template <int DIM, int EQ, int P>
__global__ __launch_bounds__(256) void k_sponge(LevelDev g, void* f, int par, int W, double sigma, double tx, double ty,
                                                double tz)
{
    using F = Form<P>;
    using T = typename F::T;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    constexpr bool SH = F::shifted;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const int k[3] = {(int)(d % g.nx), (int)((d / g.nx) % g.ny), (int)(d / ((int64_t)g.nx * g.ny))};
    const int n3[3] = {g.nx, g.ny, g.nz};
    int e = g.nx;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int ea = k[a] < n3[a] - 1 - k[a] ? k[a] : n3[a] - 1 - k[a];
        e = ea < e ? ea : e;
    }
    if (e >= W) return;
    const double r = (double)(W - e) / (double)W;
    const R sg = R(sigma * r * r);
    const Ref<R> rf = ref_of<R>(g);
    T* base = (T*)f;
    R s[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) s[i] = F::load(node_elem<DIM>(g, base, par, i, k[0], k[1], k[2]));
    R drho, j[3], du[3];
    moments<DIM, R>(s, drho, j);
    velocity<DIM, SH, R>(rf, drho, j, du);
    R f0[Q], ft[Q];
    eq_all<DIM, EQ, SH, R>(g, rf, make_mac<DIM, SH, R>(rf, drho, du), f0);
    // the target (1, u_t) in the carried variables
    const R dut[3] = {R(tx) - (SH ? rf.ur[0] : R(0)), R(ty) - (SH ? rf.ur[1] : R(0)),
                      DIM == 3 ? R(tz) - (SH ? rf.ur[2] : R(0)) : R(0)};
    eq_all<DIM, EQ, SH, R>(g, rf, make_mac<DIM, SH, R>(rf, SH ? R(0) : R(1), dut), ft);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        F::store(node_elem<DIM>(g, base, par, i, k[0], k[1], k[2]), s[i] - sg * (f0[i] - ft[i]));
}

// Centred-difference velocity divergence of a level's dense FP64 velocity
// [D][n] (NaN at holes, so a stencil touching a hole gives NaN); stencil
// points beyond a refined level's extent give NaN, level 0 wraps.
template <int DIM>
__global__ __launch_bounds__(256) void k_divergence(LevelDev g, const double* __restrict__ u, double* __restrict__ out)
{
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    const int k[3] = {(int)(d % g.nx), (int)((d / g.nx) % g.ny), (int)(d / ((int64_t)g.nx * g.ny))};
    const int n3[3] = {g.nx, g.ny, g.nz};
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        int qm[3] = {k[0], k[1], k[2]}, qp[3] = {k[0], k[1], k[2]};
        qm[c] -= 1;
        qp[c] += 1;
        if (g.periodic) {
            qm[c] = qm[c] < 0 ? qm[c] + n3[c] : qm[c];
            qp[c] = qp[c] >= n3[c] ? qp[c] - n3[c] : qp[c];
        } else if (qm[c] < 0 || qp[c] >= n3[c]) {
            s = __builtin_nan("");
            continue;
        }
        s += 0.5 * (u[c * n + dense_index<DIM>(g, qp[0], qp[1], qp[2])] - u[c * n + dense_index<DIM>(g, qm[0], qm[1], qm[2])]);
    }
    out[d] = s;
}

// ---------------------------------------------------------------- history ring init
template <int DIM, int P>
__global__ __launch_bounds__(128) void k_ring_init(LevelDev g, const typename Form<P>::T* __restrict__ src,
                                                   const int4* __restrict__ meta, int n,
                                                   typename Form<P>::R* __restrict__ H)
{
    using F = Form<P>;
    constexpr int Q = Lat<DIM>::Q;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int4 m = meta[t];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const auto v = F::load(src + eoff<DIM>(g, i, m.x, m.y, m.z));
        for (int r = 0; r < 3; ++r) H[((int64_t)r * Q + i) * n + t] = v;
    }
}

// ---------------------------------------------------------------- init / conversion
// Dense [n] / [D][n] arrays are indexed d = (z*ny + y)*nx + x.
template <int DIM, int EQ, int P>
__global__ __launch_bounds__(256) void k_init(LevelDev g, typename Form<P>::T* __restrict__ dst, int par,
                                              const double* __restrict__ rho, const double* __restrict__ u)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    if (is_hole<DIM>(g, x, y, z)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) dst[eoff<DIM>(g, i, x, y, z)] = F::nan();
        return;
    }
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t d = ((int64_t)z * g.ny + y) * g.nx + x;
    // equilibrium evaluated in FP64, then carried in the storage form
    constexpr bool SH = F::shifted;
    const Ref<double> rf = ref_of<double>(g);
    const double uu3[3] = {u[d], u[n + d], DIM == 3 ? u[2 * n + d] : 0.0};
    const double du[3] = {SH ? uu3[0] - rf.ur[0] : uu3[0], SH ? uu3[1] - rf.ur[1] : uu3[1],
                          SH ? uu3[2] - rf.ur[2] : uu3[2]};
    const Mac<double> mc = make_mac<DIM, SH, double>(rf, rho[d] - F::rho0, du);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        store_node_wb<DIM, P>(g, dst, par, i, x, y, z, R(eq_s<DIM, EQ, SH, double>(i, rf, mc)));
}

template <int DIM, int EQ, int P>
__global__ __launch_bounds__(256) void k_read(LevelDev g, const typename Form<P>::T* __restrict__ src, int par,
                                              double* __restrict__ fout, double* __restrict__ rho,
                                              double* __restrict__ u)
{
    using F = Form<P>;
    constexpr int Q = Lat<DIM>::Q;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t d = ((int64_t)z * g.ny + y) * g.nx + x;
    const bool hole = is_hole<DIM>(g, x, y, z);
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double s = hole ? __builtin_nan("") : (double)F::load(node_elem<DIM>(g, src, par, i, x, y, z));
        const double f = s + F::rho0 * ref_pop<DIM, EQ>(i, g);
        if (fout) fout[(int64_t)i * n + d] = f;
        r += f;
        j[0] += cdir<DIM>(i, 0) * f;
        j[1] += cdir<DIM>(i, 1) * f;
        j[2] += cdir<DIM>(i, 2) * f;
    }
    if (rho) rho[d] = r;
    if (u)
        for (int a = 0; a < DIM; ++a) u[(int64_t)a * n + d] = j[a] / r;
}

// X of co-located nodes scattered to a dense [4][n] FP64 array (rho, u).
template <int P>
__global__ __launch_bounds__(128) void k_read_shared(const int4* __restrict__ meta, int ntf, LevelDev g,
                                                     int64_t n, const typename Form<P>::R* __restrict__ X,
                                                     double* __restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntf) return;
    const int4 m = meta[t];
    const int64_t d = ((int64_t)m.z * g.ny + m.y) * g.nx + m.x;
    out[d] = Form<P>::rho0 + (double)X[t];
    for (int a = 1; a < 4; ++a)
        out[(int64_t)a * n + d] = (double)X[(int64_t)a * ntf + t] + (Form<P>::shifted ? g.ur[a - 1] : 0.0);
}

static __global__ void k_fill_nan_f64(double* p, int64_t n)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = __builtin_nan("");
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// Plain 16-byte copy: the bandwidth and HBM-counter reference for the
// population kernels (read n*16 bytes, write n*16 bytes).
static __global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

// ---------------------------------------------------------------- probes

// Standalone: the pending sample of the last coarse step (before the probes
// are read).
template <int DIM, int P>
__global__ __launch_bounds__(64) void k_probe(ProbeArgs a, double* __restrict__ series,
                                              int64_t* __restrict__ counter, double* __restrict__ sums)
{
    probe_pending<DIM, P>(a, series, counter, sums);
}

// ---------------------------------------------------------------- serving
// Many simulations of one (lattice, order, storage) class advance together:
// every level substep of the deepest admitted mesh is one "phase" (the
// depth-first order of the sub-cycling recursion, in which the substeps of a
// shallower mesh keep their own order), and one persistent launch per phase
// runs the workgroups of every resident simulation that has that substep.
struct SlotDev {
    int64_t step;              // coarse steps done (advanced by k_server_tail)
    int64_t target;            // coarse steps requested
    const LevelArgs* args;     // [3][n_phases]: first step, then steady steps of level-0 parity 0 and 1
    const ProbeArgs* probe;    // [2]: after a step from level-0 parity 0 and 1
    double* series;
    int64_t* counter;
};

// Phase table p at ptab + p * (3 + 2 M): n, total, slot[M], begin[M + 1]
// (begin[k] = first virtual workgroup of item k, multiples of 8; begin[n] =
// total).  The tail list follows the last phase: n, slot[M].
//
// Item k's virtual workgroups: its capture and segment workgroups (padded to
// a multiple of 8), then multi_groups(DIM, per) bulk workgroups.  Bulk
// workgroup u runs the tiles 8 (c K + r) + (u & 7), r < K, c = u >> 3, with
// K = multi_tiles(DIM): the item lookup and argument load of a serving
// workgroup are paid once per K tiles (measured +5% capacity in 2-D), and
// every tile keeps the XCD (u & 7) of a plain launch.  3-D keeps K = 1: the
// tile loop compiles the bulk arithmetic differently, and 3-D served results
// equal those of a single simulation bit for bit only with one tile.
__host__ __device__ constexpr int multi_tiles(int dim) { return dim == 2 ? 4 : 1; }
__host__ __device__ constexpr int multi_groups(int dim, int per)
{
    return 8 * ((per + multi_tiles(dim) - 1) / multi_tiles(dim));
}
struct MultiArgs {
    const SlotDev* slots;
    const int* ptab;
    int M;          // slot capacity
    int n_phases;
    int phase;
};

// Persistent: workgroup w takes virtual workgroups w, w + G, ... (G a
// multiple of 8 keeps the XCD of a virtual workgroup as in a plain launch).
// A finished simulation's workgroups do nothing, so a lagging table is safe.
// The tables are read-only while a phase runs: reading them through the
// constant address space lets the compiler keep them in scalar loads (a
// generic pointer inside the loop would be reloaded per lane after every
// store of the previous iteration).
template <class T>
using cptr = const __attribute__((address_space(4))) T*;

template <class T>
__device__ __forceinline__ T load_const(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "dword copy");
    constexpr int N = sizeof(T) / 4;
    const cptr<uint32_t> w = (cptr<uint32_t>)p;
    T out;
    uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = w[i];
    return out;
}

template <int DIM, int EQ, int P>
__global__ __launch_bounds__(kBlock) void k_level_multi(MultiArgs m)
{
    using R = typename Form<P>::R;
    __shared__ R lds[Lat<DIM>::Q * SegLimits<DIM>::TF];
    const cptr<int> pt = (cptr<int>)(m.ptab + (int64_t)m.phase * (3 + 2 * m.M));
    const int n = pt[0], total = pt[1];
    const cptr<int> slot = pt + 2;
    const cptr<int> begin = pt + 2 + m.M;
    const cptr<SlotDev> slots = (cptr<SlotDev>)m.slots;
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (begin[mid] <= v) lo = mid;
            else hi = mid - 1;
        }
        const cptr<SlotDev> sd = slots + slot[lo];
        const int64_t step = sd->step;
        if (step < sd->target) {
            const int var = step == 0 ? 0 : 1 + (int)(step & 1);
            const LevelArgs a = load_const(sd->args + var * m.n_phases + m.phase);
            const int b = v - begin[lo];
            const int na = a.nb_probe + a.nb_cap + 8 * a.seg_groups, nap = (na + 7) & ~7;
            if (b < nap) {
                // only a segment iteration leaves LDS behind; a barrier after
                // every iteration would also wait for each tile's stores.
                // Every wave runs the same iterations, so the barriers pair up.
                if (b < na && level_block<DIM, EQ, P, true>(a, b, lds)) __syncthreads();
            } else {
                constexpr int K = multi_tiles(DIM);
                const int u = b - nap, c0 = (u >> 3) * K;
                for (int r = 0; r < K && c0 + r < a.tm.per; ++r) role_bulk<DIM, EQ, P>(a, 8 * (c0 + r) + (u & 7));
            }
        }
    }
}

// After the phases of a coarse step: probes of every resident simulation
// that is still running, then its step count.  64 threads per workgroup.
template <int DIM, int P>
__global__ __launch_bounds__(64) void k_server_tail(MultiArgs m)
{
    const int* pt = m.ptab + (int64_t)m.n_phases * (3 + 2 * m.M);
    const int n = pt[0];
    for (int k = blockIdx.x; k < n; k += gridDim.x) {
        SlotDev* sd = const_cast<SlotDev*>(m.slots) + pt[1 + k];
        const int64_t step = sd->step;
        if (step < sd->target) {
            probe_sample<DIM, P>(sd->probe[step & 1], sd->series, sd->counter, nullptr);
            if (threadIdx.x == 0) sd->step = step + 1;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- balances
// Block partial sums (FP64, wavefront shuffles) of mass, momentum, kinetic
// energy over the nodes this level owns; NaN latches flag bit 2.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <int DIM, int EQ, int P>
__global__ __launch_bounds__(256) void k_balance(LevelDev g, const typename Form<P>::T* __restrict__ src, int par,
                                                 double vol, double* __restrict__ partial,
                                                 int* __restrict__ flags)
{
    using F = Form<P>;
    constexpr int Q = Lat<DIM>::Q;
    const int64_t total = (int64_t)g.nx * g.ny * g.nz;
    double acc[5] = {0, 0, 0, 0, 0};
    bool bad = false;
    for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < total;
         d += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(d % g.nx);
        const int64_t yz = d / g.nx;
        const int y = (int)(yz % g.ny);
        const int z = (int)(yz / g.ny);
        if (g.cls) {
            const uint8_t c = g.cls[d];
            if (c == kClsHole || c == kClsTfc) continue;   // no node, or owned by the finer level
        } else if (g.has_child && x >= g.clo[0] && x <= g.chi[0] && y >= g.clo[1] && y <= g.chi[1] &&
                   (DIM == 2 || (z >= g.clo[2] && z <= g.chi[2]))) {
            continue;   // hole or owned by the finer level
        }
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            const double f =
                (double)F::load(node_elem<DIM>(g, src, par, i, x, y, z)) + F::rho0 * ref_pop<DIM, EQ>(i, g);
            r += f;
            j[0] += cdir<DIM>(i, 0) * f;
            j[1] += cdir<DIM>(i, 1) * f;
            j[2] += cdir<DIM>(i, 2) * f;
        }
        if (!(r > 0.0) || !(r < 1e30)) bad = true;
        acc[0] += vol * r;
        acc[1] += vol * j[0];
        acc[2] += vol * j[1];
        acc[3] += vol * j[2];
        acc[4] += vol * 0.5 * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / r;
    }
    if (bad) atomicOr(flags, 2);
    __shared__ double sh[4][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) sh[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += sh[w][threadIdx.x];
        partial[(int64_t)blockIdx.x * 5 + threadIdx.x] = v;
    }
}

static __global__ __launch_bounds__(64) void k_balance_final(const double* __restrict__ partial, int nblocks,
                                                      double* __restrict__ out)
{
    for (int k = 0; k < 5; ++k) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 64) v += partial[(int64_t)b * 5 + k];
        v = wave_sum(v);
        if (threadIdx.x == 0) out[k] = v;
    }
}

}  // namespace dclbm
