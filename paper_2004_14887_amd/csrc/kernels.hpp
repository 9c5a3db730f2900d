// HIP kernels (gfx950) of the direct-coupling refined LBM step.
//
// Per level, populations live in two SoA buffers s[Q][z][y][x_pitch] (A/B),
// read by a pull stream and written once per node per substep.  The kernels:
//   k_bulk      fused pull-stream + BGK on every node that is not on an
//               interface (Eq.(LBMequation), Eq.(LBMscheme_reg) with BGK)
//   k_capture   coarse co-located nodes: store the streamed coarse
//               populations in a 3-deep history ring (input of Eq.(TempInt))
//   k_tf        fine co-located nodes: Newton for X (Eq.(system_fi)),
//               rebuild every Gamma=R direction (Eq.(rescff)), collide with X
//   k_ie        hanging fine nodes: 4-point 1-D Lagrange interpolation of the
//               missing directions from completed co-located values, collide
//   k_restrict  coarse co-located nodes after the synchronous fine substep:
//               Eq.(rescfc) on all directions, collide with X
// plus initialisation, conversion, probe and balance kernels.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace dclbm {

// ---------------------------------------------------------------- storage forms
// P = 0: FP64, carried value s = f.
// P = 1: FP32 arithmetic, stored s = f - w (deviation from rest).
// P = 2: FP32 arithmetic, stored FP16(256 (f - w)).
template <int P>
struct Form;
template <>
struct Form<0> {
    using T = double;
    using R = double;
    static constexpr double rho0 = 0.0;
    __device__ static __forceinline__ R load(const T* p) { return *p; }
    __device__ static __forceinline__ void store(T* p, R v) { __builtin_nontemporal_store(v, p); }
    __device__ static __forceinline__ T nan() { return __builtin_nan(""); }
};
template <>
struct Form<1> {
    using T = float;
    using R = float;
    static constexpr double rho0 = 1.0;
    __device__ static __forceinline__ R load(const T* p) { return *p; }
    __device__ static __forceinline__ void store(T* p, R v) { __builtin_nontemporal_store(v, p); }
    __device__ static __forceinline__ T nan() { return __builtin_nanf(""); }
};
template <>
struct Form<2> {
    using T = __half;
    using R = float;
    static constexpr double rho0 = 1.0;
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
    __device__ static __forceinline__ T nan() { return __ushort_as_half((unsigned short)0x7e00); }
};

// ---------------------------------------------------------------- level geometry
struct LevelDev {
    int nx, ny, nz;
    int pitch;
    int64_t plane;     // pitch * ny
    int64_t qs;        // elements between directions
    int periodic;      // level 0
    int boundary;      // own box faces are interfaces (level >= 1)
    int has_child;
    int clo[3], chi[3];// child box, closed, in this level's node coordinates
};

__device__ __forceinline__ int64_t node_off(const LevelDev& g, int x, int y, int z)
{
    return (int64_t)z * g.plane + (int64_t)y * g.pitch + x;
}

// Source node of direction i for a pull stream; periodic wrap on level 0.
template <int DIM>
__device__ __forceinline__ int64_t src_off(const LevelDev& g, int x, int y, int z, int i)
{
    int sx = x - cdir<DIM>(i, 0), sy = y - cdir<DIM>(i, 1), sz = z - cdir<DIM>(i, 2);
    if (g.periodic) {
        sx = sx < 0 ? sx + g.nx : (sx >= g.nx ? sx - g.nx : sx);
        sy = sy < 0 ? sy + g.ny : (sy >= g.ny ? sy - g.ny : sy);
        if (DIM == 3) sz = sz < 0 ? sz + g.nz : (sz >= g.nz ? sz - g.nz : sz);
    }
    return node_off(g, sx, sy, sz);
}

template <int DIM>
__device__ __forceinline__ bool in_box(const LevelDev& g, int x, int y, int z)
{
    return x >= 0 && x < g.nx && y >= 0 && y < g.ny && (DIM == 2 || (z >= 0 && z < g.nz));
}

template <int DIM>
__device__ __forceinline__ bool is_interface_or_hole(const LevelDev& g, int x, int y, int z)
{
    if (g.boundary &&
        (x == 0 || x == g.nx - 1 || y == 0 || y == g.ny - 1 || (DIM == 3 && (z == 0 || z == g.nz - 1))))
        return true;
    if (g.has_child && x >= g.clo[0] && x <= g.chi[0] && y >= g.clo[1] && y <= g.chi[1] &&
        (DIM == 2 || (z >= g.clo[2] && z <= g.chi[2])))
        return true;
    return false;
}

// ---------------------------------------------------------------- bulk stream + collide
// Tile: 64 (x, one wavefront) x 4 (y) nodes; grid (ceil(nx/64), ceil(ny/4), nz).
template <int DIM, int EQ, int P>
__global__ __launch_bounds__(256) void k_bulk(LevelDev g, const typename Form<P>::T* __restrict__ src,
                                              typename Form<P>::T* __restrict__ dst,
                                              typename Form<P>::R keep)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    if (is_interface_or_hole<DIM>(g, x, y, z)) return;
    R s[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) s[i] = F::load(src + (int64_t)i * g.qs + src_off<DIM>(g, x, y, z, i));
    R drho, j[3];
    moments<DIM, R>(s, drho, j);
    const R rho = R(F::rho0) + drho;
    const R inv = R(1) / rho;
    const R u[3] = {j[0] * inv, j[1] * inv, DIM == 3 ? j[2] * inv : R(0)};
    bgk<DIM, EQ, R>(s, R(F::rho0), drho, u, keep);
    const int64_t o = node_off(g, x, y, z);
#pragma unroll
    for (int i = 0; i < Q; ++i) F::store(dst + (int64_t)i * g.qs + o, s[i]);
}

// ---------------------------------------------------------------- coarse history capture
// meta: (x, y, z, K^c mask) of each coarse co-located node, in the order of
// the child's co-located list.  H: [3][Q][n], slot 0 = t - dt, 1 = t, 2 = t + dt.
template <int DIM, int P>
__global__ __launch_bounds__(128) void k_capture(LevelDev g, const typename Form<P>::T* __restrict__ src,
                                                 const int4* __restrict__ meta, int n,
                                                 typename Form<P>::R* __restrict__ H)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int4 m = meta[t];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!((m.w >> i) & 1)) continue;
        const R v = F::load(src + (int64_t)i * g.qs + src_off<DIM>(g, m.x, m.y, m.z, i));
        R* h = H + (int64_t)i * n + t;
        const int64_t slot = (int64_t)Q * n;
        h[0] = h[slot];
        h[slot] = h[2 * slot];
        h[2 * slot] = v;
    }
}

// Ring initialisation from the node's own initial populations.
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
    const int64_t o = node_off(g, m.x, m.y, m.z);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const auto v = F::load(src + (int64_t)i * g.qs + o);
        for (int r = 0; r < 3; ++r) H[((int64_t)r * Q + i) * n + t] = v;
    }
}

// ---------------------------------------------------------------- fine co-located nodes
struct TfArgs {
    int n;            // co-located fine nodes
    int substep;      // 1 asynchronous (mid coarse step), 2 synchronous
    int first;        // parent has made a single step: linear time interpolation
    int maxit;
    double Rfac;      // tau_f / (2 tau_c), Eq.(fneqResc)
    double keep;      // 1 - 1/tau_f
    double tol;
};

template <int DIM, int EQ, int P>
__global__ __launch_bounds__(64) void k_tf(LevelDev g, const typename Form<P>::T* __restrict__ src,
                                           typename Form<P>::T* __restrict__ dst,
                                           const int4* __restrict__ meta, TfArgs a,
                                           const typename Form<P>::R* __restrict__ H,
                                           typename Form<P>::R* __restrict__ S,
                                           typename Form<P>::R* __restrict__ X, int* __restrict__ flags)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n) return;
    const int4 m = meta[t];
    const uint32_t gR = (uint32_t)m.w;
    const int64_t slot = (int64_t)Q * a.n;
    R h[Q], gc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if ((gR >> i) & 1u) {
            const R* hp = H + (int64_t)i * a.n + t;
            const R Hm = hp[0], H0 = hp[slot], Hp = hp[2 * slot];
            R v;
            if (a.substep == 2)
                v = Hp;
            else if (a.first)
                v = R(0.5) * H0 + R(0.5) * Hp;
            else
                v = R(-0.125) * Hm + R(0.75) * H0 + R(0.375) * Hp;
            gc[i] = v;
            h[i] = v;
        } else {
            gc[i] = R(0);
            h[i] = F::load(src + (int64_t)i * g.qs + src_off<DIM>(g, m.x, m.y, m.z, i));
        }
    }
    R drho, u[3];
    const int it = newton<DIM, EQ, R>(h, gR, R(a.Rfac), R(F::rho0), R(a.tol), a.maxit, drho, u);
    if (it < 0) {
        atomicOr(flags, 1);
        R j[3];
        moments<DIM, R>(h, drho, j);
        const R rr = R(F::rho0) + drho;
        u[0] = j[0] / rr;
        u[1] = j[1] / rr;
        u[2] = DIM == 3 ? j[2] / rr : R(0);
    }
    const R uu = u[0] * u[0] + u[1] * u[1] + (DIM == 3 ? u[2] * u[2] : R(0));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if ((gR >> i) & 1u) {
            const R e = eq_s<DIM, EQ, R>(i, R(F::rho0), drho, u, uu);
            h[i] = e + R(a.Rfac) * (gc[i] - e);
        }
        S[(int64_t)i * a.n + t] = h[i];
    }
    X[t] = drho;
    X[(int64_t)a.n + t] = u[0];
    X[2 * (int64_t)a.n + t] = u[1];
    X[3 * (int64_t)a.n + t] = u[2];
    bgk<DIM, EQ, R>(h, R(F::rho0), drho, u, R(a.keep));
    const int64_t o = node_off(g, m.x, m.y, m.z);
#pragma unroll
    for (int i = 0; i < Q; ++i) F::store(dst + (int64_t)i * g.qs + o, h[i]);
}

// ---------------------------------------------------------------- hanging fine nodes
// 4-point stencil along one axis for odd position k on a line 0..N:
// centred (-1,9,9,-1)/16 at k-3..k+3, one-sided (5,15,-5,1)/16 at line ends.
__device__ __forceinline__ void line_stencil(int k, int N, int pos[4], float w[4])
{
    if (k == 1) {
        pos[0] = 0; pos[1] = 2; pos[2] = 4; pos[3] = 6;
        w[0] = 5.f / 16; w[1] = 15.f / 16; w[2] = -5.f / 16; w[3] = 1.f / 16;
    } else if (k == N - 1) {
        pos[0] = N; pos[1] = N - 2; pos[2] = N - 4; pos[3] = N - 6;
        w[0] = 5.f / 16; w[1] = 15.f / 16; w[2] = -5.f / 16; w[3] = 1.f / 16;
    } else {
        pos[0] = k - 3; pos[1] = k - 1; pos[2] = k + 1; pos[3] = k + 3;
        w[0] = -1.f / 16; w[1] = 9.f / 16; w[2] = 9.f / 16; w[3] = -1.f / 16;
    }
}

struct IeArgs {
    int n;            // hanging nodes
    int mx, my;       // dims of the co-located index map (nx/2+1, ny/2+1)
    int ntf;          // co-located nodes (stride of S)
    double keep;
};

// meta: (x, y, z, missing-direction mask).  tfmap: co-located index of the
// node at fine coords (2a, 2b, 2c) stored at (c*my + b)*mx + a, -1 elsewhere.
template <int DIM, int EQ, int P>
__global__ __launch_bounds__(64) void k_ie(LevelDev g, const typename Form<P>::T* __restrict__ src,
                                           typename Form<P>::T* __restrict__ dst,
                                           const int4* __restrict__ meta, IeArgs a,
                                           const typename Form<P>::R* __restrict__ S,
                                           const int* __restrict__ tfmap)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n) return;
    const int4 m = meta[t];
    const int k[3] = {m.x, m.y, m.z};
    const int N[3] = {g.nx - 1, g.ny - 1, g.nz - 1};
    int np[3], pos[3][4];
    float w[3][4];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (ax < DIM && (k[ax] & 1)) {
            np[ax] = 4;
            line_stencil(k[ax], N[ax], pos[ax], w[ax]);
        } else {
            np[ax] = 1;
            pos[ax][0] = k[ax];
            w[ax][0] = 1.f;
        }
    }
    // co-located indices of the (up to 16) stencil nodes and their weights
    int idx[16];
    R wt[16];
    int ns = 0;
    for (int c = 0; c < np[2]; ++c)
        for (int b = 0; b < np[1]; ++b)
            for (int aa = 0; aa < np[0]; ++aa) {
                const int64_t key = ((int64_t)(pos[2][c] >> 1) * a.my + (pos[1][b] >> 1)) * a.mx + (pos[0][aa] >> 1);
                idx[ns] = tfmap[key];
                wt[ns] = R(w[0][aa]) * R(w[1][b]) * R(w[2][c]);
                ++ns;
            }
    R s[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if ((m.w >> i) & 1) {
            R acc = R(0);
            for (int q = 0; q < ns; ++q) acc += wt[q] * S[(int64_t)i * a.ntf + idx[q]];
            s[i] = acc;
        } else {
            s[i] = F::load(src + (int64_t)i * g.qs + src_off<DIM>(g, m.x, m.y, m.z, i));
        }
    }
    R drho, j[3];
    moments<DIM, R>(s, drho, j);
    const R rho = R(F::rho0) + drho;
    const R u[3] = {j[0] / rho, j[1] / rho, DIM == 3 ? j[2] / rho : R(0)};
    bgk<DIM, EQ, R>(s, R(F::rho0), drho, u, R(a.keep));
    const int64_t o = node_off(g, m.x, m.y, m.z);
#pragma unroll
    for (int i = 0; i < Q; ++i) F::store(dst + (int64_t)i * g.qs + o, s[i]);
}

// ---------------------------------------------------------------- restriction
// Coarse co-located node t <-> child co-located node t (same ordering).
template <int DIM, int EQ, int P>
__global__ __launch_bounds__(64) void k_restrict(LevelDev g, typename Form<P>::T* __restrict__ dst,
                                                 const int4* __restrict__ meta, int n,
                                                 const typename Form<P>::R* __restrict__ S,
                                                 const typename Form<P>::R* __restrict__ X, double invR,
                                                 double keep)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int4 m = meta[t];
    const R drho = X[t];
    const R u[3] = {X[(int64_t)n + t], X[2 * (int64_t)n + t], X[3 * (int64_t)n + t]};
    const R uu = u[0] * u[0] + u[1] * u[1] + (DIM == 3 ? u[2] * u[2] : R(0));
    R s[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R e = eq_s<DIM, EQ, R>(i, R(F::rho0), drho, u, uu);
        s[i] = e + R(invR) * (S[(int64_t)i * n + t] - e);
    }
    bgk<DIM, EQ, R>(s, R(F::rho0), drho, u, R(keep));
    const int64_t o = node_off(g, m.x, m.y, m.z);
#pragma unroll
    for (int i = 0; i < Q; ++i) F::store(dst + (int64_t)i * g.qs + o, s[i]);
}

// ---------------------------------------------------------------- init / conversion
template <int DIM>
__device__ __forceinline__ bool is_hole(const LevelDev& g, int x, int y, int z)
{
    return g.has_child && x > g.clo[0] && x < g.chi[0] && y > g.clo[1] && y < g.chi[1] &&
           (DIM == 2 || (z > g.clo[2] && z < g.chi[2]));
}

template <int DIM, int EQ, int P>
__global__ __launch_bounds__(256) void k_init(LevelDev g, typename Form<P>::T* __restrict__ dst,
                                              const double* __restrict__ rho, const double* __restrict__ u)
{
    using F = Form<P>;
    using R = typename F::R;
    constexpr int Q = Lat<DIM>::Q;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const int64_t o = node_off(g, x, y, z);
    if (is_hole<DIM>(g, x, y, z)) {
#pragma unroll
        for (int i = 0; i < Q; ++i) dst[(int64_t)i * g.qs + o] = F::nan();
        return;
    }
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t d = ((int64_t)z * g.ny + y) * g.nx + x;
    // equilibrium evaluated in FP64, then carried in the storage form
    const double r = rho[d];
    const double uu3[3] = {u[d], u[n + d], DIM == 3 ? u[2 * n + d] : 0.0};
    const double uu = uu3[0] * uu3[0] + uu3[1] * uu3[1] + uu3[2] * uu3[2];
    const double drho = r - F::rho0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double e = eq_s<DIM, EQ, double>(i, F::rho0, drho, uu3, uu);
        F::store(dst + (int64_t)i * g.qs + o, R(e));
    }
}

template <int DIM, int P>
__global__ __launch_bounds__(256) void k_read(LevelDev g, const typename Form<P>::T* __restrict__ src,
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
    const int64_t o = node_off(g, x, y, z);
    const bool hole = is_hole<DIM>(g, x, y, z);
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double s = hole ? __builtin_nan("") : (double)F::load(src + (int64_t)i * g.qs + o);
        const double f = s + F::rho0 * Lat<DIM>::w[i];
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
__global__ __launch_bounds__(128) void k_read_shared(const int4* __restrict__ meta, int ntf, int nx, int ny,
                                                     int64_t n, const typename Form<P>::R* __restrict__ X,
                                                     double* __restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntf) return;
    const int4 m = meta[t];
    const int64_t d = ((int64_t)m.z * ny + m.y) * nx + m.x;
    out[d] = Form<P>::rho0 + (double)X[t];
    for (int a = 1; a < 4; ++a) out[(int64_t)a * n + d] = (double)X[(int64_t)a * ntf + t];
}

__global__ void k_fill_nan_f64(double* p, int64_t n)
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

// ---------------------------------------------------------------- probes
struct ProbeArgs {
    int n;
    int64_t capacity;
    const void* buf[32];   // storage buffer holding the probe's node
    int64_t off[32];       // node offset in that buffer
    int64_t qs[32];
};

// One workgroup; p' = (rho - 1)/3 in FP64 after each coarse step.
template <int DIM, int P>
__global__ __launch_bounds__(64) void k_probe(ProbeArgs a, double* __restrict__ series,
                                              int64_t* __restrict__ counter)
{
    using F = Form<P>;
    constexpr int Q = Lat<DIM>::Q;
    const int64_t step = *counter;
    const int p = threadIdx.x;
    if (p < a.n && step < a.capacity) {
        const typename F::T* b = reinterpret_cast<const typename F::T*>(a.buf[p]);
        double r = F::rho0;
        for (int i = 0; i < Q; ++i) r += (double)F::load(b + (int64_t)i * a.qs[p] + a.off[p]);
        series[step * a.n + p] = (r - 1.0) / 3.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) *counter = step + 1;
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

template <int DIM, int P>
__global__ __launch_bounds__(256) void k_balance(LevelDev g, const typename Form<P>::T* __restrict__ src,
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
        if (g.has_child && x >= g.clo[0] && x <= g.chi[0] && y >= g.clo[1] && y <= g.chi[1] &&
            (DIM == 2 || (z >= g.clo[2] && z <= g.chi[2])))
            continue;   // hole or owned by the finer level
        const int64_t o = node_off(g, x, y, z);
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            const double f = (double)F::load(src + (int64_t)i * g.qs + o) + F::rho0 * Lat<DIM>::w[i];
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

__global__ __launch_bounds__(64) void k_balance_final(const double* __restrict__ partial, int nblocks,
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
