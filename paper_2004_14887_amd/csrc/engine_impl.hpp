// Launchers of one (lattice, equilibrium order, storage form) class: the
// engine that a simulation drives.  Each lattice/order pair is compiled in a
// translation unit of its own (engine_d*_eq*.hip), so the device code of the
// twelve classes builds in parallel.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "engine.hpp"

namespace dclbm {

// ------------------------------------------------------------------ engine implementation
template <int DIM, int EQ, int P>
struct EngineImpl final : Engine {
    using F = Form<P>;
    using T = typename F::T;
    using R = typename F::R;

    static dim3 dense_grid(const HostLevel& L)
    {
        return dim3((unsigned)((L.nx + 63) / 64), (unsigned)((L.ny + 3) / 4), (unsigned)L.nz);
    }

    void level_step(Sim& s, int l, int substep, int first) override
    {
        unsigned grid = 0;
        const LevelArgs a = level_args(s, l, substep, first, &grid);
        if (s.hrr) {
            // H-RR on one periodic level: macroscopic fields (with the probe
            // workgroup in front), then the collision
            const HrrArgs h = hrr_args(s, a, l);
            const unsigned g_bulk = (unsigned)bulk_groups(h.a.tm.per, 1);
            if (s.timing) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                s.note(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
                s.note(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
                hipExtLaunchKernelGGL((k_hrr_macros<DIM, EQ, P, false>), dim3(a.nb_probe + g_bulk), dim3(kBlock), 0, s.stream, e0,
                                      nullptr, 0, h);
                hipExtLaunchKernelGGL((k_hrr_collide<DIM, EQ, P>), dim3(g_bulk), dim3(kBlock), 0, s.stream, nullptr, e1, 0, h);
                s.tev[l].push_back({e0, e1});
            } else {
                hipLaunchKernelGGL((k_hrr_macros<DIM, EQ, P, false>), dim3(a.nb_probe + g_bulk), dim3(kBlock), 0, s.stream, h);
                hipLaunchKernelGGL((k_hrr_collide<DIM, EQ, P>), dim3(g_bulk), dim3(kBlock), 0, s.stream, h);
            }
            return;
        }
        if (split_substep(s, a)) {
            // the bulk on the simulation's stream, the probe, capture and
            // segment workgroups beside it on the side stream (fork, launch
            // both, join)
            const unsigned g_bulk = (unsigned)bulk_groups(a.tm.per, bulk_k(DIM, P)),
                           g_if = (unsigned)(a.nb_probe + a.nb_cap + 8 * a.seg_groups);
            LevelArgs ai = a;
            ai.seg_every = 0;   // its grid holds the segments alone
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (s.timing) {
                s.note(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
                s.note(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
                s.note(hipEventRecord(e0, s.stream));
            }
            s.note(hipEventRecord(s.ev_fork, s.stream));
            s.note(hipStreamWaitEvent(s.side, s.ev_fork, 0));
            hipLaunchKernelGGL((k_iface<DIM, EQ, P>), dim3(g_if), dim3(kBlock), 0, s.side, ai);
            hipLaunchKernelGGL((k_bulk<DIM, EQ, P>), dim3(g_bulk), dim3(kBlock), 0, s.stream, a);
            s.note(hipEventRecord(s.ev_join, s.side));
            s.note(hipStreamWaitEvent(s.stream, s.ev_join, 0));
            if (s.timing) {
                s.note(hipEventRecord(e1, s.stream));
                s.tev[l].push_back({e0, e1});
            }
            return;
        }
        const void* f = level_kernel(s, l, a);
        LevelArgs arg = a;
        void* params[1] = {&arg};
        if (s.timing) {
            // start/stop events travel in the dispatch packet of the kernel
            // itself; without the system-scope fence the stop stamp is not
            // delayed by a cache write-back the next launch does not need
            hipEvent_t e0 = nullptr, e1 = nullptr;
            s.note(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
            s.note(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
            s.note(hipExtLaunchKernel(f, dim3(grid), dim3(kBlock), params, 0, s.stream, e0, e1, 0));
            s.tev[l].push_back({e0, e1});
        } else {
            s.note(hipLaunchKernel(f, dim3(grid), dim3(kBlock), params, 0, s.stream));
        }
    }
    // 3-D FP16 storage: a level substep whose bulk outweighs its segments by
    // kSplitRatio or more bulk groups per segment group runs as two kernels
    // side by side, the bulk alone at 8 waves/SIMD (49 VGPRs instead of
    // 108), which its 2-byte loads need (the 512^3 4-level mesh's finest
    // launch: 19.3 -> 18.3 ms).  Where the faces weigh more, one launch with
    // the segments interleaved over its front is faster (the 256^3 2-level
    // mesh's level 1: 365 -> 310 us).  Levels without segments use
    // k_level_top.
    static constexpr int kSplitRatio = 150;
    // (dclbm_set_split overrides the choice.)
    static bool split_substep(const Sim& s, const LevelArgs& a)
    {
        if constexpr (DIM == 3 && P == 2) {
            if (!s.side || a.seg_groups == 0 || s.split_mode == 0) return false;
            return s.split_mode == 1 || bulk_groups(a.tm.per, bulk_k(DIM, P)) / 8 >= kSplitRatio * a.seg_groups;
        }
        return false;
    }
    // The level-substep kernel of level l: without the segment role on
    // level 0 with FP16 storage (2-D: 38 VGPRs and 8 waves/SIMD instead of
    // 70 and 7; 3-D: 50 and 8 instead of 108 and 4, 239 -> 221 us on the
    // 256^3 level 0; FP32 and FP64 gain nothing, 3-D FP32 lost), and reading
    // node classes on the levels of a refined region.
    static const void* level_kernel(const Sim& s, int l, const LevelArgs& a)
    {
        const bool top = P == 2 && a.nb_seg == 0;
        if constexpr (DIM == 2) {
            if (s.lv[l].d_cls)
                return top ? reinterpret_cast<const void*>(&k_level_top<DIM, EQ, P, true>)
                           : reinterpret_cast<const void*>(&k_level<DIM, EQ, P, true>);
        }
        return top ? reinterpret_cast<const void*>(&k_level_top<DIM, EQ, P>)
                   : reinterpret_cast<const void*>(&k_level<DIM, EQ, P>);
    }
    // The same launches as level_step, as graph nodes with explicit
    // dependencies (no stream capture, so no events or side stream take part
    // in building a graph): one node per launch in a chain, except the two
    // kernels of a split substep, which both depend on the previous node(s)
    // and not on each other.
    static hipError_t kernel_node(hipGraph_t g, const void* func, unsigned grid, void* args,
                                  const std::vector<hipGraphNode_t>& deps, hipGraphNode_t* out)
    {
        hipKernelNodeParams p;
        memset(&p, 0, sizeof(p));
        void* params[1] = {args};
        p.func = const_cast<void*>(func);
        p.gridDim = dim3(grid);
        p.blockDim = dim3(kBlock);
        p.sharedMemBytes = 0;
        p.kernelParams = params;
        p.extra = nullptr;
        return hipGraphAddKernelNode(out, g, deps.empty() ? nullptr : deps.data(), deps.size(), &p);
    }
    hipError_t add_nodes(Sim& s, hipGraph_t g, const StepRecord& r, std::vector<hipGraphNode_t>& deps) override
    {
        LevelArgs a = r.args;
        hipGraphNode_t n0 = nullptr, n1 = nullptr;
        hipError_t e = hipSuccess;
        if (s.hrr) {
            HrrArgs h = hrr_args(s, a, r.level);
            const unsigned g_bulk = (unsigned)bulk_groups(h.a.tm.per, 1);
            e = kernel_node(g, reinterpret_cast<const void*>(&k_hrr_macros<DIM, EQ, P, false>), a.nb_probe + g_bulk, &h, deps, &n0);
            if (e != hipSuccess) return e;
            e = kernel_node(g, reinterpret_cast<const void*>(&k_hrr_collide<DIM, EQ, P>), g_bulk, &h, {n0}, &n1);
            deps.assign(1, n1);
            return e;
        }
        if (split_substep(s, a)) {
            const unsigned g_bulk = (unsigned)bulk_groups(a.tm.per, bulk_k(DIM, P)),
                           g_if = (unsigned)(a.nb_probe + a.nb_cap + 8 * a.seg_groups);
            LevelArgs ai = a;
            ai.seg_every = 0;   // its grid holds the segments alone
            e = kernel_node(g, reinterpret_cast<const void*>(&k_iface<DIM, EQ, P>), g_if, &ai, deps, &n0);
            if (e != hipSuccess) return e;
            e = kernel_node(g, reinterpret_cast<const void*>(&k_bulk<DIM, EQ, P>), g_bulk, &a, deps, &n1);
            if (e != hipSuccess) return e;
            deps.assign({n0, n1});
            return hipSuccess;
        }
        e = kernel_node(g, level_kernel(s, r.level, a), r.grid, &a, deps, &n0);
        deps.assign(1, n0);
        return e;
    }
    static constexpr int kHrrSegEvery = 32;
    static HrrArgs hrr_args(const Sim& s, const LevelArgs& a, int l)
    {
        const HostLevel& L = s.lv[l];
        HrrArgs h;
        memset(&h, 0, sizeof(h));
        h.a = a;
        h.a.M = L.d_M;
        h.a.M_parent = l > 0 ? s.lv[l - 1].d_M : nullptr;
        // each node's macroscopic state is read again by its 2 D axis
        // neighbours: rows go to the XCDs in slabs of 8 consecutive tile
        // rows, so the neighbour rows of a tile are read by the same L2
        h.a.tm.blk = 8;
        h.a.tm.per = h.a.tm.tx * (((h.a.tm.nrows + 63) / 64) * 8);
        h.M = L.d_M;
        h.tau = L.tau;
        h.sigma = s.cfg.hrr_sigma;
        h.psi = s.cfg.hrr_psi ? 1 : 0;
        h.Mring = L.d_Mring;
        if (L.has_child) {
            const HostLevel& C = s.lv[l + 1];
            h.M_child = C.d_M;
            h.cn[0] = C.nx;
            h.cn[1] = C.ny;
            h.cn[2] = C.nz;
        }
        // the ring's slots rotate: a level's c-th capture writes slot c % 3,
        // so after c captures the values at t - dt, t, t + dt sit in slots
        // c % 3, (c + 1) % 3, (c + 2) % 3
        h.ring_new = (int)(L.captures % 3);
        if (l > 0) {
            const int64_t cp = s.lv[l - 1].captures;
            h.Mring_parent = s.lv[l - 1].d_Mring;
            for (int e = 0; e < 3; ++e) h.pslot[e] = (int)((cp + e) % 3);
        }
        for (int e = 0; e < 3; ++e) h.plo[e] = L.plo[e];
        h.ie_tf = L.d_ie_tf;
        h.nb_bulk = bulk_groups(h.a.tm.per, 1);
        // 3-D: the segments interleaved over the front of the macroscopic
        // launch, one group of 8 after every kHrrSegEvery bulk groups
        h.a.seg_every = DIM == 3 && a.seg_groups > 0 ? std::min(kHrrSegEvery, (h.nb_bulk / 8) / a.seg_groups) : 0;
        return h;
    }
    void hrr_open(Sim& s, int l, int substep, int first) override
    {
        unsigned grid = 0;
        const LevelArgs a = level_args(s, l, substep, first, &grid);
        const HrrArgs h = hrr_args(s, a, l);
        const dim3 grid_m(a.nb_probe + a.nb_cap + (h.a.seg_every > 0 ? 8 * a.seg_groups : a.nb_seg) + h.nb_bulk);
        if (a.nb_seg > 0 && s.lv[l].d_cls)
            hipLaunchKernelGGL((k_hrr_macros<DIM, EQ, P, true, true>), grid_m, dim3(kBlock), 0, s.stream, h);
        else if (a.nb_seg > 0)
            hipLaunchKernelGGL((k_hrr_macros<DIM, EQ, P, true>), grid_m, dim3(kBlock), 0, s.stream, h);
        else
            hipLaunchKernelGGL((k_hrr_macros<DIM, EQ, P, false>), grid_m, dim3(kBlock), 0, s.stream, h);
    }
    void hrr_close(Sim& s, int l, int substep, int first) override
    {
        unsigned grid = 0;
        const LevelArgs a = level_args(s, l, substep, first, &grid);
        const HrrArgs h = hrr_args(s, a, l);
        const unsigned gtf = (unsigned)((a.n_tf + kBlock - 1) / kBlock);
        const unsigned gie = (unsigned)((a.n_ie + kBlock - 1) / kBlock);
        const unsigned gtfc = (unsigned)((a.n_cap + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((k_hrr_collide<DIM, EQ, P>), dim3(h.nb_bulk + gtf + gie + gtfc), dim3(kBlock), 0, s.stream, h);
    }
    void sponge(Sim& s) override
    {
        const HostLevel& L = s.lv[0];
        const int64_t n = L.n_dense();
        hipLaunchKernelGGL((k_sponge<DIM, EQ, P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s.stream, L.dev(),
                           L.f[L.parity], L.parity, s.sponge_w, s.sponge_sigma, s.cfg.u_ref[0], s.cfg.u_ref[1],
                           s.D == 3 ? s.cfg.u_ref[2] : 0.0);
    }
    void hrr_ring_init(Sim& s, int l, const double* rho, const double* u) override
    {
        const HostLevel& L = s.lv[l];
        const int64_t n = L.n_dense();
        hipLaunchKernelGGL((k_hrr_ring_init<DIM, P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s.stream, L.dev(),
                           L.d_Mring, rho, u);
    }
    void probe(Sim& s) override
    {
        // the pending sample of the last coarse step (a no-op if none)
        const ProbeArgs a = probe_args(s);
        hipLaunchKernelGGL((k_probe<DIM, P>), dim3(1), dim3(64), 0, s.stream, a, s.d_series, s.d_counter, s.d_psum);
    }
    void init(Sim& s, int l, const double* rho, const double* u) override
    {
        HostLevel& L = s.lv[l];
        hipLaunchKernelGGL((k_init<DIM, EQ, P>), dense_grid(L), dim3(64, 4, 1), 0, s.stream, L.dev(),
                           (T*)L.f[L.parity], L.parity, rho, u);
    }
    void ring_init(Sim& s, int l) override
    {
        HostLevel& L = s.lv[l];
        const int n = (int)L.tfc_meta.size();
        hipLaunchKernelGGL((k_ring_init<DIM, P>), dim3((n + 127) / 128), dim3(128), 0, s.stream, L.dev(),
                           (const T*)L.f[L.parity], L.d_tfc, n, (R*)L.H);
    }
    void fill_nan(Sim& s) override
    {
        for (auto& L : s.lv) {
            T nanv;
            if constexpr (P == 2) {
                unsigned short b = 0x7e00;
                memcpy(&nanv, &b, 2);
            } else {
                nanv = (T)NAN;
            }
            for (int b = 0; b < 2; ++b) {
                hipLaunchKernelGGL((k_fill<T>), dim3(2048), dim3(256), 0, s.stream, (T*)L.f[b], L.elems, nanv);
                if (L.xface)
                    hipLaunchKernelGGL((k_fill<T>), dim3(256), dim3(256), 0, s.stream, (T*)L.xf[b], L.xf_elems, nanv);
            }
            if (L.X)
                hipLaunchKernelGGL((k_fill<R>), dim3(256), dim3(256), 0, s.stream, (R*)L.X,
                                   4 * (int64_t)L.tf_meta.size(), (R)NAN);
            if (L.H)
                hipLaunchKernelGGL((k_fill<R>), dim3(256), dim3(256), 0, s.stream, (R*)L.H,
                                   3 * (int64_t)Lat<DIM>::Q * (int64_t)L.tfc_meta.size(), (R)NAN);
        }
    }
    void read(Sim& s, int l, double* f, double* rho, double* u) override
    {
        HostLevel& L = s.lv[l];
        hipLaunchKernelGGL((k_read<DIM, EQ, P>), dense_grid(L), dim3(64, 4, 1), 0, s.stream, L.dev(),
                           (const T*)L.f[L.parity], L.parity, f, rho, u);
    }
    void read_shared(Sim& s, int l, double* out) override
    {
        HostLevel& L = s.lv[l];
        const int64_t n = L.n_dense();
        hipLaunchKernelGGL(k_fill_nan_f64, dim3(1024), dim3(256), 0, s.stream, out, 4 * n);
        const int ntf = (int)L.tf_meta.size();
        if (ntf)
            hipLaunchKernelGGL((k_read_shared<P>), dim3((ntf + 127) / 128), dim3(128), 0, s.stream, L.d_tf, ntf,
                               L.dev(), n, (const R*)L.X, out);
    }
    void balance(Sim& s, int l, double* partial, int nblocks) override
    {
        HostLevel& L = s.lv[l];
        const double vol = std::ldexp(1.0, -DIM * l);
        hipLaunchKernelGGL((k_balance<DIM, EQ, P>), dim3(nblocks), dim3(256), 0, s.stream, L.dev(),
                           (const T*)L.f[L.parity], L.parity, vol, partial, s.d_flags);
    }
    void launch_multi(hipStream_t st, const MultiArgs& m, unsigned grid) override
    {
        hipLaunchKernelGGL((k_level_multi<DIM, EQ, P>), dim3(grid), dim3(kBlock), 0, st, m);
    }
    void launch_tail(hipStream_t st, const MultiArgs& m, unsigned grid) override
    {
        hipLaunchKernelGGL((k_server_tail<DIM, P>), dim3(grid), dim3(64), 0, st, m);
    }
};

}  // namespace dclbm
