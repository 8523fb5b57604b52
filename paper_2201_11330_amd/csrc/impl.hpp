// Kernel launches of one lattice kind and storage type, instantiated once per
// lattice kind in its own translation unit (lattice_*.hip).
#pragma once

#include "context.hpp"
#include "fused2d.hpp"
#include "stream2d.hpp"

namespace imexlbm {

// A captured run holds whole pairs of fused launches (see eager()).
static_assert(kGraphSteps % (2 * kFuseSteps) == 0, "graph length must be a multiple of 2 * kFuseSteps");
static_assert(kStreamLevels == kFuseSteps, "both multi-step launches take the same number of steps");

// Compile-time configuration of the step kernels: walls or masks present,
// body force, compressible equilibrium (which always takes the force path).
template <bool W, bool F, bool M>
struct Cfg {
    static constexpr bool walls = W, force = F, comp = M;
};

// Calls fn(Cfg<...>{}) for the context's configuration.
template <class Fn>
void dispatch(const lbm_ctx* c, Fn&& fn)
{
    if (c->comp) {
        if (c->walls) fn(Cfg<true, true, true>{});
        else fn(Cfg<false, true, true>{});
    } else if (c->walls) {
        if (c->force) fn(Cfg<true, true, false>{});
        else fn(Cfg<true, false, false>{});
    } else {
        if (c->force) fn(Cfg<false, true, false>{});
        else fn(Cfg<false, false, false>{});
    }
}

// Kernel instantiations of one lattice and storage.
template <int L, class S>
struct Impl {
    template <class K>
    static void step_ab(lbm_ctx* c, const S* src, S* dst)
    {
        if constexpr (std::is_same_v<S, double> && !K::walls && L != 2) {  // not D3Q27
            if (c->pairs) {
                hipLaunchKernelGGL((k_step_ab_pairs<L, K::force, K::comp, kNtStores>), c->pairs_grid, c->block,
                                   0, c->stream, src, dst, step_args<double>(c), c->pairs_shift);
                return;
            }
        }
        // Row addressing where it measured faster (D3Q19 256^3 and 512^3):
        // e4m11 storage +26 % (its step is bound by instruction issue, two
        // thirds of it the conversions), FP32 +0.5-0.9 %; FP16 and BF16 ran
        // 2-6 % slower with it.
        if constexpr (!K::walls && (std::is_same_v<S, e4m11> || std::is_same_v<S, float>)) {
            if (c->rows) {
                const auto p = one_node_step_args(c);
                hipLaunchKernelGGL((k_step_ab_rows<L, S, K::force, K::comp, kNtStores>),
                                   p.xcd_rows ? c->grid_xcd : c->grid, c->block, 0, c->stream, src, dst, p);
                return;
            }
        }
        const auto p = one_node_step_args(c);
        hipLaunchKernelGGL((k_step_ab<L, S, K::walls, K::force, K::comp, kNtStores>),
                           p.xcd_rows ? c->grid_xcd : c->grid, c->block, 0, c->stream, src, dst, p);
    }
    // Arguments of the one-node AB steps; the launch takes grid_xcd when
    // xcd_rows is set.  Placing each row's workgroups on one XCD measured on
    // MI355X, D3Q19 512^3: FP16 73.9 -> 77.2 %, BF16 73.0 -> 77.0 %, e4m11
    // 73.4 -> 74.9 % of the HBM peak, the FP64 channel 512x128x128 +0.5 %,
    // the D3Q27 sphere box unchanged, FP32 77.4 -> 74.4 % (so not for FP32).
    static StepArgs<typename Store<S>::C> one_node_step_args(const lbm_ctx* c)
    {
        auto p = step_args<typename Store<S>::C>(c);
        p.xcd_rows = c->xcd_rows && !std::is_same_v<S, float>;
        return p;
    }
    template <class K>
    static void step_aa(lbm_ctx* c, S* A, bool odd)
    {
        if constexpr (std::is_same_v<S, double> && !K::walls && L != 2) {  // not D3Q27
            if (c->pairs) {
                if (odd)
                    hipLaunchKernelGGL((k_step_aa_odd_pairs<L, K::force, K::comp, kNtStores>), c->pairs_grid,
                                       c->block, 0, c->stream, A, step_args<double>(c), c->pairs_shift);
                else
                    hipLaunchKernelGGL((k_step_aa_even_pairs<L, K::force, K::comp, kNtStores>), c->pairs_grid,
                                       c->block, 0, c->stream, A, step_args<double>(c), c->pairs_shift);
                return;
            }
        }
        if (odd)
            hipLaunchKernelGGL((k_step_aa_odd<L, S, K::walls, K::force, K::comp, kNtStores>), c->grid,
                               c->block, 0, c->stream, A, step_args<typename Store<S>::C>(c));
        else
            hipLaunchKernelGGL((k_step_aa_even<L, S, K::walls, K::force, K::comp, kNtStores>), c->grid,
                               c->block, 0, c->stream, A, step_args<typename Store<S>::C>(c));
    }

    // Captures kGraphSteps steps starting from an even step count (buffer 0
    // current, AA even parity) on a private stream; the context's launch
    // stream and counters are restored afterwards.
    static lbm_status capture(lbm_ctx* c)
    {
        if (!c->capture_stream) LBM_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipStream_t saved_stream = c->stream;
        const int saved_cur = c->cur;
        const long long saved_steps = c->steps;
        c->stream = c->capture_stream;
        c->cur = 0;
        c->steps = 0;
        const lbm_status st = eager(c, kGraphSteps);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->capture_stream, &g);
        c->stream = saved_stream;
        c->cur = saved_cur;
        c->steps = saved_steps;
        if (st != LBM_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != LBM_OK ? st : hip_fail(e, "hipStreamEndCapture");
        }
        c->graph = g;
        e = hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(c->graph);
            c->graph = nullptr;
            c->graph_exec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        return LBM_OK;
    }

    static lbm_status step(lbm_ctx* c, int n)
    {
        if (!c->use_graph || n < kGraphSteps) return eager(c, n);
        if (c->steps & 1) {  // align to the captured parity
            lbm_status st = eager(c, 1);
            if (st) return st;
            --n;
        }
        if (!c->graph_exec) {
            lbm_status st = capture(c);
            if (st) return st;
        }
        for (; n >= kGraphSteps; n -= kGraphSteps) {
            LBM_HIP(hipGraphLaunch(c->graph_exec, c->stream));
            c->steps += kGraphSteps;
        }
        return eager(c, n);
    }

    // kFuseSteps steps of a periodic D2Q9 two-lattice box in one launch:
    // 32 x 32 regions on large boxes, 16 x 16 regions otherwise (XCD-aware
    // placement from kFuseXcdMinBlocks blocks up); see fused2d.hpp.
    template <class K>
    static void step_fused2d(lbm_ctx* c, const S* src, S* dst)
    {
        constexpr int I32 = kFuseInnerOf<32>, I16 = kFuseInnerOf<16>;
        const auto blocks = [&](int inner) {
            return (long long)((c->nx + inner - 1) / inner) * ((c->ny + inner - 1) / inner);
        };
        const auto args = step_args<typename Store<S>::C>(c);
        dim3 grid;
        if (c->N >= kStreamMinNodes) {
            // Strips of kStreamStore stored columns, segments of rows chosen
            // once per context from the kernel's occupancy (stream_rows).
            const auto kernel = k_step_ab_stream2d<S, K::force, K::comp, kNtStores>;
            if (c->stream_rows == 0) {
                int per_cu = 0, cus = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
                    per_cu < 1 || cus < 1) {
                    (void)hipGetLastError();
                    per_cu = 4;  // unknown: assume a GPU of 256 CUs, 4 workgroups each
                    cus = 256;
                }
                c->stream_rows = stream_rows(c->nx, c->ny, (long long)per_cu * cus);
            }
            const int rows = c->stream_rows;
            grid = dim3(unsigned((c->nx + kStreamStore - 1) / kStreamStore), unsigned((c->ny + rows - 1) / rows), 1);
            hipLaunchKernelGGL(kernel, grid, c->block, 0, c->stream, src, dst, args, rows);
        } else if (blocks(I32) >= kFuseBigMinBlocks) {
            const FuseMap m = fuse_plan(c->nx, c->ny, I32, 0, &grid);
            hipLaunchKernelGGL((k_step_ab_fused2d<32, S, K::force, K::comp, kNtStores>), grid, c->block, 0,
                               c->stream, src, dst, args, m);
        } else {
            const FuseMap m =
                fuse_plan(c->nx, c->ny, I16, blocks(I16) >= kFuseXcdMinBlocks ? kFuseXcdTile : 0, &grid);
            hipLaunchKernelGGL((k_step_ab_fused2d<16, S, K::force, K::comp, kNtStores>), grid, c->block, 0,
                               c->stream, src, dst, args, m);
        }
    }

    static lbm_status eager(lbm_ctx* c, int n)
    {
        int i = 0;
        if constexpr (L == 0) {
            // Periodic D2Q9, two lattices: launches of kFuseSteps steps, in
            // pairs so that the current buffer keeps following the parity of
            // the step count; the remainder runs one step per launch.
            if (!c->aa && !c->walls) {
                for (; n - i >= 2 * kFuseSteps; i += 2 * kFuseSteps) {
                    for (int h = 0; h < 2; ++h) {
                        const S* src = static_cast<const S*>(c->buf[c->cur]);
                        S* dst = static_cast<S*>(c->buf[1 - c->cur]);
                        dispatch(c, [&](auto k) { step_fused2d<decltype(k)>(c, src, dst); });
                        c->cur = 1 - c->cur;
                    }
                    c->steps += 2 * kFuseSteps;
                }
            }
        }
        for (; i < n; ++i) {
            if (c->aa) {
                S* A = static_cast<S*>(c->buf[0]);
                const bool odd = c->steps & 1;
                dispatch(c, [&](auto k) { step_aa<decltype(k)>(c, A, odd); });
            } else {
                const S* src = static_cast<const S*>(c->buf[c->cur]);
                S* dst = static_cast<S*>(c->buf[1 - c->cur]);
                dispatch(c, [&](auto k) { step_ab<decltype(k)>(c, src, dst); });
                c->cur = 1 - c->cur;
            }
            ++c->steps;
        }
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    // One two-lattice step between explicit buffers.
    static void step_between_t(lbm_ctx* c, const S* src, S* dst)
    {
        dispatch(c, [&](auto k) { step_ab<decltype(k)>(c, src, dst); });
    }

    using C = typename Store<S>::C;

    static AdjArgs<C> adj_args(const lbm_ctx* c)
    {
        AdjArgs<C> p;
        p.g = dims_of(c);
        p.bx_shift = c->bx_shift;
        p.omega = C(c->omega);
        for (int d = 0; d < 3; ++d) p.F[d] = C(c->F[d]);
        p.half = C(1.0 - 0.5 * c->omega);
        return p;
    }

    template <class K>
    static void adj_step(lbm_ctx* c, const S* g, const C* lin, C* lout, double* acc)
    {
        hipLaunchKernelGGL((k_adjoint_step<L, S, K::walls, K::force, K::comp>), c->grid, c->block, 0,
                           c->stream, g, lin, lout, acc, adj_args(c));
    }

    // Transpose of Eq. (bb) on nodal walls, applied to an adjoint field.
    static void nodal_bt(lbm_ctx* c, C* lam)
    {
        if (c->nodal < 0) return;
        const int n[3] = {c->nx, c->ny, c->nz};
        const int u = c->nodal == 0 ? 1 : 0, v = c->nodal == 2 ? 1 : 2;
        const size_t work = 2 * size_t(n[u]) * size_t(n[v]);
        hipLaunchKernelGGL((k_adjoint_nodal_bt<L, C>), dim3(unsigned((work + 255) / 256)), dim3(256), 0,
                           c->stream, lam, dims_of(c));
    }

    // Backward sweep over n steps with checkpoints every k steps; see
    // lbm_adjoint.  ws holds the recomputed segment (k-1 states, plus the
    // final state in the compressible model), two lambda fields and the
    // per-workgroup accumulators.
    static lbm_status adjoint(lbm_ctx* c, int n, int k, const void* ckpt, void* ws, const double* rho0,
                              const double* u0, const double* ubar, double* u0bar, double* out4)
    {
        const WorkspaceLayout W = workspace_layout(c, k);
        char* w = static_cast<char*>(ws);
        C* lam[2] = {reinterpret_cast<C*>(w + W.lam0), reinterpret_cast<C*>(w + W.lam1)};
        double* acc = reinterpret_cast<double*>(w + W.acc);
        double* result = reinterpret_cast<double*>(w + W.result);
        const Dims g = dims_of(c);
        IoArgs io = io_args(c);
        io.mode = kPull;
        hipLaunchKernelGGL(k_fill_zero, dim3((W.acc_doubles + 255) / 256), dim3(256), 0, c->stream, acc,
                           W.acc_doubles);
        // Output map; the compressible one needs the final state, the step
        // after the last recomputed state of the last segment.
        auto seed = [&](const S* fN) {
            dispatch(c, [&](auto cfg) {
                using K = decltype(cfg);
                hipLaunchKernelGGL((k_adjoint_seed<L, S, K::walls, K::comp>), c->grid, c->block, 0, c->stream,
                                   ubar, fN, lam[0], acc, io);
            });
        };
        if (!c->comp) seed(nullptr);
        int cur = 0;
        const char* ck = static_cast<const char*>(ckpt);
        for (int s = n / k - 1; s >= 0; --s) {
            const S* state0 = reinterpret_cast<const S*>(ck + size_t(s) * W.state_bytes);
            auto state = [&](int j) -> S* {
                return j == 0 ? const_cast<S*>(state0)
                              : reinterpret_cast<S*>(w + W.seg + size_t(j - 1) * W.state_bytes);
            };
            for (int j = 1; j < k; ++j) step_between_t(c, state(j - 1), state(j));
            if (c->comp && s == n / k - 1) {
                step_between_t(c, state(k - 1), state(k));
                seed(state(k));
            }
            for (int j = k - 1; j >= 0; --j) {
                nodal_bt(c, lam[cur]);
                dispatch(c, [&](auto cfg) { adj_step<decltype(cfg)>(c, state(j), lam[cur], lam[1 - cur], acc); });
                cur = 1 - cur;
            }
        }
        nodal_bt(c, lam[cur]);
        dispatch(c, [&](auto cfg) {
            using K = decltype(cfg);
            hipLaunchKernelGGL((k_adjoint_init_map<L, S, K::walls, K::comp>), c->grid, c->block, 0, c->stream,
                               lam[cur], rho0, u0, u0bar, g, c->bx_shift);
        });
        hipLaunchKernelGGL(k_adjoint_sum, dim3(1), dim3(256), 0, c->stream, acc, W.nblocks, result);
        LBM_HIP(hipGetLastError());
        LBM_HIP(hipMemcpyAsync(out4, result, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        LBM_HIP(hipStreamSynchronize(c->stream));
        return LBM_OK;
    }

    static lbm_status build_links(lbm_ctx* c, const unsigned char* mask)
    {
        Dims g = dims_of(c);
        g.links = nullptr;
        hipLaunchKernelGGL((k_build_links<L>), c->grid, c->block, 0, c->stream, mask, c->links, g,
                           c->bx_shift);
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static lbm_status wall_force(lbm_ctx* c)
    {
        IoArgs p = io_args(c);
        const S* A = static_cast<const S*>(c->buf[c->cur]);
        hipLaunchKernelGGL((k_wall_force<L, S>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, c->stream,
                           A, c->d_partials, p);
        hipLaunchKernelGGL(k_sum3, dim3(1), dim3(kReduceThreads), 0, c->stream, c->d_partials,
                           kReduceBlocks, c->d_partials + 5 * size_t(kReduceBlocks));
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static lbm_status import(lbm_ctx* c, const double* f, const double* rho, const double* u,
                             const double* noise)
    {
        IoArgs p = io_args(c);
        S* A = static_cast<S*>(c->buf[c->cur]);
        if (c->walls)
            hipLaunchKernelGGL((k_import<L, S, true>), c->grid, c->block, 0, c->stream, A, f, rho, u,
                               noise, p);
        else
            hipLaunchKernelGGL((k_import<L, S, false>), c->grid, c->block, 0, c->stream, A, f, rho, u,
                               noise, p);
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static lbm_status export_f(lbm_ctx* c, double* f)
    {
        IoArgs p = io_args(c);
        const S* A = static_cast<const S*>(c->buf[c->cur]);
        if (c->walls)
            hipLaunchKernelGGL((k_export<L, S, true>), c->grid, c->block, 0, c->stream, A, f, p);
        else
            hipLaunchKernelGGL((k_export<L, S, false>), c->grid, c->block, 0, c->stream, A, f, p);
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    template <class O>
    static void moments_t(lbm_ctx* c, O* rho, O* u)
    {
        IoArgs p = io_args(c);
        const S* A = static_cast<const S*>(c->buf[c->cur]);
        if (c->walls)
            hipLaunchKernelGGL((k_moments<L, S, true, O>), c->grid, c->block, 0, c->stream, A, rho, u,
                               p);
        else
            hipLaunchKernelGGL((k_moments<L, S, false, O>), c->grid, c->block, 0, c->stream, A, rho,
                               u, p);
    }

    static lbm_status moments(lbm_ctx* c, void* rho, void* u, int f32)
    {
        if (f32)
            moments_t<float>(c, static_cast<float*>(rho), static_cast<float*>(u));
        else
            moments_t<double>(c, static_cast<double*>(rho), static_cast<double*>(u));
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    // Monitor reduction into partials (5 kReduceBlocks + 4 doubles; the last
    // four receive mass, kinetic energy, max |u| and the non-finite count).
    static lbm_status reduce(lbm_ctx* c, double* partials)
    {
        IoArgs p = io_args(c);
        const S* A = static_cast<const S*>(c->buf[c->cur]);
        if (c->walls)
            hipLaunchKernelGGL((k_reduce_partials<L, S, true>), dim3(kReduceBlocks),
                               dim3(kReduceThreads), 0, c->stream, A, partials, p);
        else
            hipLaunchKernelGGL((k_reduce_partials<L, S, false>), dim3(kReduceBlocks),
                               dim3(kReduceThreads), 0, c->stream, A, partials, p);
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceThreads), 0, c->stream, partials,
                           kReduceBlocks, int(Store<S>::kDeviation),
                           partials + 5 * size_t(kReduceBlocks));
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static lbm_status step_between(lbm_ctx* c, const void* src, void* dst)
    {
        step_between_t(c, static_cast<const S*>(src), static_cast<S*>(dst));
        LBM_HIP(hipGetLastError());
        return LBM_OK;
    }

    static const Ops* ops()
    {
        static const Ops table = {&step, &import, &export_f, &moments, &reduce, &adjoint,
                                  &build_links, &wall_force, &step_between};
        return &table;
    }
};

template <int L>
const Ops* make_ops(lbm_storage s)
{
    switch (s) {
    case LBM_F64: return Impl<L, double>::ops();
    case LBM_F32: return Impl<L, float>::ops();
    case LBM_F16_DEV: return Impl<L, __half>::ops();
    case LBM_BF16_DEV: return Impl<L, __hip_bfloat16>::ops();
    case LBM_E4M11_DEV: return Impl<L, e4m11>::ops();
    }
    return nullptr;
}

}  // namespace imexlbm
