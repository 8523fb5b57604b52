// Four time steps of a large periodic D2Q9 box in one pass over the state
// (two-lattice pattern), streaming up the rows of a strip of columns.
//
// A 256-item workgroup owns a strip of 256 columns (one per work-item: the
// kStreamStore = 224 columns it stores and 16 more on each side) and a
// segment of rows.  It walks up the rows once: in iteration j it loads
// stored row j (the post-collision state of the previous launch, "level
// 0"), and each level k = 1..4 pulls (Eq. (propagation)) and collides (Eq.
// (collision), the collide() of the one-step kernels) one row, lagging
// level k - 1 by one row, so that the three rows it pulls from (e_y = +1,
// 0, -1) have just been produced.  Per level a work-item keeps only what
// the next rows still need: the e_y = 0 populations of one row and the
// e_y = +1 populations of two rows, already moved along x (Eq.
// (propagation) in x: a wave shift between lanes, and between the
// wavefronts of the workgroup through LDS, one barrier per level and row).
// Level 4's rows are stored.  The two outermost columns lose one valid
// column per level, so 4 columns on each side would cover the 4 levels;
// with 16 the strip starts on a 128-byte line and each wavefront stores
// whole lines (with 8, whose 240 stored columns also start on a line, the
// wavefronts split lines between them: 4096^2 FP64 ran 2 % slower).  A
// segment re-reads 4 rows below and above its stored rows.
//
// Against the regions of fused2d.hpp (32 x 32 nodes around 24 x 24 stored
// ones), a launch fetches the state 1.14 x (256 of 224 columns) x
// (rows + 8) / rows instead of ~2.7 x, writes whole lines, and repeats
// that fraction of the collisions instead of 1.78 x.  The arithmetic per
// node and step is that of the one-step kernels, in the same order, so the
// state after 4 steps is bit for bit that of 4 one-step launches (each
// level rounds through the storage type, as a store and reload would).
#pragma once

#include "kernels.hpp"

namespace imexlbm {

constexpr int kStreamCols = 256;  // columns per workgroup, one per work-item
constexpr int kStreamHalo = 16;   // loaded columns on each side of the stored ones
constexpr int kStreamStore = kStreamCols - 2 * kStreamHalo;  // 224 stored columns
constexpr int kStreamLevels = 4;  // steps per launch
// Boxes of at least kStreamMinNodes nodes take these launches (smaller ones
// the regions of fused2d.hpp).
constexpr unsigned kStreamMinNodes = 1u << 20;

// Rows per segment for an nx x ny box when the GPU runs `slots` workgroups
// of the kernel at once.  Every workgroup runs rows + 2 H iterations, so a
// launch takes about ceil(workgroups / slots) rounds of that many: the rows
// from 8 to 256 that minimise the product (the fewest among equals).  Long
// segments re-read fewer rows (8 per segment) but leave part of the last
// round idle unless the workgroups fill it.  Measured at 4096^2 FP64 (19
// strips, 768 slots): 103 rows (760 workgroups, the rule's choice) 135,500-
// 136,700 MLUPS; 64 rows (1216) 130,400-132,300; 52 (1501) 131,900; 86
// (912) 121,400; 120 (665) 128,500.
inline int stream_rows(int nx, int ny, long long slots)
{
    const long long strips = (nx + kStreamStore - 1) / kStreamStore;
    int best = 8;
    long long best_cost = -1;
    for (int rows = 8; rows <= 256; ++rows) {
        const long long wg = strips * ((ny + rows - 1) / rows);
        const long long cost = (wg + slots - 1) / slots * (rows + 2 * kStreamLevels);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = rows;
        }
    }
    return best;
}

// Lane i receives v of lane i - 1 (SHIFT = 0x138, wave_shr:1) or of lane
// i + 1 (SHIFT = 0x130, wave_shl:1); the edge lane keeps its own v.
template <int SHIFT>
__device__ __forceinline__ float wave_shift_f(float v)
{
    int w = __builtin_bit_cast(int, v);
    w = __builtin_amdgcn_update_dpp(w, w, SHIFT, 0xf, 0xf, false);
    return __builtin_bit_cast(float, w);
}

template <int SHIFT, class C>
__device__ __forceinline__ C lane_shift(C v)
{
    if constexpr (sizeof(C) == 8) return wave_shift<SHIFT>(v);
    else return wave_shift_f<SHIFT>(v);
}

// rows: stored rows per workgroup (the last segment may have fewer).  The
// D2Q9 directions are a = 3 (e_x + 1) + (e_y + 1): a = 0, 1, 2 have
// e_x = -1, a = 6, 7, 8 e_x = +1; a = 0, 3, 6 have e_y = -1, a = 2, 5, 8
// e_y = +1.
template <class S, bool FORCE, bool COMP, bool NT>
__global__ __launch_bounds__(256) void k_step_ab_stream2d(const S* __restrict__ src, S* __restrict__ dst,
                                                          StepArgs<typename Store<S>::C> p, int rows)
{
    using C = typename Store<S>::C;
    constexpr int L = 0, Q = 9, H = kStreamLevels;
    const Dims& g = p.g;
    const int t = int(threadIdx.x), lane = t & 63, wave = t >> 6;
    const int x0 = int(blockIdx.x) * kStreamStore;  // first stored column
    const int y0 = int(blockIdx.y) * rows;          // first stored row
    const int nrows = min(rows, g.ny - y0);
    const int TS = g.S;
    int gx = (x0 - kStreamHalo + t) % g.nx;
    gx += gx < 0 ? g.nx : 0;
    const int ox = x0 + t - kStreamHalo;  // stored column of this work-item
    const bool store_col = t >= kStreamHalo && t < kStreamHalo + kStreamStore && ox < g.nx;

    // Values crossing a wavefront edge: [level][0] the e_x = +1 populations
    // of each wavefront's lane 63, [level][1] the e_x = -1 populations of
    // its lane 0.
    __shared__ C edge[H][2][4][3];
    C d0[H][3], d1[H][3], d2[H][3];  // per level: e_y = 0 of row r; e_y = +1 of rows r, r - 1
#pragma unroll
    for (int k = 0; k < H; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) d0[k][i] = d1[k][i] = d2[k][i] = C(0);
    C nxt[Q];

    const auto load_row = [&](int j, C (&out)[Q]) {
        int gy = (y0 - H + j) % g.ny;
        gy += gy < 0 ? g.ny : 0;
        const unsigned node = unsigned(gx) + unsigned(g.nx) * unsigned(gy);
        static_for<Q>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            out[a] = Store<S>::load(src[slot<Q>(a, node, TS)]);
        });
    };

    const int iters = nrows + 2 * H;
    load_row(0, nxt);
    for (int j = 0; j < iters; ++j) {
        C v[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) v[a] = nxt[a];
        if (j + 1 < iters) load_row(j + 1, nxt);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            // Move the new row of level k along x: A_a(x) = v_a(x - e_a,x).
            if (lane == 63) {
                edge[k][0][wave][0] = v[6];
                edge[k][0][wave][1] = v[7];
                edge[k][0][wave][2] = v[8];
            }
            if (lane == 0) {
                edge[k][1][wave][0] = v[0];
                edge[k][1][wave][1] = v[1];
                edge[k][1][wave][2] = v[2];
            }
            __syncthreads();
            C A[Q];
            static_for<3>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                A[6 + i] = lane_shift<0x138>(v[6 + i]);  // e_x = +1: from x - 1
                A[i] = lane_shift<0x130>(v[i]);          // e_x = -1: from x + 1
                A[3 + i] = v[3 + i];
            });
            if (lane == 0 && wave > 0) {
                A[6] = edge[k][0][wave - 1][0];
                A[7] = edge[k][0][wave - 1][1];
                A[8] = edge[k][0][wave - 1][2];
            }
            if (lane == 63 && wave < 3) {
                A[0] = edge[k][1][wave + 1][0];
                A[1] = edge[k][1][wave + 1][1];
                A[2] = edge[k][1][wave + 1][2];
            }
            // Level k + 1 at row r pulls e_y = -1 from row r + 1 (the new
            // row), e_y = 0 from row r, e_y = +1 from row r - 1.
            C f[Q];
            static_for<3>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                f[3 * i] = A[3 * i];             // e_y = -1
                f[3 * i + 1] = d0[k][i];         // e_y = 0
                f[3 * i + 2] = d2[k][i];         // e_y = +1
                d2[k][i] = d1[k][i];
                d1[k][i] = A[3 * i + 2];
                d0[k][i] = A[3 * i + 1];
            });
            if (j >= 2 * (k + 1)) {  // uniform: the rows it pulls from exist
                collide<L, C, FORCE, COMP, Store<S>::kDeviation>(f, p.c);
                if constexpr (!std::is_same_v<S, C>) {
                    static_for<Q>([&](auto ac) {
                        constexpr int a = decltype(ac)::value;
                        f[a] = Store<S>::load(Store<S>::save(f[a]));
                    });
                }
            }
#pragma unroll
            for (int a = 0; a < Q; ++a) v[a] = f[a];
        }
        if (j >= 2 * H && store_col) {
            const unsigned own = unsigned(ox) + unsigned(g.nx) * unsigned(y0 + j - 2 * H);
            static_for<Q>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                put<NT>(dst + slot<Q>(a, own, TS), Store<S>::save(v[a]));
            });
        }
    }
}

}  // namespace imexlbm
