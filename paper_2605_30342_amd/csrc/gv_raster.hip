// gv_raster.hip -- per-tile front-to-back blending for gfx950.
//
//   k_raster_vis  single-view particle visibility (Alg. 2): every pixel walks
//                 its tile's depth-sorted list; each Gaussian that overlaps the
//                 pixel (Mahalanobis^2 <= cut) and is reached before T < eps_T
//                 receives the pixel's transmittance and a count.  The 64
//                 contributions of a wave are summed with DPP and the four
//                 waves' sums combined in LDS, so each (tile, Gaussian) pair
//                 costs one pair of global atomics (the pair count of the
//                 blend is the sum of the counts, taken by k_vf_accum).
//   k_raster_uq   uncertainty rasterisation (Alg. 6): compensated opacity
//                 (eq. alpha_comp), per-pixel entropy bound (eq. huber) and
//                 per-tile partial sums of the score.
//   k_vf_accum    SH accumulation (Alg. 3): gamma_k += (sum T / count) a_l Y_k(d).
//
// Workgroup = one 16x16 tile, 256 threads, one pixel per lane.  The tile's
// list is staged through LDS in batches of 256 records; a batch loop stops
// as soon as every pixel of the tile has terminated.
#include <type_traits>

#include "gv_device.hpp"
#include "gv_launch.hpp"

namespace gv {

constexpr float LN2 = 0.6931471805599453f;

__device__ __forceinline__ int find_view(const ViewDev *__restrict__ views, int nv, int gt) {
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= gt) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Adds the block's total of a per-thread count to *out (one atomic per block).
__device__ __forceinline__ void block_count(uint32_t c, unsigned long long *out) {
    if (!out) return;
    __shared__ unsigned long long red[WAVES];
    unsigned long long x = c;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < WAVES; ++w) tot += red[w];
        if (tot) atomicAdd(out, tot);
    }
}
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

// Compile-time loop: f(std::integral_constant<int, J>{}) for J = I .. N-1.
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// x as held by lane J of this lane's row of 16 (DPP row broadcast).  Used as
// the first operand of a VALU instruction, the compiler folds the broadcast
// into that instruction, so a value staged once per row costs no extra move.
template <int J>
__device__ __forceinline__ float row_bcast(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x150 + J, 0xF, 0xF, true));
}

// c + a_J b, where a_J is a in lane J of this lane's row of 16 (the compiler
// does not fold a broadcast into v_fmac, so it is written out; the s_nop
// provides the two wait states a DPP read needs after a VALU write of a).
template <int J>
__device__ __forceinline__ float fmac_row_bcast(float c, float a, float b) {
    asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
        : "+v"(c)
        : "v"(a), "v"(b), "i"(J));
    return c;
}

// x from the lane of this lane's quad that the DPP quad_perm control CTRL selects.
template <int CTRL>
__device__ __forceinline__ float quad_perm_f(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}

// x from lane i - 4 of this lane's row (0 in lanes 0..3 of the row).
__device__ __forceinline__ float row_shr4_f(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x114, 0xF, 0xF, true));
}

// ---------------------------------------------------------------- batch staging

// A 16x16 tile is split into four 8x8 quadrants, one per wave.  Lane l of wave
// w owns pixel ((w & 1) * 8 + (l & 7), (w >> 1) * 8 + (l >> 3)) of the tile.
__device__ __forceinline__ void quadrant_pixel(int t, int &qx, int &qy) {
    const int w = t >> 6, l = t & 63;
    qx = ((w & 1) << 3) + (l & 7);
    qy = ((w >> 1) << 3) + (l >> 3);
}

// Records are staged in batches of RB (a launch-time choice: 64, 128 or 256);
// a wave blends its lists in groups of LGROUP entries.
constexpr int LGROUP = 16;
// Row stride (floats) of the per-wave transpose buffer: a multiple of 4 so that
// 16-byte reads stay aligned, and 4 mod 64 banks so that the four quads'
// reads of one pass fall in different banks.
constexpr int SCR_STRIDE = 68;

// Wave-level counts of one batch go through LDS in [list][wave] order, so
// that a list's four counts are one 16-byte read.  With the counts, each
// wave also posts whether any of its pixels is still live; both are read
// back after the batch's first barrier.
template <int NLISTS>
struct BatchCounts {
    int4 cnt[NLISTS];   // .x .. .w: records of waves 0 .. 3 in the list
    int4 live;          // .x .. .w: wave 0 .. 3 still has a live pixel
};

// Records of waves below w in a list, from the list's four wave counts (w uniform).
__device__ __forceinline__ int waves_below(const int4 c, int w) {
    return (w > 0 ? c.x : 0) + (w > 1 ? c.y : 0) + (w > 2 ? c.z : 0);
}

__device__ __forceinline__ int list_total(const int4 c) { return (c.x + c.y) + (c.z + c.w); }

// Lists are padded with never-hit entries to a multiple of LPAD; a list is
// consumed in groups of LGROUP entries and, for its last 1..LPAD entries, one
// group of LPAD.  Index of the pad slot thread t fills in list q (q = t / LPAD),
// or -1 (threads 0 .. 4 LPAD - 1 pad the four lists); n = length of list q.
constexpr int LPAD = LGROUP / 2;
__device__ __forceinline__ int pad_slot(int n) {
    const int t = threadIdx.x;
    if (t >= WAVES * LPAD) return -1;
    const int k = n + (t % LPAD);
    return k < ((n + LPAD - 1) / LPAD) * LPAD ? k : -1;
}

// ---------------------------------------------------------------- tile schedule

// Tile blended by workgroup b of a grid of T.  The workgroups of a launch are
// dealt to the eight XCDs in turn (b mod 8), and each XCD has its own L2.
// order 0: workgroup b takes tile b, so neighbouring tiles, which share most
// of their records, run on different XCDs and every XCD's L2 fetches them;
// order 1: XCD x takes a contiguous run of the tile ids (row-major tiles of
// one view after another), so neighbours share an L2.  A bijection of
// [0, T): XCD x holds the ceil((T - x) / 8) workgroups x, x + 8, ...
// order 2: torder[b], the tiles of all views by decreasing list length (the
// dispatcher hands workgroups to free slots in launch order, so the longest
// tiles start first and the short ones fill the end: no straggler tail).
// order 3 and 4 (persistent): a grid of about one round of resident
// workgroups; each workgroup takes queue positions until the queue is empty:
// position q is tile q (order 3) or torder[q] (order 4).  The queue is dealt
// to the eight XCDs (workgroup b runs on XCD b mod 8): XCD x takes positions
// x, x + 8, x + 16, ... through a counter of its own (cleared with the call's
// status words), so that no single counter serialises every workgroup's
// atomic and every XCD gets an equal share of long and short tiles.
__device__ __forceinline__ int tile_of_block(int b, int T, int order, const uint32_t *torder) {
    if (order == 2) return (int)torder[b];
    if (order == 0) return b;
    const int x = b & 7, k = b >> 3;
    const int per = T >> 3, rem = T & 7;
    return x * per + min(x, rem) + k;
}

// Queue positions of a persistent workgroup (ticket: the eight XCD
// counters).  Thread 0 asks for the next position when a tile starts, so the
// atomic's round trip overlaps the tile's work: take_tile() issues the
// request, next_tile() publishes its result to the workgroup.  The first
// barrier keeps the previous tile's LDS in use until every thread has left
// it; sq is read by all threads between the two barriers.
struct TileQueue {
    uint32_t *ctr;   // this XCD's counter
    uint32_t x;      // this XCD
    uint32_t pend;   // thread 0: the requested position's counter value
    __device__ __forceinline__ void take_tile() {
        if (threadIdx.x == 0) pend = atomicAdd(ctr, 1u);
    }
    __device__ __forceinline__ int next_tile(int &sq) {
        __syncthreads();
        if (threadIdx.x == 0) sq = (int)(pend * 8u + x);
        __syncthreads();
        return sq;
    }
};

__device__ __forceinline__ TileQueue tile_queue(uint32_t *ticket) {
    TileQueue tq;
    tq.x = blockIdx.x & 7u;
    tq.ctr = ticket + tq.x;
    tq.pend = 0;
    tq.take_tile();
    return tq;
}

// ---------------------------------------------------------------- VF CONST raster (Alg. 2)

// Contributions of LGROUP consecutive list entries are kept per lane (acc[])
// and summed over the wave's 64 pixels with one transpose through LDS,
// instead of a cross-lane reduction per Gaussian.
// With RB = 64 the registers and LDS of a workgroup fit six per CU.
template <int RB>
__device__ __forceinline__ void vis_tile(const int gt, const ViewDev *__restrict__ views, int nv,
                                         const uint2 *__restrict__ ranges, const uint32_t *__restrict__ ival,
                                         const uint32_t *__restrict__ ikey, const Rec *__restrict__ rec, float eps_T,
                                         float qcut, float *__restrict__ acc_T, uint32_t *__restrict__ acc_c) {
    constexpr int LCAP = RB + LGROUP;
    __shared__ float4 wA[WAVES][LCAP];     // ux, uy, l11, l21 (tile-local centre)
    __shared__ float2 wB[WAVES][LCAP];     // l22, o
    __shared__ uint16_t wS[WAVES][LCAP];   // batch slot of the entry
    // per batch slot (two batches: a batch is flushed while the next one blends)
    __shared__ BatchCounts<WAVES> bc;      // per quadrant list: counts of the four waves
    __shared__ float part[2 * RB];         // sum of T over the tile's hit pixels
    __shared__ uint32_t cpart[2 * RB];     // number of hit pixels
    __shared__ __align__(16) float scr[WAVES][LGROUP][SCR_STRIDE];

    const int vi = find_view(views, nv, gt);
    const ViewDev &V = views[vi];
    const int lt = gt - V.tile_base;
    const int ox = (lt % V.tiles_x) * TILE, oy = (lt / V.tiles_x) * TILE;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int qx, qy;
    quadrant_pixel(t, qx, qy);
    const float px = (float)qx + 0.5f, py = (float)qy + 0.5f;
    // transmittance; pixels outside the image start inactive (T = 0 < eps_T)
    float T = (ox + qx < V.w && oy + qy < V.h) ? 1.0f : 0.0f;
    const uint2 rg = ranges[gt];

    // records are prefetched: while batch k is blended, the records of batch
    // k + 1 and the record indices of batch k + 2 are in flight
    const bool loader = t < RB;
    uint32_t r1 = 0, r2 = 0, k1 = 0, k2 = 0;   // record indices and instance keys
    Rec R1 = {};
    if (loader && rg.x + t < rg.y) {
        r1 = ival[rg.x + t];
        k1 = ikey[rg.x + t];
    }
    if (loader && rg.x + RB + t < rg.y) {
        r2 = ival[rg.x + RB + t];
        k2 = ikey[rg.x + RB + t];
    }
    if (loader && rg.x + t < rg.y) R1 = rec[r1];

    // Adds a finished batch's per-slot sums to the per-record accumulators
    // (thread t holds slot t: record rlast).  Done one batch late, in the
    // middle of the next batch, so that the atomics are long complete when
    // the next record prefetch is waited for.
    uint32_t rlast = 0;
    auto flush = [&](int buf, uint32_t bstart) {
        const int cnt = (int)min((uint32_t)RB, rg.y - bstart);
        if (t < cnt) {
            const int sl = buf * RB + t;
            const uint32_t c = cpart[sl];
            if (c) {
                atomicAdd(&acc_T[rlast], part[sl]);
                atomicAdd(&acc_c[rlast], c);
            }
        }
    };
    int cur = 0;
    uint32_t blast = rg.y;   // start of the last blended batch (none yet)
    const int wu = __builtin_amdgcn_readfirstlane(w);
    for (uint32_t b = rg.x; b < rg.y; b += RB) {
        // Two barriers per batch.  Before the first: registers, this batch's
        // slot buffers (sR, part, cpart: the previous batch uses the other
        // half) and the wave counts.  Between the two: the lists, which the
        // previous batch's blend has finished reading at the first barrier.
        const bool have = loader && b + t < rg.y;
        const Rec R = R1;
        const uint32_t r = r1, kq = k1;
        r1 = r2;
        k1 = k2;
        if (loader && b + RB + t < rg.y) R1 = rec[r1];
        if (loader && b + 2 * RB + t < rg.y) {
            r2 = ival[b + 2 * RB + t];
            k2 = ikey[b + 2 * RB + t];
        }
        // quadrants of this tile the record's ellipse reaches (from the binning)
        const uint32_t mask = have ? kq >> QMASK_SHIFT : 0u;
        float ux = 0.f, uy = 0.f;
        if (have) local_centre(R, ox, oy, ux, uy);
        if (t < RB) {
            part[cur * RB + t] = 0.0f;
            cpart[cur * RB + t] = 0u;
        }
        // ONE (RB = 64): only wave 0 holds records, so a record's position in a
        // list is its lanes below, and wave 0 posts the four list lengths in
        // bc.cnt[0]; the other waves post only their liveness.
        constexpr bool ONE = RB == 64;
        uint32_t pre[WAVES];
        if (!ONE || wu == 0) {
            int c[WAVES];
#pragma unroll
            for (int q = 0; q < WAVES; ++q) {
                const unsigned long long bal = __builtin_amdgcn_ballot_w64(((mask >> q) & 1u) != 0u);
                pre[q] = lanes_below(bal);
                c[q] = (int)__popcll(bal);
                if (!ONE && lane == 0) (&bc.cnt[q].x)[wu] = c[q];
            }
            if (ONE && lane == 0) bc.cnt[0] = make_int4(c[0], c[1], c[2], c[3]);
        }
        {
            const bool alive = __builtin_amdgcn_ballot_w64(T >= eps_T) != 0ull;
            if (lane == 0) (&bc.live.x)[wu] = alive ? 1 : 0;
        }
        __syncthreads();
        {
            const int4 a = bc.live;
            if ((a.x | a.y | a.z | a.w) == 0) break;   // every pixel of the tile has terminated
        }
        // entries in batch (= depth) order: records of the lower waves first
        // (every wave stages when RB > 64, so nq is set on every path)
        int nq[WAVES];
        if constexpr (ONE) {
            const int4 c = bc.cnt[0];
            nq[0] = c.x; nq[1] = c.y; nq[2] = c.z; nq[3] = c.w;
        }
        if (!ONE || wu == 0) {
#pragma unroll
            for (int q = 0; q < WAVES; ++q) {
                int below = 0;
                if constexpr (!ONE) {
                    const int4 c = bc.cnt[q];
                    nq[q] = list_total(c);
                    below = waves_below(c, wu);
                }
                if ((mask >> q) & 1u) {
                    const int pos = below + (int)pre[q];
                    wA[q][pos] = make_float4(ux, uy, R.l11, R.l21);
                    wB[q][pos] = make_float2(R.l22, R.o);
                    wS[q][pos] = (uint16_t)(cur * RB + t);
                }
            }
            const int q = (t / LPAD) & (WAVES - 1);
            const int k = pad_slot(q == 0 ? nq[0] : q == 1 ? nq[1] : q == 2 ? nq[2] : nq[3]);
            if (k >= 0) {
                wA[q][k] = make_float4(1e18f, 1e18f, 1.0f, 0.0f);
                wB[q][k] = make_float2(1.0f, 0.0f);
                wS[q][k] = 0;
            }
        }
        const int len = wu == 0 ? nq[0] : wu == 1 ? nq[1] : wu == 2 ? nq[2] : nq[3];
        __syncthreads();
        if (blast != rg.y) flush(cur ^ 1, blast);
        const int jl = lane & (LGROUP - 1);
        // one group of G entries (G = LGROUP, or LPAD for the last few)
        auto group = [&](int i0, auto gs) {
            constexpr int G = decltype(gs)::value;
            // lane j of every row loads entry i0 + j; entry jj then reaches all
            // 64 pixels by row broadcast, so LDS is read once per group
            const float4 A = wA[w][i0 + jl];
            const float2 B = wB[w][i0 + jl];
            float acc[G];
            // hit counts of the group's entries, one byte each (at most 64 hits)
            unsigned long long cnt8[2] = {0ull, 0ull};
            static_for<0, G>([&](auto jc) {
                constexpr int jj = decltype(jc)::value;
                // centre minus pixel: the sign flip leaves the quadratic form unchanged
                const float ex = row_bcast<jj>(A.x) - px, ey = row_bcast<jj>(A.y) - py;
                const float w1 = fmac_row_bcast<jj>(row_bcast<jj>(A.z) * ex, A.w, ey);
                const float w2 = row_bcast<jj>(B.x) * ey;
                const float p = fmaf(w1, w1, w2 * w2);
                const bool ov = p <= qcut, live = T >= eps_T;
                const unsigned long long bal = __builtin_amdgcn_ballot_w64(ov) & __builtin_amdgcn_ballot_w64(live);
                const float a = (ov && live) ? T : 0.0f;
                acc[jj] = a;
                // T (1 - alpha), alpha = o 2^-p; a = 0 leaves T unchanged where there is no hit
                T = fmaf(-a, row_bcast<jj>(B.y) * fast_exp2(-p), T);
                cnt8[jj / 8] |= (unsigned long long)__popcll(bal) << (8 * (jj % 8));
            });
            // transpose: the 64 / G lanes of entry e = lane / (64 / G) each sum G
            // pixels; their partial sums are combined by DPP within the row
            constexpr int LPE = 64 / G;
#pragma unroll
            for (int jj = 0; jj < G; ++jj) scr[w][jj][lane] = acc[jj];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int ge = lane / LPE, gc = lane % LPE;
            const float4 *row = reinterpret_cast<const float4 *>(&scr[w][ge][gc * G]);
            float sum = 0.0f;
            static_for<0, G / 4>([&](auto rc) {
                const float4 r = row[decltype(rc)::value];
                sum += (r.x + r.y) + (r.z + r.w);
            });
            sum += quad_perm_f<0xB1>(sum);   // lanes (0 1 2 3) <- (1 0 3 2)
            sum += quad_perm_f<0x4E>(sum);   // lanes (0 1 2 3) <- (2 3 0 1)
            if constexpr (LPE == 8) sum += row_shr4_f(sum);   // lanes 4..7 <- 0..3 of the 8
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const uint32_t cv = (uint32_t)(((ge < 8 ? cnt8[0] : cnt8[1]) >> (8 * (ge & 7))) & 0xFFull);
            if (gc == (LPE == 8 ? 4 : 0) && cv > 0u) {
                const int slot = wS[w][i0 + ge];
                atomicAdd(&part[slot], sum);
                atomicAdd(&cpart[slot], cv);
            }
        };
        for (int i0 = 0; i0 < len; i0 += LGROUP) {
            if (__builtin_amdgcn_ballot_w64(T >= eps_T) == 0) break;
            if (len - i0 > LPAD) group(i0, std::integral_constant<int, LGROUP>{});
            else group(i0, std::integral_constant<int, LPAD>{});
        }
        blast = b;
        rlast = r;
        cur ^= 1;
    }
    __syncthreads();
    if (blast != rg.y) flush(cur ^ 1, blast);
}

// PERSIST: the persistent schedules (orders 3 and 4), a kernel of its own so
// that the one-tile form keeps its registers.
template <int RB, bool PERSIST>
__global__ __launch_bounds__(WG, RB == 64 ? 6 : 1) void k_raster_vis(const ViewDev *__restrict__ views, int nv,
                                                   const uint2 *__restrict__ ranges,
                                                   const uint32_t *__restrict__ ival, const uint32_t *__restrict__ ikey,
                                                   const Rec *__restrict__ rec,
                                                   float eps_T, float qcut, float *__restrict__ acc_T,
                                                   uint32_t *__restrict__ acc_c, int order,
                                                   const uint32_t *__restrict__ torder, int ntiles,
                                                   uint32_t *__restrict__ ticket) {
    if constexpr (!PERSIST) {
        vis_tile<RB>(tile_of_block(blockIdx.x, ntiles, order, torder), views, nv, ranges, ival, ikey, rec, eps_T,
                     qcut, acc_T, acc_c);
    } else {
        __shared__ int sq;
        TileQueue tq = tile_queue(ticket);
        for (;;) {
            const int q = tq.next_tile(sq);
            if (q >= ntiles) break;
            tq.take_tile();
            vis_tile<RB>(order == 4 ? (int)torder[q] : q, views, nv, ranges, ival, ikey, rec, eps_T, qcut, acc_T,
                         acc_c);
        }
    }
}

// ---------------------------------------------------------------- VF QUERY raster (Alg. 6)

// Lane -> pixel of the query blend: wave w covers quadrant w (8 x 8 pixels)
// and DPP row r of the wave (16 lanes) the 4 x 4 sub-block r of it.
__device__ __forceinline__ void subblock_pixel(int t, int &qx, int &qy) {
    const int w = t >> 6, l = t & 63, r = l >> 4, j = l & 15;
    qx = ((w & 1) << 3) + ((r & 1) << 2) + (j & 3);
    qy = ((w >> 1) << 3) + ((r >> 1) << 2) + (j >> 2);
}

// Each record of a batch is staged once (slot = its index in the batch); the
// 16 sub-blocks of the tile keep depth-ordered lists of slot indices, built
// from a 16-bit sub-block mask computed per record at staging.  A wave
// walks the four lists of its quadrant side by side: lane j of row r reads
// entry i0 + j of sub-block r's list (or a never-hit slot past its end), and
// entry jj reaches the row's 16 pixels by row broadcast, so every row
// composites its own list.  The wave iterates as long as its longest list.
// CC: the colour term's constant c_c = 1/2 log|Q_c| + 3/2 log(2 pi e) comes
// per record from rcc[] (a per-Gaussian colour covariance seen from this
// view) instead of the uniform u.cQc; costs one more LDS value per entry and
// one multiply-add per evaluated pair.
// DEPTH: also the expected depth of every pixel under the same weights,
// sum w* z / sum w* (0 where nothing contributes), from the per-record depths
// rz[], into dmaps (packed like maps); the same cost again.
// Blends tile gt; returns the thread's composited pairs (COUNT).
template <int RB, bool MAPS, bool COUNT, bool CC, bool DEPTH>
__device__ __forceinline__ uint32_t uq_tile(const int gt, const ViewDev *__restrict__ views, int nv,
                                            const uint2 *__restrict__ ranges, const uint32_t *__restrict__ ival,
                                            const Rec *__restrict__ rec, const float *__restrict__ rcc,
                                            const float *__restrict__ rz, const UqArgs &u,
                                            float *__restrict__ tile_part, float *__restrict__ maps,
                                            float *__restrict__ dmaps) {
    constexpr int NL = 4 * WAVES;          // sub-block lists per tile
    __shared__ float4 wA[RB + 1];          // ux, uy, l11, l21 per batch slot (slot RB: never hit)
    __shared__ float4 wB[RB + 1];          // l22, o (v + beta (1 - v)), o0 (1 - beta)(1 - v), v
    __shared__ float wC[CC ? RB + 1 : 1];        // c_c of the record
    __shared__ float wD[DEPTH ? RB + 1 : 1];     // depth of the record
    __shared__ uint16_t idx[NL][RB];       // per sub-block: slots in batch (= depth) order
    __shared__ BatchCounts<NL> bc;         // per sub-block list: counts of the four waves
    __shared__ float red[WAVES];

    const int vi = find_view(views, nv, gt);
    const ViewDev &V = views[vi];
    const int lt = gt - V.tile_base;
    const int ox = (lt % V.tiles_x) * TILE, oy = (lt / V.tiles_x) * TILE;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    int qx, qy;
    subblock_pixel(t, qx, qy);
    const float px = (float)qx + 0.5f, py = (float)qy + 0.5f;
    const bool inside = (ox + qx < V.w) && (oy + qy < V.h);
    // per pixel: sx = sum w* v, sxl = sum w* v log2(w* v); the entropy bound is
    // formed from them after the last Gaussian, with sum w* = 1 - T (every
    // composited w* = alpha* T is taken off T)
    float T = inside ? 1.0f : 0.0f, sx = 0.0f, sxl = 0.0f;
    float sxc = 0.0f;   // sum w* v c_c, with per-record constants
    float swz = 0.0f;   // sum w* z
    uint32_t npairs = 0;
    const uint2 rg = ranges[gt];
    const float ob = u.o0 * (1.0f - u.beta);
    const float qcb = band_threshold(u.qcut), sqb = sqrtf(qcb);
    const int mylist = 4 * w + (lane >> 4);
    if (t == 0) {
        wA[RB] = make_float4(1e18f, 1e18f, 1.0f, 0.0f);
        wB[RB] = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
        if (CC) wC[RB] = 0.0f;
        if (DEPTH) wD[RB] = 0.0f;
    }

    // records are prefetched as in the VF CONST blend
    const bool loader = t < RB;
    uint32_t r1 = 0, r2 = 0;   // record indices
    Rec R1 = {};
    float C1 = 0.0f, Z1 = 0.0f;
    if (loader && rg.x + t < rg.y) r1 = ival[rg.x + t];
    if (loader && rg.x + RB + t < rg.y) r2 = ival[rg.x + RB + t];
    if (loader && rg.x + t < rg.y) {
        R1 = rec[r1];
        if (CC) C1 = rcc[r1];
        if (DEPTH) Z1 = rz[r1];
    }

    const int wu = __builtin_amdgcn_readfirstlane(w);
    for (uint32_t b = rg.x; b < rg.y; b += RB) {
        // Two barriers per batch: registers and wave counts before the first;
        // the staged records and the lists (which the previous batch's blend
        // has finished reading at the first barrier) between the two.
        const bool have = loader && b + t < rg.y;
        const Rec R = R1;
        const float Cr = C1, Zr = Z1;
        r1 = r2;
        if (loader && b + RB + t < rg.y) {
            R1 = rec[r1];
            if (CC) C1 = rcc[r1];
            if (DEPTH) Z1 = rz[r1];
        }
        if (loader && b + 2 * RB + t < rg.y) r2 = ival[b + 2 * RB + t];
        // the sub-blocks the record reaches
        uint32_t smask = 0u;
        float ux = 0.0f, uy = 0.0f;
        if (have) {
            local_centre(R, ox, oy, ux, uy);
            const EllipseBands E = ellipse_bands(R.l11, R.l21, R.l22, sqb);
            smask = subblock_mask_bands(ux, uy, E.kx, E.ia, R.l22, E.eyR, E.hy, qcb);
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const unsigned long long bal = __builtin_amdgcn_ballot_w64(((smask >> l) & 1u) != 0u);
            if (lane == 0) (&bc.cnt[l].x)[wu] = (int)__popcll(bal);
        }
        {
            const bool alive = __builtin_amdgcn_ballot_w64(T >= u.eps_T) != 0ull;
            if (lane == 0) (&bc.live.x)[wu] = alive ? 1 : 0;
        }
        __syncthreads();
        {
            const int4 a = bc.live;
            if ((a.x | a.y | a.z | a.w) == 0) break;   // every pixel of the tile has terminated
        }
        // stage the record in its slot; slot lists in batch (= depth) order,
        // records of the lower waves first
        if (have) {
            const float v = R.v;
            wA[t] = make_float4(ux, uy, R.l11, R.l21);
            wB[t] = make_float4(R.l22, R.o * fmaf(u.beta, 1.0f - v, v), ob * (1.0f - v), v);
            if (CC) wC[t] = Cr;
            if (DEPTH) wD[t] = Zr;
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const unsigned long long bal = __builtin_amdgcn_ballot_w64(((smask >> l) & 1u) != 0u);
            if ((smask >> l) & 1u) idx[l][waves_below(bc.cnt[l], wu) + (int)lanes_below(bal)] = (uint16_t)t;
        }
        const int mylen = list_total(bc.cnt[mylist]);
        const int len = max(max(list_total(bc.cnt[4 * wu]), list_total(bc.cnt[4 * wu + 1])),
                            max(list_total(bc.cnt[4 * wu + 2]), list_total(bc.cnt[4 * wu + 3])));
        __syncthreads();
        const int jl = lane & (LGROUP - 1);
        // one group of G entries per row (G = LGROUP, or LPAD for the last few)
        auto group = [&](int i0, auto gs) {
            constexpr int G = decltype(gs)::value;
            const int slot = i0 + jl < mylen ? (int)idx[mylist][i0 + jl] : RB;
            const float4 A = wA[slot];
            const float4 B = wB[slot];
            const float Cg = CC ? wC[slot] : 0.0f;
            const float Zg = DEPTH ? wD[slot] : 0.0f;
            static_for<0, G>([&](auto jc) {
                // products and sums are rounded separately, so that every
                // broadcast operand folds into its instruction
#pragma clang fp contract(off)
                constexpr int jj = decltype(jc)::value;
                const float ex = row_bcast<jj>(A.x) - px, ey = row_bcast<jj>(A.y) - py;
                const float w1 = fmac_row_bcast<jj>(row_bcast<jj>(A.z) * ex, A.w, ey);
                const float w2 = row_bcast<jj>(B.x) * ey;
                const float p = fmaf(w1, w1, w2 * w2);
                const bool ov = p <= u.qcut, live = T >= u.eps_T;
                const unsigned long long bal = __builtin_amdgcn_ballot_w64(ov) & __builtin_amdgcn_ballot_w64(live);
                if (bal) {
                    const bool hit = ov && live;
                    const float as = row_bcast<jj>(B.z) + row_bcast<jj>(B.y) * fast_exp2(-p);      // alpha*
                    const float wt = hit ? as * T : 0.0f;                                            // w*
                    const float x = row_bcast<jj>(B.w) * wt;                                         // w* v
                    sxl = fmaf(x, fast_log2(fmaxf(x, 1e-30f)), sxl);
                    sx += x;
                    if (CC) sxc = fmac_row_bcast<jj>(sxc, Cg, x);                                    // x c_c
                    if (DEPTH) swz = fmac_row_bcast<jj>(swz, Zg, wt);                                // w* z
                    T -= wt;                                                                         // T (1 - alpha*)
                    if (COUNT) npairs += hit ? 1u : 0u;
                }
            });
        };
        for (int i0 = 0; i0 < len; i0 += LGROUP) {
            if (__builtin_amdgcn_ballot_w64(T >= u.eps_T) == 0) break;
            if (len - i0 > LPAD) group(i0, std::integral_constant<int, LGROUP>{});
            else group(i0, std::integral_constant<int, LPAD>{});
        }
        __syncthreads();
    }
    // H = sum_hits x (cQc - ln x) + w0 (cQ0 - ln w0), w0 = sum w* (1 - v) = sw - sx >= 0
    float H = CC ? fmaf(-LN2, sxl, sxc) : fmaf(u.cQc, sx, -LN2 * sxl);
    const float sw = inside ? 1.0f - T : 0.0f;
    const float w0 = sw - sx;
    if (w0 > 0.0f) H = fmaf(w0, fmaf(-LN2, fast_log2(w0), u.cQ0), H);
    if (!inside) H = 0.0f;
    if (MAPS && inside) maps[V.pix_base + (int64_t)(oy + qy) * V.w + (ox + qx)] = H;
    if (DEPTH && inside) dmaps[V.pix_base + (int64_t)(oy + qy) * V.w + (ox + qx)] = sw > 0.0f ? swz / sw : 0.0f;
    const float s = wave_sum(H);
    if (lane == 0) red[w] = s;
    __syncthreads();
    if (t == 0) {
        float tot = 0.0f;
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) tot += red[ww];
        tile_part[gt] = tot;
    }
    return npairs;
}

template <int RB, bool MAPS, bool COUNT, bool CC, bool DEPTH, bool PERSIST>
__global__ __launch_bounds__(WG) void k_raster_uq(const ViewDev *__restrict__ views, int nv,
                                                  const uint2 *__restrict__ ranges,
                                                  const uint32_t *__restrict__ ival,
                                                  const Rec *__restrict__ rec, const float *__restrict__ rcc,
                                                  const float *__restrict__ rz,
                                                  UqArgs u, float *__restrict__ tile_part, float *__restrict__ maps,
                                                  float *__restrict__ dmaps, unsigned long long *__restrict__ pairs,
                                                  int order, const uint32_t *__restrict__ torder, int ntiles,
                                                  uint32_t *__restrict__ ticket) {
    uint32_t npairs = 0;
    if constexpr (!PERSIST) {
        npairs = uq_tile<RB, MAPS, COUNT, CC, DEPTH>(tile_of_block(blockIdx.x, ntiles, order, torder), views, nv,
                                                     ranges, ival, rec, rcc, rz, u, tile_part, maps, dmaps);
    } else {
        __shared__ int sq;
        TileQueue tq = tile_queue(ticket);
        for (;;) {
            const int q = tq.next_tile(sq);
            if (q >= ntiles) break;
            tq.take_tile();
            npairs += uq_tile<RB, MAPS, COUNT, CC, DEPTH>(order == 4 ? (int)torder[q] : q, views, nv, ranges, ival,
                                                          rec, rcc, rz, u, tile_part, maps, dmaps);
        }
    }
    if (COUNT) block_count(npairs, pairs);
}

// ---------------------------------------------------------------- scores and argmax

// S_v = sum of the view's tile partials, accumulated in FP64.
__global__ __launch_bounds__(WG) void k_scores(const ViewDev *__restrict__ views, const float *__restrict__ tile_part,
                                               const Status *__restrict__ st, float *__restrict__ scores) {
    const ViewDev &V = views[blockIdx.x];
    const int n = V.tiles_x * V.tiles_y;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += WG) s += (double)tile_part[V.tile_base + i];
    __shared__ double red[WG];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = WG / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) scores[blockIdx.x] = st->overflow ? __int_as_float(0x7fc00000) : (float)red[0];
}

__device__ __forceinline__ bool better(float a, int ia, float b, int ib) {
    if (ia < 0) return false;
    if (ib < 0) return true;
    return a > b || (a == b && ia < ib);
}

__global__ __launch_bounds__(1024) void k_argmax(const float *__restrict__ scores, int n, int32_t *__restrict__ best) {
    float bv = 0.0f;
    int bi = -1;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const float v = scores[i];
        if (v != v) continue;
        if (better(v, i, bv, bi)) { bv = v; bi = i; }
    }
    __shared__ float sv[1024];
    __shared__ int si[1024];
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            if (better(sv[threadIdx.x + off], si[threadIdx.x + off], sv[threadIdx.x], si[threadIdx.x])) {
                sv[threadIdx.x] = sv[threadIdx.x + off];
                si[threadIdx.x] = si[threadIdx.x + off];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *best = si[0];
}

// ---------------------------------------------------------------- VF accumulation (Alg. 3)

struct ALs { float a[4]; };

__device__ __forceinline__ void store_f(float *p, int64_t i, float v) { p[i] = v; }
__device__ __forceinline__ void store_f(_Float16 *p, int64_t i, float v) { p[i] = (_Float16)v; }
__device__ __forceinline__ void store_f(uint16_t *p, int64_t i, float v) {   // bfloat16, round to nearest even
    uint32_t b = __float_as_uint(v);
    if ((b & 0x7f800000u) != 0x7f800000u) b += 0x7fffu + ((b >> 16) & 1u);
    p[i] = (uint16_t)(b >> 16);
}

template <typename TG, typename TGam, int L>
__global__ __launch_bounds__(WG) void k_vf_accum(GaussArgs a, const ViewDev *__restrict__ views,
                                                 const uint32_t *__restrict__ offs, const uint32_t *__restrict__ vmask,
                                                 int mw,
                                                 const float *__restrict__ acc_T, const uint32_t *__restrict__ acc_c,
                                                 const Status *__restrict__ st, ALs al, TGam *__restrict__ gamma,
                                                 bool accumulate, unsigned long long *__restrict__ pairs) {
    constexpr int K = (L + 1) * (L + 1);
    const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (st->overflow) return;
    uint32_t npairs = 0;   // pixels composited over this Gaussian's records
    if (g < a.n) {
        float m[3];
        {
            const TG *mp = (const TG *)a.means;
            if constexpr (sizeof(TG) == 4) {
                m[0] = load_f(mp, 3 * g); m[1] = load_f(mp, 3 * g + 1); m[2] = load_f(mp, 3 * g + 2);
            } else {
                const int64_t blk = g / (a.anchor_block > 0 ? a.anchor_block : 1);
                m[0] = a.anchors[3 * blk] + load_f(mp, 3 * g);
                m[1] = a.anchors[3 * blk + 1] + load_f(mp, 3 * g + 1);
                m[2] = a.anchors[3 * blk + 2] + load_f(mp, 3 * g + 2);
            }
        }
        float acc[K];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = accumulate ? load_f((const TGam *)gamma, (int64_t)k * a.n + g) : 0.0f;
        // records of g in order: per view subset, the views whose bit is set in
        // the cull's mask, ascending
        const uint32_t rlim = st->R_eff;
        for (int sub = 0; sub < PROJ_SPLIT; ++sub) {
            const int64_t e = g * PROJ_SPLIT + sub;
            uint32_t r = offs[e];
            const uint32_t rend = min(offs[e + 1], rlim);
            for (int wi = 0; wi < mw && r < rend; ++wi) {
                uint32_t x = vmask[e * mw + wi];
                while (x != 0u && r < rend) {
                    const int vw = sub + PROJ_SPLIT * (32 * wi + __builtin_ctz(x));
                    x &= x - 1u;
                    const uint32_t c = acc_c[r];
                    if (c == 0) { ++r; continue; }
                    npairs += c;
                    const float v = acc_T[r] / (float)c;
                    const ViewDev &V = views[vw];
                    float dx = m[0] - V.C[0], dy = m[1] - V.C[1], dz = m[2] - V.C[2];
                    const float nrm = sqrtf(dx * dx + dy * dy + dz * dz);
                    if (!(nrm > 0.0f)) { ++r; continue; }
                    const float inv = 1.0f / nrm;
                    dx *= inv; dy *= inv; dz *= inv;
                    float Y[K];
                    sh_eval<L>(dx, dy, dz, Y);
#pragma unroll
                    for (int l = 0; l <= L; ++l) {
                        const float va = v * al.a[l];
#pragma unroll
                        for (int k = l * l; k < (l + 1) * (l + 1); ++k) acc[k] = fmaf(va, Y[k], acc[k]);
                    }
                    ++r;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) store_f(gamma, (int64_t)k * a.n + g, acc[k]);
    }
    block_count(npairs, pairs);
}

// ---------------------------------------------------------------- multi-view visibility (Alg. 5)

// out[g] += sum over this pass's views of log(1 - v_p[g]), v_p = sum T / count
// (a view that reaches no pixel of g contributes log 1 = 0).
__global__ __launch_bounds__(WG) void k_vis_logsum(int64_t n, const uint32_t *__restrict__ offs,
                                                   const float *__restrict__ acc_T,
                                                   const uint32_t *__restrict__ acc_c, const Status *__restrict__ st,
                                                   float *__restrict__ out, bool accumulate,
                                                   unsigned long long *__restrict__ pairs) {
    const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (st->overflow) return;
    uint32_t npairs = 0;
    if (g < n) {
        float s = accumulate ? out[g] : 0.0f;
        const uint32_t r0 = offs[g * PROJ_SPLIT], r1 = min(offs[(g + 1) * PROJ_SPLIT], st->R_eff);
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t c = acc_c[r];
            if (c == 0) continue;
            npairs += c;
            const float v = fminf(acc_T[r] / (float)c, 1.0f);
            s += log1pf(-v);
        }
        out[g] = s;
    }
    block_count(npairs, pairs);
}

// out[g] = 1 - exp(out[g]) = 1 - prod_p (1 - v_p[g]).
__global__ __launch_bounds__(WG) void k_vis_finish(int64_t n, float *__restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (g < n) out[g] = 1.0f - expf(out[g]);
}

// Per-view single-view visibility (Alg. 2): out[view * n + g] = v_p[g] =
// sum T / count over the pixels the view composites for g, for every record
// of g in this pass (the caller clears the pass's rows first, so a view that
// culls g or reaches none of its pixels leaves 0).  Walks g's records in the
// order of the projection: per view subset, the views of the cull's mask,
// ascending.
__global__ __launch_bounds__(WG) void k_view_vis(int64_t n, const uint32_t *__restrict__ offs,
                                                 const uint32_t *__restrict__ vmask, int mw,
                                                 const float *__restrict__ acc_T, const uint32_t *__restrict__ acc_c,
                                                 const Status *__restrict__ st, float *__restrict__ out,
                                                 unsigned long long *__restrict__ pairs) {
    const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (st->overflow) return;
    uint32_t npairs = 0;
    if (g < n) {
        const uint32_t rlim = st->R_eff;
        for (int sub = 0; sub < PROJ_SPLIT; ++sub) {
            const int64_t e = g * PROJ_SPLIT + sub;
            uint32_t r = offs[e];
            const uint32_t rend = min(offs[e + 1], rlim);
            for (int wi = 0; wi < mw && r < rend; ++wi) {
                uint32_t x = vmask[e * mw + wi];
                while (x != 0u && r < rend) {
                    const int vw = sub + PROJ_SPLIT * (32 * wi + __builtin_ctz(x));
                    x &= x - 1u;
                    const uint32_t c = acc_c[r];
                    if (c != 0) {
                        npairs += c;
                        out[(int64_t)vw * n + g] = acc_T[r] / (float)c;
                    }
                    ++r;
                }
            }
        }
    }
    block_count(npairs, pairs);
}

void launch_view_vis(const GaussArgs &a, const uint32_t *offs, const uint32_t *vmask, int mw, const float *acc_T,
                     const uint32_t *acc_c, const Status *st, float *out, unsigned long long *pairs, hipStream_t s) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_view_vis, dim3((unsigned)((a.n + WG - 1) / WG)), dim3(WG), 0, s, a.n, offs, vmask, mw,
                       acc_T, acc_c, st, out, pairs);
}

void launch_vis_logsum(int64_t n, const uint32_t *offs, const float *acc_T, const uint32_t *acc_c, const Status *st,
                       float *out, bool accumulate, unsigned long long *pairs, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_vis_logsum, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, n, offs, acc_T, acc_c, st,
                       out, accumulate, pairs);
}

void launch_vis_finish(int64_t n, float *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_vis_finish, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, s, n, out);
}

// ---------------------------------------------------------------- density control (Alg. 5)

// Virtual particle i of nv at lo + u_i (hi - lo), formed in FP64 (the product
// of the FP32 draw and the FP32 box side is exact there) and stored in FP32
// like every Gaussian attribute; isotropic scale s, identity rotation,
// opacity 0: rows n_real + i of the FP32 attribute arrays.
__global__ __launch_bounds__(WG) void k_place_virtual(float *__restrict__ means, float *__restrict__ scales,
                                                      float *__restrict__ quats, float *__restrict__ opac,
                                                      const float *__restrict__ u, int64_t n_real, int64_t nv,
                                                      VirtArgs v) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= nv) return;
    const int64_t g = n_real + i;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        means[3 * g + k] = (float)fma((double)u[3 * i + k], v.span[k], v.lo[k]);
        scales[3 * g + k] = v.s;
    }
    quats[4 * g] = 1.0f;
    quats[4 * g + 1] = 0.0f;
    quats[4 * g + 2] = 0.0f;
    quats[4 * g + 3] = 0.0f;
    opac[g] = 0.0f;
}

// flags[i] = 1 where particle i is kept: its multi-view visibility is at most
// eps_v (Alg. 5's pruning rule).
__global__ __launch_bounds__(WG) void k_virtual_flags(const float *__restrict__ vis, int64_t n_real, int64_t nv,
                                                      float eps_v, uint32_t *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < nv) flags[i] = vis[n_real + i] <= eps_v ? 1u : 0u;
}

// The kept particles in draw order: kept[offs[i]] = i, and their attributes
// packed into rows offs[i] of tmp (11 floats: mean, scale, quaternion,
// opacity).
__global__ __launch_bounds__(WG) void k_virtual_pack(const uint32_t *__restrict__ flags,
                                                     const uint32_t *__restrict__ offs, int64_t n_real, int64_t nv,
                                                     const float *__restrict__ means, const float *__restrict__ scales,
                                                     const float *__restrict__ quats, const float *__restrict__ opac,
                                                     int32_t *__restrict__ kept, float *__restrict__ tmp) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= nv || !flags[i]) return;
    const uint32_t j = offs[i];
    const int64_t g = n_real + i;
    kept[j] = (int32_t)i;
    float *t = tmp + (int64_t)j * 11;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        t[k] = means[3 * g + k];
        t[3 + k] = scales[3 * g + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) t[6 + k] = quats[4 * g + k];
    t[10] = opac[g];
}

// Rows n_real .. n_real + n_kept - 1 of the attribute arrays <- the packed
// kept particles.
__global__ __launch_bounds__(WG) void k_virtual_store(const float *__restrict__ tmp, int64_t n_real, int64_t n_kept,
                                                      float *__restrict__ means, float *__restrict__ scales,
                                                      float *__restrict__ quats, float *__restrict__ opac) {
    const int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (j >= n_kept) return;
    const int64_t g = n_real + j;
    const float *t = tmp + j * 11;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        means[3 * g + k] = t[k];
        scales[3 * g + k] = t[3 + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) quats[4 * g + k] = t[6 + k];
    opac[g] = t[10];
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + WG - 1) / WG); }

void launch_place_virtual(float *means, float *scales, float *quats, float *opac, const float *u, int64_t n_real,
                          int64_t nv, const VirtArgs &v, hipStream_t s) {
    if (nv <= 0) return;
    hipLaunchKernelGGL(k_place_virtual, dim3(blocks_for(nv)), dim3(WG), 0, s, means, scales, quats, opac, u, n_real,
                       nv, v);
}

void launch_virtual_flags(const float *vis, int64_t n_real, int64_t nv, float eps_v, uint32_t *flags, hipStream_t s) {
    if (nv <= 0) return;
    hipLaunchKernelGGL(k_virtual_flags, dim3(blocks_for(nv)), dim3(WG), 0, s, vis, n_real, nv, eps_v, flags);
}

void launch_virtual_pack(const uint32_t *flags, const uint32_t *offs, int64_t n_real, int64_t nv, const float *means,
                         const float *scales, const float *quats, const float *opac, int32_t *kept, float *tmp,
                         hipStream_t s) {
    if (nv <= 0) return;
    hipLaunchKernelGGL(k_virtual_pack, dim3(blocks_for(nv)), dim3(WG), 0, s, flags, offs, n_real, nv, means, scales,
                       quats, opac, kept, tmp);
}

void launch_virtual_store(const float *tmp, int64_t n_real, int64_t n_kept, float *means, float *scales, float *quats,
                          float *opac, hipStream_t s) {
    if (n_kept <= 0) return;
    hipLaunchKernelGGL(k_virtual_store, dim3(blocks_for(n_kept)), dim3(WG), 0, s, tmp, n_real, n_kept, means, scales,
                       quats, opac);
}

// ---------------------------------------------------------------- dtype conversion

template <typename TS, typename TD>
__global__ __launch_bounds__(WG) void k_convert(const TS *__restrict__ src, TD *__restrict__ dst, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (uint64_t)gridDim.x * WG)
        store_f(dst, (int64_t)i, load_f(src, (int64_t)i));
}

template <typename TS>
static void convert_to(const TS *src, void *dst, int ddt, uint64_t n, hipStream_t s) {
    const dim3 grid(4096), block(WG);
    switch (ddt) {
    case 0: hipLaunchKernelGGL((k_convert<TS, float>), grid, block, 0, s, src, (float *)dst, n); break;
    case 1: hipLaunchKernelGGL((k_convert<TS, _Float16>), grid, block, 0, s, src, (_Float16 *)dst, n); break;
    default: hipLaunchKernelGGL((k_convert<TS, uint16_t>), grid, block, 0, s, src, (uint16_t *)dst, n); break;
    }
}

void launch_convert(const void *src, int sdt, void *dst, int ddt, uint64_t n, hipStream_t s) {
    if (n == 0) return;
    switch (sdt) {
    case 0: convert_to((const float *)src, dst, ddt, n, s); break;
    case 1: convert_to((const _Float16 *)src, dst, ddt, n, s); break;
    default: convert_to((const uint16_t *)src, dst, ddt, n, s); break;
    }
}

// ---------------------------------------------------------------- launchers

// Grid of a blend: one workgroup per tile, or for the persistent orders (3,
// 4) one round of resident workgroups at most (eight per CU; where fewer fit,
// the rest start as the first ones finish, find the queue empty and exit).
static unsigned blend_grid(int total_tiles, int order) {
    if (order < 3) return (unsigned)total_tiles;
    static const int cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            n = 256;
        return n > 0 ? n : 256;
    }();
    return (unsigned)std::min<int64_t>(total_tiles, (int64_t)cus * 8);
}

template <int RB>
static void raster_vis_rb(const ViewDev *views, int nv, int total_tiles, const uint2 *ranges, const uint32_t *ival,
                          const uint32_t *ikey, const Rec *rec, float eps_T, float qcut, float *acc_T, uint32_t *acc_c,
                          int order, const uint32_t *torder, uint32_t *ticket, hipStream_t s) {
    if (order >= 3)
        hipLaunchKernelGGL((k_raster_vis<RB, true>), dim3(blend_grid(total_tiles, order)), dim3(WG), 0, s, views, nv,
                           ranges, ival, ikey, rec, eps_T, qcut, acc_T, acc_c, order, torder, total_tiles, ticket);
    else
        hipLaunchKernelGGL((k_raster_vis<RB, false>), dim3(total_tiles), dim3(WG), 0, s, views, nv, ranges, ival, ikey,
                           rec, eps_T, qcut, acc_T, acc_c, order, torder, total_tiles, ticket);
}

void launch_raster_vis(const ViewDev *views, int nv, int total_tiles, const uint2 *ranges, const uint32_t *ival,
                       const uint32_t *ikey, const Rec *rec, float eps_T, float qcut, float *acc_T, uint32_t *acc_c, int batch,
                       int order, const uint32_t *torder, uint32_t *ticket, hipStream_t s) {
    if (total_tiles <= 0) return;
#define GV_VIS_ARGS views, nv, total_tiles, ranges, ival, ikey, rec, eps_T, qcut, acc_T, acc_c, order, torder, ticket, s
    switch (batch) {
    case 64: raster_vis_rb<64>(GV_VIS_ARGS); break;
    case 256: raster_vis_rb<256>(GV_VIS_ARGS); break;
    default: raster_vis_rb<128>(GV_VIS_ARGS); break;
    }
#undef GV_VIS_ARGS
}

template <int RB, bool CC, bool DEPTH, bool P>
static void raster_uq_rb(const ViewDev *views, int nv, int total_tiles, const uint2 *ranges, const uint32_t *ival,
                         const Rec *rec, const float *rcc, const float *rz, const UqArgs &u,
                         float *tile_part, float *maps, float *dmaps, unsigned long long *pairs, int order,
                         const uint32_t *torder, uint32_t *ticket, hipStream_t s) {
    const dim3 g(blend_grid(total_tiles, order)), b(WG);
#define GV_UQ_ARGS views, nv, ranges, ival, rec, rcc, rz, u, tile_part, maps, dmaps, pairs, order, torder, total_tiles, ticket
    if constexpr (DEPTH) {   // depth maps come with the entropy maps
        if (pairs)
            hipLaunchKernelGGL((k_raster_uq<RB, true, true, CC, true, P>), g, b, 0, s, GV_UQ_ARGS);
        else
            hipLaunchKernelGGL((k_raster_uq<RB, true, false, CC, true, P>), g, b, 0, s, GV_UQ_ARGS);
    } else {
        if (maps && pairs)
            hipLaunchKernelGGL((k_raster_uq<RB, true, true, CC, false, P>), g, b, 0, s, GV_UQ_ARGS);
        else if (maps)
            hipLaunchKernelGGL((k_raster_uq<RB, true, false, CC, false, P>), g, b, 0, s, GV_UQ_ARGS);
        else if (pairs)
            hipLaunchKernelGGL((k_raster_uq<RB, false, true, CC, false, P>), g, b, 0, s, GV_UQ_ARGS);
        else
            hipLaunchKernelGGL((k_raster_uq<RB, false, false, CC, false, P>), g, b, 0, s, GV_UQ_ARGS);
    }
#undef GV_UQ_ARGS
}

template <int RB>
static void raster_uq_var(const ViewDev *views, int nv, int total_tiles, const uint2 *ranges, const uint32_t *ival,
                          const Rec *rec, const float *rcc, const float *rz, const UqArgs &u,
                          float *tile_part, float *maps, float *dmaps, unsigned long long *pairs, int order,
                          const uint32_t *torder, uint32_t *ticket, hipStream_t s) {
#define GV_UQ_ARGS views, nv, total_tiles, ranges, ival, rec, rcc, rz, u, tile_part, maps, dmaps, pairs, order, torder, ticket, s
    const bool depth = dmaps && maps && rz;
    // the persistent schedules are built for the plain query; the colour and
    // depth variants take the matching one-tile schedule (same tiles, same
    // results)
    if ((rcc || depth) && order >= 3) {
        order = order == 4 ? 2 : 0;
        ticket = nullptr;
    }
    if (rcc && depth) raster_uq_rb<RB, true, true, false>(GV_UQ_ARGS);
    else if (rcc) raster_uq_rb<RB, true, false, false>(GV_UQ_ARGS);
    else if (depth) raster_uq_rb<RB, false, true, false>(GV_UQ_ARGS);
    else if (order >= 3) raster_uq_rb<RB, false, false, true>(GV_UQ_ARGS);
    else raster_uq_rb<RB, false, false, false>(GV_UQ_ARGS);
#undef GV_UQ_ARGS
}

void launch_raster_uq(const ViewDev *views, int nv, int total_tiles, const uint2 *ranges, const uint32_t *ival,
                      const Rec *rec, const float *rcc, const float *rz, const UqArgs &u,
                      float *tile_part, float *maps, float *dmaps, unsigned long long *pairs, int batch,
                      int order, const uint32_t *torder, uint32_t *ticket, hipStream_t s) {
    if (total_tiles <= 0) return;
#define GV_UQ_ARGS views, nv, total_tiles, ranges, ival, rec, rcc, rz, u, tile_part, maps, dmaps, pairs, order, torder, ticket, s
    switch (batch) {
    case 64: raster_uq_var<64>(GV_UQ_ARGS); break;
    case 256: raster_uq_var<256>(GV_UQ_ARGS); break;
    default: raster_uq_var<128>(GV_UQ_ARGS); break;
    }
#undef GV_UQ_ARGS
}

void launch_scores(const ViewDev *views, int nv, const float *tile_part, const Status *st, float *scores,
                   hipStream_t s) {
    if (nv <= 0) return;
    hipLaunchKernelGGL(k_scores, dim3(nv), dim3(WG), 0, s, views, tile_part, st, scores);
}

void launch_argmax(const float *scores, int n, int32_t *best, hipStream_t s) {
    hipLaunchKernelGGL(k_argmax, dim3(1), dim3(1024), 0, s, scores, n, best);
}

template <typename TG, typename TGam>
static void accum_L(int L, const GaussArgs &a, const ViewDev *views, const uint32_t *offs, const uint32_t *vmask, int mw,
                    const float *acc_T, const uint32_t *acc_c, const Status *st, const ALs &al, void *gamma,
                    bool accumulate, unsigned long long *pairs, hipStream_t s) {
    const unsigned grid = (unsigned)((a.n + WG - 1) / WG);
    TGam *gm = (TGam *)gamma;
    switch (L) {
    case 0: hipLaunchKernelGGL((k_vf_accum<TG, TGam, 0>), dim3(grid), dim3(WG), 0, s, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gm, accumulate, pairs); break;
    case 1: hipLaunchKernelGGL((k_vf_accum<TG, TGam, 1>), dim3(grid), dim3(WG), 0, s, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gm, accumulate, pairs); break;
    case 2: hipLaunchKernelGGL((k_vf_accum<TG, TGam, 2>), dim3(grid), dim3(WG), 0, s, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gm, accumulate, pairs); break;
    default: hipLaunchKernelGGL((k_vf_accum<TG, TGam, 3>), dim3(grid), dim3(WG), 0, s, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gm, accumulate, pairs); break;
    }
}

template <typename TG>
static void accum_gam(int gdt, int L, const GaussArgs &a, const ViewDev *views, const uint32_t *offs, const uint32_t *vmask, int mw,
                      const float *acc_T, const uint32_t *acc_c, const Status *st, const ALs &al, void *gamma,
                      bool accumulate, unsigned long long *pairs, hipStream_t s) {
    switch (gdt) {
    case 0: accum_L<TG, float>(L, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gamma, accumulate, pairs, s); break;
    case 1: accum_L<TG, _Float16>(L, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gamma, accumulate, pairs, s); break;
    default: accum_L<TG, uint16_t>(L, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gamma, accumulate, pairs, s); break;
    }
}

void launch_vf_accum(const GaussArgs &a, const ViewDev *views, const uint32_t *offs, const uint32_t *vmask, int mw,
                     const float *acc_T, const uint32_t *acc_c, const Status *st, int L, const float *al_in,
                     void *gamma, int gamma_dtype, bool accumulate, unsigned long long *pairs, hipStream_t s) {
    if (a.n == 0) return;
    ALs al;
    for (int l = 0; l < 4; ++l) al.a[l] = l <= L ? al_in[l] : 0.0f;
    switch (a.dtype) {
    case 0: accum_gam<float>(gamma_dtype, L, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gamma, accumulate, pairs, s); break;
    case 1: accum_gam<_Float16>(gamma_dtype, L, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gamma, accumulate, pairs, s); break;
    default: accum_gam<uint16_t>(gamma_dtype, L, a, views, offs, vmask, mw, acc_T, acc_c, st, al, gamma, accumulate, pairs, s); break;
    }
}

}  // namespace gv
