// gv_bin.hip -- culling, projection (with the fused visibility-field query),
// device scans, LSD radix sort and tile binning for gfx950.
//
// Layout of the work: a record is one (Gaussian, view) pair that survives a
// conservative frustum test; records are numbered Gaussian-major (all views
// of Gaussian 0, then Gaussian 1, ...) so that the build can accumulate a
// Gaussian's views without atomics.  Records are sorted by FP32 depth (stable,
// so equal depths keep index order), expanded into one instance per touched
// 16x16 tile, and the instances are stably sorted by global tile id: every
// tile's list is then in increasing (depth, Gaussian) order, the front-to-back
// order that Alg. 2 and Alg. 6 composite in.
#include <algorithm>

#include "gv_device.hpp"
#include "gv_launch.hpp"

#include <type_traits>

namespace gv {

// ---------------------------------------------------------------- small kernels

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ---------------------------------------------------------------- Gaussian loads

template <typename TG>
struct GaussIn {
    const TG *means;
    const TG *scales;
    const TG *quats;
    const TG *opac;
    const float *anchors;
    int32_t anchor_block;
    int64_t n;
    int64_t n_virtual;

    __device__ __forceinline__ void mean(int64_t g, float m[3]) const {
        if constexpr (std::is_same<TG, float>::value) {
            m[0] = means[3 * g];
            m[1] = means[3 * g + 1];
            m[2] = means[3 * g + 2];
        } else {
            const int64_t b = g / anchor_block;
            m[0] = anchors[3 * b] + load_f(means, 3 * g);
            m[1] = anchors[3 * b + 1] + load_f(means, 3 * g + 1);
            m[2] = anchors[3 * b + 2] + load_f(means, 3 * g + 2);
        }
    }
    __device__ __forceinline__ void scale(int64_t g, float s[3]) const {
        s[0] = load_f(scales, 3 * g);
        s[1] = load_f(scales, 3 * g + 1);
        s[2] = load_f(scales, 3 * g + 2);
    }
    __device__ __forceinline__ void quat(int64_t g, float q[4]) const {
        q[0] = load_f(quats, 4 * g);
        q[1] = load_f(quats, 4 * g + 1);
        q[2] = load_f(quats, 4 * g + 2);
        q[3] = load_f(quats, 4 * g + 3);
    }
    __device__ __forceinline__ float opacity(int64_t g) const { return load_f(opac, g); }
};

// ---------------------------------------------------------------- culling

// Conservative in-view test, evaluated identically by the count, measure and
// projection kernels (no FP contraction, so every kernel takes the same
// decision).  It keeps every Gaussian whose exact EWA ellipse bounding box can
// touch the image: the 2D x-variance is at most |J_x R|^2 s_max^2 + lowpass,
// with |J_x R|^2 = (fx/z)^2 (1 + (x/z)^2).
__device__ __forceinline__ bool cons_visible(const float m[3], float smax, const ViewDev &V, float znear,
                                          float lowpass, float cut) {
#pragma clang fp contract(off)
    const float pz = V.R[6] * m[0] + V.R[7] * m[1] + V.R[8] * m[2] + V.t[2];
    const float amax = fmaxf(fmaxf(fabsf(m[0]), fabsf(m[1])), fmaxf(fabsf(m[2]), 1.0f)) +
                       fmaxf(fmaxf(fabsf(V.t[0]), fabsf(V.t[1])), fabsf(V.t[2]));
    const float mg = 1e-4f * (1.0f + fabsf(pz) + amax);
    if (!(pz > znear - mg)) return false;
    if (pz < znear + mg) return true;
    const float px = V.R[0] * m[0] + V.R[1] * m[1] + V.R[2] * m[2] + V.t[0];
    const float py = V.R[3] * m[0] + V.R[4] * m[1] + V.R[5] * m[2] + V.t[1];
    // hardware reciprocal and square roots: their 1-ulp error is far inside
    // the test's margins
    const float iz = __builtin_amdgcn_rcpf(pz);
    const float ax = px * iz, ay = py * iz;
    const float s2 = smax * smax;
    const float wx2 = V.fx * V.fx * iz * iz * (1.0f + ax * ax);
    const float wy2 = V.fy * V.fy * iz * iz * (1.0f + ay * ay);
    const float rx = __builtin_amdgcn_sqrtf(cut * (wx2 * s2 + lowpass)) * 1.01f + 2.0f;
    const float ry = __builtin_amdgcn_sqrtf(cut * (wy2 * s2 + lowpass)) * 1.01f + 2.0f;
    const float ux = V.fx * ax + V.cx, uy = V.fy * ay + V.cy;
    const float slx = 1e-4f * (fabsf(ux) + V.fx * fabsf(ax) + 1.0f);
    const float sly = 1e-4f * (fabsf(uy) + V.fy * fabsf(ay) + 1.0f);
    return (ux + rx + slx >= 0.0f) && (ux - rx - slx <= (float)V.w) && (uy + ry + sly >= 0.0f) &&
           (uy - ry - sly <= (float)V.h);
}

// FP64 reciprocal and square root of positive arguments, about 1e-16
// relative: the hardware estimates refined by two Newton steps each (the
// results are rounded to FP32 or padded by conservative margins, so correct
// rounding is not needed).  sqrt_pos(0) = 0.
__device__ __forceinline__ double rcp_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
}

__device__ __forceinline__ double sqrt_pos(double x) {
    if (!(x > 0.0)) return 0.0;
    double y = __builtin_amdgcn_rsq(x);          // 1 / sqrt(x)
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    const double r = x * y;
    return fma(fma(-r, r, x), 0.5 * y, r);       // one more step on the root itself
}

// 3D covariance (R_q S)(R_q S)^T of one Gaussian in FP64: s00 s01 s02 s11 s12 s22.
__device__ __forceinline__ void cov3d(const float s[3], const float q[4], double S[6]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    const double qn = sqrt(w * w + x * x + y * y + z * z);
    const double iq = qn > 0.0 ? 1.0 / qn : 0.0;
    w *= iq; x *= iq; y *= iq; z *= iq;
    const double r00 = 1 - 2 * (y * y + z * z), r01 = 2 * (x * y - w * z), r02 = 2 * (x * z + w * y);
    const double r10 = 2 * (x * y + w * z), r11 = 1 - 2 * (x * x + z * z), r12 = 2 * (y * z - w * x);
    const double r20 = 2 * (x * z - w * y), r21 = 2 * (y * z + w * x), r22 = 1 - 2 * (x * x + y * y);
    const double a = s[0], b = s[1], c = s[2];
    const double m00 = r00 * a, m01 = r01 * b, m02 = r02 * c;
    const double m10 = r10 * a, m11 = r11 * b, m12 = r12 * c;
    const double m20 = r20 * a, m21 = r21 * b, m22 = r22 * c;
    S[0] = m00 * m00 + m01 * m01 + m02 * m02;
    S[1] = m00 * m10 + m01 * m11 + m02 * m12;
    S[2] = m00 * m20 + m01 * m21 + m02 * m22;
    S[3] = m10 * m10 + m11 * m11 + m12 * m12;
    S[4] = m10 * m20 + m11 * m21 + m12 * m22;
    S[5] = m20 * m20 + m21 * m21 + m22 * m22;
}

struct Proj {
    bool ok;
    double z, ux, uy, ca, cb, cc;
    int x0, x1, y0, y1;   // tile rectangle, half open
};

// Exact EWA projection in FP64 (the camera values and the attributes are the
// FP32 inputs): z, centre u, conic = inverse of J R S3 R^T J^T + lowpass I,
// and the tiles whose pixel centres can lie inside the m <= cut ellipse.
__device__ __forceinline__ void project_exact(const float m[3], const double S[6], const ViewDev &V, float znear,
                                           float lowpass, float cut, Proj &P) {
    // multiply-adds fused within an expression only (decided per expression,
    // so the sizing and the projection kernels compute the same values)
#pragma clang fp contract(on)
    P.ok = false;
    const double mx = m[0], my = m[1], mz = m[2];
    const double px = (double)V.R[0] * mx + (double)V.R[1] * my + (double)V.R[2] * mz + (double)V.t[0];
    const double py = (double)V.R[3] * mx + (double)V.R[4] * my + (double)V.R[5] * mz + (double)V.t[1];
    const double pz = (double)V.R[6] * mx + (double)V.R[7] * my + (double)V.R[8] * mz + (double)V.t[2];
    P.z = pz;
    if (!(pz > (double)znear)) return;
    const double iz = rcp_pos(pz);
    const double fx = V.fx, fy = V.fy;
    const double jx0 = fx * iz, jx2 = -fx * px * iz * iz;
    const double jy1 = fy * iz, jy2 = -fy * py * iz * iz;
    // W = J R (2x3)
    const double w00 = jx0 * V.R[0] + jx2 * V.R[6], w01 = jx0 * V.R[1] + jx2 * V.R[7], w02 = jx0 * V.R[2] + jx2 * V.R[8];
    const double w10 = jy1 * V.R[3] + jy2 * V.R[6], w11 = jy1 * V.R[4] + jy2 * V.R[7], w12 = jy1 * V.R[5] + jy2 * V.R[8];
    const double t0 = S[0] * w00 + S[1] * w01 + S[2] * w02;
    const double t1 = S[1] * w00 + S[3] * w01 + S[4] * w02;
    const double t2 = S[2] * w00 + S[4] * w01 + S[5] * w02;
    const double u0 = S[0] * w10 + S[1] * w11 + S[2] * w12;
    const double u1 = S[1] * w10 + S[3] * w11 + S[4] * w12;
    const double u2 = S[2] * w10 + S[4] * w11 + S[5] * w12;
    const double a = w00 * t0 + w01 * t1 + w02 * t2 + (double)lowpass;
    const double b = w10 * t0 + w11 * t1 + w12 * t2;
    const double c = w10 * u0 + w11 * u1 + w12 * u2 + (double)lowpass;
    const double det = a * c - b * b;
    if (!(det > 1e-12)) return;
    const double idet = rcp_pos(det);
    P.ca = c * idet;
    P.cb = -b * idet;
    P.cc = a * idet;
    P.ux = fx * px * iz + (double)V.cx;
    P.uy = fy * py * iz + (double)V.cy;
    const double rx = sqrt_pos((double)cut * a) * (1.0 + 1e-6) + 1e-4;
    const double ry = sqrt_pos((double)cut * c) * (1.0 + 1e-6) + 1e-4;
    double i0 = ceil(P.ux - rx - 0.5), i1 = floor(P.ux + rx - 0.5);
    double j0 = ceil(P.uy - ry - 0.5), j1 = floor(P.uy + ry - 0.5);
    i0 = fmax(i0, 0.0); j0 = fmax(j0, 0.0);
    i1 = fmin(i1, (double)(V.w - 1)); j1 = fmin(j1, (double)(V.h - 1));
    if (!(i0 <= i1) || !(j0 <= j1)) return;
    P.x0 = (int)i0 >> TILE_SHIFT;
    P.x1 = ((int)i1 >> TILE_SHIFT) + 1;
    P.y0 = (int)j0 >> TILE_SHIFT;
    P.y1 = ((int)j1 >> TILE_SHIFT) + 1;
    P.ok = true;
}

template <typename TG>
// Wave w of a block takes view subset sub = w (views sub, sub + PROJ_SPLIT,
// ...) for the block's 64 Gaussians, one per lane, so that the view read in
// each step is the same for the whole wave (scalar loads).
__global__ __launch_bounds__(WG) void k_count(GaussIn<TG> G, const ViewDev *__restrict__ views, int nv,
                                              float znear, float lowpass, float cut, uint32_t *__restrict__ cnt,
                                              uint32_t *__restrict__ vmask, int mw, uint32_t *__restrict__ clr0,
                                              uint32_t n0, uint32_t *__restrict__ clr1, uint64_t n1) {
    // the call's zero fills (status words, tile ranges) ride along, so
    // that they need no launches of their own
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < n1; i += (uint64_t)gridDim.x * WG) {
        if (i < n0) clr0[i] = 0u;
        clr1[i] = 0u;
    }
    if (blockIdx.x == 0 && n0 > n1)
        for (uint32_t i = n1 + threadIdx.x; i < n0; i += WG) clr0[i] = 0u;
    const int sub = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int64_t g = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (g >= G.n) return;
    const int64_t e = g * PROJ_SPLIT + sub;
    float m[3], s[3];
    G.mean(g, m);
    G.scale(g, s);
    const float smax = fmaxf(fmaxf(s[0], s[1]), s[2]);
    // bit i % 32 of word i / 32 set when view sub + PROJ_SPLIT i passes the test
    uint32_t c = 0, word = 0;
    int i = 0;
    for (int v = sub; v < nv; v += PROJ_SPLIT, ++i) {
        if (cons_visible(m, smax, views[v], znear, lowpass, cut)) {
            ++c;
            word |= 1u << (i & 31);
        }
        if ((i & 31) == 31) {
            vmask[e * mw + (i >> 5)] = word;
            word = 0;
        }
    }
    if (i & 31) vmask[e * mw + (i >> 5)] = word;
    cnt[e] = c;
}

// Sizing pass: counts records (conservative test) and exact instances.
template <typename TG>
__global__ __launch_bounds__(WG) void k_measure(GaussIn<TG> G, const ViewDev *__restrict__ views, int nv,
                                                float znear, float lowpass, float cut,
                                                unsigned long long *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
    const int64_t g = e / PROJ_SPLIT;
    const int sub = (int)(e % PROJ_SPLIT);
    unsigned long long rc = 0, mc = 0;
    if (g < G.n) {
        float m[3], s[3], q[4];
        G.mean(g, m);
        G.scale(g, s);
        G.quat(g, q);
        const float smax = fmaxf(fmaxf(s[0], s[1]), s[2]);
        double S[6];
        cov3d(s, q, S);
        for (int v = sub; v < nv; v += PROJ_SPLIT) {
            if (!cons_visible(m, smax, views[v], znear, lowpass, cut)) continue;
            ++rc;
            Proj P;
            project_exact(m, S, views[v], znear, lowpass, cut, P);
            if (P.ok) mc += (unsigned long long)(P.x1 - P.x0) * (unsigned long long)(P.y1 - P.y0);
        }
    }
    // wave totals, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        rc += __shfl_xor(rc, off);
        mc += __shfl_xor(mc, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&out[0], rc);
        atomicAdd(&out[1], mc);
    }
}

// Index of the k-th (from 0) set bit of x; x has more than k set bits.
__device__ __forceinline__ int kth_set_bit(uint32_t x, uint32_t k) {
    int pos = 0;
#pragma unroll
    for (int sh = 16; sh >= 1; sh >>= 1) {
        const uint32_t low = (uint32_t)__popc(x & ((1u << sh) - 1u));
        if (k >= low) {
            k -= low;
            x >>= sh;
            pos += sh;
        }
    }
    return pos;
}

// log(1 - a) for a in [0, 1], accurate also for small a: with u = 1 - a
// rounded, log(u) a / (1 - u) cancels the rounding error of u (the log1p
// identity of Goldberg, "What every computer scientist should know about
// floating-point arithmetic", 1991).  u = 1 gives -a, u = 0 gives -infinity.
__device__ __forceinline__ float log_one_minus(float a) {
    const float u = 1.0f - a;
    const float l = __builtin_amdgcn_logf(u) * 0.6931471805599453f * (a * __builtin_amdgcn_rcpf(1.0f - u));
    return u == 1.0f ? -a : l;
}

// Projection of every surviving (Gaussian, view) pair into its record slot,
// one record per lane.  A wave takes 64 consecutive (Gaussian, view subset)
// entries and enumerates their records in chunks of 64: the entry owning a
// record is found from start marks and a ballot (as in the instance
// emission), the view from the entry's visibility mask.  Lanes therefore stay
// busy however few views of a Gaussian survive the cull.
// MODE 0 (build) leaves the record's visibility at 0 and zeroes zr0[r], zr1[r] (the
// per-record accumulators of the blend, when given).  The query modes store
// the Gaussian's visibility in direction d = camera -> Gaussian:
// MODE 1, the visibility field (Alg. 4): V~ = sum_k gamma_k Y_k(d), clamped to
//   [0, |P|], then V = 1 - (1 - V~/|P|)^|P| as 1 - exp(|P| log1p(-V~/|P|));
// MODE 2, the exact multi-view visibility (eq. vis_all with eq. vis_p):
//   V = 1 - prod_p (1 - v_p nu_p), nu_p = exp(kappa (d . d_p - 1)), d_p the
//   unit direction from training camera p, summed as logs and finished with
//   expm1 so that small V keep their relative precision.  A training camera
//   at the Gaussian's centre contributes nothing.
// With rz (query modes), also the record's depth rz[r] = z (FP32).
// With cvar (query modes), also the colour term's constant of the record,
// rcc[r] = 1/2 log|Q_c(d)| + 3/2 log(2 pi e), where channel k of the colour
// covariance is Q_k(d) = sum_j Y_j(d)^2 cvar[(k Kc + j) n + g] (the colour is
// linear in its SH coefficients, whose variances cvar holds), floored at
// 1e-30; 3/2 log(2 pi e) alone for a Gaussian at the camera centre.
// EXTRA: the colour constants and depths above are requested (compiled out
// otherwise, so that the plain query keeps its scalar registers).
template <typename TG, typename TGam, int MODE, int L, bool EXTRA>
__global__ __launch_bounds__(WG) void k_project(GaussIn<TG> G, const ViewDev *__restrict__ views, int nv,
                                                float znear, float lowpass, float cut,
                                                const uint32_t *__restrict__ offs, const uint32_t *__restrict__ vmask,
                                                int mw, const Status *__restrict__ st, uint32_t rcap,
                                                const TGam *__restrict__ gamma, float n_train,
                                                const float *__restrict__ vtrain, const float *__restrict__ tc,
                                                int ntv, float kappa_log2e, const float *__restrict__ cvar, int Lc,
                                                float c3, float *__restrict__ rcc, float *__restrict__ rz,
                                                Rec *__restrict__ rec, uint32_t *__restrict__ key,
                                                Bin *__restrict__ bin, uint32_t *__restrict__ ntr, int pack,
                                                uint32_t *__restrict__ zr0, uint32_t *__restrict__ zr1) {
    constexpr int K = (L + 1) * (L + 1);
    __shared__ uint32_t srel[WAVES][64];   // first record of each entry (relative)
    __shared__ uint8_t cl[WAVES][64];      // lanes of the entries that own records, in order
    __shared__ uint8_t mk[WAVES][64];      // 1 where an entry starts at that record of the chunk
    __shared__ float4 sgm[WAVES][64];      // each entry's Gaussian: mean, opacity
    __shared__ double sgS[WAVES][6][64];   // its 3D covariance (six terms, one row per term)
    // the query's SH coefficients of each entry's Gaussian (K per entry, rows
    // of K + 1 floats so that entries fall in different banks)
    constexpr int GROW = MODE == 1 ? K + 1 : 1;
    __shared__ float sgG[WAVES][MODE == 1 ? 64 : 1][GROW];
    if (st->overflow & 1u) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t ne = (uint64_t)G.n * PROJ_SPLIT;
    const uint64_t nwaves = (uint64_t)gridDim.x * WAVES;
    const double sc = 0.8493218002880191;   // sqrt(log2(e) / 2)
    for (uint64_t c = (uint64_t)blockIdx.x * WAVES + w; c * 64 < ne; c += nwaves) {
        const uint64_t e = c * 64 + lane;
        const bool valid = e < ne;
        uint32_t o = 0, cnt = 0;
        if (valid) {
            o = offs[e];
            cnt = offs[e + 1] - o;
        }
        const uint32_t o0 = __builtin_amdgcn_readfirstlane(o);
        const uint32_t rel = o - o0;
        const bool owns = valid && cnt > 0;
        const unsigned long long own = __builtin_amdgcn_ballot_w64(owns);
        if (owns) cl[w][lanes_below(own)] = (uint8_t)lane;
        srel[w][lane] = rel;
        if (owns) {
            // the Gaussian's attributes and 3D covariance, once per entry
            // for all of its records
            const int64_t g = (int64_t)(e / PROJ_SPLIT);
            float m[3], sc3[3], qt[4];
            G.mean(g, m);
            G.scale(g, sc3);
            G.quat(g, qt);
            double S[6];
            cov3d(sc3, qt, S);
            sgm[w][lane] = make_float4(m[0], m[1], m[2], G.opacity(g));
#pragma unroll
            for (int k = 0; k < 6; ++k) sgS[w][k][lane] = S[k];
            if constexpr (MODE == 1) {
                // read only where the records use them (real Gaussians, |P| > 0)
                if (n_train > 0.0f && g < G.n - G.n_virtual) {
#pragma unroll
                    for (int kk = 0; kk < K; ++kk) sgG[w][lane][kk] = load_f(gamma, (int64_t)kk * G.n + g);
                }
            }
        }
        uint32_t total = 0;
        if (own) {
            const int last = 63 - __builtin_clzll(own);
            total = __shfl(rel + cnt, last);
        }
        uint32_t started = 0;
        for (uint32_t J = 0; J < total; J += 64) {
            mk[w][lane] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (owns && rel >= J && rel < J + 64) mk[w][rel - J] = 1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const unsigned long long P = __builtin_amdgcn_ballot_w64(mk[w][lane] != 0);
            const uint32_t upto = started + lanes_below(P) + (uint32_t)((P >> lane) & 1ull);
            const uint32_t j = J + lane;
            const uint32_t r = o0 + j;
            if (j < total && r < rcap) {
                const int q = cl[w][upto - 1];
                uint32_t k = j - srel[w][q];
                const uint64_t eq = c * 64 + (uint64_t)q;
                const int64_t g = (int64_t)(eq / PROJ_SPLIT);
                const int sub = (int)(eq % PROJ_SPLIT);
                // the k-th view of the entry that passed the cull
                int wi = 0;
                uint32_t word = vmask[eq * mw];
                for (uint32_t pc = (uint32_t)__popc(word); k >= pc; pc = (uint32_t)__popc(word)) {
                    k -= pc;
                    word = vmask[eq * mw + ++wi];
                }
                const int v = sub + PROJ_SPLIT * (32 * wi + kth_set_bit(word, k));
                const ViewDev &V = views[v];
                const float4 gm = sgm[w][q];
                const float m[3] = {gm.x, gm.y, gm.z};
                double S[6];
#pragma unroll
                for (int kk = 0; kk < 6; ++kk) S[kk] = sgS[w][kk][q];
                Proj Pj;
                project_exact(m, S, V, znear, lowpass, cut, Pj);
                if constexpr (MODE == 0) {
                    // the build's per-record accumulators start at zero
                    if (zr0) zr0[r] = 0u;
                    if (zr1) zr1[r] = 0u;
                }
                Bin b = {};
                if (!Pj.ok) {
                    bin[r] = b;
                    if (ntr) ntr[r] = pack ? r : 0u;
                    key[r] = DEAD_KEY;
                    rec[r] = Rec{0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                } else {
                    const double ax = fmin(fmax(rint(Pj.ux), -32768.0), 32767.0);
                    const double ay = fmin(fmax(rint(Pj.uy), -32768.0), 32767.0);
                    Rec R;
                    R.uv = (int32_t)(((uint32_t)(int)ax & 0xFFFFu) | ((uint32_t)(int)ay << 16));
                    R.fx = (float)(Pj.ux - ax);
                    R.fy = (float)(Pj.uy - ay);
                    const double l11 = sqrt_pos(Pj.ca);          // ca > 0: det > 0
                    const double l21 = Pj.cb * rcp_pos(l11);
                    const double l22 = sqrt_pos(Pj.cc - l21 * l21);
                    R.l11 = (float)(sc * l11);
                    R.l21 = (float)(sc * l21);
                    R.l22 = (float)(sc * l22);
                    R.o = gm.w;
                    float vis = 0.0f;
                    if constexpr (MODE == 2) {
                        const bool virt = g >= G.n - G.n_virtual;
                        float dx = m[0] - V.C[0], dy = m[1] - V.C[1], dz = m[2] - V.C[2];
                        const float nrm = sqrtf(dx * dx + dy * dy + dz * dz);
                        if (!virt && ntv > 0 && nrm > 0.0f) {
                            const float inv = 1.0f / nrm;
                            dx *= inv; dy *= inv; dz *= inv;
                            float lsum = 0.0f;   // sum_p log(1 - v_p nu_p)
#pragma unroll 4
                            for (int p = 0; p < ntv; ++p) {
                                const float vp = vtrain[(int64_t)p * G.n + g];
                                const float ex = m[0] - tc[3 * p], ey = m[1] - tc[3 * p + 1], ez = m[2] - tc[3 * p + 2];
                                const float e2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
                                const float cosang = fmaf(dx, ex, fmaf(dy, ey, dz * ez)) * rsqrtf(e2);
                                const float nu = exp2f(kappa_log2e * (cosang - 1.0f));
                                const float a = e2 > 0.0f ? fminf(vp * nu, 1.0f) : 0.0f;
                                lsum += log_one_minus(a);
                            }
                            vis = -expm1f(lsum);
                        }
                    }
                    if constexpr (MODE == 1) {
                        const bool virt = g >= G.n - G.n_virtual;
                        if (!virt && n_train > 0.0f) {
                            float dx = m[0] - V.C[0], dy = m[1] - V.C[1], dz = m[2] - V.C[2];
                            const float nrm = sqrtf(dx * dx + dy * dy + dz * dz);
                            if (nrm > 0.0f) {
                                const float inv = 1.0f / nrm;
                                dx *= inv; dy *= inv; dz *= inv;
                                float Y[K];
                                sh_eval<L>(dx, dy, dz, Y);
                                float vt = 0.0f;
#pragma unroll
                                for (int kk = 0; kk < K; ++kk) vt = fmaf(sgG[w][q][kk], Y[kk], vt);
                                vt = fminf(fmaxf(vt, 0.0f), n_train);
                                vis = (vt >= n_train) ? 1.0f : 1.0f - expf(n_train * log1pf(-vt / n_train));
                            }
                        }
                    }
                    R.v = vis;
                    if constexpr (MODE != 0 && EXTRA) {
                        if (cvar) {
                            float cc = c3;
                            float dx = m[0] - V.C[0], dy = m[1] - V.C[1], dz = m[2] - V.C[2];
                            const float nrm = sqrtf(dx * dx + dy * dy + dz * dz);
                            if (nrm > 0.0f) {
                                const float inv = 1.0f / nrm;
                                float Y[16];
                                sh_eval<3>(dx * inv, dy * inv, dz * inv, Y);
                                const int Kc = (Lc + 1) * (Lc + 1);
                                float h = 0.0f;
#pragma unroll
                                for (int k = 0; k < 3; ++k) {
                                    float Q = 0.0f;
#pragma unroll
                                    for (int j = 0; j < 16; ++j)
                                        if (j < Kc) Q = fmaf(Y[j] * Y[j], cvar[(int64_t)(k * Kc + j) * G.n + g], Q);
                                    h += logf(fmaxf(Q, 1e-30f));
                                }
                                cc = fmaf(0.5f, h, c3);
                            }
                            rcc[r] = cc;
                        }
                        if (rz) rz[r] = (float)Pj.z;
                    }
                    rec[r] = R;
                    key[r] = __float_as_uint((float)Pj.z);
                    b.tile0 = (uint32_t)(V.tile_base + Pj.y0 * V.tiles_x + Pj.x0);
                    b.dims = (uint32_t)V.tiles_x | (uint32_t)(Pj.x1 - Pj.x0 - 1) << 11 |
                             (uint32_t)(Pj.y1 - Pj.y0 - 1) << 21 | 1u << 31;
                    // the anchor is at least one pixel left of / above the first
                    // tile only when that tile is the first of the image row, so
                    // the offsets fit int16
                    b.uvr = (int32_t)(((uint32_t)((int)ax - TILE * Pj.x0) & 0xFFFFu) |
                                      ((uint32_t)((int)ay - TILE * Pj.y0) << 16));
                    b.fx = R.fx;
                    b.fy = R.fy;
                    b.l11 = R.l11;
                    b.l21 = R.l21;
                    b.l22 = R.l22;
                    bin[r] = b;
                    if (ntr) {
                        const uint32_t nt = bin_ntiles(b.dims);
                        ntr[r] = pack ? r | (min(nt, PACK_SAT) << PACK_SHIFT) : nt;
                    }
                }
            }
            started += (uint32_t)__popcll(P);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- device exclusive scan

// Three phases over up to n = min(*n_dev or n_host, cap) uint32 values:
// block sums, a single-block scan of the block sums (64-bit totals), and the
// per-block scan.  out[n] receives the total (wrapped to 32 bits); the
// 64-bit total goes to *total and min(total, tcap) to *eff; a total above
// tcap sets `flag_bit` in *overflow.  Scans of at most SCAN_OWN_BLOCKS blocks
// (8M values) skip the middle phase: each block of the last one adds up the
// sums of the blocks before it (at most 16 KiB of reads), one launch fewer.
constexpr int SCAN_OWN_BLOCKS = 2048;

__device__ __forceinline__ uint64_t scan_n(const uint32_t *n_dev, uint64_t n_host) {
    return n_dev ? (uint64_t)(*n_dev) : n_host;
}

__global__ __launch_bounds__(WG) void k_scan_reduce(const uint32_t *__restrict__ in, const uint32_t *n_dev,
                                                    uint64_t n_host, unsigned long long *__restrict__ blk) {
    const uint64_t n = scan_n(n_dev, n_host);
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK;
    if (base >= n) {
        if (threadIdx.x == 0) blk[blockIdx.x] = 0ull;
        return;
    }
    unsigned long long s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const uint64_t i = base + (uint64_t)k * WG + threadIdx.x;
        if (i < n) s += in[i];
    }
    __shared__ unsigned long long red[WAVES];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < WAVES; ++w) t += red[w];
        blk[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_blocks(unsigned long long *__restrict__ blk, const uint32_t *n_dev,
                                                      uint64_t n_host, unsigned long long *total, uint32_t *eff,
                                                      uint64_t tcap, uint32_t *overflow, uint32_t flag_bit) {
    const uint64_t n = scan_n(n_dev, n_host);
    const uint64_t nb = n / SCAN_BLOCK + 1;   // includes the block that holds out[n]
    __shared__ unsigned long long buf[1024];
    __shared__ unsigned long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t s = 0; s < nb; s += 1024) {
        const uint64_t i = s + threadIdx.x;
        const unsigned long long x = i < nb ? blk[i] : 0ull;
        buf[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const unsigned long long y = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0ull;
            __syncthreads();
            buf[threadIdx.x] += y;
            __syncthreads();
        }
        if (i < nb) blk[i] = carry + buf[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long t = carry;
        if (total) *total = t;
        if (eff) *eff = (uint32_t)(t < tcap ? t : tcap);
        if (t > tcap && overflow) atomicOr(overflow, flag_bit);
    }
}

// Slot of element i of a scan block in LDS: one pad word per 32, so that a
// thread reading its SCAN_ITEMS consecutive elements and a wave reading 64
// consecutive ones both spread over the banks.
__device__ __forceinline__ int scan_slot(int i) { return i + (i >> 5); }

// OWN: the block adds up the sums of the blocks before it itself (a scan of
// at most SCAN_OWN_BLOCKS blocks, so that k_scan_blocks is not launched), and
// the block that holds out[n] writes the totals and the overflow flag as
// k_scan_blocks does; otherwise blk[b] already holds the prefix of block b.
template <bool OWN>
__global__ __launch_bounds__(WG) void k_scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                  const uint32_t *n_dev, uint64_t n_host,
                                                  const unsigned long long *__restrict__ blk,
                                                  unsigned long long *total, uint32_t *eff, uint64_t tcap,
                                                  uint32_t *overflow, uint32_t flag_bit) {
    const uint64_t n = scan_n(n_dev, n_host);
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_BLOCK;
    if (base > n) return;
    __shared__ uint32_t tile[SCAN_BLOCK + SCAN_BLOCK / 32];
    __shared__ unsigned long long wsum[WAVES];
    __shared__ unsigned long long wpre[WAVES];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    unsigned long long pre = 0;
    if constexpr (OWN) {
#pragma unroll
        for (int k = 0; k < SCAN_OWN_BLOCKS / WG; ++k) {
            const uint32_t b = (uint32_t)(k * WG + t);
            pre += b < blockIdx.x ? blk[b] : 0ull;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) pre += __shfl_xor(pre, off);
        if (lane == 0) wpre[w] = pre;
    }
    // the block's elements, read with consecutive lanes on consecutive
    // elements (zero past n)
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int i = k * WG + t;
        const uint64_t e = base + (uint64_t)i;
        tile[scan_slot(i)] = e < n ? in[e] : 0u;
    }
    __syncthreads();
    // each thread owns SCAN_ITEMS consecutive elements
    uint32_t v[SCAN_ITEMS];
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = tile[scan_slot(t * SCAN_ITEMS + k)];
        s += v[k];
    }
    // exclusive scan of the threads' sums: within the wave, then over waves
    unsigned long long inc = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if constexpr (OWN) {
        pre = 0;
#pragma unroll
        for (int q = 0; q < WAVES; ++q) pre += wpre[q];
    } else {
        pre = blk[blockIdx.x];
    }
    unsigned long long run = pre + inc - s;
#pragma unroll
    for (int q = 0; q < WAVES; ++q) run += q < w ? wsum[q] : 0ull;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        tile[scan_slot(t * SCAN_ITEMS + k)] = (uint32_t)run;
        run += v[k];
    }
    if constexpr (OWN) {
        // the last thread of the block holding out[n] ends at the total
        // (elements past n are zero)
        if (t == WG - 1 && n < base + SCAN_BLOCK) {
            if (total) *total = run;
            if (eff) *eff = (uint32_t)(run < tcap ? run : tcap);
            if (run > tcap && overflow) atomicOr(overflow, flag_bit);
        }
    }
    __syncthreads();
    // out[e] for e <= n (out[n]: the total), consecutive lanes again
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int i = k * WG + t;
        const uint64_t e = base + (uint64_t)i;
        if (e <= n) out[e] = tile[scan_slot(i)];
    }
}

// ---------------------------------------------------------------- LSD radix sort

// Each pass sorts (key, value) pairs stably by one digit of up to 8 bits.
// The n pairs are cut into one contiguous chunk of whole tiles per block (the
// grid is sized from the capacity so that a block gets about one tile)
// (RTILE = 4096 pairs).  Block b histograms its chunk; the histograms are
// scanned digit-major; block b then walks its chunk tile by tile.  In a tile,
// wave w owns pairs [w * 1024, (w + 1) * 1024) and loads all sixteen of its
// keys per lane up front; it ranks equal digits with ballot matching, sub-round by
// sub-round, against wave-private LDS counters (no barrier).  One block-wide
// step turns the four waves' counts into slots of the tile sorted by digit;
// the tile is staged in LDS in that order and written out so that
// consecutive lanes store consecutive positions of each digit's run.
constexpr int RITEMS = 16;
constexpr int RTILE = WG * RITEMS;
constexpr int RWAVE = 64 * RITEMS;

__device__ __forceinline__ void radix_chunk(uint64_t n, uint64_t &start, uint64_t &end) {
    uint64_t ch = (n + gridDim.x - 1) / gridDim.x;
    ch = (ch + RTILE - 1) / RTILE * RTILE;
    if (ch == 0) ch = RTILE;
    start = (uint64_t)blockIdx.x * ch;
    end = start + ch;
    if (end > n) end = n;
    if (start > n) start = n;
}

// drop: keys whose tile field (key & TILE_KEY_MASK) equals it are left out of
// the pass (DEAD_KEY: none); their count does not enter the histogram.
__global__ __launch_bounds__(WG) void k_radix_hist(const uint32_t *__restrict__ keys, const uint32_t *n_dev,
                                                   int shift, int nbits, uint32_t drop, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[WAVES][RADIX];
    const int t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int q = 0; q < WAVES; ++q) h[q][t] = 0;
    __syncthreads();
    uint64_t start, end;
    radix_chunk(*n_dev, start, end);
    const uint32_t mask = (1u << nbits) - 1u;
    for (uint64_t s = start; s < end; s += RTILE) {
        uint32_t k[RITEMS];
#pragma unroll
        for (int i = 0; i < RITEMS; ++i) {
            const uint64_t e = s + (uint64_t)i * WG + t;
            k[i] = e < end ? keys[e] : 0u;
        }
        // runs of equal digits among a thread's items are counted before
        // one atomic each: where most keys share a digit (the high digit of
        // depths, the view bits of tile ids) this avoids 64-way conflicts
        // on one LDS counter per item
        uint32_t dprev = 0, run = 0;
#pragma unroll
        for (int i = 0; i < RITEMS; ++i) {
            const uint64_t e = s + (uint64_t)i * WG + t;
            if (e < end && (k[i] & TILE_KEY_MASK) != drop) {
                const uint32_t d = (k[i] >> shift) & mask;
                if (run != 0 && d != dprev) {
                    atomicAdd(&h[w][dprev], run);
                    run = 0;
                }
                dprev = d;
                ++run;
            }
        }
        if (run != 0) atomicAdd(&h[w][dprev], run);
    }
    __syncthreads();
    hist[(size_t)t * gridDim.x + blockIdx.x] = h[0][t] + h[1][t] + h[2][t] + h[3][t];
}

// Exclusive prefix sum over the block's 256 threads (one value each).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *wtot) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    uint32_t base = 0;
#pragma unroll
    for (int ww = 0; ww < WAVES; ++ww) base += ww < w ? wtot[ww] : 0u;
    return base + inc - x;
}

// One block per digit: exclusive scan of that digit's nblk counts (one per
// block of the histogram pass, nblk <= RADIX_BLOCKS), read and written with
// consecutive lanes on consecutive counts; in LDS each thread scans
// RADIX_BLOCKS / WG consecutive counts after one block-wide scan of the
// threads' sums.  dtot[digit] receives the digit's total.
__global__ __launch_bounds__(WG) void k_radix_scan(uint32_t *__restrict__ hist, uint32_t *__restrict__ dtot,
                                                   int nblk) {
    constexpr int PER = RADIX_BLOCKS / WG;
    __shared__ uint32_t tile[RADIX_BLOCKS + RADIX_BLOCKS / 32];
    __shared__ uint32_t wtot[WAVES];
    uint32_t *row = hist + (size_t)blockIdx.x * nblk;
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = k * WG + t;
        tile[scan_slot(i)] = i < nblk ? row[i] : 0u;
    }
    __syncthreads();
    uint32_t v[PER], s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = tile[scan_slot(t * PER + k)];
        s += v[k];
    }
    // a thread rewrites only its own slots, which no other thread reads
    // before the barrier below
    uint32_t run = block_excl_scan(s, wtot);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        tile[scan_slot(t * PER + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = k * WG + t;
        if (i < nblk) row[i] = tile[scan_slot(i)];
    }
    if (t == WG - 1) dtot[blockIdx.x] = run;
}

// kout NULL: only the values are written (the last pass of a sort whose
// sorted keys are not needed).
// With drop (see k_radix_hist) the kept pairs are written compacted and their
// total goes to *n_kept (by one thread of block 0), the count the following
// passes take.  With gdst and gbin set, gdst[o] is the tile count a packed
// value carries (see PACK_SHIFT; a saturated one from gbin[record]); with
// gdst alone, gdst[o] = gsrc[value]; either is also written for
// every output position o (a per-value word gathered into sorted order).
__global__ __launch_bounds__(WG) void k_radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                      uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                      const uint32_t *n_dev, int shift, int nbits, uint32_t drop,
                                                      const uint32_t *__restrict__ hist,
                                                      const uint32_t *__restrict__ dtot,
                                                      uint32_t *__restrict__ n_kept,
                                                      const uint32_t *__restrict__ gsrc, uint32_t *__restrict__ gdst,
                                                      const Bin *__restrict__ gbin) {
    __shared__ uint32_t run[RADIX];          // output position of this block's next pair of each digit
    __shared__ uint32_t wcnt[WAVES][RADIX];  // wave counts, then wave offsets inside the digit
    __shared__ uint32_t lbase[RADIX];        // first slot of each digit in the staged tile
    __shared__ uint32_t goff[RADIX];         // output position minus staged slot, per digit
    __shared__ uint32_t wtot[WAVES];
    __shared__ uint32_t skept;               // pairs staged in the current tile
    __shared__ uint32_t sk[RTILE], sv[RTILE];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    {   // digit bases: exclusive scan of the digit totals plus this block's offset
        const uint32_t d = dtot[t];
        const uint32_t ex = block_excl_scan(d, wtot);
        run[t] = ex + hist[(size_t)t * gridDim.x + blockIdx.x];
        if (n_kept && blockIdx.x == 0 && t == RADIX - 1) *n_kept = ex + d;
    }
    const uint64_t n = *n_dev;
    uint64_t start, end;
    radix_chunk(n, start, end);
    const uint32_t mask = (1u << nbits) - 1u;
    for (uint64_t s = start; s < end; s += RTILE) {
        const uint64_t base = s + (uint64_t)w * RWAVE + lane;
        uint32_t k[RITEMS], v[RITEMS], pos[RITEMS];
        bool keep[RITEMS];
#pragma unroll
        for (int i = 0; i < RITEMS; ++i) {
            const uint64_t e = base + (uint64_t)i * 64;
            k[i] = e < end ? kin[e] : 0u;
            v[i] = e < end ? (vin ? vin[e] : (uint32_t)e) : 0u;
            keep[i] = e < end && (k[i] & TILE_KEY_MASK) != drop;
        }
        // this wave's counters start the tile at zero (wave-private row)
#pragma unroll
        for (int q = 0; q < RADIX / 64; ++q) wcnt[w][q * 64 + lane] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int i = 0; i < RITEMS; ++i) {
            const bool valid = keep[i];
            const uint32_t d = (k[i] >> shift) & mask;
            unsigned long long peers = __builtin_amdgcn_ballot_w64(valid);
            for (int bb = 0; bb < nbits; ++bb) {
                const bool bit = (d >> bb) & 1u;
                const unsigned long long bal = __builtin_amdgcn_ballot_w64(bit);
                peers &= bit ? bal : ~bal;
            }
            const uint32_t rank = lanes_below(peers);
            const uint32_t before = wcnt[w][d];
            pos[i] = before + rank;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (valid && rank == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
        {   // digit t: wave offsets inside the digit, the digit's staged slot and output base
            uint32_t c[WAVES], tot = 0;
#pragma unroll
            for (int ww = 0; ww < WAVES; ++ww) {
                c[ww] = wcnt[ww][t];
                wcnt[ww][t] = tot;
                tot += c[ww];
            }
            const uint32_t lb = block_excl_scan(tot, wtot);
            lbase[t] = lb;
            goff[t] = run[t] - lb;
            run[t] += tot;
            if (t == RADIX - 1) skept = lb + tot;
        }
        __syncthreads();
        // stage the tile in digit order ...
#pragma unroll
        for (int i = 0; i < RITEMS; ++i) {
            if (keep[i]) {
                const uint32_t d = (k[i] >> shift) & mask;
                const uint32_t slot = lbase[d] + wcnt[w][d] + pos[i];
                sk[slot] = k[i];
                sv[slot] = v[i];
            }
        }
        __syncthreads();
        // ... and write it out: consecutive lanes write consecutive positions of a digit run
        const uint32_t cnt = skept;
        if (gdst) {
            for (uint32_t j = t; j < cnt; j += WG) {
                const uint32_t key = sk[j], val = sv[j];
                const uint32_t o = goff[(key >> shift) & mask] + j;
                if (kout) kout[o] = key;
                vout[o] = val;
                // the gathered index is a value's record index, below n in a
                // call that projected its records; a call whose records
                // overflowed skips the projection and sorts the workspace's
                // stale contents, so the index is checked before every read
                // (the call then reports the overflow and emits nothing)
                if (gbin) {   // packed values: the count they carry, or the binning line's
                    uint32_t c = val >> PACK_SHIFT;
                    const uint32_t rr = val & PACK_RMASK;
                    if (c == PACK_SAT) c = rr < n ? bin_ntiles(gbin[rr].dims) : 0u;
                    gdst[o] = c;
                } else {
                    gdst[o] = val < n ? gsrc[val] : 0u;
                }
            }
        } else if (!kout) {
            for (uint32_t j = t; j < cnt; j += WG) vout[goff[(sk[j] >> shift) & mask] + j] = sv[j];
        } else {
            for (uint32_t j = t; j < cnt; j += WG) {
                const uint32_t key = sk[j];
                const uint32_t o = goff[(key >> shift) & mask] + j;
                kout[o] = key;
                vout[o] = sv[j];
            }
        }
        // no barrier here: the next tile writes sk / sv / goff only after its
        // first block-wide barrier, which every thread reaches after this loop
    }
}

// ---------------------------------------------------------------- binning

// One (global tile id, record) instance per tile of every record, written in
// depth order so that a stable sort by tile id keeps depth order in a tile.
// The key also carries the record's quadrant mask for the tile (which
// quadrants of the tile its ellipse reaches); an instance whose ellipse
// reaches none of them is given the tile id past the last tile.
//
// A wave takes a chunk of 64 depth-ordered records and writes their instances
// as one contiguous range, lane j writing output J + j, in two levels.  The
// records' tile rows are taken 64 at a time: lane j computes row R0 + j's
// band extents (the part of the quadrant test that depends on the row only,
// done once per row instead of once per tile), its first output and its
// first tile id, kept in LDS.  Then the outputs of those 64 rows are written
// 64 at a time; each needs only its row's extents, its column and the
// comparisons.  At both levels the owner of a row or an output is found
// without a search: the owners starting inside the chunk mark their first
// position in LDS, and a ballot over the marks gives every lane the number of
// owners started up to its position (for rows, the compacted list of records
// that own tiles turns that count into a lane).  Two kernels differ only in
// where a chunk's output offsets come from: a scan of the records' tile
// counts done before (k_emit_scanned), or the kernel's own single-pass scan
// (k_emit).
struct EmitLds {
    float4 sgA[WAVES][64];      // band-test constants of each record: fx, fy, kx, 1 / a
    float4 sgB[WAVES][64];      // c, ey of the rightmost point, half height, anchor (bits)
    uint2 sgC[WAVES][64];       // first tile, rectangle dims
    float4 rwE[WAVES][64];      // rows of the current 64: band extents (band_extents)
    uint4 rwI[WAVES][64];       // rows: first output, first tile id, record index, anchor x (float bits)
    uint8_t cl[WAVES][64];      // lanes of the records that own at least one tile, in order
    uint8_t mk[WAVES][64];      // 1 where a row / an output owner starts at that position
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// This lane's record r (binning line B, nt tiles, first output rel after the
// chunk's first output cbase); outputs at or past icap are not written.
__device__ __forceinline__ void emit_chunk(EmitLds &S, int w, int lane, uint32_t r, const Bin &B, uint32_t nt,
                                           uint32_t rel, unsigned long long cbase, unsigned long long icap, float qc,
                                           float sq, uint32_t dead_tile, uint32_t *__restrict__ ikey,
                                           uint32_t *__restrict__ ival) {
    const bool owns = nt > 0;
    const unsigned long long own = __builtin_amdgcn_ballot_w64(owns);
    if (owns) S.cl[w][lanes_below(own)] = (uint8_t)lane;
    // the records' tile rows, numbered in record order
    const uint32_t wy = owns ? bin_wy(B.dims) : 0u;
    uint32_t rinc = wy;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(rinc, off);
        if (lane >= off) rinc += y;
    }
    const uint32_t rrel = rinc - wy;
    const uint32_t rtot = __shfl(rinc, 63);
    if (owns) {
        const EllipseBands E = ellipse_bands(B.l11, B.l21, B.l22, sq);
        S.sgA[w][lane] = make_float4(B.fx, B.fy, E.kx, E.ia);
        S.sgB[w][lane] = make_float4(B.l22, E.eyR, E.hy, __int_as_float(B.uvr));
        S.sgC[w][lane] = make_uint2(B.tile0, B.dims);
    }
    uint32_t rstarted = 0;   // records (owning tiles) whose rows start before the row chunk
    for (uint32_t R0 = 0; R0 < rtot; R0 += 64) {
        // row R0 + lane: its record, band extents, first output and first tile
        S.mk[w][lane] = 0;
        wave_sync();
        if (owns && rrel >= R0 && rrel < R0 + 64) S.mk[w][rrel - R0] = 1;
        wave_sync();
        const unsigned long long PR = __builtin_amdgcn_ballot_w64(S.mk[w][lane] != 0);
        const uint32_t ri = R0 + lane;
        const bool rv = ri < rtot;
        // the row's record: its lane q; its index, first output and first row
        // come from that lane's registers (every lane takes part in the shuffles)
        const int q = rv ? (int)S.cl[w][rstarted + lanes_below(PR) + (uint32_t)((PR >> lane) & 1ull) - 1] : 0;
        const uint32_t q_r = __shfl(r, q), q_rel = __shfl(rel, q), q_row = __shfl(rrel, q);
        float4 ext = make_float4(0.f, 0.f, 0.f, 0.f);
        uint4 rinfo = make_uint4(0u, 0u, 0u, 0u);
        uint32_t rend = 0;   // first output past the row
        if (rv) {
            const uint32_t ty = ri - q_row;
            const float4 A = S.sgA[w][q], Bq = S.sgB[w][q];
            const uint2 C = S.sgC[w][q];
            const uint32_t wx = bin_wx(C.y);
            const int uvr = __float_as_int(Bq.w);
            const float uy = (float)((uvr >> 16) - (int)ty * TILE) + A.y;
            ext = band_extents(uy, A.z, A.w, Bq.x, Bq.y, Bq.z, qc);
            const uint32_t first = q_rel + ty * wx;
            rinfo = make_uint4(first, C.x + ty * bin_tiles_x(C.y), q_r,
                               __float_as_uint((float)(int)(int16_t)(uvr & 0xFFFF) + A.x));
            rend = first + wx;
        }
        rstarted += (uint32_t)__popcll(PR);
        S.rwE[w][lane] = ext;
        S.rwI[w][lane] = rinfo;
        // the rows' outputs: [first output of row R0, end of the chunk's last row)
        const uint32_t nr = min(rtot - R0, 64u);
        const uint32_t o_first = __shfl(rinfo.x, 0);
        const uint32_t o_end = __shfl(rend, (int)nr - 1);
        uint32_t started = 0;   // rows of this chunk that start before the output chunk
        for (uint32_t J = o_first; J < o_end; J += 64) {
            wave_sync();
            S.mk[w][lane] = 0;
            wave_sync();
            if (rv && rinfo.x >= J && rinfo.x < J + 64) S.mk[w][rinfo.x - J] = 1;
            wave_sync();
            const unsigned long long P = __builtin_amdgcn_ballot_w64(S.mk[w][lane] != 0);
            const uint32_t jo = J + lane;
            const unsigned long long o = cbase + jo;
            if (jo < o_end && o < icap) {
                const int row = (int)(started + lanes_below(P) + (uint32_t)((P >> lane) & 1ull)) - 1;
                const uint4 I = S.rwI[w][row];
                const float4 X = S.rwE[w][row];
                const uint32_t rem = jo - I.x;
                const float ux = __uint_as_float(I.w) - (float)(int)(rem * TILE);
                const uint32_t qm = quadrant_mask_ext(ux, X);
                const uint32_t tile = qm ? I.y + rem : dead_tile;
                ikey[o] = tile | (qm << QMASK_SHIFT);
                ival[o] = I.z;
            }
            started += (uint32_t)__popcll(P);
        }
        wave_sync();
    }
    wave_sync();
}

// Offsets from a scan done before (ioff[i]: first output of depth-ordered
// record i; the scan has set the instance totals and the overflow flag, and
// nothing is emitted on overflow).  Waves take chunks of 64 records in turn.
// rmask: the record index bits of the values (PACK_RMASK for packed values).
__global__ __launch_bounds__(WG) void k_emit_scanned(const uint32_t *__restrict__ sval, const Bin *__restrict__ bin,
                                                     const uint32_t *__restrict__ ioff,
                                                     const Status *__restrict__ st, float qcut, uint32_t dead_tile,
                                                     uint32_t *__restrict__ ikey, uint32_t *__restrict__ ival,
                                                     uint32_t rmask) {
    __shared__ EmitLds S;
    if (st->overflow) return;
    const uint64_t n = st->R_eff;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t nwaves = (uint64_t)gridDim.x * WAVES;
    const float qc = band_threshold(qcut), sq = sqrtf(qc);
    for (uint64_t c = (uint64_t)blockIdx.x * WAVES + w; c * 64 < n; c += nwaves) {
        const uint64_t i = c * 64 + lane;
        uint32_t r = 0, o = 0, nt = 0;
        Bin B = {};
        if (i < n) {
            r = sval[i] & rmask;
            B = bin[r];
            o = ioff[i];
            nt = bin_ntiles(B.dims);
        }
        const uint32_t o0 = __builtin_amdgcn_readfirstlane(o);
        emit_chunk(S, w, lane, r, B, nt, o - o0, o0, ~0ull, qc, sq, dead_tile, ikey, ival);
    }
}

// Offsets found by the kernel itself.  A block starts by taking a ticket (the
// order in which blocks begin) and with it the next EMIT_RPB records in depth
// order; it reads their binning lines, sums their tile counts, posts that sum
// and then the sum of all earlier blocks, which it learns by looking back
// over what the blocks with smaller tickets posted: a single-pass scan with
// decoupled look-back (Merrill and Garland, "Single-pass parallel prefix scan
// with decoupled look-back", NVIDIA technical report NVR-2016-002).  A block
// with a smaller ticket started earlier, so it is running or done, and it
// posts its own sum before it waits for anything: every wait ends.
// Post words: bits 62-63 the kind (0 nothing yet, 1 the block's own sum,
// 2 the sum of it and every earlier block), bits 0-61 the value.  Within a
// block, wave w owns chunks 4w .. 4w + 3.  The block holding the last record
// sets the instance totals and the overflow flag; outputs past the capacity
// are not written.
constexpr int EMIT_CHUNKS = 4;                       // chunks of 64 records per wave
constexpr int EMIT_RPB = WG * EMIT_CHUNKS;           // records per block
constexpr unsigned long long LB_AGG = 1ull << 62, LB_INCL = 2ull << 62, LB_VALUE = (1ull << 62) - 1ull;

// A post word carries everything its reader needs (kind and value in one
// 64-bit atomic), and nothing else is published through it, so the posts
// and reads are relaxed atomics at device scope: coherent across the XCDs'
// L2 caches without the L2 write-back / invalidate that release and acquire
// ordering would add to every post and every read of the spin.
__device__ __forceinline__ void lb_post(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long lb_read(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(WG) void k_emit(const uint32_t *__restrict__ sval, const Bin *__restrict__ bin,
                                             unsigned long long *__restrict__ lb, Status *__restrict__ st,
                                             uint64_t icap, float qcut, uint32_t dead_tile,
                                             uint32_t *__restrict__ ikey, uint32_t *__restrict__ ival) {
    __shared__ EmitLds S;
    __shared__ uint32_t wsum[WAVES];       // tile counts of each wave's records
    __shared__ uint32_t sticket;
    __shared__ unsigned long long sbase;   // instances of all earlier blocks
    if (st->overflow) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) sticket = atomicAdd(&st->emit_ticket, 1u);
    __syncthreads();
    const uint32_t blk = sticket;
    const uint64_t n = st->R_eff;
    const uint64_t first = (uint64_t)blk * EMIT_RPB;
    if (first >= n) return;                // the whole block: no record left for this ticket
    // this lane's records, their binning lines and tile counts
    uint32_t r[EMIT_CHUNKS], nt[EMIT_CHUNKS], pre[EMIT_CHUNKS];
    Bin B[EMIT_CHUNKS];
    uint32_t wtot = 0;
#pragma unroll
    for (int j = 0; j < EMIT_CHUNKS; ++j) {
        const uint64_t i = first + (uint64_t)(w * EMIT_CHUNKS + j) * 64 + lane;
        r[j] = 0;
        nt[j] = 0;
        B[j] = Bin{};
        if (i < n) {
            r[j] = sval[i];
            B[j] = bin[r[j]];
            nt[j] = bin_ntiles(B[j].dims);
        }
        // inclusive scan over the wave's lanes, then exclusive with the
        // chunk's offset inside the wave
        uint32_t inc = nt[j];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off);
            if (lane >= off) inc += y;
        }
        pre[j] = wtot + inc - nt[j];
        wtot += __shfl(inc, 63);
    }
    if (lane == 0) wsum[w] = wtot;
    __syncthreads();
    uint32_t wbase = 0, btot = 0;
#pragma unroll
    for (int q = 0; q < WAVES; ++q) {
        wbase += q < w ? wsum[q] : 0u;
        btot += wsum[q];
    }
    // post this block's sum; learn the sum of all earlier blocks
    if (w == 0) {
        if (blk == 0) {
            if (lane == 0) {
                lb_post(&lb[0], LB_INCL | (unsigned long long)btot);
                sbase = 0;
            }
        } else {
            if (lane == 0) lb_post(&lb[blk], LB_AGG | (unsigned long long)btot);
            unsigned long long acc = 0;
            int64_t j = (int64_t)blk - 1;      // the newest earlier block not yet added
            while (true) {
                const int64_t jj = j - lane;
                unsigned long long word = jj >= 0 ? lb_read(&lb[jj]) : LB_INCL;
                const unsigned long long incl = __builtin_amdgcn_ballot_w64((word >> 62) == 2ull);
                const unsigned long long empty = __builtin_amdgcn_ballot_w64((word >> 62) == 0ull);
                // lanes up to the first inclusive one (all lanes if none)
                const int stop = incl ? __builtin_ctzll(incl) : 63;
                const unsigned long long need = stop == 63 ? ~0ull : ((2ull << stop) - 1ull);
                if (empty & need) continue;    // an earlier block has not posted yet: read again
                unsigned long long v = lane <= stop ? (word & LB_VALUE) : 0ull;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                acc += v;
                if (incl) break;
                j -= 64;
            }
            if (lane == 0) {
                lb_post(&lb[blk], LB_INCL | ((acc + btot) & LB_VALUE));
                sbase = acc;
            }
        }
    }
    __syncthreads();
    const unsigned long long base = sbase;
    if (threadIdx.x == 0 && first + EMIT_RPB >= n) {   // the block holding the last record: the totals
        const unsigned long long tot = base + btot;
        st->M_total = tot;
        st->M_eff = (uint32_t)(tot < icap ? tot : icap);
        if (tot > icap) st->overflow |= 2u;
    }
    const float qc = band_threshold(qcut), sq = sqrtf(qc);
#pragma unroll
    for (int j = 0; j < EMIT_CHUNKS; ++j) {
        const uint32_t p0 = __shfl(pre[j], 0);
        emit_chunk(S, w, lane, r[j], B[j], nt[j], pre[j] - p0, base + wbase + p0, icap, qc, sq, dead_tile, ikey,
                   ival);
    }
}

// [start, end) of every tile's run in the sorted instance list (instances
// past the last tile are dead and belong to no run).
__global__ __launch_bounds__(WG) void k_ranges(const uint32_t *__restrict__ key, const Status *__restrict__ st,
                                               uint32_t dead_tile, uint2 *__restrict__ ranges) {
    if (st->overflow) return;
    const uint64_t n = st->M_live;
    // four consecutive keys per thread (one 16-byte load where aligned and
    // complete) and the key before them; run ends are found against the next
    // key, which is the first of the following thread's four
    for (uint64_t i0 = ((uint64_t)blockIdx.x * WG + threadIdx.x) * 4; i0 < n; i0 += (uint64_t)gridDim.x * WG * 4) {
        uint32_t k[6];
        k[0] = i0 > 0 ? key[i0 - 1] & TILE_KEY_MASK : 0xFFFFFFFFu;
        if (i0 + 4 <= n) {
            const uint4 v = *reinterpret_cast<const uint4 *>(key + i0);
            k[1] = v.x & TILE_KEY_MASK; k[2] = v.y & TILE_KEY_MASK; k[3] = v.z & TILE_KEY_MASK; k[4] = v.w & TILE_KEY_MASK;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) k[1 + j] = i0 + j < n ? key[i0 + j] & TILE_KEY_MASK : 0xFFFFFFFFu;
        }
        k[5] = i0 + 4 < n ? key[i0 + 4] & TILE_KEY_MASK : 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t i = i0 + j;
            const uint32_t kk = k[1 + j];
            if (i >= n || kk >= dead_tile) continue;
            if (k[j] != kk) ranges[kk].x = (uint32_t)i;
            if (k[2 + j] != kk) ranges[kk].y = (uint32_t)(i + 1);
        }
    }
}

// Sort keys of the cost-ordered tile schedule: tile t's list length, capped
// at 2^16 - 1 and complemented in 16 bits so that an ascending two-pass sort
// puts the longest first (lists past the cap, rare, keep tile order among
// themselves); values the tile ids; *count = T for the sort.
constexpr int TILE_COST_BITS = 16;
__global__ __launch_bounds__(WG) void k_tile_cost(const uint2 *__restrict__ ranges, uint32_t T,
                                                  uint32_t *__restrict__ key, uint32_t *__restrict__ val,
                                                  uint32_t *__restrict__ count) {
    const uint32_t t = blockIdx.x * WG + threadIdx.x;
    if (t == 0) *count = T;
    if (t >= T) return;
    const uint2 r = ranges[t];
    constexpr uint32_t cap = (1u << TILE_COST_BITS) - 1u;
    key[t] = cap - min(r.y - r.x, cap);
    val[t] = t;
}

// ---------------------------------------------------------------- host launchers

static inline unsigned grid_for(uint64_t n, unsigned cap = 65535u * 4u) {
    uint64_t g = (n + WG - 1) / WG;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 4096)), dim3(WG), 0, s, p, n, value);
}

template <typename TG>
static GaussIn<TG> gin(const GaussArgs &a) {
    GaussIn<TG> G;
    G.means = (const TG *)a.means;
    G.scales = (const TG *)a.scales;
    G.quats = (const TG *)a.quats;
    G.opac = (const TG *)a.opacity;
    G.anchors = a.anchors;
    G.anchor_block = a.anchor_block > 0 ? a.anchor_block : 1;
    G.n = a.n;
    G.n_virtual = a.n_virtual;
    return G;
}

int mask_words(int nv) {
    const int per = (nv + PROJ_SPLIT - 1) / PROJ_SPLIT;
    return per > 32 ? (per + 31) / 32 : 1;
}

void launch_count(const GaussArgs &a, const ViewDev *views, int nv, const GeomArgs &p, uint32_t *cnt,
                  uint32_t *vmask, uint32_t *clr0, uint32_t n0, uint32_t *clr1, uint64_t n1, hipStream_t s) {
    static_assert(PROJ_SPLIT == WAVES, "one view subset per wave");
    const unsigned grid = (unsigned)((a.n + 63) / 64);
    if (grid == 0) {   // no Gaussian: the fills alone
        launch_fill_u32(clr0, n0, 0u, s);
        launch_fill_u32(clr1, n1, 0u, s);
        return;
    }
    const int mw = mask_words(nv);
    switch (a.dtype) {
    case 0: hipLaunchKernelGGL(k_count<float>, dim3(grid), dim3(WG), 0, s, gin<float>(a), views, nv, p.znear, p.lowpass, p.cut, cnt, vmask, mw, clr0, n0, clr1, n1); break;
    case 1: hipLaunchKernelGGL(k_count<_Float16>, dim3(grid), dim3(WG), 0, s, gin<_Float16>(a), views, nv, p.znear, p.lowpass, p.cut, cnt, vmask, mw, clr0, n0, clr1, n1); break;
    default: hipLaunchKernelGGL(k_count<uint16_t>, dim3(grid), dim3(WG), 0, s, gin<uint16_t>(a), views, nv, p.znear, p.lowpass, p.cut, cnt, vmask, mw, clr0, n0, clr1, n1); break;
    }
}

void launch_measure(const GaussArgs &a, const ViewDev *views, int nv, const GeomArgs &p, unsigned long long *out,
                    hipStream_t s) {
    const unsigned grid = (unsigned)((a.n * PROJ_SPLIT + WG - 1) / WG);
    if (grid == 0) return;
    switch (a.dtype) {
    case 0: hipLaunchKernelGGL(k_measure<float>, dim3(grid), dim3(WG), 0, s, gin<float>(a), views, nv, p.znear, p.lowpass, p.cut, out); break;
    case 1: hipLaunchKernelGGL(k_measure<_Float16>, dim3(grid), dim3(WG), 0, s, gin<_Float16>(a), views, nv, p.znear, p.lowpass, p.cut, out); break;
    default: hipLaunchKernelGGL(k_measure<uint16_t>, dim3(grid), dim3(WG), 0, s, gin<uint16_t>(a), views, nv, p.znear, p.lowpass, p.cut, out); break;
    }
}

template <typename TG, typename TGam, int MODE>
static void project_dispatch_L(int L, const GaussArgs &a, const ViewDev *views, int nv, const GeomArgs &p,
                               const uint32_t *offs, const uint32_t *vmask, const Status *st, uint32_t rcap,
                               const QueryArgs &q, Rec *rec, uint32_t *key, Bin *bin, uint32_t *ntr, int pack,
                               uint32_t *zr0, uint32_t *zr1, hipStream_t s) {
    const uint64_t chunks = ((uint64_t)a.n * PROJ_SPLIT + 63) / 64;
    const unsigned grid = (unsigned)std::min<uint64_t>((chunks + WAVES - 1) / WAVES, 4096);
    const int mw = mask_words(nv);
    const TGam *gm = (const TGam *)q.gamma;
    const float kl = (float)(q.kappa * 1.4426950408889634);
#define GV_PROJECT_ARGS gin<TG>(a), views, nv, p.znear, p.lowpass, p.cut, offs, vmask, mw, st, rcap, gm, q.n_train, \
        q.view_vis, q.train_centres, q.n_train_views, kl, q.color_var, q.color_sh_degree, q.c3, q.rcc, q.rz, rec, key, bin, ntr, pack, zr0, zr1
    const bool extra = q.color_var || q.rz;
#define GV_PROJECT_LAUNCH(LL) \
    do { \
        if (extra) hipLaunchKernelGGL((k_project<TG, TGam, MODE, LL, true>), dim3(grid), dim3(WG), 0, s, GV_PROJECT_ARGS); \
        else hipLaunchKernelGGL((k_project<TG, TGam, MODE, LL, false>), dim3(grid), dim3(WG), 0, s, GV_PROJECT_ARGS); \
    } while (0)
    if constexpr (MODE == 0) {   // the build: no SH evaluation, no side outputs
        hipLaunchKernelGGL((k_project<TG, TGam, 0, 0, false>), dim3(grid), dim3(WG), 0, s, GV_PROJECT_ARGS);
    } else if constexpr (MODE == 2) {
        GV_PROJECT_LAUNCH(0);
    } else {
        switch (L) {
        case 0: GV_PROJECT_LAUNCH(0); break;
        case 1: GV_PROJECT_LAUNCH(1); break;
        case 2: GV_PROJECT_LAUNCH(2); break;
        default: GV_PROJECT_LAUNCH(3); break;
        }
    }
#undef GV_PROJECT_LAUNCH
#undef GV_PROJECT_ARGS
}

template <typename TG>
static void project_dispatch_gam(int L, const GaussArgs &a, const ViewDev *views, int nv, const GeomArgs &p,
                                 const uint32_t *offs, const uint32_t *vmask, const Status *st, uint32_t rcap,
                                 const QueryArgs *q, Rec *rec, uint32_t *key, Bin *bin, uint32_t *ntr, int pack,
                                 uint32_t *zr0, uint32_t *zr1, hipStream_t s) {
    if (!q) {
        const QueryArgs none = {0, 0, nullptr, 0, 0.f, nullptr, nullptr, 0, 0.f, nullptr, 0, 0.f, nullptr, nullptr};
        project_dispatch_L<TG, float, 0>(0, a, views, nv, p, offs, vmask, st, rcap, none, rec, key, bin, ntr, pack, zr0, zr1, s);
        return;
    }
    if (q->mode == 2) {
        project_dispatch_L<TG, float, 2>(0, a, views, nv, p, offs, vmask, st, rcap, *q, rec, key, bin, ntr, pack, zr0, zr1, s);
        return;
    }
    switch (q->gamma_dtype) {
    case 0: project_dispatch_L<TG, float, 1>(L, a, views, nv, p, offs, vmask, st, rcap, *q, rec, key, bin, ntr, pack, zr0, zr1, s); break;
    case 1: project_dispatch_L<TG, _Float16, 1>(L, a, views, nv, p, offs, vmask, st, rcap, *q, rec, key, bin, ntr, pack, zr0, zr1, s); break;
    default: project_dispatch_L<TG, uint16_t, 1>(L, a, views, nv, p, offs, vmask, st, rcap, *q, rec, key, bin, ntr, pack, zr0, zr1, s); break;
    }
}

void launch_project(const GaussArgs &a, const ViewDev *views, int nv, const GeomArgs &p, const uint32_t *offs,
                    const uint32_t *vmask, const Status *st, uint32_t rcap, const QueryArgs *q, Rec *rec,
                    uint32_t *key, Bin *bin, uint32_t *ntr, int pack, uint32_t *zr0, uint32_t *zr1,
                    hipStream_t s) {
    if (a.n == 0) return;
    const int L = q ? q->sh_degree : 0;
    switch (a.dtype) {
    case 0: project_dispatch_gam<float>(L, a, views, nv, p, offs, vmask, st, rcap, q, rec, key, bin, ntr, pack, zr0, zr1, s); break;
    case 1: project_dispatch_gam<_Float16>(L, a, views, nv, p, offs, vmask, st, rcap, q, rec, key, bin, ntr, pack, zr0, zr1, s); break;
    default: project_dispatch_gam<uint16_t>(L, a, views, nv, p, offs, vmask, st, rcap, q, rec, key, bin, ntr, pack, zr0, zr1, s); break;
    }
}

void launch_scan(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint64_t n_host, uint64_t n_cap,
                 unsigned long long *blk, unsigned long long *total, uint32_t *eff, uint64_t tcap,
                 uint32_t *overflow, uint32_t flag_bit, hipStream_t s) {
    const unsigned nb = (unsigned)((n_cap + SCAN_BLOCK) / SCAN_BLOCK);   // covers out[n] too
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(WG), 0, s, in, n_dev, n_host, blk);
    if (nb <= SCAN_OWN_BLOCKS) {
        hipLaunchKernelGGL(k_scan_down<true>, dim3(nb), dim3(WG), 0, s, in, out, n_dev, n_host, blk, total, eff, tcap,
                           overflow, flag_bit);
    } else {
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, blk, n_dev, n_host, total, eff, tcap, overflow,
                           flag_bit);
        hipLaunchKernelGGL(k_scan_down<false>, dim3(nb), dim3(WG), 0, s, in, out, n_dev, n_host, blk, nullptr,
                           nullptr, 0, nullptr, 0u);
    }
}

size_t scan_blk_count(uint64_t n_cap) { return (size_t)((n_cap + SCAN_BLOCK) / SCAN_BLOCK) + 1; }

// Sorts n = *n_dev pairs on key bits [0, bits).  Returns 0 if the result is
// in (k0, v0), 1 if it is in (k1, v1).  With iota set, the input values are
// the indices 0..n-1 and v0 is only used as a buffer.
int launch_radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const uint32_t *n_dev, int bits,
                      bool iota, uint32_t *hist, uint32_t *dtot, hipStream_t s, uint32_t drop, uint32_t *n_kept,
                      uint64_t n_cap, const uint32_t *gather_src, uint32_t *gather_dst, bool keys_out,
                      const Bin *gather_bin) {
    int cur = 0;
    // about one tile of pairs per block at the capacity: fewer, fuller blocks
    // than a fixed grid when the sort is short
    const int nblk = (int)std::min<uint64_t>(std::max<uint64_t>((n_cap + RTILE - 1) / RTILE, 256), RADIX_BLOCKS);
    const uint32_t *vin = iota ? nullptr : v0;
    // digits of equal width (at most RADIX_BITS): a narrow last digit would
    // pile the whole histogram onto a few counters
    const int passes = (bits + RADIX_BITS - 1) / RADIX_BITS;
    for (int p = 0, shift = 0; p < passes; ++p) {
        const int nb = (bits - shift + (passes - p) - 1) / (passes - p);
        uint32_t *ki = cur ? k1 : k0, *ko = cur ? k0 : k1;
        uint32_t *vo = cur ? v0 : v1;
        // the first pass drops the `drop` keys; later passes sort the kept ones
        const uint32_t dk = p == 0 ? drop : DEAD_KEY;
        uint32_t *kept = p == 0 && drop != DEAD_KEY ? n_kept : nullptr;
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(WG), 0, s, ki, n_dev, shift, nb, dk, hist);
        hipLaunchKernelGGL(k_radix_scan, dim3(RADIX), dim3(WG), 0, s, hist, dtot, nblk);
        const bool last = p == passes - 1;
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(WG), 0, s, ki, vin, last && !keys_out ? nullptr : ko, vo,
                           n_dev, shift, nb, dk,
                           hist, dtot, kept, last ? gather_src : nullptr, last ? gather_dst : nullptr,
                           last ? gather_bin : nullptr);
        if (kept) n_dev = kept;
        cur ^= 1;
        vin = cur ? v1 : v0;
        shift += nb;
    }
    return cur;
}


size_t emit_post_words(uint64_t rcap) { return (size_t)((rcap + EMIT_RPB - 1) / EMIT_RPB) + 1; }

void launch_emit_scanned(const uint32_t *sval, const Bin *bin, const uint32_t *ioff, const Status *st, float qcut,
                         uint32_t dead_tile, uint32_t *ikey, uint32_t *ival, uint32_t rmask, hipStream_t s) {
    hipLaunchKernelGGL(k_emit_scanned, dim3(8192), dim3(WG), 0, s, sval, bin, ioff, st, qcut, dead_tile, ikey, ival,
                       rmask);
}

void launch_emit(const uint32_t *sval, const Bin *bin, unsigned long long *lb, Status *st, uint64_t rcap,
                 uint64_t icap, float qcut, uint32_t dead_tile, uint32_t *ikey, uint32_t *ival, hipStream_t s) {
    // the post words start empty (a fill kernel, not a memset: the sequence
    // may be captured in a graph); st->emit_ticket was cleared with the status
    const size_t words = emit_post_words(rcap);
    launch_fill_u32(reinterpret_cast<uint32_t *>(lb), 2 * (uint64_t)words, 0u, s);
    hipLaunchKernelGGL(k_emit, dim3((unsigned)words), dim3(WG), 0, s, sval, bin, lb, st, icap, qcut, dead_tile,
                       ikey, ival);
}

const uint32_t *launch_tile_order(const uint2 *ranges, uint32_t T, uint32_t *buf, uint32_t *count, uint32_t *hist,
                                  uint32_t *dtot, hipStream_t s) {
    uint32_t *k0 = buf, *v0 = buf + T, *k1 = buf + 2 * (uint64_t)T, *v1 = buf + 3 * (uint64_t)T;
    hipLaunchKernelGGL(k_tile_cost, dim3((T + WG - 1) / WG), dim3(WG), 0, s, ranges, T, k0, v0, count);
    const int r = launch_radix_sort(k0, v0, k1, v1, count, TILE_COST_BITS, false, hist, dtot, s, DEAD_KEY, nullptr, T);
    return r ? v1 : v0;
}

void launch_ranges(const uint32_t *key, const Status *st, uint32_t dead_tile, uint2 *ranges, hipStream_t s) {
    hipLaunchKernelGGL(k_ranges, dim3(4096), dim3(WG), 0, s, key, st, dead_tile, ranges);
}

}  // namespace gv
