// gv_launch.hpp -- host-side launchers of the HIP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gv_device.hpp"

namespace gv {

struct GaussArgs {
    int64_t n;
    int64_t n_virtual;
    int dtype;               // 0 f32, 1 f16, 2 bf16
    const void *means, *scales, *quats, *opacity;
    const float *anchors;
    int32_t anchor_block;
};

struct GeomArgs {
    float znear, lowpass, cut;
};

// Per-pixel constants of the uncertainty rasterisation (Alg. 6).
struct UqArgs {
    float beta, o0;
    float cQc;       // 1/2 log|Q_c| + 3/2 log(2 pi e)
    float cQ0;       // 1/2 log|Q0| + 3/2 log(2 pi e)
    float eps_T;
    float qcut;      // log2(e) cut / 2, the overlap threshold on the scaled quadratic form
};

// Where the query takes a Gaussian's visibility in a candidate view from.
struct QueryArgs {
    int mode;                     // 1: SH field with the AM-GM bound (Alg. 4)
                                  // 2: exact product over the training views (eq. vis_all)
    int sh_degree;                // mode 1
    const void *gamma;            // mode 1: planar [K][n]
    int gamma_dtype;              // mode 1
    float n_train;                // |P|
    const float *view_vis;        // mode 2: v_p of every Gaussian, [n_train][n]
    const float *train_centres;   // mode 2: [n_train][3]
    int32_t n_train_views;        // mode 2
    float kappa;                  // mode 2
    // optional per-Gaussian colour covariance (both modes): variances of the
    // colour SH coefficients, planar [3][Kc][n], Kc = (color_sh_degree + 1)^2;
    // the projection writes c_c per record into rcc
    const float *color_var;
    int color_sh_degree;
    float c3;                     // 3/2 log(2 pi e)
    float *rcc;
    float *rz;                    // optional: the projection writes each record's depth here
};

void launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s);

// Words of the per-(Gaussian, view subset) visibility mask for nv views.
int mask_words(int nv);
// Also zeroes n0 words at clr0 and n1 words at clr1 (one launch for all).
void launch_count(const GaussArgs &a, const ViewDev *views, int nv, const GeomArgs &p, uint32_t *cnt, uint32_t *vmask,
                  uint32_t *clr0, uint32_t n0, uint32_t *clr1, uint64_t n1, hipStream_t s);
void launch_measure(const GaussArgs &a, const ViewDev *views, int nv, const GeomArgs &p, unsigned long long *out,
                    hipStream_t s);
// Build (q NULL): zr0[r] and zr1[r], if given, are set to zero for every record r written.
void launch_project(const GaussArgs &a, const ViewDev *views, int nv, const GeomArgs &p, const uint32_t *offs,
                    const uint32_t *vmask, const Status *st, uint32_t rcap, const QueryArgs *q, Rec *rec,
                    uint32_t *key, Bin *bin, uint32_t *ntr, int pack, uint32_t *zr0, uint32_t *zr1,
                    hipStream_t s);

size_t scan_blk_count(uint64_t n_cap);
void launch_scan(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint64_t n_host, uint64_t n_cap,
                 unsigned long long *blk, unsigned long long *total, uint32_t *eff, uint64_t tcap,
                 uint32_t *overflow, uint32_t flag_bit, hipStream_t s);
// LSD radix sort of (key, value) pairs on the low `bits` bits; returns 1 when
// the result is in (k1, v1).  drop (DEAD_KEY: none): pairs whose tile field
// equals it are removed by the first pass, which writes the kept count to
// *n_kept for the rest of the sort.  n_cap: the most pairs *n_dev can hold
// (sizes the grid).  gather_dst (optional): the last pass also writes
// gather_dst[i] = gather_src[sorted value i] for every output position i,
// or, with gather_bin, the tile count the sorted value carries (PACK_SHIFT;
// a saturated count from gather_bin[record]).
// keys_out false: the sorted keys are not written (only the values are
// sorted into the result buffer).
int launch_radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const uint32_t *n_dev, int bits,
                      bool iota, uint32_t *hist, uint32_t *dtot, hipStream_t s, uint32_t drop, uint32_t *n_kept,
                      uint64_t n_cap, const uint32_t *gather_src = nullptr, uint32_t *gather_dst = nullptr,
                      bool keys_out = true, const Bin *gather_bin = nullptr);
void launch_convert(const void *src, int sdt, void *dst, int ddt, uint64_t n, hipStream_t s);
// Density control (Alg. 5): box corner and sides in FP64, particle scale.
struct VirtArgs {
    double lo[3], span[3];
    float s;
};
void launch_place_virtual(float *means, float *scales, float *quats, float *opac, const float *u, int64_t n_real,
                          int64_t nv, const VirtArgs &v, hipStream_t s);
void launch_virtual_flags(const float *vis, int64_t n_real, int64_t nv, float eps_v, uint32_t *flags, hipStream_t s);
void launch_virtual_pack(const uint32_t *flags, const uint32_t *offs, int64_t n_real, int64_t nv, const float *means,
                         const float *scales, const float *quats, const float *opac, int32_t *kept, float *tmp,
                         hipStream_t s);
void launch_virtual_store(const float *tmp, int64_t n_real, int64_t n_kept, float *means, float *scales, float *quats,
                          float *opac, hipStream_t s);
void launch_vis_logsum(int64_t n, const uint32_t *offs, const float *acc_T, const uint32_t *acc_c, const Status *st,
                       float *out, bool accumulate, unsigned long long *pairs, hipStream_t s);
void launch_vis_finish(int64_t n, float *out, hipStream_t s);
void launch_view_vis(const GaussArgs &a, const uint32_t *offs, const uint32_t *vmask, int mw, const float *acc_T,
                     const uint32_t *acc_c, const Status *st, float *out, unsigned long long *pairs, hipStream_t s);
// Instances of the first st->R_eff depth-ordered records (sval) at the output
// offsets ioff of a scan done before (nothing on overflow).
void launch_emit_scanned(const uint32_t *sval, const Bin *bin, const uint32_t *ioff, const Status *st, float qcut,
                         uint32_t dead_tile, uint32_t *ikey, uint32_t *ival, uint32_t rmask, hipStream_t s);
// Post words the instance emission needs for rcap records (its look-back).
size_t emit_post_words(uint64_t rcap);
// Instances of the first st->R_eff depth-ordered records (sval) into
// (ikey, ival), at most icap of them; sets st->M_total, M_eff and the
// instance overflow bit.  lb: emit_post_words(rcap) words of workspace.
void launch_emit(const uint32_t *sval, const Bin *bin, unsigned long long *lb, Status *st, uint64_t rcap,
                 uint64_t icap, float qcut, uint32_t dead_tile, uint32_t *ikey, uint32_t *ival, hipStream_t s);
void launch_ranges(const uint32_t *key, const Status *st, uint32_t dead_tile, uint2 *ranges, hipStream_t s);

// order: tile schedule of the blend's workgroups (0 linear, 1 contiguous runs
// of tiles per XCD, 2 the tiles listed by torder; 3 and 4 persistent
// workgroups taking tiles from a queue, in tile order or in torder's order,
// through the eight ticket words, which must be zero at launch); batch:
// records staged per LDS batch (64, 128, 256)
void launch_raster_vis(const ViewDev *views, int nv, int total_tiles, const uint2 *ranges, const uint32_t *ival,
                       const uint32_t *ikey, const Rec *rec, float eps_T, float qcut, float *acc_T, uint32_t *acc_c,
                       int batch, int order, const uint32_t *torder, uint32_t *ticket, hipStream_t s);
// The tiles 0..T-1 by decreasing list length (ties by tile id), for the
// blends' schedule 2: four T-word buffers and a count word of workspace;
// returns the ordered ids (one of the buffers).
const uint32_t *launch_tile_order(const uint2 *ranges, uint32_t T, uint32_t *buf, uint32_t *count, uint32_t *hist,
                                  uint32_t *dtot, hipStream_t s);
// rcc: per-record colour constants c_c (NULL: the uniform u.cQc); rz and
// dmaps: per-record depths and the expected-depth maps (both NULL: none;
// depth maps need maps)
void launch_raster_uq(const ViewDev *views, int nv, int total_tiles, const uint2 *ranges, const uint32_t *ival,
                      const Rec *rec, const float *rcc, const float *rz, const UqArgs &u,
                      float *tile_part, float *maps, float *dmaps, unsigned long long *pairs, int batch,
                      int order, const uint32_t *torder, uint32_t *ticket, hipStream_t s);
void launch_scores(const ViewDev *views, int nv, const float *tile_part, const Status *st, float *scores,
                   hipStream_t s);
void launch_argmax(const float *scores, int n, int32_t *best, hipStream_t s);
void launch_vf_accum(const GaussArgs &a, const ViewDev *views, const uint32_t *offs, const uint32_t *vmask, int mw,
                     const float *acc_T, const uint32_t *acc_c, const Status *st, int L, const float *al,
                     void *gamma, int gamma_dtype, bool accumulate, unsigned long long *pairs, hipStream_t s);

}  // namespace gv
