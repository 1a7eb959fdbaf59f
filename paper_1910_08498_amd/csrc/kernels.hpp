// Device-side declarations shared by the gfx950 kernels and their host
// launchers (internal to librecon.so; the public interface is include/recon.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace recon {

// Geometry and blob constants of one reconstruction, passed by value.
struct Geom {
    int n;          // slice edge (even)
    int h;          // n / 2
    int dim;        // n + 1, volume edge
    int sw;         // h + 1, stored half-plane row length
    float a;        // blob radius
    float a2;       // a * a
    float tscale;   // (N - 1) / a^2 : table index per unit squared distance
    int N;          // table entries
    float r2max;    // r_max^2 : samples with kx^2 + ky^2 < r2max are inserted
    int dtype;      // slice storage: 0 complex64, 1 half pairs x per-slice scale, 2 bfloat16 pairs
    const float *scales;  // per-slice scales of the current batch (half storage), else NULL
    int nterms;     // on-the-fly weights: coefficients of the blob polynomial (a multiple of 4)
    float inv_a2;   // 1 / a^2
};

// Source of the interpolation weights (the paper's "precomputed or on the
// fly" option, Sect. 4.2 "3D Fourier Reconstruction").
//   WEIGHT_TRUNC, WEIGHT_LERP: the FP64-built table T[i] = b(i a^2/(N-1)),
//     looked up at t = d^2 (N-1)/a^2 by truncation or linear interpolation;
//   WEIGHT_OTF: the blob itself, b = s^m sum_j c_j s^j with s = 1 - d^2/a^2
//     (the power series of I_m, divided by I_m(alpha)), evaluated by Horner's
//     rule in FP32.  The coefficients c (nterms of them, leading ones of the
//     highest degree padded with zeros) follow the table in the workspace.
constexpr int WEIGHT_TRUNC = 0;
constexpr int WEIGHT_LERP = 1;
constexpr int WEIGHT_OTF = 2;
constexpr int kMaxTerms = 72;   // coefficients of the on-the-fly polynomial, at most

// Horner's rule over the polynomial's coefficients c[0..nterms-1] (c[0] the
// constant term; stored as the .x of float2 entries), four at a time.
__device__ __forceinline__ float blob_poly(const float2 *__restrict__ c, int nterms, float s)
{
    float acc = 0.f;
    for (int j = nterms - 4; j >= 0; j -= 4) {
        acc = fmaf(acc, s, c[j + 3].x);
        acc = fmaf(acc, s, c[j + 2].x);
        acc = fmaf(acc, s, c[j + 1].x);
        acc = fmaf(acc, s, c[j].x);
    }
    return acc;
}

// Bytes per stored sample for a storage type.
__host__ __device__ inline int sample_bytes(int dtype) { return dtype == 0 ? 8 : 4; }

// Decodes one stored sample (element index idx of the slice starting at
// `base`); `scale` multiplies half-precision samples.
__device__ __forceinline__ float2 decode_sample(const unsigned char *__restrict__ base, int idx, int dtype,
                                                float scale)
{
    if (dtype == 0) return reinterpret_cast<const float2 *>(base)[idx];
    const unsigned raw = reinterpret_cast<const unsigned *>(base)[idx];
    if (dtype == 1) {
        const _Float16 lo = __builtin_bit_cast(_Float16, static_cast<unsigned short>(raw & 0xffffu));
        const _Float16 hi = __builtin_bit_cast(_Float16, static_cast<unsigned short>(raw >> 16));
        return make_float2(static_cast<float>(lo) * scale, static_cast<float>(hi) * scale);
    }
    return make_float2(__uint_as_float(raw << 16), __uint_as_float(raw & 0xffff0000u));
}

// Per-slice orientation record written by the prep kernel (128 bytes).
// e1, e2 are the images of the slice's x and y axes in the volume, e3 the
// plane normal (columns of R), each component the correctly rounded value
// for the given quaternion.  e1.w is 1 for a usable slice, 0 otherwise.
// The rest are per-slice constants of the slab kernel, computed once here
// instead of once per (tile, slice):
//   e1s, e2s, e3s  the axes scaled by sqrt((N-1)/a^2) (table units),
//                  rounded to FP32; with exact geometry, their part on a
//                  grid of a power-of-two step gs instead, with the
//                  remainders in a separate array of three float4 per slice
//                  (xyz: the remainders of e1s, e2s, e3s; see exact_geometry);
//   e1s.w          the axes' order as int bits d | ia << 8 | ib << 16: d is
//                  e3's dominant axis, ia < ib the other two;
//   e2s.w          1 / e3[d];  e3s.w  e3[d];
//   p1, p2         (e[d], e[ia], e[ib], .) of e1 and e2; p1.w = e3[ia],
//                  p2.w = e3[ib].
struct Orient {
    float4 e1, e2, e3;
    float4 e1s, e2s, e3s;
    float4 p1, p2;
};

// Exact window geometry for the slab kernel.  A voxel's position in table
// units, c . v for a scaled axis c, is formed in FP32; at |v| ~ 500 its
// rounding (an ulp of ~27000) moves the table index by ~0.1 steps, a
// relative weight error of ~1e-4 per sample far from the origin.  With
// exact geometry c = g + b with g on a grid fine enough that g . v is exact
// for |v_i| <= 512, and b . v (|b| <= gs / 2) is added after the large part
// has cancelled, so the error drops to an ulp of the offset itself.  It costs
// three FMAs per coordinate and hit, so it is used where the weight error
// of one position ulp is large: it grows with the distance from the origin
// over the blob radius (a weight's slope in d^2 is of order 1/a^2, and the
// rounding of d^2 of order a ulp(|v|)), so boxes with h > 67.4 a, i.e. boxes
// above 256 for the default blob radius 1.9, and smaller boxes for smaller
// blobs.
inline bool exact_geometry(const Geom &g) { return static_cast<float>(g.h) > 67.4f * g.a; }

// Workspace counters (device, 256 bytes at the start of the workspace).
struct Counters {
    unsigned long long inserted;   // slices passed to the insertion kernels
    unsigned long long rejected;   // slices with zero / non-finite quaternion
    unsigned int queue;            // work-queue head of the persistent kernel
    unsigned int pad[59];
};

// Work item of the queue kernels: one voxel tile and one slice range.
struct Item {
    int tile;      // tile index (tx + TX * (ty + TY * tz)); slab kernel: job id in bits 24..31
    int part;      // k-th of nparts slice ranges
    int nparts;    // number of ranges the tile's slices are split into
    int slot;      // partial-sum slot (when nparts > 1), else -1
};

// One reconstruction of a slab launch.  Several reconstructions (jobs) with
// the same blob parameters can share one persistent launch.
constexpr int kMaxJobs = 8;
struct JobDesc {
    Geom g;
    const void *slices;      // this batch's stored slices
    const Orient *orient;    // orientation records of this batch
    const float4 *rem;       // exact geometry: axis remainders, 3 per slice
    float4 *partials;        // partial-sum slots of split tiles (slab: re, im, w planes of 512 floats)
    float2 *G;
    float *W;
    int count;               // slices in this batch
    int pad;
};
struct JobTable {
    JobDesc job[kMaxJobs];
    int njobs;
};

// Host launchers (defined in kernels.hip).
hipError_t launch_zero(float *p, size_t count, hipStream_t st);
// Orientation records for a batch; adds `count` to ctr->inserted; zeroes
// *queue (a work-queue head) when given.  `exact`: split the scaled axes for
// the slab kernel's exact geometry (the launch that reads the records must
// be built for the same choice).
hipError_t launch_prep(const float *quats, int count, float tscale, bool exact, Orient *orient, float4 *rem,
                       Counters *ctr, unsigned *queue, hipStream_t st);
hipError_t launch_insert_naive(const Geom &g, int mode, const void *slices,
                               const Orient *orient, int count, const float2 *table,
                               int inner_chunk, int waves_per_block, float2 *G, float *W,
                               hipStream_t st);
hipError_t launch_insert_binned(const Geom &g, int mode, const void *slices,
                                const Orient *orient, int count, const float2 *table,
                                const Item *items, int nitems, float4 *partials,
                                int inner_chunk, int blocks, int waves_per_block,
                                Counters *ctr, float2 *G, float *W, hipStream_t st);
hipError_t launch_reduce_partials(const Geom &g, const Item *items, int nitems,
                                  const float4 *partials, float2 *G, float *W,
                                  hipStream_t st);
// Slab-enumeration gather over 8x8x8 tiles (one wavefront per item).
// lane_order: which in-plane axis of a tile's columns varies fastest across
// the lanes (0: the first, 1: the second).
size_t slab_lds_bytes(const Geom &g, int mode, int waves_per_block);
hipError_t launch_insert_slab(const JobTable &jt, int mode, int flags, bool exact, const float2 *table,
                              const Item *items, int nitems, int inner_chunk, int lane_order, int blocks,
                              int waves_per_block, Counters *ctr, hipStream_t st);
hipError_t launch_reduce_partials8(const JobTable &jt, const Item *items, int nitems, hipStream_t st);
hipError_t launch_finalize(const Geom &g, float2 *G, float *W, float2 *V, float thr,
                           hipStream_t st);

// Learned configuration predictor (mlp.hip).
size_t mlp_param_count(int n_in, int H, int C);
size_t mlp_ws_floats(int n_in, int H, int C, int B);
hipError_t mlp_forward(const float *params, int n_in, int H, int C, const float *x, int B, float *ws, float *probs,
                       hipStream_t st);
hipError_t mlp_train_step(float *params, int n_in, int H, int C, const float *x, const float *y, int B, float lr,
                          float *ws, float *loss, float *grads_out, hipStream_t st);

}  // namespace recon
