// gfx950 kernels of the Fourier-slice insertion path.
//
// Insertion follows the paper's Algorithm 1 (Sect. 5.3.1) and the insertion
// step of Sect. 4.2 ("3D Fourier Reconstruction"): every sample k of a slice
// with rotation R lands at p = R (kx, ky, 0)^T and adds b(|v-p|^2) F(k) to G
// and b(|v-p|^2) to W at every voxel v within the blob radius a.  The paper's
// own kernel is a gather (each output owned by one thread, no atomics); the
// kernels here are gathers too: for a voxel v and a slice with axes e1, e2 and
// normal e3, |v - p|^2 = (ux-kx)^2 + (uy-ky)^2 + uz^2 with u = (e1.v, e2.v,
// e3.v), so only slices with |uz| <= a contribute, through the samples of the
// WIN x WIN integer window starting at (ceil(ux-a), ceil(uy-a)),
// WIN = floor(2a) + 1.
//
// Only the half box x >= 0 is accumulated; the finalize kernel mirrors the
// rest (G(-v) = conj G(v), W(-v) = W(v), which holds because every slice is
// the transform of a real image and its full plane is Hermitian).
#include "kernels.hpp"

namespace recon {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Blob weight at squared distance d2 <= a^2.  Table modes: t = d^2 (N-1)/a^2,
// entry i of `tab` holds (T[i], T[i+1]-T[i]).  On-the-fly mode: `tab` holds
// the polynomial's coefficients, evaluated at s = 1 - d^2/a^2 (clamped at 0,
// where rounding leaves a tiny negative s for d2 = a^2).
template <int MODE>
__device__ __forceinline__ float blob_weight(const float2 *__restrict__ tab, float d2, const Geom &g)
{
    if constexpr (MODE == WEIGHT_OTF) {
        return blob_poly(tab, g.nterms, fmaxf(fmaf(-d2, g.inv_a2, 1.0f), 0.0f));
    } else {
        const float t = d2 * g.tscale;
        const int i = min(static_cast<int>(t), g.N - 1);
        const float2 e = tab[i];
        if (MODE == WEIGHT_LERP) return fmaf(t - static_cast<float>(i), e.y, e.x);
        return e.x;
    }
}

// Full-plane sample F~(k) from the stored half plane of one slice.
__device__ __forceinline__ float2 fetch_full(const unsigned char *__restrict__ Fs, float scale, const Geom &g,
                                             int kx, int ky)
{
    const bool direct = kx > 0 || (kx == 0 && ky >= 0);
    const int row = direct ? ky + g.h : g.h - ky;
    const int col = direct ? kx : -kx;
    float2 f = decode_sample(Fs, row * g.sw + col, g.dtype, scale);
    if (!direct) f.y = -f.y;
    return f;
}

// Start of slice s in a batch of stored slices, and its scale.
__device__ __forceinline__ const unsigned char *slice_base(const void *slices, int s, const Geom &g)
{
    return static_cast<const unsigned char *>(slices) +
           static_cast<size_t>(s) * static_cast<size_t>(g.n) * g.sw * sample_bytes(g.dtype);
}
__device__ __forceinline__ float slice_scale(int s, const Geom &g) { return g.scales ? g.scales[s] : 1.0f; }

// Accumulates the WIN x WIN window of one (voxel, slice) pair.
template <int WIN, int MODE>
__device__ __forceinline__ void window_global(const unsigned char *__restrict__ Fs, float scale, const Geom &g,
                                              const float2 *__restrict__ tab, float ux, float uy,
                                              float uz, float &pr, float &pi, float &pw)
{
    const float uz2 = uz * uz;
    const int kx0 = static_cast<int>(ceilf(ux - g.a));
    const int ky0 = static_cast<int>(ceilf(uy - g.a));
#pragma unroll
    for (int j = 0; j < WIN; ++j) {
        const int ky = ky0 + j;
        const float dy = uy - static_cast<float>(ky);
        const float dyz = fmaf(dy, dy, uz2);
#pragma unroll
        for (int i = 0; i < WIN; ++i) {
            const int kx = kx0 + i;
            const float dx = ux - static_cast<float>(kx);
            const float d2 = fmaf(dx, dx, dyz);
            const bool in_disk = static_cast<float>(kx * kx + ky * ky) < g.r2max;
            if (d2 <= g.a2 && in_disk) {
                const float w = blob_weight<MODE>(tab, d2, g);
                const float2 f = fetch_full(Fs, scale, g, kx, ky);
                pr = fmaf(w, f.x, pr);
                pi = fmaf(w, f.y, pi);
                pw += w;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// zero fill (used instead of a memset so callers may capture it in a graph)
// ---------------------------------------------------------------------------
__global__ void k_zero(float *__restrict__ p, size_t count)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
         i += stride)
        p[i] = 0.0f;
}

hipError_t launch_zero(float *p, size_t count, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// orientation prep: quaternion (w, x, y, z) -> columns of R, in FP32
// ---------------------------------------------------------------------------
// R is formed in double-float arithmetic (a value is the unevaluated sum
// hi + lo of two floats: error-free two-sum and fma two-product, about 44
// bits) and rounded to FP32 once, so every stored axis component is the
// exact rotation of the given FP32 quaternion, correctly rounded.  Plain FP32
// evaluation loses a few bits per component, and the position error it
// causes grows with the distance from the origin (at |v| = 500 it dominates
// the geometry error of a window).  Contraction is off in these helpers and
// in the prep kernel: a product fused into a following sum after inlining
// would break the error-free transformations.
struct DF {
    float hi, lo;
};
__device__ __forceinline__ DF df_quick(float a, float b)   // |a| >= |b| or a == 0
{
#pragma clang fp contract(off)
    const float s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ DF df_sum(float a, float b)
{
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ DF df_prod(float a, float b)
{
#pragma clang fp contract(off)
    const float p = a * b;
    return {p, fmaf(a, b, -p)};
}
__device__ __forceinline__ DF df_add(DF a, DF b)
{
#pragma clang fp contract(off)
    DF s = df_sum(a.hi, b.hi);
    const DF t = df_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = df_quick(s.hi, s.lo);
    s.lo += t.lo;
    return df_quick(s.hi, s.lo);
}
__device__ __forceinline__ DF df_neg(DF a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ DF df_scale(DF a, float b)
{
#pragma clang fp contract(off)
    DF p = df_prod(a.hi, b);
    p.lo = fmaf(a.lo, b, p.lo);
    return df_quick(p.hi, p.lo);
}
// a / b for b > 0: quotient of the leading parts, then one correction from
// the remainder
__device__ __forceinline__ DF df_div(DF a, DF b)
{
#pragma clang fp contract(off)
    const float q1 = a.hi / b.hi;
    const DF r = df_add(a, df_neg(df_scale(b, q1)));
    return df_quick(q1, r.hi / b.hi);
}

__global__ void k_prep(const float4 *__restrict__ quats, int count, float tscale, int exact,
                       Orient *__restrict__ orient, float4 *__restrict__ rem, Counters *__restrict__ ctr,
                       unsigned *__restrict__ queue)
{
#pragma clang fp contract(off)
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        if (queue) *queue = 0u;
        atomicAdd(&ctr->inserted, static_cast<unsigned long long>(count));
    }
    if (s >= count) return;
    float4 q = quats[s];
    const float nn = q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w;
    Orient o;
    if (!(nn > 0.0f) || !isfinite(nn)) {
        o.e1 = make_float4(0.f, 0.f, 0.f, 0.f);
        o.e2 = o.e3 = o.e1s = o.e2s = o.e3s = o.p1 = o.p2 = o.e1;
        orient[s] = o;
        atomicAdd(&ctr->rejected, 1ull);
        return;
    }
    // R(q) = M(q) / |q|^2 for the unnormalised q (Hamilton, active rotation):
    //   M = [[ww+xx-yy-zz, 2(xy-wz),    2(xz+wy)],
    //        [2(xy+wz),    ww-xx+yy-zz, 2(yz-wx)],
    //        [2(xz-wy),    2(yz+wx),    ww-xx-yy+zz]]
    // which equals the normalised form 1 - 2(y^2 + z^2), ... exactly.
    const float w = q.x, x = q.y, y = q.z, z = q.w;
    const DF ww = df_prod(w, w), xx = df_prod(x, x), yy = df_prod(y, y), zz = df_prod(z, z);
    const DF xy = df_prod(x, y), wz = df_prod(w, z), xz = df_prod(x, z), wy = df_prod(w, y);
    const DF yz = df_prod(y, z), wx = df_prod(w, x);
    const DF n2 = df_add(df_add(ww, xx), df_add(yy, zz));
    // the factor 2 of the off-diagonal terms is exact in any precision
    auto ent = [&](DF m, float two) { return df_div(df_scale(m, two), n2); };
    const DF r00 = ent(df_add(df_add(ww, xx), df_neg(df_add(yy, zz))), 1.f);
    const DF r11 = ent(df_add(df_add(ww, yy), df_neg(df_add(xx, zz))), 1.f);
    const DF r22 = ent(df_add(df_add(ww, zz), df_neg(df_add(xx, yy))), 1.f);
    const DF r01 = ent(df_add(xy, df_neg(wz)), 2.f), r10 = ent(df_add(xy, wz), 2.f);
    const DF r02 = ent(df_add(xz, wy), 2.f), r20 = ent(df_add(xz, df_neg(wy)), 2.f);
    const DF r12 = ent(df_add(yz, df_neg(wx)), 2.f), r21 = ent(df_add(yz, wx), 2.f);
    o.e1 = make_float4(r00.hi, r10.hi, r20.hi, 1.f);
    o.e2 = make_float4(r01.hi, r11.hi, r21.hi, 0.f);
    o.e3 = make_float4(r02.hi, r12.hi, r22.hi, 0.f);
    // slab-kernel constants; the scaled axes are rounded once from the
    // double-float product as well
    const float r = sqrtf(tscale);
    const float n[3] = {o.e3.x, o.e3.y, o.e3.z};
    const float a1[3] = {o.e1.x, o.e1.y, o.e1.z};
    const float a2[3] = {o.e2.x, o.e2.y, o.e2.z};
    const float m0 = fabsf(n[0]), m1 = fabsf(n[1]), m2 = fabsf(n[2]);
    const int d = (m0 >= m1 && m0 >= m2) ? 0 : (m1 >= m2 ? 1 : 2);
    const int ia = d == 0 ? 1 : 0;
    const int ib = d == 2 ? 1 : 2;
    // Exact geometry: each scaled component c = r e is split into a part on
    // a grid of step gs (a power of two) and the remainder: with |v_i| <= 512
    // every partial sum of (grid part) . v is a multiple of gs below 2^24 gs,
    // so the slab kernel forms it exactly in FP32, and the remainder
    // (|.| <= gs / 2) adds the rest with an error far below a table step.
    // Otherwise the component is rounded once and the remainder is zero.
    int ex;
    frexpf(1.7321f * 512.f * r * 0x1p-24f * 1.001f, &ex);
    const float gs = ldexpf(1.f, ex);
    float g3[9], b3[9];
    const DF cols[9] = {r00, r10, r20, r01, r11, r21, r02, r12, r22};
    for (int k = 0; k < 9; ++k) {
        const DF c = df_scale(cols[k], r);
        g3[k] = exact ? rintf(c.hi / gs) * gs : c.hi;
        b3[k] = exact ? (c.hi - g3[k]) + c.lo : 0.f;
    }
    o.e1s = make_float4(g3[0], g3[1], g3[2], __int_as_float(d | (ia << 8) | (ib << 16)));
    o.e2s = make_float4(g3[3], g3[4], g3[5], 1.0f / n[d]);
    o.e3s = make_float4(g3[6], g3[7], g3[8], n[d]);
    if (exact) {
        rem[3 * s] = make_float4(b3[0], b3[1], b3[2], 0.f);
        rem[3 * s + 1] = make_float4(b3[3], b3[4], b3[5], 0.f);
        rem[3 * s + 2] = make_float4(b3[6], b3[7], b3[8], 0.f);
    }
    o.p1 = make_float4(a1[d], a1[ia], a1[ib], n[ia]);
    o.p2 = make_float4(a2[d], a2[ia], a2[ib], n[ib]);
    orient[s] = o;
}

hipError_t launch_prep(const float *quats, int count, float tscale, bool exact, Orient *orient, float4 *rem,
                       Counters *ctr, unsigned *queue, hipStream_t st)
{
    const int blocks = count > 0 ? (count + 255) / 256 : 1;
    hipLaunchKernelGGL(k_prep, dim3(blocks), dim3(256), 0, st,
                       reinterpret_cast<const float4 *>(quats), count, tscale, exact ? 1 : 0, orient, rem, ctr,
                       queue);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// naive gather: one thread per voxel of the half box, every slice
// ---------------------------------------------------------------------------
template <int WIN, int MODE>
__global__ __launch_bounds__(1024) void k_insert_naive(Geom g, const void *__restrict__ slices,
                                                       const Orient *__restrict__ orient, int count,
                                                       const float2 *__restrict__ tab, int inner_chunk,
                                                       float2 *__restrict__ G, float *__restrict__ W)
{
    const int hx = g.h + 1;
    const long total = static_cast<long>(hx) * g.dim * g.dim;
    const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int ix = static_cast<int>(idx % hx);
    const long rest = idx / hx;
    const int iy = static_cast<int>(rest % g.dim);
    const int iz = static_cast<int>(rest / g.dim);
    const float vx = static_cast<float>(ix);
    const float vy = static_cast<float>(iy - g.h);
    const float vz = static_cast<float>(iz - g.h);

    float ore = 0.f, oim = 0.f, ow = 0.f;
    float ire = 0.f, iim = 0.f, iw = 0.f;
    int inner = 0;
    for (int s = 0; s < count; ++s) {
        const Orient o = orient[s];
        if (o.e1.w == 0.f) continue;
        const float uz = fmaf(o.e3.x, vx, fmaf(o.e3.y, vy, o.e3.z * vz));
        if (fabsf(uz) <= g.a) {
            const float ux = fmaf(o.e1.x, vx, fmaf(o.e1.y, vy, o.e1.z * vz));
            const float uy = fmaf(o.e2.x, vx, fmaf(o.e2.y, vy, o.e2.z * vz));
            window_global<WIN, MODE>(slice_base(slices, s, g), slice_scale(s, g), g, tab, ux, uy, uz, ire, iim,
                                     iw);
        }
        if (++inner == inner_chunk) {
            ore += ire; oim += iim; ow += iw;
            ire = iim = iw = 0.f;
            inner = 0;
        }
    }
    ore += ire; oim += iim; ow += iw;
    const size_t vi = (static_cast<size_t>(iz) * g.dim + iy) * g.dim + (ix + g.h);
    float2 gv = G[vi];
    gv.x += ore;
    gv.y += oim;
    G[vi] = gv;
    W[vi] += ow;
}

template <int WIN, int MODE>
static hipError_t launch_naive_t(const Geom &g, const void *slices, const Orient *orient, int count,
                                 const float2 *tab, int inner_chunk, int wpb, float2 *G, float *W,
                                 hipStream_t st)
{
    const long total = static_cast<long>(g.h + 1) * g.dim * g.dim;
    const int threads = 64 * wpb;
    const long blocks = (total + threads - 1) / threads;
    // on the fly: the coefficients follow the table's N entries
    const float2 *w = MODE == WEIGHT_OTF ? tab + g.N : tab;
    hipLaunchKernelGGL((k_insert_naive<WIN, MODE>), dim3(static_cast<unsigned>(blocks)),
                       dim3(threads), 0, st, g, slices, orient, count, w, inner_chunk, G, W);
    return hipGetLastError();
}

// window sizes of blob radii in [1, 2.95]: floor(2a) + 1 = 3 .. 6
#define RECON_DISPATCH_MODE(WV, FN, ...)                                                  \
    case WV:                                                                              \
        return mode == WEIGHT_OTF    ? FN<WV, WEIGHT_OTF>(__VA_ARGS__)                    \
               : mode == WEIGHT_LERP ? FN<WV, WEIGHT_LERP>(__VA_ARGS__)                   \
                                     : FN<WV, WEIGHT_TRUNC>(__VA_ARGS__);
#define RECON_DISPATCH_WIN(WINV, FN, ...)          \
    switch (WINV) {                                \
        RECON_DISPATCH_MODE(3, FN, __VA_ARGS__)    \
        RECON_DISPATCH_MODE(4, FN, __VA_ARGS__)    \
        RECON_DISPATCH_MODE(5, FN, __VA_ARGS__)    \
        RECON_DISPATCH_MODE(6, FN, __VA_ARGS__)    \
    default: return hipErrorInvalidValue;          \
    }

static inline int window_size(float a) { return static_cast<int>(floorf(2.0f * a)) + 1; }

hipError_t launch_insert_naive(const Geom &g, int mode, const void *slices, const Orient *orient,
                               int count, const float2 *table, int inner_chunk, int waves_per_block,
                               float2 *G, float *W, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    RECON_DISPATCH_WIN(window_size(g.a), launch_naive_t, g, slices, orient, count, table, inner_chunk,
                       waves_per_block, G, W, st)
}

// ---------------------------------------------------------------------------
// binned gather: persistent wavefronts pull (4x4x4 tile, slice range) items
// from a queue; each wave tests the slices of its range against the tile
// (ballot), then every lane (one voxel) gathers from the slices that pass.
// The blob table lives in LDS, shared by the work-group's waves.
// ---------------------------------------------------------------------------
template <int WIN, int MODE>
__global__ __launch_bounds__(1024) void k_insert_binned(
    Geom g, const void *__restrict__ slices, const Orient *__restrict__ orient, int count,
    const float2 *__restrict__ table_g, const Item *__restrict__ items, int nitems,
    float4 *__restrict__ partials, int inner_chunk, Counters *__restrict__ ctr,
    float2 *__restrict__ G, float *__restrict__ W)
{
    // the table, or on the fly the polynomial's coefficients (after the table)
    extern __shared__ float2 tab[];
    if constexpr (MODE == WEIGHT_OTF) {
        for (int i = threadIdx.x; i < g.nterms; i += blockDim.x) tab[i] = table_g[g.N + i];
    } else {
        for (int i = threadIdx.x; i < g.N; i += blockDim.x) tab[i] = table_g[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int TX = (g.h + 1 + 3) >> 2;
    const int TY = (g.dim + 3) >> 2;
    // conservative in-plane reach of a tile: r_max + a + 1.5 * sqrt(6)
    const float reach = sqrtf(g.r2max) + g.a + 3.675f;
    const float reach2 = reach * reach;

    for (;;) {
        unsigned it = 0;
        if (lane == 0) it = atomicAdd(&ctr->queue, 1u);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
        if (it >= static_cast<unsigned>(nitems)) break;
        const Item item = items[it];
        const int tx = item.tile % TX;
        const int ty = (item.tile / TX) % TY;
        const int tz = item.tile / (TX * TY);
        const int ix = 4 * tx + (lane & 3);
        const int iy = 4 * ty + ((lane >> 2) & 3);
        const int iz = 4 * tz + (lane >> 4);
        const bool in_box = ix <= g.h && iy < g.dim && iz < g.dim;
        const float vx = static_cast<float>(ix);
        const float vy = static_cast<float>(iy - g.h);
        const float vz = static_cast<float>(iz - g.h);
        const float cx = 4.f * tx + 1.5f;
        const float cy = 4.f * ty + 1.5f - g.h;
        const float cz = 4.f * tz + 1.5f - g.h;
        const int s0 = static_cast<int>(static_cast<long>(count) * item.part / item.nparts);
        const int s1 = static_cast<int>(static_cast<long>(count) * (item.part + 1) / item.nparts);

        float ore = 0.f, oim = 0.f, ow = 0.f;
        float ire = 0.f, iim = 0.f, iw = 0.f;
        int inner = 0;
        for (int base = s0; base < s1; base += 64) {
            const int s = base + lane;
            bool pass = false;
            if (s < s1) {
                const Orient o = orient[s];
                if (o.e1.w != 0.f) {
                    const float dz = fmaf(o.e3.x, cx, fmaf(o.e3.y, cy, o.e3.z * cz));
                    const float ext = 1.5f * (fabsf(o.e3.x) + fabsf(o.e3.y) + fabsf(o.e3.z));
                    const float px = fmaf(o.e1.x, cx, fmaf(o.e1.y, cy, o.e1.z * cz));
                    const float py = fmaf(o.e2.x, cx, fmaf(o.e2.y, cy, o.e2.z * cz));
                    pass = fabsf(dz) <= g.a + ext + 1e-3f && fmaf(px, px, py * py) <= reach2;
                }
            }
            unsigned long long mask = __ballot(pass);
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1ull;
                const int ss = base + b;
                const Orient o = orient[ss];
                const float uz = fmaf(o.e3.x, vx, fmaf(o.e3.y, vy, o.e3.z * vz));
                if (in_box && fabsf(uz) <= g.a) {
                    const float ux = fmaf(o.e1.x, vx, fmaf(o.e1.y, vy, o.e1.z * vz));
                    const float uy = fmaf(o.e2.x, vx, fmaf(o.e2.y, vy, o.e2.z * vz));
                    window_global<WIN, MODE>(slice_base(slices, ss, g), slice_scale(ss, g), g, tab, ux, uy, uz, ire,
                                             iim, iw);
                }
                if (++inner == inner_chunk) {
                    ore += ire; oim += iim; ow += iw;
                    ire = iim = iw = 0.f;
                    inner = 0;
                }
            }
        }
        ore += ire; oim += iim; ow += iw;
        if (item.nparts == 1) {
            if (in_box) {
                const size_t vi = (static_cast<size_t>(iz) * g.dim + iy) * g.dim + (ix + g.h);
                float2 gv = G[vi];
                gv.x += ore;
                gv.y += oim;
                G[vi] = gv;
                W[vi] += ow;
            }
        } else {
            partials[static_cast<size_t>(item.slot) * 64 + lane] = make_float4(ore, oim, ow, 0.f);
        }
    }
}

template <int WIN, int MODE>
static hipError_t launch_binned_t(const Geom &g, const void *slices, const Orient *orient, int count,
                                  const float2 *table, const Item *items, int nitems, float4 *partials,
                                  int inner_chunk, int blocks, int wpb, Counters *ctr, float2 *G,
                                  float *W, hipStream_t st)
{
    const size_t lds = static_cast<size_t>(MODE == WEIGHT_OTF ? g.nterms : g.N) * sizeof(float2);
    hipLaunchKernelGGL((k_insert_binned<WIN, MODE>), dim3(blocks), dim3(64 * wpb), lds, st, g, slices,
                       orient, count, table, items, nitems, partials, inner_chunk, ctr, G, W);
    return hipGetLastError();
}

hipError_t launch_insert_binned(const Geom &g, int mode, const void *slices, const Orient *orient,
                                int count, const float2 *table, const Item *items, int nitems,
                                float4 *partials, int inner_chunk, int blocks, int waves_per_block,
                                Counters *ctr, float2 *G, float *W, hipStream_t st)
{
    if (count <= 0 || nitems <= 0) return hipSuccess;
    RECON_DISPATCH_WIN(window_size(g.a), launch_binned_t, g, slices, orient, count, table, items, nitems,
                       partials, inner_chunk, blocks, waves_per_block, ctr, G, W, st)
}

// Adds the partial sums of split tiles, in part order, into G and W.
// One wavefront per item; only items with part == 0 of a split tile work.
__global__ __launch_bounds__(64) void k_reduce_partials(Geom g, const Item *__restrict__ items,
                                                        const float4 *__restrict__ partials,
                                                        float2 *__restrict__ G, float *__restrict__ W)
{
    const Item item = items[blockIdx.x];
    if (item.nparts == 1 || item.part != 0) return;
    const int lane = threadIdx.x;
    const int TX = (g.h + 1 + 3) >> 2;
    const int TY = (g.dim + 3) >> 2;
    const int tx = item.tile % TX;
    const int ty = (item.tile / TX) % TY;
    const int tz = item.tile / (TX * TY);
    const int ix = 4 * tx + (lane & 3);
    const int iy = 4 * ty + ((lane >> 2) & 3);
    const int iz = 4 * tz + (lane >> 4);
    if (!(ix <= g.h && iy < g.dim && iz < g.dim)) return;
    float re = 0.f, im = 0.f, w = 0.f;
    for (int k = 0; k < item.nparts; ++k) {
        const float4 p = partials[static_cast<size_t>(item.slot + k) * 64 + lane];
        re += p.x;
        im += p.y;
        w += p.z;
    }
    const size_t vi = (static_cast<size_t>(iz) * g.dim + iy) * g.dim + (ix + g.h);
    float2 gv = G[vi];
    gv.x += re;
    gv.y += im;
    G[vi] = gv;
    W[vi] += w;
}

hipError_t launch_reduce_partials(const Geom &g, const Item *items, int nitems, const float4 *partials,
                                  float2 *G, float *W, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials, dim3(nitems), dim3(64), 0, st, g, items, partials, G, W);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// finalize: Hermitian mirror of the x < 0 half, then V = G / W (FP64 divide)
// ---------------------------------------------------------------------------
__global__ void k_finalize(Geom g, float2 *__restrict__ G, float *__restrict__ W,
                           float2 *__restrict__ V, float thr)
{
    const long total = static_cast<long>(g.dim) * g.dim * g.dim;
    const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int ix = static_cast<int>(idx % g.dim);
    float2 gv;
    float wv;
    if (ix < g.h) {
        const long mirror = total - 1 - idx;   // (-x, -y, -z)
        gv = G[mirror];
        gv.y = -gv.y;
        wv = W[mirror];
        G[idx] = gv;
        W[idx] = wv;
    } else {
        gv = G[idx];
        wv = W[idx];
    }
    if (V) {
        float2 out = make_float2(0.f, 0.f);
        if (wv > thr) {
            const double inv = 1.0 / static_cast<double>(wv);
            out.x = static_cast<float>(static_cast<double>(gv.x) * inv);
            out.y = static_cast<float>(static_cast<double>(gv.y) * inv);
        }
        V[idx] = out;
    }
}

hipError_t launch_finalize(const Geom &g, float2 *G, float *W, float2 *V, float thr, hipStream_t st)
{
    const long total = static_cast<long>(g.dim) * g.dim * g.dim;
    const long blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, g, G, W, V, thr);
    return hipGetLastError();
}

}  // namespace recon
