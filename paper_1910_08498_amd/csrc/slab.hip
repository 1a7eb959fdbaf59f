// Slab-enumeration gather: the main gfx950 insertion kernel.
//
// Same arithmetic as the other gathers (Sect. 4.2, "3D Fourier
// Reconstruction"; Algorithm 1 of Sect. 5.3.1): voxel v receives
// b(|v - R(k,0)|^2) F~(k) and b(.) from every sample k within the blob radius.
// What differs is how the work is laid out on a CDNA wavefront:
//
//  * Work items are (8x8x8 voxel tile of the half box x >= 0, slice range);
//    each wavefront pulls items from a queue and owns the tile's 512
//    accumulators in its own LDS region, so no voxel has two writers and no
//    atomics leave the wavefront.
//  * A slice passes the tile's bin test when its plane's slab |e3.v| <= a can
//    meet the tile.  For each passing slice the wavefront
//      1. enumerates exactly the voxels inside the slab: lane = one of the
//         64 columns of the tile along the normal's dominant axis, whose slab
//         run is a contiguous range; a wave prefix scan packs the runs into a
//         hit list, and the ends of the runs bound the hits' windows (slices
//         without hits stop here);
//      2. stages that rectangle of the slice into LDS, resolving the
//         Hermitian half plane and the |k| < r_max disk once per sample (zero
//         outside the disk);
//      3. processes the hits 64 per round, each lane evaluating the
//         branch-free WIN x WIN window from LDS (blob table lerp from LDS)
//         and adding its partial sums to the voxel's LDS accumulator; only
//         rounds whose windows can reach the disk edge gate each cell's
//         weight by |k| < r_max.
//    Steps 1 and the loads of step 2 for the next slice are issued before
//    step 3 of the current one, so the loads overlap the window evaluation.
//  * One kernel instance per slice storage type (complex64, half, bfloat16).
//  * Two-level FP32 accumulation: LDS accumulators hold at most
//    `inner_chunk` slices before they are folded into per-lane registers.
//    A tile split into slice ranges writes its parts' sums to partial-sum
//    slots, added in part order by k_reduce_partials8, so results are
//    bitwise reproducible.
#include <type_traits>

#include "kernels.hpp"

namespace recon {

namespace {

constexpr int TE = 8;                  // tile edge
constexpr int TV = TE * TE * TE;       // voxels per tile
constexpr int ACC_WORDS = 3 * TV;      // (re, im) pairs [512], then w [512]
constexpr int LIST_WORDS = TV / 2;     // 512 uint16 voxel ids

// The staged rectangle spans columns floor(u_min - a - 1e-3) to
// ceil(u_max - a + 1e-3) + WIN - 1 over the hits' in-plane coordinate u, so
// its width is below u_max - u_min + WIN + 2.002; the hits are voxels of one
// tile, so u_max - u_min <= 7 (|e_x| + |e_y| + |e_z|) <= 7 sqrt(3) < 12.13,
// and WIN + 14 cells always suffice.
__host__ __device__ constexpr int slab_rect(int win) { return win + 14; }
__host__ __device__ constexpr int slab_wave_words(int win)
{
    return ACC_WORDS + 2 * slab_rect(win) * slab_rect(win) + 2 * LIST_WORDS;
}

template <int WIN>
struct SlabShape {
    static constexpr int RECT = slab_rect(WIN);
    static constexpr int RECT2 = RECT * RECT;
    static constexpr int WAVE_WORDS = slab_wave_words(WIN);
};

// Table in LDS: T[0..N-1], then two sentinels T[N] = T[N+1] = -2^30 T[N-1].
// With i = min(floor(t), N) and w = clamp(T[i] + frac(t) (T[i+1] - T[i]), 0, 1),
// t = N-1 gives exactly T[N-1], and any representable t > N-1 gives 0, so the
// blob's inclusive cut-off at d^2 = a^2 costs no compare: past N-1 >= 1 the
// float spacing, and so frac(t), is at least 2^-23, and the sentinel slope
// exceeds T[N-1] by 2^30, so the lerp is at most T[N-1] (1 - 2^7) < 0; from N
// on, both sentinels give T[N] < 0.  (The table lies in [0, 1], so the upper
// clamp never acts; the clamp is the fma's output modifier.)
__host__ __device__ inline int table_words(int N) { return (N + 2 + 3) & ~3; }
// LDS words of the weight source: the table with its sentinels, or on the
// fly the polynomial's coefficients (a multiple of 4, so float4 reads)
__host__ __device__ inline int weight_words(const Geom &g, int mode)
{
    return mode == WEIGHT_OTF ? g.nterms : table_words(g.N);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Componentwise minimum over the 64 lanes of a wavefront (all lanes active)
// of two int16 values packed in one register: DPP permutations reduce each
// row of 16 lanes, then row broadcasts carry rows 0-2 into row 3, whose last
// lane holds the result.
typedef short short2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int pk_min(int a, int b)
{
    return __builtin_bit_cast(int, __builtin_elementwise_min(__builtin_bit_cast(short2_t, a),
                                                             __builtin_bit_cast(short2_t, b)));
}
// Two such reductions run interleaved, so each DPP step's wait for its
// source overlaps the other's.  The quad and mirror steps read valid lanes
// only (no fill value needed); the row broadcasts leave rows outside their
// mask at the neutral value.
__device__ __forceinline__ void wave_min_pk2(int &a, int &b)
{
    constexpr int NEUTRAL = 0x7fff7fff;
    a = pk_min(a, __builtin_amdgcn_mov_dpp(a, 0xB1, 0xF, 0xF, false));            // quad_perm [1,0,3,2]
    b = pk_min(b, __builtin_amdgcn_mov_dpp(b, 0xB1, 0xF, 0xF, false));
    a = pk_min(a, __builtin_amdgcn_mov_dpp(a, 0x4E, 0xF, 0xF, false));            // quad_perm [2,3,0,1]
    b = pk_min(b, __builtin_amdgcn_mov_dpp(b, 0x4E, 0xF, 0xF, false));
    a = pk_min(a, __builtin_amdgcn_mov_dpp(a, 0x141, 0xF, 0xF, false));           // row_half_mirror
    b = pk_min(b, __builtin_amdgcn_mov_dpp(b, 0x141, 0xF, 0xF, false));
    a = pk_min(a, __builtin_amdgcn_mov_dpp(a, 0x140, 0xF, 0xF, false));           // row_mirror
    b = pk_min(b, __builtin_amdgcn_mov_dpp(b, 0x140, 0xF, 0xF, false));
    a = pk_min(a, __builtin_amdgcn_update_dpp(NEUTRAL, a, 0x142, 0xA, 0xF, false));  // row_bcast:15
    b = pk_min(b, __builtin_amdgcn_update_dpp(NEUTRAL, b, 0x142, 0xA, 0xF, false));
    a = pk_min(a, __builtin_amdgcn_update_dpp(NEUTRAL, a, 0x143, 0xC, 0xF, false));  // row_bcast:31
    b = pk_min(b, __builtin_amdgcn_update_dpp(NEUTRAL, b, 0x143, 0xC, 0xF, false));
    a = __builtin_amdgcn_readlane(a, 63);
    b = __builtin_amdgcn_readlane(b, 63);
}

// Inclusive prefix sum over the 64 lanes (all lanes active): Hillis-Steele
// steps of 1, 2, 4 and 8 lanes inside each row of 16 (DPP row_shr; lanes
// shifted in from outside the row add 0), then the last lane of row 0 (and 2)
// is added to row 1 (and 3) and the last lane of row 1 to rows 2 and 3 (DPP
// row_bcast:15 and row_bcast:31).
__device__ __forceinline__ int wave_inclusive_sum(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);   // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);   // row_bcast:31 into rows 2, 3
    return x;
}

__device__ __forceinline__ int pack16(int lo, int hi)
{
    return static_cast<int>((static_cast<unsigned>(lo) & 0xffffu) | (static_cast<unsigned>(hi) << 16));
}
__device__ __forceinline__ int unpack16_lo(int v) { return static_cast<short>(v & 0xffff); }
__device__ __forceinline__ int unpack16_hi(int v) { return v >> 16; }

// The same global buffer seen through the constant address space: loads
// with a wave-uniform index become scalar loads into scalar registers.
template <typename T>
__device__ __forceinline__ const T __attribute__((address_space(4))) *const_space(const T *p)
{
    return (const T __attribute__((address_space(4))) *)reinterpret_cast<unsigned long long>(p);
}

__device__ __forceinline__ int sel3i(int i, int x, int y, int z)
{
    return i == 0 ? x : (i == 1 ? y : z);
}

// Window of one (voxel, slice) hit from the LDS rectangle (row stride RECT)
// whose cell (0, 0) is sample (kx_lo, ky_lo).  The hit's coordinates arrive
// scaled by s = sqrt(table scale), so squared distances are table positions
// directly (on the fly, the scale is 1/a^2: positions are d^2/a^2).  RIM: the
// rectangle reaches the disk edge, so each candidate's |k| < r_max
// membership gates its weight.  PRELOAD: all LDS reads of the window are
// issued before any is consumed.  EXACT: uxs and uys are exact grid-part
// products and uxl, uyl the remainders' products, added once the large parts
// have cancelled (else uxl, uyl are unused).  MODE: the weight source (tab
// holds the table, or on the fly the polynomial's coefficients).
template <int WIN, int ROWS, bool RIM, int MODE, bool PRELOAD, bool EXACT>
__device__ __forceinline__ void window_lds(const float2 *__restrict__ rect, const float *__restrict__ tab,
                                           const Geom &g, float uxs, float uxl, float uys, float uyl, float uzs,
                                           float s, float inv_s, int kx_lo, int ky_lo, int j0, float &pr, float &pi,
                                           float &pw)
{
    constexpr int RECT = SlabShape<WIN>::RECT;
    // largest first-cell offset that keeps the window inside the buffer
    constexpr int MAXOFF = RECT * RECT - 1 - (WIN - 1) * (RECT + 1);
    // first window column / row: ceil(u - a)
    const float fx0 = ceilf(fmaf(EXACT ? uxs + uxl : uxs, inv_s, -g.a));
    const float fy0 = ceilf(fmaf(EXACT ? uys + uyl : uys, inv_s, -g.a));
    // the staged rectangle holds every window; the clamp only guards the buffer
    const int off = min(max(__mul24(static_cast<int>(fy0) - ky_lo, RECT) + (static_cast<int>(fx0) - kx_lo), 0), MAXOFF);
    // rows j0 .. j0 + ROWS - 1 of the window (all of them when ROWS == WIN)
    const float2 *base = rect + off + (ROWS == WIN ? 0 : __mul24(j0, RECT));
    float dxs[WIN], dys[ROWS];
    float dx0 = fmaf(-s, fx0, uxs), dy0 = fmaf(-s, fy0, uys);
    if constexpr (EXACT) {
        // uxs and s fx0 are exact, so the fma rounds once at the size of the
        // offset; then the small remainder
        dx0 += uxl;
        dy0 += uyl;
    }
    const float uz2 = uzs * uzs;
#pragma unroll
    for (int i = 0; i < WIN; ++i) {
        const float dx = i == 0 ? dx0 : fmaf(-s, static_cast<float>(i), dx0);
        dxs[i] = dx * dx;
    }
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
        const float dy = ROWS == WIN ? (j == 0 ? dy0 : fmaf(-s, static_cast<float>(j), dy0))
                                     : fmaf(-s, static_cast<float>(j0 + j), dy0);
        dys[j] = fmaf(dy, dy, uz2);
    }
    // rim gate per cell: kx^2 < r_max^2 - ky^2 (integers below 2^24: exact,
    // so the same test as kx^2 + ky^2 < r_max^2), per column and per row
    float kx2[WIN], rem[ROWS];
    if (RIM) {
#pragma unroll
        for (int i = 0; i < WIN; ++i) {
            const float kx = fx0 + static_cast<float>(i);
            kx2[i] = kx * kx;
        }
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const float ky = fy0 + static_cast<float>(ROWS == WIN ? j : j0 + j);
            rem[j] = fmaf(-ky, ky, g.r2max);
        }
    }
    float sr = 0.f, si = 0.f, sw = 0.f;
    if constexpr (MODE == WEIGHT_OTF) {
        // every cell's s = 1 - d^2/a^2 (clamped at 0: far cells are cut off
        // below and must not feed large powers into Horner's rule), then the
        // polynomial for all cells at once, four coefficients per LDS read
        // (the same address in every lane)
        float sv[ROWS * WIN], acc[ROWS * WIN];
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
#pragma unroll
            for (int i = 0; i < WIN; ++i) {
                sv[j * WIN + i] = fmaxf(1.0f - (dxs[i] + dys[j]), 0.f);
                acc[j * WIN + i] = 0.f;
            }
        for (int c = g.nterms - 4; c >= 0; c -= 4) {
            const float4 k4 = *reinterpret_cast<const float4 *>(tab + c);
#pragma unroll
            for (int k = 0; k < ROWS * WIN; ++k) acc[k] = fmaf(acc[k], sv[k], k4.w);
#pragma unroll
            for (int k = 0; k < ROWS * WIN; ++k) acc[k] = fmaf(acc[k], sv[k], k4.z);
#pragma unroll
            for (int k = 0; k < ROWS * WIN; ++k) acc[k] = fmaf(acc[k], sv[k], k4.y);
#pragma unroll
            for (int k = 0; k < ROWS * WIN; ++k) acc[k] = fmaf(acc[k], sv[k], k4.x);
        }
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
#pragma unroll
            for (int i = 0; i < WIN; ++i) {
                const int k = j * WIN + i;
                // inclusive cut-off d^2 <= a^2
                float w = dxs[i] + dys[j] <= 1.0f ? acc[k] : 0.f;
                if (RIM) w = kx2[i] < rem[j] ? w : 0.f;
                const float2 f2 = base[j * RECT + i];
                sr = fmaf(w, f2.x, sr);
                si = fmaf(w, f2.y, si);
                sw += w;
            }
        pr = sr;
        pi = si;
        pw = sw;
        return;
    }
    constexpr bool LERP = MODE == WEIGHT_LERP;
    auto weight = [&](float tk, float t0k, float t1k, int i, int j) {
        float w;
        if (LERP) {
            const float f = __builtin_amdgcn_fractf(tk);
            // the table lies in [0, 1] and decreases (b(0) = 1), so the lerp
            // never exceeds 1 and clamping to [0, 1] is the cut-off's max(., 0)
            // in one instruction (the fma's clamp modifier)
            w = fminf(fmaxf(fmaf(f, t1k - t0k, t0k), 0.f), 1.f);
        } else {
            w = tk <= static_cast<float>(g.N - 1) ? t0k : 0.f;
        }
        if (RIM) w = kx2[i] < rem[j] ? w : 0.f;
        return w;
    };
    if (PRELOAD) {
        // every LDS read of the window is issued before any is consumed
        float t[ROWS * WIN];
        unsigned idx[ROWS * WIN];
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
#pragma unroll
            for (int i = 0; i < WIN; ++i) {
                t[j * WIN + i] = dxs[i] + dys[j];
                idx[j * WIN + i] = min(static_cast<unsigned>(t[j * WIN + i]), static_cast<unsigned>(g.N));
            }
        float t0[ROWS * WIN], t1[ROWS * WIN];
        float2 fv[ROWS * WIN];
#pragma unroll
        for (int k = 0; k < ROWS * WIN; ++k) {
            t0[k] = tab[idx[k]];
            t1[k] = LERP ? tab[idx[k] + 1] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
#pragma unroll
            for (int i = 0; i < WIN; ++i) fv[j * WIN + i] = base[j * RECT + i];
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
#pragma unroll
            for (int i = 0; i < WIN; ++i) {
                const int k = j * WIN + i;
                const float w = weight(t[k], t0[k], t1[k], i, j);
                sr = fmaf(w, fv[k].x, sr);
                si = fmaf(w, fv[k].y, si);
                sw += w;
            }
    } else {
#pragma unroll
        for (int j = 0; j < ROWS; ++j)
#pragma unroll
            for (int i = 0; i < WIN; ++i) {
                const float tk = dxs[i] + dys[j];
                const unsigned ik = min(static_cast<unsigned>(tk), static_cast<unsigned>(g.N));
                const float w = weight(tk, tab[ik], LERP ? tab[ik + 1] : 0.f, i, j);
                const float2 f2 = base[j * RECT + i];
                sr = fmaf(w, f2.x, sr);
                si = fmaf(w, f2.y, si);
                sw += w;
            }
    }
    pr = sr;
    pi = si;
    pw = sw;
}

// Variant flags of the slab kernel (tuning knobs).
constexpr int SLAB_ATOMIC = 1;    // LDS float atomics for the accumulators (else read-add-write)
constexpr int SLAB_PRELOAD = 2;   // issue all window reads before use
// windows of 5x5 and more keep too many reads in flight; they interleave
template <int WIN>
constexpr int slab_default_flags() { return WIN <= 4 ? SLAB_PRELOAD : 0; }

// MAXW: largest work-group (in waves) the instance is built for; it sets the
// register budget (8 waves: 256 VGPRs, two waves per SIMD; 11 waves: 168
// VGPRs, three waves on three of the four SIMDs).
template <int WIN, int MODE, int FLAGS, int MAXW, bool EXACT, int STORE>
__global__ __launch_bounds__(64 * MAXW) void k_insert_slab(JobTable jt, const float2 *__restrict__ table_g,
                                                     const Item *__restrict__ items, int nitems, int inner_chunk,
                                                     int lane_order, Counters *__restrict__ ctr)
{
    using SS = SlabShape<WIN>;
    constexpr int RECT = SS::RECT;
    constexpr int RECT2 = SS::RECT2;
    constexpr int NC = (RECT2 + 63) / 64;
    extern __shared__ float smem[];
    // blob parameters (and so the table) are common to every job of a launch
    const int N = jt.job[0].g.N;
    float *tab = smem;
    if constexpr (MODE == WEIGHT_OTF) {
        // the polynomial's coefficients, stored after the table
        for (int i = threadIdx.x; i < jt.job[0].g.nterms; i += blockDim.x) tab[i] = table_g[N + i].x;
    } else {
        for (int i = threadIdx.x; i < N; i += blockDim.x) tab[i] = table_g[i].x;
        if (threadIdx.x == 0) {
            const float sentinel = -1073741824.0f * table_g[N - 1].x;
            tab[N] = sentinel;
            tab[N + 1] = sentinel;
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // per-wave region: the staged rectangle first (its base has no constant
    // part, so the window's cell offsets fit the LDS instructions' offset
    // fields), then the accumulators (re, im pairs and weights), then two
    // hit lists
    float *wregion = smem + weight_words(jt.job[0].g, MODE) + wave * SS::WAVE_WORDS;
    float2 *rect = reinterpret_cast<float2 *>(wregion);
    float *accs = wregion + 2 * RECT2;
    float2 *acc_c = reinterpret_cast<float2 *>(accs);
    float *acc_w = accs + 2 * TV;
    unsigned short *list = reinterpret_cast<unsigned short *>(wregion + 2 * RECT2 + ACC_WORDS);

    // Queue positions are taken by lane 0; an item's successor is taken
    // before the item's final writes, so the atomic's round trip overlaps
    // them.  Every wave ends on a position at or past nitems.
    unsigned pos = 0;
    if (lane == 0) pos = atomicAdd(&ctr->queue, 1u);
    for (;;) {
        const unsigned it = __builtin_amdgcn_readfirstlane(pos);
        if (it >= static_cast<unsigned>(nitems)) break;
        const Item item = items[it];
        // the item's reconstruction (job) and its geometry and buffers
        const int job = __builtin_amdgcn_readfirstlane(item.tile >> 24);
        // a job without slices in this launch (a batch whose reconstructions
        // hold different slice counts) adds nothing: its items and their
        // partial sums are skipped
        if (jt.job[job].count == 0) {
            if (lane == 0) pos = atomicAdd(&ctr->queue, 1u);
            continue;
        }
        const int tile = item.tile & 0xffffff;
        const Geom g = jt.job[job].g;
        const void *__restrict__ slices = jt.job[job].slices;
        const Orient *__restrict__ orient = jt.job[job].orient;
        float4 *__restrict__ partials = jt.job[job].partials;
        float2 *__restrict__ G = jt.job[job].G;
        float *__restrict__ W = jt.job[job].W;
        const int count = jt.job[job].count;
        const int TX = (g.h + 1 + TE - 1) / TE;
        const int TY = (g.dim + TE - 1) / TE;
        const size_t slen = static_cast<size_t>(g.n) * g.sw;
        const float rmax = sqrtf(g.r2max);
        // voxels with |v| >= r_max + a receive nothing (every sample has |p| < r_max)
        const float R2 = (rmax + g.a + 1e-3f) * (rmax + g.a + 1e-3f);
        const float a_run = g.a * (1.0f + 1e-5f) + 1e-5f;
        // square root of the table scale (N - 1) / a^2 and its inverse
        const float ts_root = sqrtf(g.tscale);
        const float ts_rinv = 1.0f / ts_root;
        const int tx = tile % TX;
        const int ty = (tile / TX) % TY;
        const int tz = tile / (TX * TY);
        // voxel box of the tile, clipped to the half box
        const int X0 = TE * tx, Y0 = TE * ty - g.h, Z0 = TE * tz - g.h;
        const int X1 = min(X0 + TE - 1, g.h), Y1 = min(Y0 + TE - 1, g.h), Z1 = min(Z0 + TE - 1, g.h);
        const float cx = 0.5f * (X0 + X1), cy = 0.5f * (Y0 + Y1), cz = 0.5f * (Z0 + Z1);
        const float hx = 0.5f * (X1 - X0), hy = 0.5f * (Y1 - Y0), hz = 0.5f * (Z1 - Z0);
        const float reach = rmax + g.a + sqrtf(hx * hx + hy * hy + hz * hz) + 0.01f;
        const float reach2 = reach * reach;
        const int s0 = static_cast<int>(static_cast<long>(count) * item.part / item.nparts);
        const int s1 = static_cast<int>(static_cast<long>(count) * (item.part + 1) / item.nparts);

        for (int k = lane; k < ACC_WORDS; k += 64) accs[k] = 0.f;
        float ore[TV / 64], oim[TV / 64], ow[TV / 64];
#pragma unroll
        for (int k = 0; k < TV / 64; ++k) ore[k] = oim[k] = ow[k] = 0.f;
        int inner = 0;
        wave_sync();

        // Iterator over the item's slices that pass the tile's bin test: a
        // ballot over 64 slices at a time (wave-uniform state).
        int it_base = s0 - 64;
        unsigned long long it_mask = 0ull;
        auto next_slice = [&]() -> int {
            while (it_mask == 0ull) {
                it_base += 64;
                if (it_base >= s1) return -1;
                const int sl = it_base + lane;
                bool pass = false;
                if (sl < s1) {
                    const Orient o = orient[sl];
                    if (o.e1.w != 0.f) {
                        const float dz = fmaf(o.e3.x, cx, fmaf(o.e3.y, cy, o.e3.z * cz));
                        const float ext = fmaf(hx, fabsf(o.e3.x), fmaf(hy, fabsf(o.e3.y), hz * fabsf(o.e3.z)));
                        const float px = fmaf(o.e1.x, cx, fmaf(o.e1.y, cy, o.e1.z * cz));
                        const float py = fmaf(o.e2.x, cx, fmaf(o.e2.y, cy, o.e2.z * cz));
                        pass = fabsf(dz) <= g.a + ext + 1e-3f && fmaf(px, px, py * py) <= reach2;
                    }
                }
                it_mask = __ballot(pass);
            }
            const int b = __builtin_ctzll(it_mask);
            it_mask &= it_mask - 1ull;
            return __builtin_amdgcn_readfirstlane(it_base + b);
        };

        // The slice loop is compiled once per storage type, so no load of
        // one type shares registers with the other's.
        auto slice_loop = [&](auto dt_tag) {
            constexpr int DT = decltype(dt_tag)::value;
            // Per slice with hits: (1) enumerate the tile's voxels inside the
            // slab into a hit list and bound their windows; (2) issue the loads
            // of exactly that rectangle of samples; (3) commit it to LDS; (4) run
            // the windows.  The next slice's (1) and (2) run before this slice's
            // (4), so its loads are in flight while these windows are evaluated
            // (two hit lists alternate).
            struct Stage {
                float4 e1s, e2s, e3s;        // axes in table units; .w: axis order, 1/e3[d], e3[d]
                float4 p1, p2;               // e1, e2 along (d, ia, ib); .w: e3[ia], e3[ib]
                float4 b1, b2, b3;           // remainders of the scaled axes (exact geometry)
                int kx_lo, ky_lo, wx, wy;    // staged rectangle: columns kx_lo.., rows ky_lo..
                int rim;                     // int, not bool: no padding bytes in the struct copies
                int fast;                    // staging: 1 all direct, -1 all mirrored (inside the disk), 0 mixed
                int H;                       // hits
                int nq;                      // loads per lane
                float scale;
            };
            // cell[] holds the raw sample words between issue and commit: the
            // complex64 value, or the packed 16-bit pair in .x.  Decoding waits
            // for the loads, so it happens at commit.
            float2 cell[NC];
            int neg[NC];      // mixed staging: the sample is mirrored (conjugated at commit)
            // Staged cells: rows of RECT cells, cell c = 64 q + lane of load q at
            // row c / RECT, column c % RECT, so its LDS slot is c itself.  Its
            // offset within the slice relative to the rectangle's first sample
            // (row stride sw) is a constant of the item.
            constexpr int eb = DT == 0 ? 8 : 4;
            int loff[NC];
#pragma unroll
            for (int qq = 0; qq < NC; ++qq) {
                const int c = qq * 64 + lane;
                loff[qq] = (__mul24(c / RECT, g.sw) + c % RECT) * eb;
            }

            auto setup = [&](int s, Stage &st) {
                // s is wave-uniform: the orientation and scale are read with scalar
                // loads (constant address space) straight into scalar registers, so
                // no later copy of the stage waits on the sample loads
                // (the slab kernel's per-slice constants, words 12..31 of the record)
                const float __attribute__((address_space(4))) *o =
                    const_space(reinterpret_cast<const float *>(orient)) + static_cast<long>(s) * (sizeof(Orient) / 4);
                st.e1s = make_float4(o[12], o[13], o[14], o[15]);
                st.e2s = make_float4(o[16], o[17], o[18], o[19]);
                st.e3s = make_float4(o[20], o[21], o[22], o[23]);
                st.p1 = make_float4(o[24], o[25], o[26], o[27]);
                st.p2 = make_float4(o[28], o[29], o[30], o[31]);
                if constexpr (EXACT) {
                    const float __attribute__((address_space(4))) *rm =
                        const_space(reinterpret_cast<const float *>(jt.job[job].rem)) + static_cast<long>(s) * 12;
                    st.b1 = make_float4(rm[0], rm[1], rm[2], 0.f);
                    st.b2 = make_float4(rm[4], rm[5], rm[6], 0.f);
                    st.b3 = make_float4(rm[8], rm[9], rm[10], 0.f);
                }
                st.scale = g.scales ? const_space(g.scales)[s] : 1.0f;
            };

            // (1) Voxels inside the slab |e3.v| <= a (and inside the reach sphere
            // |v| < r_max + a): lane = one of the 64 columns of the tile along
            // the normal's dominant axis, whose run is a contiguous range; a wave
            // prefix scan packs the runs into the list.  The rectangle holds every
            // window [ceil(u - a), ceil(u - a) + WIN - 1] of the hits, with 1e-3
            // of slack for rounding (u is linear along a run, so the run's end
            // voxels bound it).  Returns the hit count.
            auto enumerate = [&](Stage &st, unsigned short *lst) -> int {
                // axis order and normal components, precomputed per slice
                const int axes = __float_as_int(st.e1s.w);
                const int d = axes & 0xff, ia = (axes >> 8) & 0xff, ib = axes >> 16;
                const float na = st.p1.w, nb = st.p2.w;
                const int D0 = sel3i(d, X0, Y0, Z0), D1 = sel3i(d, X1, Y1, Z1);
                const int A0 = sel3i(ia, X0, Y0, Z0), A1 = sel3i(ia, X1, Y1, Z1);
                const int B0 = sel3i(ib, X0, Y0, Z0), B1 = sel3i(ib, X1, Y1, Z1);
                const int sd = sel3i(d, 1, TE, TE * TE);
                const int sa = sel3i(ia, 1, TE, TE * TE);
                const int sb = sel3i(ib, 1, TE, TE * TE);
                // lane_order 0: the first in-plane axis varies fastest across the
                // lanes (and so along the hit list), 1: the second
                const int cs = lane_order ? 3 : 0;
                const int ca = (lane >> cs) & (TE - 1), cb = (lane >> (3 - cs)) & (TE - 1);
                const int va = A0 + ca, vb = B0 + cb;
                const float fva = static_cast<float>(va), fvb = static_cast<float>(vb);
                const float rem = R2 - fmaf(fva, fva, fvb * fvb);
                const bool col_in = va <= A1 && vb <= B1 && rem >= 0.f;
                // hardware square root: R2 carries far more slack than its last-bit
                // error
                const float lim = __builtin_amdgcn_sqrtf(fmaxf(rem, 0.f));
                const float q = fmaf(na, fva, nb * fvb);
                const float inv = st.e2s.w;                  // 1 / e3[d]
                const float t1 = (-a_run - q) * inv, t2 = (a_run - q) * inv;
                const int lo = max(static_cast<int>(ceilf(fmaxf(fminf(t1, t2), -lim))), D0);
                const int hi = min(static_cast<int>(floorf(fminf(fmaxf(t1, t2), lim))), D1);
                const int cnt = col_in ? max(hi - lo + 1, 0) : 0;
                const int incl = wave_inclusive_sum(cnt);
                const int H = __builtin_amdgcn_readlane(incl, 63);
                st.H = H;
                if (H == 0) return 0;
                const int excl = incl - cnt;
                const int lid0 = __mul24(ca, sa) + __mul24(cb, sb) + __mul24(lo - D0, sd);
                // a run never exceeds the tile edge: a fixed, predicated loop
#pragma unroll
                for (int k = 0; k < TE; ++k)
                    if (k < cnt) lst[excl + k] = static_cast<unsigned short>(lid0 + k * sd);
                // Bounds of the hits' windows from the ends of each column's run: u
                // along a column is u(va, vb) + k e_d, and the 1e-3 slack covers the
                // rounding against the windows' own evaluation.  Every lane computes;
                // columns without hits give the neutral 0x7fff.  |coordinates| stay
                // below n / 2 + 8 <= 520, so they fit in int16.
                const float e1d = st.p1.x, e1a = st.p1.y, e1b = st.p1.z;
                const float e2d = st.p2.x, e2a = st.p2.y, e2b = st.p2.z;
                const float am = g.a + 1e-3f, ap = g.a - 1e-3f;
                const float uxc = fmaf(e1a, fva, e1b * fvb), uyc = fmaf(e2a, fva, e2b * fvb);
                const float flo = static_cast<float>(lo), fhi = static_cast<float>(hi);
                const float ux0 = fmaf(flo, e1d, uxc), ux1 = fmaf(fhi, e1d, uxc);
                const float uy0 = fmaf(flo, e2d, uyc), uy1 = fmaf(fhi, e2d, uyc);
                const int xl = static_cast<int>(floorf(fminf(ux0, ux1) - am));
                const int xh = static_cast<int>(ceilf(fmaxf(ux0, ux1) - ap)) + (WIN - 1);
                const int yl = static_cast<int>(floorf(fminf(uy0, uy1) - am));
                const int yh = static_cast<int>(ceilf(fmaxf(uy0, uy1) - ap)) + (WIN - 1);
                int lows = cnt > 0 ? pack16(xl, yl) : 0x7fff7fff;
                int highs = cnt > 0 ? pack16(-xh, -yh) : 0x7fff7fff;
                wave_min_pk2(lows, highs);
                st.kx_lo = unpack16_lo(lows);
                st.ky_lo = unpack16_hi(lows);
                // never wider than RECT; min() only guards the buffer
                st.wx = min(-unpack16_lo(highs) - st.kx_lo + 1, RECT);
                st.wy = min(-unpack16_hi(highs) - st.ky_lo + 1, RECT);
                const int fxm = max(abs(st.kx_lo), abs(st.kx_lo + st.wx - 1));
                const int fym = max(abs(st.ky_lo), abs(st.ky_lo + st.wy - 1));
                st.rim = static_cast<float>(fxm * fxm + fym * fym) < g.r2max ? 0 : 1;
                // inside the disk and on one side of kx = 0: every sample comes
                // from one run of rows, directly (kx >= 1) or mirrored (kx <= -1)
                st.fast = st.rim ? 0 : (st.kx_lo >= 1 ? 1 : (st.kx_lo + st.wx <= 0 ? -1 : 0));
                st.nq = (RECT * st.wy + 63) >> 6;
                return H;
            };

            // (2) loads of the staged rows, Hermitian rule and disk applied
            auto issue = [&](int s, const Stage &st) {
                // buffer resource over this slice: 32-bit offsets, hardware bounds check
                // (reads at or past the record size return zero: cells outside
                // the disk are loaded from there and so stage as zero)
                const int bytes = static_cast<int>(slen * eb);
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<unsigned char *>(static_cast<const unsigned char *>(slices) +
                                                static_cast<size_t>(s) * slen * eb),
                    static_cast<short>(0), bytes, 0x00020000);
                int off[NC];
                if (st.fast != 0) {
                    // one run of rows: direct samples at row ky + h, column kx;
                    // mirrored ones at row h - ky, column -kx, i.e. the same
                    // offsets counted backwards from the first sample's mirror.
                    // Cells right of the rectangle may wrap into the next stored
                    // row and cells below it may fall past the slice (zero); no
                    // window reads them.
                    const int base = st.fast > 0 ? (__mul24(st.ky_lo + g.h, g.sw) + st.kx_lo) * eb
                                                 : (__mul24(g.h - st.ky_lo, g.sw) - st.kx_lo) * eb;
    #pragma unroll
                    for (int qq = 0; qq < NC; ++qq) off[qq] = st.fast > 0 ? base + loff[qq] : base - loff[qq];
                } else {
    #pragma unroll
                    for (int qq = 0; qq < NC; ++qq) {
                        if (qq >= st.nq) break;
                        const int c = qq * 64 + lane;
                        const int cy_ = c / RECT, cx_ = c % RECT;
                        const int kx = st.kx_lo + cx_, ky = st.ky_lo + cy_;
                        // (operands below 2^11: 24-bit multiplies run at full rate)
                        const bool valid = cx_ < st.wx && cy_ < st.wy &&
                                           static_cast<float>(__mul24(kx, kx) + __mul24(ky, ky)) < g.r2max;
                        const bool direct = kx > 0 || (kx == 0 && ky >= 0);
                        const int row = direct ? ky + g.h : g.h - ky;
                        const int col = direct ? kx : -kx;
                        off[qq] = valid ? (__mul24(row, g.sw) + col) * eb : bytes;
                        // the sign flip of mirrored samples is applied at commit
                        neg[qq] = direct ? 0 : 1;
                    }
                }
                // all loads back to back; only as many as the rectangle's rows
                // need (st.nq is wave-uniform)
                if constexpr (DT == 0) {
    #pragma unroll
                    for (int qq = 0; qq < NC; ++qq)
                        if (qq < st.nq)
                            cell[qq] = __builtin_bit_cast(float2,
                                                          __builtin_amdgcn_raw_buffer_load_b64(rs, off[qq], 0, 0));
                } else {
    #pragma unroll
                    for (int qq = 0; qq < NC; ++qq)
                        if (qq < st.nq)
                            cell[qq].x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off[qq], 0, 0));
                }
            };

            // (3) decode and write the staged samples to LDS (cell c to slot c;
            // the last load's lanes past the rectangle write nothing)
            auto commit = [&](const Stage &st) {
    #pragma unroll
                for (int qq = 0; qq < NC; ++qq) {
                    const int c = qq * 64 + lane;
                    if (qq < st.nq && (qq < NC - 1 || c < RECT2)) {
                        float2 v;
                        if constexpr (DT == 0) {
                            v = cell[qq];
                        } else {
                            const unsigned raw = __float_as_uint(cell[qq].x);
                            if constexpr (DT == 1) {
                                const _Float16 lo = __builtin_bit_cast(_Float16, static_cast<unsigned short>(raw & 0xffffu));
                                const _Float16 hi = __builtin_bit_cast(_Float16, static_cast<unsigned short>(raw >> 16));
                                v = make_float2(static_cast<float>(lo) * st.scale, static_cast<float>(hi) * st.scale);
                            } else {
                                v = make_float2(__uint_as_float(raw << 16), __uint_as_float(raw & 0xffff0000u));
                            }
                        }
                        if (st.fast < 0 || (st.fast == 0 && neg[qq])) v.y = -v.y;
                        rect[c] = v;
                    }
                }
            };

            // next slice of the item that has hits: enumerated into lst, loads issued
            auto advance = [&](Stage &st, unsigned short *lst) -> int {
                for (;;) {
                    const int s = next_slice();
                    if (s < 0) return -1;
                    setup(s, st);
                    if (enumerate(st, lst) > 0) {
                        issue(s, st);
                        return s;
                    }
                }
            };

            Stage cur, nxt;
            unsigned short *list_cur = list, *list_nxt = list + TV;
            int s = advance(cur, list_cur);
            while (s >= 0) {
                commit(cur);
                const int s_next = advance(nxt, list_nxt);
                wave_sync();

                // (4) windows of the hits, 64 per round
                const int H = cur.H;
                // slice axes in table units
                const float4 e1s = cur.e1s, e2s = cur.e2s, e3s = cur.e3s;
                // (remainders: read only with exact geometry)
                const float4 b1 = cur.b1, b2 = cur.b2, b3 = cur.b3;
                // One round: hits r .. r + 64 / K - 1, K lanes per hit (the lanes
                // of a quad), each evaluating WIN / K rows of the window; the K
                // partial sums are added across the lanes (DPP within the quad)
                // and the first lane of each hit updates the voxel's
                // accumulator.  Full rounds take K = 1; a last round of at most
                // 32 (16) hits takes K = 2 (4), so its lanes are not left idle.
                auto round = [&](auto kk, int r) {
                    constexpr int K = decltype(kk)::value;
                    constexpr int LK = K == 1 ? 0 : (K == 2 ? 1 : 2);
                    constexpr int ROWS = WIN / K;
                    constexpr bool PRE = (FLAGS & SLAB_PRELOAD) != 0 && K == 1;
                    const int hh = r + (lane >> LK);
                    const int part = lane & (K - 1);
                    float pr = 0.f, pi = 0.f, pw = 0.f;
                    int lid = 0;
                    if (hh < H) {
                        lid = list_cur[hh];
                        const float vx = static_cast<float>(X0 + (lid & 7));
                        const float vy = static_cast<float>(Y0 + ((lid >> 3) & 7));
                        const float vz = static_cast<float>(Z0 + (lid >> 6));
                        const float uxs = fmaf(e1s.x, vx, fmaf(e1s.y, vy, e1s.z * vz));
                        const float uys = fmaf(e2s.x, vx, fmaf(e2s.y, vy, e2s.z * vz));
                        const float uzs = fmaf(e3s.x, vx, fmaf(e3s.y, vy, e3s.z * vz));
                        float uxl = 0.f, uyl = 0.f, uz = uzs;
                        if constexpr (EXACT) {
                            uxl = fmaf(b1.x, vx, fmaf(b1.y, vy, b1.z * vz));
                            uyl = fmaf(b2.x, vx, fmaf(b2.y, vy, b2.z * vz));
                            uz += fmaf(b3.x, vx, fmaf(b3.y, vy, b3.z * vz));
                        }
                        // The rectangle reaches the disk edge: gate each window
                        // cell by |k| < r_max only in rounds where some hit's
                        // window reaches it, i.e. where the window's farthest
                        // corner (columns ceil(u_x - a) .. + WIN - 1, likewise
                        // rows; the window's own origins, remainders included)
                        // lies outside.
                        bool rim_round = false;
                        if (cur.rim) {
                            const float fx0 = ceilf(fmaf(EXACT ? uxs + uxl : uxs, ts_rinv, -g.a));
                            const float fy0 = ceilf(fmaf(EXACT ? uys + uyl : uys, ts_rinv, -g.a));
                            const float fx1 = fx0 + static_cast<float>(WIN - 1), fy1 = fy0 + static_cast<float>(WIN - 1);
                            const float mx = fmaxf(fx0 * fx0, fx1 * fx1), my = fmaxf(fy0 * fy0, fy1 * fy1);
                            rim_round = __ballot(mx + my >= g.r2max) != 0ull;
                        }
                        const int j0 = part * ROWS;
                        if (rim_round)
                            window_lds<WIN, ROWS, true, MODE, PRE, EXACT>(rect, tab, g, uxs, uxl, uys, uyl, uz,
                                                                          ts_root, ts_rinv, cur.kx_lo, cur.ky_lo,
                                                                          j0, pr, pi, pw);
                        else
                            window_lds<WIN, ROWS, false, MODE, PRE, EXACT>(rect, tab, g, uxs, uxl, uys, uyl, uz,
                                                                           ts_root, ts_rinv, cur.kx_lo, cur.ky_lo,
                                                                           j0, pr, pi, pw);
                    }
                    if constexpr (K > 1) {
                        // every lane takes part (idle ones with zeros)
                        auto swap1 = [](float v) {     // quad_perm [1,0,3,2]
                            return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF,
                                                                               false));
                        };
                        auto swap2 = [](float v) {     // quad_perm [2,3,0,1]
                            return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF,
                                                                               false));
                        };
                        pr = swap1(pr);
                        pi = swap1(pi);
                        pw = swap1(pw);
                        if constexpr (K == 4) {
                            pr = swap2(pr);
                            pi = swap2(pi);
                            pw = swap2(pw);
                        }
                    }
                    if (hh < H && part == 0) {
                        // a voxel appears once per slice: single writer within the wave
                        if (FLAGS & SLAB_ATOMIC) {
                            atomicAdd(&acc_c[lid].x, pr);
                            atomicAdd(&acc_c[lid].y, pi);
                            atomicAdd(acc_w + lid, pw);
                        } else {
                            float2 c = acc_c[lid];
                            c.x += pr;
                            c.y += pi;
                            acc_c[lid] = c;
                            acc_w[lid] += pw;
                        }
                    }
                };
                const int full = H & ~63;
                for (int r = 0; r < full; r += 64) round(std::integral_constant<int, 1>{}, r);
                const int tail = H - full;
                if (tail > 0) {
                    bool done = false;
                    if constexpr (WIN % 4 == 0) {
                        if (tail <= 16) {
                            round(std::integral_constant<int, 4>{}, full);
                            done = true;
                        }
                    }
                    if constexpr (WIN % 2 == 0) {
                        if (!done && tail <= 32) {
                            round(std::integral_constant<int, 2>{}, full);
                            done = true;
                        }
                    }
                    if (!done) round(std::integral_constant<int, 1>{}, full);
                }
                wave_sync();
                if (++inner == inner_chunk) {
    #pragma unroll
                    for (int k = 0; k < TV / 64; ++k) {
                        const int lid = lane + 64 * k;
                        const float2 c = acc_c[lid];
                        ore[k] += c.x;
                        oim[k] += c.y;
                        ow[k] += acc_w[lid];
                        acc_c[lid] = make_float2(0.f, 0.f);
                        acc_w[lid] = 0.f;
                    }
                    inner = 0;
                    wave_sync();
                }
                cur = nxt;
                unsigned short *t = list_cur;
                list_cur = list_nxt;
                list_nxt = t;
                s = s_next;
            }
        };
        slice_loop(std::integral_constant<int, STORE>{});
#pragma unroll
        for (int k = 0; k < TV / 64; ++k) {
            const int lid = lane + 64 * k;
            const float2 c = acc_c[lid];
            ore[k] += c.x;
            oim[k] += c.y;
            ow[k] += acc_w[lid];
        }
        wave_sync();
        if (lane == 0) pos = atomicAdd(&ctr->queue, 1u);
        if (item.nparts == 1) {
            // all reads first, then all writes: G and W may not be proven
            // disjoint, and interleaving would serialise every read
            float2 gv[TV / 64];
            float wv[TV / 64];
            size_t vi[TV / 64];
            bool in[TV / 64];
#pragma unroll
            for (int k = 0; k < TV / 64; ++k) {
                const int lid = lane + 64 * k;
                const int ix = X0 + (lid & 7);
                const int iy = Y0 + ((lid >> 3) & 7) + g.h;
                const int iz = Z0 + (lid >> 6) + g.h;
                in[k] = ix <= g.h && iy < g.dim && iz < g.dim;
                vi[k] = (static_cast<size_t>(iz) * g.dim + iy) * g.dim + (ix + g.h);
                if (in[k]) {
                    gv[k] = G[vi[k]];
                    wv[k] = W[vi[k]];
                }
            }
#pragma unroll
            for (int k = 0; k < TV / 64; ++k) {
                if (in[k]) {
                    G[vi[k]] = make_float2(gv[k].x + ore[k], gv[k].y + oim[k]);
                    W[vi[k]] = wv[k] + ow[k];
                }
            }
        } else {
            // partial sums of a split tile: three planes (re, im, w) of TV
            // floats per slot, so the stores and the reduction's loads are
            // coalesced dwords with no padding
            float *__restrict__ pp = reinterpret_cast<float *>(partials) + static_cast<size_t>(item.slot) * 3 * TV;
#pragma unroll
            for (int k = 0; k < TV / 64; ++k) {
                const int lid = lane + 64 * k;
                pp[lid] = ore[k];
                pp[TV + lid] = oim[k];
                pp[2 * TV + lid] = ow[k];
            }
        }
    }
}

template <int WIN, int MODE, int FLAGS, bool EXACT, int MAXW = 8>
hipError_t launch_slab_t(const JobTable &jt, const float2 *table, const Item *items, int nitems, int inner_chunk,
                         int lane_order, int blocks, int wpb, Counters *ctr, hipStream_t st)
{
    const size_t lds = (static_cast<size_t>(weight_words(jt.job[0].g, MODE)) +
                        static_cast<size_t>(wpb) * SlabShape<WIN>::WAVE_WORDS) * sizeof(float);
    if (wpb > MAXW) return hipErrorInvalidConfiguration;
    // one instance per slice storage type (every job of a launch shares it)
    switch (jt.job[0].g.dtype) {
    case 0:
        hipLaunchKernelGGL((k_insert_slab<WIN, MODE, FLAGS, MAXW, EXACT, 0>), dim3(blocks), dim3(64 * wpb), lds, st, jt,
                           table, items, nitems, inner_chunk, lane_order, ctr);
        break;
    case 1:
        hipLaunchKernelGGL((k_insert_slab<WIN, MODE, FLAGS, MAXW, EXACT, 1>), dim3(blocks), dim3(64 * wpb), lds, st, jt,
                           table, items, nitems, inner_chunk, lane_order, ctr);
        break;
    case 2:
        hipLaunchKernelGGL((k_insert_slab<WIN, MODE, FLAGS, MAXW, EXACT, 2>), dim3(blocks), dim3(64 * wpb), lds, st, jt,
                           table, items, nitems, inner_chunk, lane_order, ctr);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Adds the partial sums of split 8x8x8 tiles, in part order, into G and W
// (one work-group per entry of the list of split tiles).
__global__ __launch_bounds__(512) void k_reduce_partials8(JobTable jt, const Item *__restrict__ items)
{
    const Item item = items[blockIdx.x];
    if (item.nparts == 1 || item.part != 0) return;
    const int job = item.tile >> 24;
    if (jt.job[job].count == 0) return;    // skipped by the insertion kernel too
    const int tile = item.tile & 0xffffff;
    const Geom g = jt.job[job].g;
    const float *__restrict__ partials = reinterpret_cast<const float *>(jt.job[job].partials);
    float2 *__restrict__ G = jt.job[job].G;
    float *__restrict__ W = jt.job[job].W;
    const int lid = threadIdx.x;
    const int TX = (g.h + 1 + TE - 1) / TE;
    const int TY = (g.dim + TE - 1) / TE;
    const int tx = tile % TX;
    const int ty = (tile / TX) % TY;
    const int tz = tile / (TX * TY);
    const int ix = TE * tx + (lid & 7);
    const int iy = TE * ty + ((lid >> 3) & 7);
    const int iz = TE * tz + (lid >> 6);
    if (!(ix <= g.h && iy < g.dim && iz < g.dim)) return;
    float re = 0.f, im = 0.f, w = 0.f;
    // sums in part order; the loads of several parts are in flight together
#pragma unroll 4
    for (int k = 0; k < item.nparts; ++k) {
        const float *__restrict__ pp = partials + static_cast<size_t>(item.slot + k) * 3 * TV;
        re += pp[lid];
        im += pp[TV + lid];
        w += pp[2 * TV + lid];
    }
    const size_t vi = (static_cast<size_t>(iz) * g.dim + iy) * g.dim + (ix + g.h);
    float2 gv = G[vi];
    gv.x += re;
    gv.y += im;
    G[vi] = gv;
    W[vi] += w;
}

}  // namespace

size_t slab_lds_bytes(const Geom &g, int mode, int waves_per_block)
{
    const int win = static_cast<int>(floorf(2.0f * g.a)) + 1;
    return (static_cast<size_t>(weight_words(g, mode)) +
            static_cast<size_t>(waves_per_block) * slab_wave_words(win)) * sizeof(float);
}

template <bool EXACT>
static hipError_t dispatch_slab(const JobTable &jt, int mode, int flags, const float2 *table, const Item *items,
                                int nitems, int inner_chunk, int lane_order, int blocks, int wpb, Counters *ctr,
                                hipStream_t st)
{
#define RECON_SLAB_ARGS jt, table, items, nitems, inner_chunk, lane_order, blocks, wpb, ctr, st
    const Geom &g = jt.job[0].g;
    const int win = static_cast<int>(floorf(2.0f * g.a)) + 1;
    if (mode == WEIGHT_OTF) {
        // on the fly: 8-wave instances (at most), window reads interleaved;
        // LDS float atomics as a knob for the common window
        if (win == 4 && (flags & SLAB_ATOMIC)) return launch_slab_t<4, WEIGHT_OTF, SLAB_ATOMIC, EXACT>(RECON_SLAB_ARGS);
        switch (win) {
        case 3: return launch_slab_t<3, WEIGHT_OTF, 0, EXACT>(RECON_SLAB_ARGS);
        case 4: return launch_slab_t<4, WEIGHT_OTF, 0, EXACT>(RECON_SLAB_ARGS);
        case 5: return launch_slab_t<5, WEIGHT_OTF, 0, EXACT>(RECON_SLAB_ARGS);
        case 6: return launch_slab_t<6, WEIGHT_OTF, 0, EXACT>(RECON_SLAB_ARGS);
        default: return hipErrorInvalidValue;
        }
    }
    const bool lerp = mode == WEIGHT_LERP;
    // every flag combination exists for the common window (a in [1.5, 2)) with
    // linear interpolation; other windows and truncation use the default flags
    if (win == 4 && lerp && wpb > 8) {
        // three waves per SIMD: register budget of 168, window reads interleaved
        if (flags & SLAB_ATOMIC) return launch_slab_t<4, WEIGHT_LERP, SLAB_ATOMIC, EXACT, 11>(RECON_SLAB_ARGS);
        return launch_slab_t<4, WEIGHT_LERP, 0, EXACT, 11>(RECON_SLAB_ARGS);
    }
    if (win == 4 && lerp) {
        switch (flags & 3) {
        case 0: return launch_slab_t<4, WEIGHT_LERP, 0, EXACT>(RECON_SLAB_ARGS);
        case 1: return launch_slab_t<4, WEIGHT_LERP, 1, EXACT>(RECON_SLAB_ARGS);
        case 2: return launch_slab_t<4, WEIGHT_LERP, 2, EXACT>(RECON_SLAB_ARGS);
        default: return launch_slab_t<4, WEIGHT_LERP, 3, EXACT>(RECON_SLAB_ARGS);
        }
    }
#define RECON_SLAB_CASE(WV)                                                                                   \
    case WV:                                                                                                  \
        return lerp ? launch_slab_t<WV, WEIGHT_LERP, slab_default_flags<WV>(), EXACT>(RECON_SLAB_ARGS)        \
                    : launch_slab_t<WV, WEIGHT_TRUNC, slab_default_flags<WV>(), EXACT>(RECON_SLAB_ARGS);
    switch (win) {
        RECON_SLAB_CASE(3)
        RECON_SLAB_CASE(4)
        RECON_SLAB_CASE(5)
        RECON_SLAB_CASE(6)
    default:
        return hipErrorInvalidValue;
    }
#undef RECON_SLAB_CASE
#undef RECON_SLAB_ARGS
}

hipError_t launch_insert_slab(const JobTable &jt, int mode, int flags, bool exact, const float2 *table,
                              const Item *items, int nitems, int inner_chunk, int lane_order, int blocks, int wpb,
                              Counters *ctr, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    return exact ? dispatch_slab<true>(jt, mode, flags, table, items, nitems, inner_chunk, lane_order, blocks, wpb,
                                       ctr, st)
                 : dispatch_slab<false>(jt, mode, flags, table, items, nitems, inner_chunk, lane_order, blocks, wpb,
                                        ctr, st);
}

hipError_t launch_reduce_partials8(const JobTable &jt, const Item *items, int nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials8, dim3(nitems), dim3(TV), 0, st, jt, items);
    return hipGetLastError();
}

}  // namespace recon
