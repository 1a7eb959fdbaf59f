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
//      1. stages the (WIN+16)^2 rectangle of the slice that the tile's
//         windows can touch into LDS, resolving the Hermitian half plane and
//         the |k| < r_max disk once per sample (zero outside the disk);
//      2. enumerates exactly the voxels inside the slab: lane = one of the
//         64 columns of the tile along the normal's dominant axis, whose slab
//         run is a contiguous range; a wave prefix scan packs the runs into a
//         hit list;
//      3. processes the hits 64 per round, each lane evaluating the
//         branch-free WIN x WIN window from LDS (blob table lerp from LDS)
//         and adding its partial sums to the voxel's LDS accumulator.
//  * Two-level FP32 accumulation: LDS accumulators hold at most
//    `inner_chunk` slices before they are folded into per-lane registers.
#include "kernels.hpp"

namespace recon {

namespace {

constexpr int TE = 8;                  // tile edge
constexpr int TV = TE * TE * TE;       // voxels per tile
constexpr int ACC_WORDS = 3 * TV;      // re[512], im[512], w[512]
constexpr int LIST_WORDS = TV / 2;     // 512 uint16 voxel ids

template <int WIN>
struct SlabShape {
    // The rectangle must hold every window of the tile: its width is at most
    // 2 * ext + 2a + 4 with ext <= 3.5 * sqrt(3) (half the tile diagonal
    // projected on a slice axis) and WIN = floor(2a) + 1, so WIN + 17 cells
    // always suffice.
    static constexpr int RECT = WIN + 17;
    static constexpr int RECT2 = RECT * RECT;
    static constexpr int WAVE_WORDS = ACC_WORDS + 2 * RECT2 + LIST_WORDS;
};

// Table in LDS: T[0..N-1], then two sentinels T[N] = T[N+1] = -2^20 T[N-1].
// With i = min(floor(t), N) and w = max(T[i] + frac(t) (T[i+1] - T[i]), 0),
// t = N-1 gives exactly T[N-1], and any representable t > N-1 gives 0 (the
// sentinel slope exceeds T[N-1] by 2^20 while frac(t) >= 2^-10 there), so the
// blob's inclusive cut-off at d^2 = a^2 costs no compare.
__host__ __device__ inline int table_words(int N) { return (N + 2 + 3) & ~3; }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float uniformf(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ float4 uniform4(float4 v)
{
    return make_float4(uniformf(v.x), uniformf(v.y), uniformf(v.z), uniformf(v.w));
}

__device__ __forceinline__ float sel3(int i, float x, float y, float z)
{
    return i == 0 ? x : (i == 1 ? y : z);
}
__device__ __forceinline__ int sel3i(int i, int x, int y, int z)
{
    return i == 0 ? x : (i == 1 ? y : z);
}

// Window of one (voxel, slice) hit from the LDS rectangle (row stride RECT)
// whose cell (0, 0) is sample (kx_lo, ky_lo).  All LDS reads of the window
// are issued before any is consumed.  RIM: the rectangle reaches the disk
// edge, so each candidate's |k| < r_max membership gates its weight.
template <int WIN, bool RIM, bool LERP, bool PRELOAD>
__device__ __forceinline__ void window_lds(const float2 *__restrict__ rect, const float *__restrict__ tab,
                                           const Geom &g, float ux, float uy, float uz, float kx_lo,
                                           float ky_lo, float &pr, float &pi, float &pw)
{
    constexpr int RECT = SlabShape<WIN>::RECT;
    const float span = static_cast<float>(RECT - WIN);
    // first window column / row as floats, kept inside the staged rectangle
    const float fx0 = fminf(fmaxf(ceilf(ux - g.a), kx_lo), kx_lo + span);
    const float fy0 = fminf(fmaxf(ceilf(uy - g.a), ky_lo), ky_lo + span);
    const int ox = static_cast<int>(fx0 - kx_lo);
    const int oy = static_cast<int>(fy0 - ky_lo);
    const float2 *base = rect + oy * RECT + ox;
    const float ts = g.tscale;
    float dxs[WIN], dys[WIN];
    const float uzs = uz * uz;
#pragma unroll
    for (int i = 0; i < WIN; ++i) {
        const float dx = ux - (fx0 + static_cast<float>(i));
        dxs[i] = dx * dx * ts;
        const float dy = uy - (fy0 + static_cast<float>(i));
        dys[i] = fmaf(dy, dy, uzs) * ts;
    }
    float sr = 0.f, si = 0.f, sw = 0.f;
    auto weight = [&](float tk, float t0k, float t1k, int i, int j) {
        float w;
        if (LERP) {
            const float f = __builtin_amdgcn_fractf(tk);
            w = fmaxf(fmaf(f, t1k - t0k, t0k), 0.f);
        } else {
            w = tk <= static_cast<float>(g.N - 1) ? t0k : 0.f;
        }
        if (RIM) {
            const float kx = fx0 + static_cast<float>(i), ky = fy0 + static_cast<float>(j);
            w = fmaf(kx, kx, ky * ky) < g.r2max ? w : 0.f;
        }
        return w;
    };
    if (PRELOAD) {
        // every LDS read of the window is issued before any is consumed
        float t[WIN * WIN];
        unsigned idx[WIN * WIN];
#pragma unroll
        for (int j = 0; j < WIN; ++j)
#pragma unroll
            for (int i = 0; i < WIN; ++i) {
                t[j * WIN + i] = dxs[i] + dys[j];
                idx[j * WIN + i] = min(static_cast<unsigned>(t[j * WIN + i]), static_cast<unsigned>(g.N));
            }
        float t0[WIN * WIN], t1[WIN * WIN];
        float2 fv[WIN * WIN];
#pragma unroll
        for (int k = 0; k < WIN * WIN; ++k) {
            t0[k] = tab[idx[k]];
            t1[k] = LERP ? tab[idx[k] + 1] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < WIN; ++j)
#pragma unroll
            for (int i = 0; i < WIN; ++i) fv[j * WIN + i] = base[j * RECT + i];
#pragma unroll
        for (int j = 0; j < WIN; ++j)
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
        for (int j = 0; j < WIN; ++j)
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

template <int WIN, bool LERP, int FLAGS>
__global__ __launch_bounds__(512) void k_insert_slab(JobTable jt, const float2 *__restrict__ table_g,
                                                     const Item *__restrict__ items, int nitems, int inner_chunk,
                                                     Counters *__restrict__ ctr)
{
    using SS = SlabShape<WIN>;
    constexpr int RECT = SS::RECT;
    constexpr int RECT2 = SS::RECT2;
    constexpr int NC = (RECT2 + 63) / 64;
    extern __shared__ float smem[];
    // blob parameters (and so the table) are common to every job of a launch
    const int N = jt.job[0].g.N;
    float *tab = smem;
    for (int i = threadIdx.x; i < N; i += blockDim.x) tab[i] = table_g[i].x;
    if (threadIdx.x == 0) {
        const float sentinel = -1048576.0f * table_g[N - 1].x;
        tab[N] = sentinel;
        tab[N + 1] = sentinel;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    float *wregion = smem + table_words(N) + wave * SS::WAVE_WORDS;
    float *acc_re = wregion;
    float *acc_im = wregion + TV;
    float *acc_w = wregion + 2 * TV;
    float2 *rect = reinterpret_cast<float2 *>(wregion + ACC_WORDS);
    unsigned short *list = reinterpret_cast<unsigned short *>(wregion + ACC_WORDS + 2 * RECT2);

    for (;;) {
        unsigned it = 0;
        if (lane == 0) it = atomicAdd(&ctr->queue, 1u);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
        if (it >= static_cast<unsigned>(nitems)) break;
        const Item item = items[it];
        // the item's reconstruction (job) and its geometry and buffers
        const int job = __builtin_amdgcn_readfirstlane(item.tile >> 24);
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

        for (int k = lane; k < ACC_WORDS; k += 64) wregion[k] = 0.f;
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

        // Staging of one slice, split into issue (global loads into registers)
        // and commit (LDS writes) so that the next slice's loads are in flight
        // while the current slice's windows are evaluated.
        struct Stage {
            float4 e1, e2, e3;
            int kx_lo, ky_lo;
            int rim;          // int, not bool: no padding bytes in the struct copies
            float scale;
        };
        // cell[] holds the raw sample words between issue and commit: the
        // complex64 value, or the packed 16-bit pair in .x.  Decoding waits
        // for the loads, so it happens at commit, after the previous slice's
        // windows have hidden their latency.
        float2 cell[NC];
        bool keep[NC];
        int dst[NC];
        auto issue = [&](int s, Stage &st) {
            // s is wave-uniform: the orientation and scale go to scalar
            // registers here, so no later copy of the stage waits on the
            // sample loads issued below
            const Orient ov = orient[s];
            Orient o;
            o.e1 = uniform4(ov.e1);
            o.e2 = uniform4(ov.e2);
            o.e3 = uniform4(ov.e3);
            st.e1 = o.e1;
            st.e2 = o.e2;
            st.e3 = o.e3;
            const float ucx = fmaf(o.e1.x, cx, fmaf(o.e1.y, cy, o.e1.z * cz));
            const float ucy = fmaf(o.e2.x, cx, fmaf(o.e2.y, cy, o.e2.z * cz));
            const float extx = fmaf(hx, fabsf(o.e1.x), fmaf(hy, fabsf(o.e1.y), hz * fabsf(o.e1.z)));
            const float exty = fmaf(hx, fabsf(o.e2.x), fmaf(hy, fabsf(o.e2.y), hz * fabsf(o.e2.z)));
            const int kx_lo = static_cast<int>(floorf(ucx - extx - g.a)) - 1;
            const int ky_lo = static_cast<int>(floorf(ucy - exty - g.a)) - 1;
            const int wx = min(static_cast<int>(floorf(ucx + extx + g.a)) + 2 - kx_lo, RECT);
            const int wy = min(static_cast<int>(floorf(ucy + exty + g.a)) + 2 - ky_lo, RECT);
            const int fxm = max(abs(kx_lo), abs(kx_lo + wx - 1));
            const int fym = max(abs(ky_lo), abs(ky_lo + wy - 1));
            st.kx_lo = kx_lo;
            st.ky_lo = ky_lo;
            st.rim = static_cast<float>(fxm * fxm + fym * fym) < g.r2max ? 0 : 1;
            st.scale = g.scales ? uniformf(g.scales[s]) : 1.0f;
            const int ncell = wx * wy;
            const float inv_wx = 1.0f / static_cast<float>(wx);
            // buffer resource over this slice: 32-bit offsets, hardware bounds check
            const int eb = sample_bytes(g.dtype);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<unsigned char *>(static_cast<const unsigned char *>(slices) +
                                            static_cast<size_t>(s) * slen * eb),
                static_cast<short>(0), static_cast<int>(slen * eb), 0x00020000);
            int off[NC];
#pragma unroll
            for (int qq = 0; qq < NC; ++qq) {
                const int c = qq * 64 + lane;
                const int cy_ = static_cast<int>((static_cast<float>(c) + 0.5f) * inv_wx);
                const int cx_ = c - cy_ * wx;
                const int kx = kx_lo + cx_, ky = ky_lo + cy_;
                const bool valid = c < ncell && static_cast<float>(kx * kx + ky * ky) < g.r2max;
                const bool direct = kx > 0 || (kx == 0 && ky >= 0);
                int row = direct ? ky + g.h : g.h - ky;
                int col = direct ? kx : -kx;
                row = valid ? row : g.h;
                col = valid ? col : 0;
                off[qq] = (row * g.sw + col) * eb;
                // the sign flip of mirrored samples is applied at commit
                keep[qq] = valid;
                dst[qq] = c < ncell ? (direct ? 1 : -1) * (cy_ * RECT + cx_ + 1) : 0;
            }
            // all loads back to back (dtype is uniform over the launch)
            if (g.dtype == 0) {
#pragma unroll
                for (int qq = 0; qq < NC; ++qq)
                    cell[qq] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, off[qq], 0, 0));
            } else {
#pragma unroll
                for (int qq = 0; qq < NC; ++qq)
                    cell[qq].x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off[qq], 0, 0));
            }
        };
        auto commit = [&](const Stage &st) {
            const int dt = g.dtype;
#pragma unroll
            for (int qq = 0; qq < NC; ++qq) {
                if (dst[qq] != 0) {
                    float2 v;
                    if (dt == 0) {
                        v = cell[qq];
                    } else {
                        const unsigned raw = __float_as_uint(cell[qq].x);
                        if (dt == 1) {
                            const _Float16 lo = __builtin_bit_cast(_Float16, static_cast<unsigned short>(raw & 0xffffu));
                            const _Float16 hi = __builtin_bit_cast(_Float16, static_cast<unsigned short>(raw >> 16));
                            v = make_float2(static_cast<float>(lo) * st.scale, static_cast<float>(hi) * st.scale);
                        } else {
                            v = make_float2(__uint_as_float(raw << 16), __uint_as_float(raw & 0xffff0000u));
                        }
                    }
                    v = keep[qq] ? v : make_float2(0.f, 0.f);
                    if (dst[qq] < 0) v.y = -v.y;
                    rect[abs(dst[qq]) - 1] = v;
                }
            }
        };

        Stage cur;
        int s = next_slice();
        if (s >= 0) issue(s, cur);
        while (s >= 0) {
            // 1. enumerate the tile's voxels inside the slab |e3.v| <= a
            //    (and inside the reach sphere |v| < r_max + a)
            const float4 e3 = cur.e3;
            const float n0 = fabsf(e3.x), n1 = fabsf(e3.y), n2 = fabsf(e3.z);
            const int d = (n0 >= n1 && n0 >= n2) ? 0 : (n1 >= n2 ? 1 : 2);
            const int ia = d == 0 ? 1 : 0;
            const int ib = d == 2 ? 1 : 2;
            const float nd = sel3(d, e3.x, e3.y, e3.z);
            const float na = sel3(ia, e3.x, e3.y, e3.z);
            const float nb = sel3(ib, e3.x, e3.y, e3.z);
            const int D0 = sel3i(d, X0, Y0, Z0), D1 = sel3i(d, X1, Y1, Z1);
            const int A0 = sel3i(ia, X0, Y0, Z0), A1 = sel3i(ia, X1, Y1, Z1);
            const int B0 = sel3i(ib, X0, Y0, Z0), B1 = sel3i(ib, X1, Y1, Z1);
            const int sd = sel3i(d, 1, TE, TE * TE);
            const int sa = sel3i(ia, 1, TE, TE * TE);
            const int sb = sel3i(ib, 1, TE, TE * TE);
            const int ca = lane & (TE - 1), cb = lane >> 3;
            const int va = A0 + ca, vb = B0 + cb;
            const float fva = static_cast<float>(va), fvb = static_cast<float>(vb);
            const float rem = R2 - fmaf(fva, fva, fvb * fvb);
            const bool col_in = va <= A1 && vb <= B1 && rem >= 0.f;
            const float lim = sqrtf(fmaxf(rem, 0.f));
            const float q = fmaf(na, fva, nb * fvb);
            const float inv = 1.0f / nd;
            const float t1 = (-a_run - q) * inv, t2 = (a_run - q) * inv;
            const int lo = max(static_cast<int>(ceilf(fmaxf(fminf(t1, t2), -lim))), D0);
            const int hi = min(static_cast<int>(floorf(fminf(fmaxf(t1, t2), lim))), D1);
            const int cnt = col_in ? max(hi - lo + 1, 0) : 0;
            int incl = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(incl, off);
                if (lane >= off) incl += y;
            }
            const int H = __builtin_amdgcn_readfirstlane(__shfl(incl, 63));
            if (H > 0) {
                const int excl = incl - cnt;
                const int lid0 = ca * sa + cb * sb + (lo - D0) * sd;
                for (int k = 0; k < cnt; ++k) list[excl + k] = static_cast<unsigned short>(lid0 + k * sd);
                // 2. the staged samples of this slice go to LDS
                commit(cur);
            }
            // next slice's loads are issued before this slice's windows
            Stage nxt = cur;
            const int s_next = next_slice();
            if (s_next >= 0) issue(s_next, nxt);
            wave_sync();

            if (H > 0) {
                // 3. windows of the hits, 64 per round
                const float fkx_lo = static_cast<float>(cur.kx_lo), fky_lo = static_cast<float>(cur.ky_lo);
                for (int r = 0; r < H; r += 64) {
                    const int hh = r + lane;
                    if (hh < H) {
                        const int lid = list[hh];
                        const float vx = static_cast<float>(X0 + (lid & 7));
                        const float vy = static_cast<float>(Y0 + ((lid >> 3) & 7));
                        const float vz = static_cast<float>(Z0 + (lid >> 6));
                        const float ux = fmaf(cur.e1.x, vx, fmaf(cur.e1.y, vy, cur.e1.z * vz));
                        const float uy = fmaf(cur.e2.x, vx, fmaf(cur.e2.y, vy, cur.e2.z * vz));
                        const float uz = fmaf(e3.x, vx, fmaf(e3.y, vy, e3.z * vz));
                        float pr, pi, pw;
                        constexpr bool PRE = (FLAGS & SLAB_PRELOAD) != 0;
                        if (cur.rim)
                            window_lds<WIN, true, LERP, PRE>(rect, tab, g, ux, uy, uz, fkx_lo, fky_lo, pr, pi, pw);
                        else
                            window_lds<WIN, false, LERP, PRE>(rect, tab, g, ux, uy, uz, fkx_lo, fky_lo, pr, pi, pw);
                        // a voxel appears once per slice: single writer within the wave
                        if (FLAGS & SLAB_ATOMIC) {
                            atomicAdd(acc_re + lid, pr);
                            atomicAdd(acc_im + lid, pi);
                            atomicAdd(acc_w + lid, pw);
                        } else {
                            acc_re[lid] += pr;
                            acc_im[lid] += pi;
                            acc_w[lid] += pw;
                        }
                    }
                }
                wave_sync();
                if (++inner == inner_chunk) {
#pragma unroll
                    for (int k = 0; k < TV / 64; ++k) {
                        const int lid = lane + 64 * k;
                        ore[k] += acc_re[lid];
                        oim[k] += acc_im[lid];
                        ow[k] += acc_w[lid];
                        acc_re[lid] = 0.f;
                        acc_im[lid] = 0.f;
                        acc_w[lid] = 0.f;
                    }
                    inner = 0;
                    wave_sync();
                }
            }
            cur = nxt;
            s = s_next;
        }
#pragma unroll
        for (int k = 0; k < TV / 64; ++k) {
            const int lid = lane + 64 * k;
            ore[k] += acc_re[lid];
            oim[k] += acc_im[lid];
            ow[k] += acc_w[lid];
        }
        wave_sync();
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
#pragma unroll
            for (int k = 0; k < TV / 64; ++k) {
                const int lid = lane + 64 * k;
                partials[static_cast<size_t>(item.slot) * TV + lid] = make_float4(ore[k], oim[k], ow[k], 0.f);
            }
        }
    }
}

template <int WIN, bool LERP, int FLAGS>
hipError_t launch_slab_t(const JobTable &jt, const float2 *table, const Item *items, int nitems, int inner_chunk,
                         int blocks, int wpb, Counters *ctr, hipStream_t st)
{
    const size_t lds = (static_cast<size_t>(table_words(jt.job[0].g.N)) +
                        static_cast<size_t>(wpb) * SlabShape<WIN>::WAVE_WORDS) * sizeof(float);
    hipLaunchKernelGGL((k_insert_slab<WIN, LERP, FLAGS>), dim3(blocks), dim3(64 * wpb), lds, st, jt, table, items,
                       nitems, inner_chunk, ctr);
    return hipGetLastError();
}

// Adds the partial sums of split 8x8x8 tiles, in part order, into G and W.
__global__ __launch_bounds__(512) void k_reduce_partials8(JobTable jt, const Item *__restrict__ items)
{
    const Item item = items[blockIdx.x];
    if (item.nparts == 1 || item.part != 0) return;
    const int job = item.tile >> 24;
    const int tile = item.tile & 0xffffff;
    const Geom g = jt.job[job].g;
    const float4 *__restrict__ partials = jt.job[job].partials;
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
    for (int k = 0; k < item.nparts; ++k) {
        const float4 p = partials[static_cast<size_t>(item.slot + k) * TV + lid];
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

}  // namespace

size_t slab_lds_bytes(const Geom &g, int waves_per_block)
{
    const int win = static_cast<int>(floorf(2.0f * g.a)) + 1;
    const int rect = win + 17;
    const size_t wave_words = ACC_WORDS + 2 * rect * rect + LIST_WORDS;
    return (static_cast<size_t>(table_words(g.N)) + waves_per_block * wave_words) * sizeof(float);
}

hipError_t launch_insert_slab(const JobTable &jt, bool lerp, int flags, const float2 *table, const Item *items,
                              int nitems, int inner_chunk, int blocks, int wpb, Counters *ctr, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    const Geom &g = jt.job[0].g;
    const int win = static_cast<int>(floorf(2.0f * g.a)) + 1;
    // every flag combination exists for the common window (a in [1.5, 2)) with
    // linear interpolation; other windows and truncation use the default flags
    if (win == 4 && lerp) {
        switch (flags & 3) {
        case 0: return launch_slab_t<4, true, 0>(jt, table, items, nitems, inner_chunk, blocks, wpb, ctr, st);
        case 1: return launch_slab_t<4, true, 1>(jt, table, items, nitems, inner_chunk, blocks, wpb, ctr, st);
        case 2: return launch_slab_t<4, true, 2>(jt, table, items, nitems, inner_chunk, blocks, wpb, ctr, st);
        default: return launch_slab_t<4, true, 3>(jt, table, items, nitems, inner_chunk, blocks, wpb, ctr, st);
        }
    }
#define RECON_SLAB_CASE(WV)                                                                                    \
    case WV:                                                                                                   \
        return lerp ? launch_slab_t<WV, true, slab_default_flags<WV>()>(jt, table, items, nitems, inner_chunk,  \
                                                                        blocks, wpb, ctr, st)                  \
                    : launch_slab_t<WV, false, slab_default_flags<WV>()>(jt, table, items, nitems, inner_chunk, \
                                                                         blocks, wpb, ctr, st);
    switch (win) {
        RECON_SLAB_CASE(1)
        RECON_SLAB_CASE(2)
        RECON_SLAB_CASE(3)
        RECON_SLAB_CASE(4)
        RECON_SLAB_CASE(5)
        RECON_SLAB_CASE(6)
    default:
        return hipErrorInvalidValue;
    }
#undef RECON_SLAB_CASE
}

hipError_t launch_reduce_partials8(const JobTable &jt, const Item *items, int nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials8, dim3(nitems), dim3(TV), 0, st, jt, items);
    return hipGetLastError();
}

}  // namespace recon
