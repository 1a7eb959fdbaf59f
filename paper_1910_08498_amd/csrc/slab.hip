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
    static constexpr int RECT = WIN + 16;   // >= 2 * 3.5 * sqrt(3) + WIN + 3
    static constexpr int RECT2 = RECT * RECT;
    static constexpr int WAVE_WORDS = ACC_WORDS + 2 * RECT2 + LIST_WORDS;
};

__host__ __device__ inline int table_words(int N) { return (N + 1 + 3) & ~3; }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float sel3(int i, float x, float y, float z)
{
    return i == 0 ? x : (i == 1 ? y : z);
}
__device__ __forceinline__ int sel3i(int i, int x, int y, int z)
{
    return i == 0 ? x : (i == 1 ? y : z);
}

// Window of one (voxel, slice) hit from the LDS rectangle whose cell (0, 0)
// is sample (kx_lo, ky_lo).  RIM: the rectangle reaches the disk edge, so
// each candidate's |k| < r_max membership is checked for the weight sum.
template <int WIN, bool RIM, bool LERP>
__device__ __forceinline__ void window_lds(const float2 *__restrict__ rect, const float *__restrict__ tab,
                                           const Geom &g, float tmax, float ux, float uy, float uz,
                                           int kx_lo, int ky_lo, float &pr, float &pi, float &pw)
{
    constexpr int RECT = SlabShape<WIN>::RECT;
    const int kx0 = static_cast<int>(ceilf(ux - g.a));
    const int ky0 = static_cast<int>(ceilf(uy - g.a));
    const int ox = min(max(kx0 - kx_lo, 0), RECT - WIN);
    const int oy = min(max(ky0 - ky_lo, 0), RECT - WIN);
    const float2 *base = rect + oy * RECT + ox;
    float dxs[WIN], dys[WIN];
    int kx2[WIN], ky2[WIN];
    const float uzs = uz * uz;
#pragma unroll
    for (int i = 0; i < WIN; ++i) {
        const int kx = kx_lo + ox + i;
        const float dx = ux - static_cast<float>(kx);
        dxs[i] = dx * dx * g.tscale;
        const int ky = ky_lo + oy + i;
        const float dy = uy - static_cast<float>(ky);
        dys[i] = fmaf(dy, dy, uzs) * g.tscale;
        if (RIM) {
            kx2[i] = kx * kx;
            ky2[i] = ky * ky;
        }
    }
    float sr = 0.f, si = 0.f, sw = 0.f;
#pragma unroll
    for (int j = 0; j < WIN; ++j) {
#pragma unroll
        for (int i = 0; i < WIN; ++i) {
            const float t = dxs[i] + dys[j];
            const float tc = fminf(t, tmax);
            const int it = static_cast<int>(tc);
            float w;
            if (LERP) {
                const float f = tc - static_cast<float>(it);
                const float t0 = tab[it], t1 = tab[it + 1];
                w = fmaf(f, t1 - t0, t0);
            } else {
                w = tab[it];
            }
            bool ok = t <= tmax;
            if (RIM) ok = ok && static_cast<float>(kx2[i] + ky2[j]) < g.r2max;
            w = ok ? w : 0.f;
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

template <int WIN, bool LERP>
__global__ __launch_bounds__(1024) void k_insert_slab(
    Geom g, const float2 *__restrict__ slices, const Orient *__restrict__ orient, int count,
    const float2 *__restrict__ table_g, const Item *__restrict__ items, int nitems,
    float4 *__restrict__ partials, int inner_chunk, Counters *__restrict__ ctr,
    float2 *__restrict__ G, float *__restrict__ W)
{
    using SS = SlabShape<WIN>;
    constexpr int RECT = SS::RECT;
    constexpr int RECT2 = SS::RECT2;
    extern __shared__ float smem[];
    float *tab = smem;
    for (int i = threadIdx.x; i < g.N; i += blockDim.x) tab[i] = table_g[i].x;
    if (threadIdx.x == 0) tab[g.N] = table_g[g.N - 1].x;
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    float *wregion = smem + table_words(g.N) + wave * SS::WAVE_WORDS;
    float *acc_re = wregion;
    float *acc_im = wregion + TV;
    float *acc_w = wregion + 2 * TV;
    float2 *rect = reinterpret_cast<float2 *>(wregion + ACC_WORDS);
    unsigned short *list = reinterpret_cast<unsigned short *>(wregion + ACC_WORDS + 2 * RECT2);

    const int TX = (g.h + 1 + TE - 1) / TE;
    const int TY = (g.dim + TE - 1) / TE;
    const size_t slen = static_cast<size_t>(g.n) * g.sw;
    const float reach = sqrtf(g.r2max) + g.a + 3.5f * 1.7320508f + 0.01f;
    const float reach2 = reach * reach;
    const float tmax = static_cast<float>(g.N - 1);
    const float a_run = g.a * (1.0f + 1e-5f) + 1e-5f;

    for (;;) {
        unsigned it = 0;
        if (lane == 0) it = atomicAdd(&ctr->queue, 1u);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
        if (it >= static_cast<unsigned>(nitems)) break;
        const Item item = items[it];
        const int tx = item.tile % TX;
        const int ty = (item.tile / TX) % TY;
        const int tz = item.tile / (TX * TY);
        const int X0 = TE * tx, Y0 = TE * ty - g.h, Z0 = TE * tz - g.h;
        const float cx = X0 + 3.5f, cy = Y0 + 3.5f, cz = Z0 + 3.5f;
        const int s0 = static_cast<int>(static_cast<long>(count) * item.part / item.nparts);
        const int s1 = static_cast<int>(static_cast<long>(count) * (item.part + 1) / item.nparts);

        for (int k = lane; k < ACC_WORDS; k += 64) wregion[k] = 0.f;
        float ore[TV / 64], oim[TV / 64], ow[TV / 64];
#pragma unroll
        for (int k = 0; k < TV / 64; ++k) ore[k] = oim[k] = ow[k] = 0.f;
        int inner = 0;
        wave_sync();

        for (int base0 = s0; base0 < s1; base0 += 64) {
            const int sl = base0 + lane;
            bool pass = false;
            if (sl < s1) {
                const Orient o = orient[sl];
                if (o.e1.w != 0.f) {
                    const float dz = fmaf(o.e3.x, cx, fmaf(o.e3.y, cy, o.e3.z * cz));
                    const float ext = 3.5f * (fabsf(o.e3.x) + fabsf(o.e3.y) + fabsf(o.e3.z));
                    const float px = fmaf(o.e1.x, cx, fmaf(o.e1.y, cy, o.e1.z * cz));
                    const float py = fmaf(o.e2.x, cx, fmaf(o.e2.y, cy, o.e2.z * cz));
                    pass = fabsf(dz) <= g.a + ext + 1e-3f && fmaf(px, px, py * py) <= reach2;
                }
            }
            unsigned long long mask = __ballot(pass);
            while (mask) {
                const int b = __builtin_ctzll(mask);
                mask &= mask - 1ull;
                const int s = base0 + b;
                const Orient o = orient[s];
                const float2 *Fs = slices + s * slen;

                // 1. stage the rectangle of samples the tile's windows can touch
                const float ucx = fmaf(o.e1.x, cx, fmaf(o.e1.y, cy, o.e1.z * cz));
                const float ucy = fmaf(o.e2.x, cx, fmaf(o.e2.y, cy, o.e2.z * cz));
                const float extx = 3.5f * (fabsf(o.e1.x) + fabsf(o.e1.y) + fabsf(o.e1.z));
                const float exty = 3.5f * (fabsf(o.e2.x) + fabsf(o.e2.y) + fabsf(o.e2.z));
                const int kx_lo = static_cast<int>(floorf(ucx - extx - g.a)) - 1;
                const int ky_lo = static_cast<int>(floorf(ucy - exty - g.a)) - 1;
                const int fx = max(abs(kx_lo), abs(kx_lo + RECT - 1));
                const int fy = max(abs(ky_lo), abs(ky_lo + RECT - 1));
                const bool rim = !(static_cast<float>(fx * fx + fy * fy) < g.r2max);
                constexpr int NC = (RECT2 + 63) / 64;
                float2 cell[NC];
                bool keep[NC];
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    const int c = q * 64 + lane;
                    const int cy_ = c / RECT, cx_ = c - cy_ * RECT;
                    const int kx = kx_lo + cx_, ky = ky_lo + cy_;
                    const bool valid = c < RECT2 && static_cast<float>(kx * kx + ky * ky) < g.r2max;
                    const bool direct = kx > 0 || (kx == 0 && ky >= 0);
                    int row = direct ? ky + g.h : g.h - ky;
                    int col = direct ? kx : -kx;
                    row = valid ? row : g.h;
                    col = valid ? col : 0;
                    cell[q] = Fs[row * g.sw + col];
                    cell[q].y = direct ? cell[q].y : -cell[q].y;
                    keep[q] = valid;
                }
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    const int c = q * 64 + lane;
                    if (q < NC - 1 || c < RECT2) rect[c] = keep[q] ? cell[q] : make_float2(0.f, 0.f);
                }

                // 2. enumerate the tile's voxels inside the slab |e3.v| <= a
                const float n0 = fabsf(o.e3.x), n1 = fabsf(o.e3.y), n2 = fabsf(o.e3.z);
                const int d = (n0 >= n1 && n0 >= n2) ? 0 : (n1 >= n2 ? 1 : 2);
                const int ia = d == 0 ? 1 : 0;
                const int ib = d == 2 ? 1 : 2;
                const float nd = sel3(d, o.e3.x, o.e3.y, o.e3.z);
                const float na = sel3(ia, o.e3.x, o.e3.y, o.e3.z);
                const float nb = sel3(ib, o.e3.x, o.e3.y, o.e3.z);
                const int D0 = sel3i(d, X0, Y0, Z0);
                const int A0 = sel3i(ia, X0, Y0, Z0);
                const int B0 = sel3i(ib, X0, Y0, Z0);
                const int sd = sel3i(d, 1, TE, TE * TE);
                const int sa = sel3i(ia, 1, TE, TE * TE);
                const int sb = sel3i(ib, 1, TE, TE * TE);
                const int ca = lane & (TE - 1), cb = lane >> 3;
                const int va = A0 + ca, vb = B0 + cb;
                // every axis ends at +h; the x axis starts at 0, y and z at -h
                const bool col_in = va <= g.h && vb <= g.h;
                const float q = fmaf(na, static_cast<float>(va), nb * static_cast<float>(vb));
                const float inv = 1.0f / nd;
                const float t1 = (-a_run - q) * inv, t2 = (a_run - q) * inv;
                const int lo = max(static_cast<int>(ceilf(fminf(t1, t2))), D0);
                const int hi = min(static_cast<int>(floorf(fmaxf(t1, t2))), min(D0 + TE - 1, g.h));
                const int cnt = col_in ? max(hi - lo + 1, 0) : 0;
                int incl = cnt;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const int y = __shfl_up(incl, off);
                    if (lane >= off) incl += y;
                }
                const int excl = incl - cnt;
                const int H = __builtin_amdgcn_readfirstlane(__shfl(incl, 63));
                const int lid0 = ca * sa + cb * sb + (lo - D0) * sd;
                for (int k = 0; k < cnt; ++k) list[excl + k] = static_cast<unsigned short>(lid0 + k * sd);
                wave_sync();

                // 3. windows of the hits, 64 per round
                for (int r = 0; r < H; r += 64) {
                    const int hh = r + lane;
                    if (hh < H) {
                        const int lid = list[hh];
                        const float vx = static_cast<float>(X0 + (lid & 7));
                        const float vy = static_cast<float>(Y0 + ((lid >> 3) & 7));
                        const float vz = static_cast<float>(Z0 + (lid >> 6));
                        const float ux = fmaf(o.e1.x, vx, fmaf(o.e1.y, vy, o.e1.z * vz));
                        const float uy = fmaf(o.e2.x, vx, fmaf(o.e2.y, vy, o.e2.z * vz));
                        const float uz = fmaf(o.e3.x, vx, fmaf(o.e3.y, vy, o.e3.z * vz));
                        float pr, pi, pw;
                        if (rim)
                            window_lds<WIN, true, LERP>(rect, tab, g, tmax, ux, uy, uz, kx_lo, ky_lo, pr, pi, pw);
                        else
                            window_lds<WIN, false, LERP>(rect, tab, g, tmax, ux, uy, uz, kx_lo, ky_lo, pr, pi, pw);
                        acc_re[lid] += pr;
                        acc_im[lid] += pi;
                        acc_w[lid] += pw;
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
#pragma unroll
            for (int k = 0; k < TV / 64; ++k) {
                const int lid = lane + 64 * k;
                const int ix = X0 + (lid & 7);
                const int iy = Y0 + ((lid >> 3) & 7) + g.h;
                const int iz = Z0 + (lid >> 6) + g.h;
                if (ix <= g.h && iy < g.dim && iz < g.dim) {
                    const size_t vi = (static_cast<size_t>(iz) * g.dim + iy) * g.dim + (ix + g.h);
                    float2 gv = G[vi];
                    gv.x += ore[k];
                    gv.y += oim[k];
                    G[vi] = gv;
                    W[vi] += ow[k];
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

template <int WIN, bool LERP>
hipError_t launch_slab_t(const Geom &g, const float2 *slices, const Orient *orient, int count, const float2 *table,
                         const Item *items, int nitems, float4 *partials, int inner_chunk, int blocks, int wpb,
                         Counters *ctr, float2 *G, float *W, hipStream_t st)
{
    const size_t lds = (static_cast<size_t>(table_words(g.N)) + static_cast<size_t>(wpb) * SlabShape<WIN>::WAVE_WORDS) *
                       sizeof(float);
    hipLaunchKernelGGL((k_insert_slab<WIN, LERP>), dim3(blocks), dim3(64 * wpb), lds, st, g, slices, orient, count,
                       table, items, nitems, partials, inner_chunk, ctr, G, W);
    return hipGetLastError();
}

// Adds the partial sums of split 8x8x8 tiles, in part order, into G and W.
__global__ __launch_bounds__(512) void k_reduce_partials8(Geom g, const Item *__restrict__ items,
                                                          const float4 *__restrict__ partials,
                                                          float2 *__restrict__ G, float *__restrict__ W)
{
    const Item item = items[blockIdx.x];
    if (item.nparts == 1 || item.part != 0) return;
    const int lid = threadIdx.x;
    const int TX = (g.h + 1 + TE - 1) / TE;
    const int TY = (g.dim + TE - 1) / TE;
    const int tx = item.tile % TX;
    const int ty = (item.tile / TX) % TY;
    const int tz = item.tile / (TX * TY);
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
    const int rect = win + 16;
    const size_t wave_words = ACC_WORDS + 2 * rect * rect + LIST_WORDS;
    return (static_cast<size_t>(table_words(g.N)) + waves_per_block * wave_words) * sizeof(float);
}

hipError_t launch_insert_slab(const Geom &g, bool lerp, const float2 *slices, const Orient *orient, int count,
                              const float2 *table, const Item *items, int nitems, float4 *partials,
                              int inner_chunk, int blocks, int wpb, Counters *ctr, float2 *G, float *W,
                              hipStream_t st)
{
    if (count <= 0 || nitems <= 0) return hipSuccess;
    const int win = static_cast<int>(floorf(2.0f * g.a)) + 1;
#define RECON_SLAB_CASE(WV)                                                                                   \
    case WV:                                                                                                  \
        return lerp ? launch_slab_t<WV, true>(g, slices, orient, count, table, items, nitems, partials,      \
                                              inner_chunk, blocks, wpb, ctr, G, W, st)                        \
                    : launch_slab_t<WV, false>(g, slices, orient, count, table, items, nitems, partials,     \
                                               inner_chunk, blocks, wpb, ctr, G, W, st);
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

hipError_t launch_reduce_partials8(const Geom &g, const Item *items, int nitems, const float4 *partials, float2 *G,
                                   float *W, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials8, dim3(nitems), dim3(TV), 0, st, g, items, partials, G, W);
    return hipGetLastError();
}

}  // namespace recon
