// Host side of librecon.so: the C ABI declared in include/recon.h.
//
// Responsibilities: argument validation, the FP64 blob table (the paper lets
// the interpolation weights be precomputed, Sect. 4.2 "3D Fourier
// Reconstruction"), the workspace layout, the static work plan of the binned
// kernel (tiles, slice-range splits, cost order) and kernel dispatch on the
// caller's stream.  No device memory is allocated here: G, W, V and the
// workspace belong to the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/recon.h"
#include "kernels.hpp"

using recon::Counters;
using recon::Geom;
using recon::Item;
using recon::Orient;

namespace {

thread_local std::string g_err;

recon_status fail(recon_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

recon_status hip_fail(hipError_t e, const char *what)
{
    return fail(RECON_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// I_m(x) by its power series sum_j (x/2)^(2j+m) / (j! (j+m)!), in FP64.
double bessel_i(int m, double x)
{
    const double half = 0.5 * x, q = half * half;
    double term = 1.0;
    for (int j = 1; j <= m; ++j) term *= half / j;
    double total = term;
    for (int j = 1; j < 400; ++j) {
        term *= q / (static_cast<double>(j) * (j + m));
        total += term;
        if (term <= 1e-18 * total) break;
    }
    return total;
}

// Kaiser-Bessel blob normalised to b(0) = 1, as a function of squared distance.
double kb_blob(double d2, double a, double alpha, int m)
{
    if (d2 > a * a) return 0.0;
    double s = 1.0 - d2 / (a * a);
    if (s < 0.0) s = 0.0;
    const double scale = m == 0 ? 1.0 : std::pow(s, 0.5 * m);
    return scale * bessel_i(m, alpha * std::sqrt(s)) / bessel_i(m, alpha);
}

// Coefficients of the blob as a polynomial in s = 1 - d^2/a^2, built in FP64:
// b = s^(m/2) I_m(alpha sqrt(s)) / I_m(alpha) = s^m sum_j c_j s^j with
// c_j = (alpha/2)^(2j+m) / (j! (j+m)! I_m(alpha)) (the power series of I_m,
// whose terms carry s^(j + m/2)).  Output: out[k] = coefficient of s^k, m
// leading zeros, terms until the rest sums below 1e-10 (b <= 1 on [0, 1], all
// terms positive), zero-padded to a multiple of 4.  Returns the count, or 0
// if more than kMaxTerms would be needed (a very large alpha).
int blob_coefficients(double alpha, int m, std::vector<double> *out)
{
    std::vector<double> c(m, 0.0);
    const double half = 0.5 * alpha;
    double term = 1.0;                                  // (alpha/2)^m / m!
    for (int j = 1; j <= m; ++j) term *= half / j;
    const double norm = bessel_i(m, alpha);
    bool converged = false;
    for (int j = 0; m + j < recon::kMaxTerms; ++j) {
        if (j > 0) term *= half * half / (static_cast<double>(j) * (j + m));
        c.push_back(term / norm);
        // the remaining terms shrink at least geometrically with this ratio
        // once j (j + m) exceeds (alpha/2)^2
        const double ratio = half * half / ((j + 1.0) * (j + 1.0 + m));
        if (ratio < 0.5 && term / norm * ratio / (1.0 - ratio) < 1e-10) {
            converged = true;
            break;
        }
    }
    while (c.size() % 4) c.push_back(0.0);
    if (!converged || static_cast<int>(c.size()) > recon::kMaxTerms) return 0;
    *out = c;
    return static_cast<int>(c.size());
}

recon_status validate(const recon_params *p)
{
    if (!p) return fail(RECON_EINVAL, "params is NULL");
    if (p->n < 4 || p->n > 1024 || (p->n & 1))
        return fail(RECON_EINVAL, "n must be even and in [4, 1024] (got %d)", p->n);
    // below a = 1 a voxel sees few samples (4/3 pi a^3 < 4.2 on average),
    // so the FP32 position rounding of single samples is not averaged out
    if (!(p->blob_radius >= 1.0f) || p->blob_radius > 2.95f)
        return fail(RECON_EINVAL, "blob_radius must be in [1, 2.95] (got %g)", p->blob_radius);
    if (!(p->blob_alpha >= 0.0f) || !std::isfinite(p->blob_alpha) || p->blob_alpha > 60.0f)
        return fail(RECON_EINVAL, "blob_alpha must be in [0, 60] (got %g)", p->blob_alpha);
    if (p->blob_order < 0 || p->blob_order > 8)
        return fail(RECON_EINVAL, "blob_order must be in [0, 8] (got %d)", p->blob_order);
    if (p->blob_alpha == 0.0f && p->blob_order > 0)
        return fail(RECON_EINVAL, "blob_alpha 0 needs blob_order 0 (I_m(0) = 0 cannot normalise the blob)");
    if (p->table_size != 0 && (p->table_size < 2 || p->table_size > 65536))
        return fail(RECON_EINVAL, "table_size must be 0 (weights on the fly) or in [2, 65536] (got %d)",
                    p->table_size);
    std::vector<double> coef;
    if (p->table_size == 0 && blob_coefficients(p->blob_alpha, p->blob_order, &coef) == 0)
        return fail(RECON_EINVAL, "weights on the fly need at most %d polynomial terms (alpha %g, order %d is "
                                  "too steep); use a table", recon::kMaxTerms, p->blob_alpha, p->blob_order);
    if (p->table_lerp != 0 && p->table_lerp != 1)
        return fail(RECON_EINVAL, "table_lerp must be 0 or 1");
    if (!(p->r_max > 0.0f) || p->r_max > 0.5f * p->n)
        return fail(RECON_EINVAL, "r_max must be in (0, n/2] (got %g)", p->r_max);
    if (p->slice_dtype != RECON_SLICE_C64 && p->slice_dtype != RECON_SLICE_F16 && p->slice_dtype != RECON_SLICE_BF16)
        return fail(RECON_EINVAL, "slice_dtype must be 0 (complex64), 1 (half) or 2 (bfloat16) (got %d)",
                    p->slice_dtype);
    if (p->max_batch < 1 || p->max_batch > (1 << 24))
        return fail(RECON_EINVAL, "max_batch must be in [1, 2^24] (got %d)", p->max_batch);
    return RECON_OK;
}

// ---------------------------------------------------------------------------
// static work plan of the binned kernel
// ---------------------------------------------------------------------------
struct Plan {
    std::vector<Item> items;
    std::vector<double> cost;   // estimated cost of each item (slice visits)
    std::vector<Item> ritems;   // split tiles (uploaded after the items)
    int nslots = 0;
};

// Tiles of E x E x E voxels (E = 4 or 8) over the half box x in [0, h],
// y, z in [-h, h].  A tile at centre distance r sees, for uniformly
// distributed slice normals, about min(1, (a + ext) / r) of the slices
// (ext = half the tile diagonal); its cost is that share of the slice visits,
// scaled by the part of its voxels inside the box and inside the reach
// sphere |v| < r_max + a (sampled on a 3 x 3 x 3 grid); tiles whose every
// voxel is out of reach are dropped.  Tiles are split into up to `split`
// slice ranges: the persistent waves pull items largest first, so the items
// that start last set the tail of the launch.  The costliest tiles, holding
// the first 40 % of the cost, are cut into items of twice the target cost,
// the next 40 % into items of the target, and the cheapest 20 %, which run
// last, into items of a quarter of it.  Items are ordered by decreasing
// estimated cost or, with `spatial`, tier by tier with the tiles of a tier
// in Morton order of their tile coordinates (a tile's parts together, in
// part order), so that the waves running at one time hold neighbouring tiles.
// `launch_total`, when positive, is the estimated cost of the whole launch
// the plan is part of (a batch of reconstructions): the item sizes follow
// it rather than this reconstruction's own total.
Plan make_plan(const recon_params &p, int split, int E, bool spatial, double launch_total = 0.0)
{
    Plan plan;
    const int h = p.n / 2, dim = p.n + 1;
    const int TX = (h + 1 + E - 1) / E, TY = (dim + E - 1) / E, TZ = TY;
    const double ext = 0.5 * (E - 1) * std::sqrt(3.0);
    const double a = p.blob_radius;
    struct Est { int tile; double cost; };
    std::vector<Est> tiles;
    double total = 0.0;
    const double R = p.r_max + a + 1e-3;   // no voxel at |v| >= R receives anything
    for (int tz = 0; tz < TZ; ++tz)
        for (int ty = 0; ty < TY; ++ty)
            for (int tx = 0; tx < TX; ++tx) {
                // voxel box of the tile clipped to the half box
                const double x0 = E * tx, x1 = std::min(x0 + E - 1, static_cast<double>(h));
                const double y0 = E * ty - h, y1 = std::min(y0 + E - 1, static_cast<double>(h));
                const double z0 = E * tz - h, z1 = std::min(z0 + E - 1, static_cast<double>(h));
                auto closest = [](double lo, double hi) { return lo > 0 ? lo : (hi < 0 ? hi : 0.0); };
                const double qx = closest(x0, x1), qy = closest(y0, y1), qz = closest(z0, z1);
                if (qx * qx + qy * qy + qz * qz >= R * R) continue;
                const double cx = 0.5 * (x0 + x1), cy = 0.5 * (y0 + y1), cz = 0.5 * (z0 + z1);
                const double r = std::sqrt(cx * cx + cy * cy + cz * cz);
                const double vol = (x1 - x0 + 1) * (y1 - y0 + 1) * (z1 - z0 + 1) / (E * E * E);
                int in = 0;
                for (int k = 0; k < 27; ++k) {
                    const double sx = x0 + 0.5 * (k % 3) * (x1 - x0), sy = y0 + 0.5 * ((k / 3) % 3) * (y1 - y0),
                                 sz = z0 + 0.5 * (k / 9) * (z1 - z0);
                    in += sx * sx + sy * sy + sz * sz < R * R ? 1 : 0;
                }
                const double frac = std::min(1.0, (a + ext) / std::max(r, 1e-9));
                const double share = vol * std::max(in, 1) / 27.0;
                const double cost = frac * p.max_batch * (E == 8 ? std::max(share, 0.25) : 1.0);
                tiles.push_back({tx + TX * (ty + TY * tz), cost});
                total += cost;
            }
    // target item cost: an eighth of the mean cost per wavefront slot of a
    // 256-CU device (16 slots per CU for 4^3 tiles, 8 for 8^3), >= 24 visits
    const double slots = 256.0 * (E == 4 ? 16.0 : 8.0);
    const double target = std::max(24.0, std::max(total, launch_total) / (slots * 8.0));
    std::vector<int> order(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tiles[x].cost > tiles[y].cost; });
    std::vector<int> np_of(tiles.size()), tier_of(tiles.size());
    double cum = 0.0;
    for (int i : order) {
        const double at = cum / std::max(total, 1e-30);
        tier_of[i] = at < 0.4 ? 0 : (at < 0.8 ? 1 : 2);
        const double t = tier_of[i] == 0 ? 2.0 * target : (tier_of[i] == 1 ? target : std::max(6.0, 0.25 * target));
        cum += tiles[i].cost;
        int np = static_cast<int>(std::ceil(tiles[i].cost / t));
        np = std::max(1, std::min(np, split));
        np_of[i] = std::min(np, std::max(1, p.max_batch));
    }
    struct Tmp { Item it; double cost; };
    std::vector<Tmp> tmp;
    for (size_t i = 0; i < tiles.size(); ++i) {
        const Est &e = tiles[i];
        const int np = np_of[i];
        const int slot = np > 1 ? plan.nslots : -1;
        if (np > 1) plan.nslots += np;
        for (int k = 0; k < np; ++k) tmp.push_back({{e.tile, k, np, np > 1 ? slot + k : -1}, e.cost / np});
    }
    if (spatial) {
        // key: tier, then the Morton code of (tx, ty, tz) (10 bits each)
        auto spread = [](uint64_t v) {
            uint64_t r = 0;
            for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
            return r;
        };
        std::vector<uint64_t> key(tiles.size());
        for (size_t i = 0; i < tiles.size(); ++i) {
            const uint64_t t = static_cast<uint64_t>(tiles[i].tile);
            const uint64_t tx = t % TX, ty = (t / TX) % TY, tz = t / (static_cast<uint64_t>(TX) * TY);
            key[i] = (static_cast<uint64_t>(tier_of[i]) << 32) | spread(tx) | (spread(ty) << 1) | (spread(tz) << 2);
        }
        std::vector<int> by(tiles.size());
        for (size_t i = 0; i < by.size(); ++i) by[i] = static_cast<int>(i);
        std::sort(by.begin(), by.end(), [&](int x, int y) { return key[x] < key[y]; });
        // items of tile i start at the sum of the parts of tiles before it
        std::vector<size_t> first(tiles.size() + 1, 0);
        for (size_t i = 0; i < tiles.size(); ++i) first[i + 1] = first[i] + np_of[i];
        plan.items.reserve(tmp.size());
        plan.cost.reserve(tmp.size());
        for (int i : by)
            for (size_t k = first[i]; k < first[i + 1]; ++k) {
                plan.items.push_back(tmp[k].it);
                plan.cost.push_back(tmp[k].cost);
            }
        return plan;
    }
    std::stable_sort(tmp.begin(), tmp.end(), [](const Tmp &x, const Tmp &y) { return x.cost > y.cost; });
    plan.items.reserve(tmp.size());
    plan.cost.reserve(tmp.size());
    for (const Tmp &t : tmp) {
        plan.items.push_back(t.it);
        plan.cost.push_back(t.cost);
    }
    return plan;
}

int tile_edge(int variant) { return variant == RECON_VARIANT_SLAB ? 8 : 4; }
bool spatial_queue(const recon_config &c) { return (c.traversal & RECON_TRAVERSAL_SPATIAL_QUEUE) != 0; }

constexpr int kMaxSplit = 64;

struct Layout {
    size_t ctr = 0, table = 0, orient = 0, items = 0, partials = 0, total = 0;
};

Layout layout_for(const recon_params &p, int nitems, size_t partial_vox)
{
    Layout L;
    size_t off = 0;
    L.ctr = off;
    off = align_up(off + sizeof(Counters), 256);
    // the blob table (N entries), then the on-the-fly polynomial's coefficients
    L.table = off;
    off = align_up(off + (static_cast<size_t>(p.table_size) + recon::kMaxTerms) * sizeof(float2), 256);
    // orientation records, then the exact-geometry axis remainders (3 float4
    // per slice)
    L.orient = off;
    off = align_up(off + static_cast<size_t>(p.max_batch) * (sizeof(Orient) + 3 * sizeof(float4)), 256);
    // work items, then (slab) the list of split tiles for the partial-sum
    // reduction: at most as many entries as items
    L.items = off;
    off = align_up(off + 2 * static_cast<size_t>(nitems) * sizeof(Item), 256);
    L.partials = off;
    off = align_up(off + partial_vox * sizeof(float4), 256);
    L.total = off;
    return L;
}

// Workspace layout large enough for the plan of every variant at the largest split.
Layout worst_layout(const recon_params &p)
{
    Plan p4 = make_plan(p, kMaxSplit, 4, false), p8 = make_plan(p, kMaxSplit, 8, false);
    const int nitems = static_cast<int>(std::max(p4.items.size(), p8.items.size()));
    // partial sums per split-tile slot: a float4 per voxel for the binned
    // kernel (64 voxels), three planes of 512 floats for the slab kernel
    const size_t pv = std::max(static_cast<size_t>(p4.nslots) * 64, static_cast<size_t>(p8.nslots) * 384);
    return layout_for(p, nitems, pv);
}

// Library default: the slab kernel, 8 waves per work-group with window reads
// preloaded, inner chunks of 64 slices and up to 32 slice-range splits (the
// 8-wave configuration of least mean regret over the timed workloads of the
// learned tuner's data); recon_init takes the 11-wave instance where it
// applies.  Other variants keep inner chunks of 32 and 16 splits.
recon_config default_config()
{
    recon_config c;
    std::memset(&c, 0, sizeof(c));
    c.variant = RECON_VARIANT_SLAB;
    c.waves_per_block = 8;
    c.group = 1;
    c.inner_chunk = 64;
    c.split = 32;
    c.slab_flags = 4 | 2;
    return c;
}
int default_inner_chunk(int variant) { return variant == RECON_VARIANT_SLAB ? 64 : 32; }
int default_split(int variant) { return variant == RECON_VARIANT_SLAB ? 32 : 16; }

int default_waves(int variant) { return variant == RECON_VARIANT_SLAB ? 8 : 16; }

// The slab kernel's 11-wave instance exists for the 4 x 4 window (blob
// radius in [1.5, 2)) with table interpolation, and needs its LDS to fit.
bool slab_wide_ok(const recon::Geom &g, int mode, size_t max_lds)
{
    const int win = static_cast<int>(std::floor(2.0f * g.a)) + 1;
    return win == 4 && mode == recon::WEIGHT_LERP && recon::slab_lds_bytes(g, mode, 11) <= max_lds;
}

// Weight source of a configuration: RECON_WEIGHTS_DEFAULT means the table
// when the parameters build one, else on the fly.
int weight_source(const recon_params &p, int weights)
{
    if (weights == RECON_WEIGHTS_OTF || (weights == RECON_WEIGHTS_DEFAULT && p.table_size == 0))
        return recon::WEIGHT_OTF;
    return p.table_lerp ? recon::WEIGHT_LERP : recon::WEIGHT_TRUNC;
}

// Geometry as the kernels of a weight source see it: on the fly, positions
// are scaled by 1/a (squared distances in units of a^2), not in table steps.
recon::Geom launch_geom(const recon::Geom &g, int mode)
{
    recon::Geom r = g;
    if (mode == recon::WEIGHT_OTF) r.tscale = r.inv_a2;
    return r;
}

// State of a dynamic-tuning search (random search over the tuning space).
struct TuneState {
    bool active = false;
    std::vector<recon_config> space;
    std::vector<int> order;       // random permutation of space indices
    size_t next = 0;              // next position in order
    int max_steps = 0;
    double target = 0.0;
    int steps_done = 0;
    int pending = -1;             // space index of the step in flight
    int pending_count = 0;        // slices of that step
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<double> ns;       // ns per slice per space index (< 0: not measured)
    int best = -1;
    double best_ns = std::numeric_limits<double>::infinity();
    double sum_ns = 0.0;
};

// splitmix64: the random search's generator (seeded, reproducible)
uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

}  // namespace

struct recon_ctx {
    recon_params p;
    Geom g;
    hipStream_t stream;
    float2 *G;
    float *W;
    unsigned char *ws;
    size_t ws_bytes;
    Layout L;
    recon_config cfg;
    Plan plan;           // plan for cfg.split
    int device;
    int num_cu;
    size_t max_lds;
    int max_threads;
    hipEvent_t ev_start;  // optional timing events around the insertion kernel
    hipEvent_t ev_stop;
    TuneState tune;
    int static_device = -1;   // >= 0: ws is that device's static workspace (recon_init_static)
};

// exact-geometry axis remainders: after the max_batch orientation records
static float4 *orient_rem(recon_ctx *c)
{
    return reinterpret_cast<float4 *>(c->ws + c->L.orient + static_cast<size_t>(c->p.max_batch) * sizeof(Orient));
}

// ---------------------------------------------------------------------------
// static workspace (recon_init_static): the workspace of one context per
// device in a device array of the library's own, for callers that cannot
// allocate device memory.  In host code `scratch` only names the symbol; its
// device address comes from hipGetSymbolAddress, resolved once per device
// with that device current, and only that address is handed to kernels and
// copies.
// ---------------------------------------------------------------------------
constexpr size_t kStaticWsBytes = RECON_STATIC_WS_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

namespace {
constexpr int kMaxDevices = 64;
struct StaticWs {
    unsigned char *ptr = nullptr;   // device address of `scratch` on this device (nullptr: not resolved)
    bool in_use = false;            // a live context holds it
};
std::mutex g_static_mu;
StaticWs g_static_ws[kMaxDevices];
}  // namespace

// Resolves the current device's static workspace and marks it in use.
static recon_status acquire_static_workspace(int *dev, unsigned char **ws)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (*dev < 0 || *dev >= kMaxDevices) return fail(RECON_EDEVICE, "device %d beyond the static table", *dev);
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticWs &s = g_static_ws[*dev];
    if (s.in_use)
        return fail(RECON_EINVAL, "the static workspace of device %d belongs to a live context: destroy it first",
                    *dev);
    if (!s.ptr) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(static workspace)");
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u))
            return fail(RECON_EDEVICE, "static workspace address is NULL or not 256-byte aligned");
        s.ptr = static_cast<unsigned char *>(ptr);
    }
    s.in_use = true;
    *ws = s.ptr;
    return RECON_OK;
}

static void release_static_workspace(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_ws[dev].in_use = false;
}

static recon_status tune_collect(recon_ctx *c);
static recon_status tune_finish(recon_ctx *c);
static recon_status apply_config(recon_ctx *c, const recon_config &n);

extern "C" {

const char *recon_last_error(void) { return g_err.c_str(); }

const char *recon_version(void) { return "recon-mi355x 0.1 (gfx950)"; }

recon_status recon_default_params(int32_t n, recon_params *out)
{
    if (!out) return fail(RECON_EINVAL, "out is NULL");
    out->n = n;
    out->blob_radius = 1.9f;
    out->blob_alpha = 15.0f;
    out->blob_order = 0;
    out->table_size = 10000;
    out->table_lerp = 1;
    out->r_max = 0.5f * static_cast<float>(n);
    out->slice_dtype = RECON_SLICE_C64;
    out->max_batch = 1500;
    return RECON_OK;
}

recon_status recon_query_sizes(const recon_params *p, size_t *g_bytes, size_t *w_bytes, size_t *ws_bytes)
{
    recon_status st = validate(p);
    if (st != RECON_OK) return st;
    const size_t dim = static_cast<size_t>(p->n) + 1;
    const size_t nvox = dim * dim * dim;
    if (g_bytes) *g_bytes = nvox * sizeof(float2);
    if (w_bytes) *w_bytes = nvox * sizeof(float);
    if (ws_bytes) *ws_bytes = worst_layout(*p).total;
    return RECON_OK;
}

// The split tiles of a work plan (their first part's item), for the
// reduction of their partial sums.
static std::vector<Item> split_tiles(const std::vector<Item> &items)
{
    std::vector<Item> r;
    for (const Item &it : items)
        if (it.nparts > 1 && it.part == 0) r.push_back(it);
    return r;
}

static recon_status upload_plan(recon_ctx *c)
{
    c->plan.ritems = split_tiles(c->plan.items);
    if (c->plan.items.empty()) return RECON_OK;
    // items, then the split tiles right after them
    std::vector<Item> all(c->plan.items);
    all.insert(all.end(), c->plan.ritems.begin(), c->plan.ritems.end());
    hipError_t e = hipMemcpyAsync(c->ws + c->L.items, all.data(), all.size() * sizeof(Item),
                                  hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(e, "upload work plan");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "upload work plan (sync)");
    return RECON_OK;
}

recon_status recon_init(const recon_params *p, void *d_G, void *d_W, void *d_ws, size_t ws_bytes,
                        void *stream, recon_ctx **out)
{
    if (!out) return fail(RECON_EINVAL, "out is NULL");
    *out = nullptr;
    recon_status st = validate(p);
    if (st != RECON_OK) return st;
    if (!d_G || !d_W || !d_ws) return fail(RECON_EINVAL, "G, W and workspace must be non-NULL");
    if ((reinterpret_cast<uintptr_t>(d_G) | reinterpret_cast<uintptr_t>(d_W) |
         reinterpret_cast<uintptr_t>(d_ws)) & 255u)
        return fail(RECON_EINVAL, "G, W and workspace must be 256-byte aligned");
    size_t need = 0;
    recon_query_sizes(p, nullptr, nullptr, &need);
    if (ws_bytes < need)
        return fail(RECON_ENOMEM, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);

    recon_ctx *c = new (std::nothrow) recon_ctx();
    if (!c) return fail(RECON_ENOMEM, "host allocation failed");
    c->p = *p;
    c->G = static_cast<float2 *>(d_G);
    c->W = static_cast<float *>(d_W);
    c->ws = static_cast<unsigned char *>(d_ws);
    c->ws_bytes = ws_bytes;
    c->stream = static_cast<hipStream_t>(stream);
    c->cfg = default_config();

    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipGetDevice"); }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, c->device);
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipGetDeviceProperties"); }
    c->num_cu = prop.multiProcessorCount;
    c->max_lds = prop.sharedMemPerBlock;
    c->max_threads = prop.maxThreadsPerBlock;

    const int h = p->n / 2;
    c->g.n = p->n;
    c->g.h = h;
    c->g.dim = p->n + 1;
    c->g.sw = h + 1;
    c->g.a = p->blob_radius;
    c->g.a2 = p->blob_radius * p->blob_radius;
    c->g.N = p->table_size;
    const double a = p->blob_radius;
    // table steps per unit squared distance (on the fly: none, positions in units of a)
    c->g.tscale = p->table_size > 0 ? static_cast<float>((p->table_size - 1) / (a * a))
                                    : static_cast<float>(1.0 / (a * a));
    c->g.inv_a2 = static_cast<float>(1.0 / (a * a));
    c->g.r2max = p->r_max * p->r_max;
    c->g.dtype = p->slice_dtype;
    c->g.scales = nullptr;
    // the blob as a polynomial in s = 1 - d^2/a^2, for weights on the fly
    std::vector<double> coef;
    c->g.nterms = blob_coefficients(p->blob_alpha, p->blob_order, &coef);   // > 0 if table_size == 0 (validated)
    const int mode = weight_source(*p, RECON_WEIGHTS_DEFAULT);
    // the current configuration names its weight source, as the tuning space does
    c->cfg.weights = mode == recon::WEIGHT_OTF ? RECON_WEIGHTS_OTF : RECON_WEIGHTS_TABLE;
    if (mode == recon::WEIGHT_OTF) c->cfg.slab_flags = 4;   // no window preload on the fly
    if (slab_wide_ok(c->g, mode, c->max_lds)) {
        // three waves per SIMD where the 11-wave instance applies (the
        // fastest measured configuration for the 4 x 4 window)
        c->cfg.waves_per_block = 11;
        c->cfg.slab_flags = 4;
        c->cfg.inner_chunk = 64;
        c->cfg.split = 32;
    }
    if (recon::slab_lds_bytes(c->g, mode, c->cfg.waves_per_block) > c->max_lds) {
        // blob table too large for the slab kernel's LDS budget
        c->cfg.variant = static_cast<size_t>(p->table_size) * sizeof(float2) <= c->max_lds ? RECON_VARIANT_BINNED
                                                                                             : RECON_VARIANT_NAIVE;
        c->cfg.waves_per_block = 16;
    }

    c->L = worst_layout(*p);
    c->plan = make_plan(*p, c->cfg.split, tile_edge(c->cfg.variant), spatial_queue(c->cfg));

    // blob table: entry i = (T[i], T[i+1] - T[i]), T[i] = b(i a^2 / (N-1)), built in FP64;
    // then the polynomial's coefficients (coefficient, 0)
    const int N = p->table_size;
    std::vector<double> T(N);
    for (int i = 0; i < N; ++i)
        T[i] = kb_blob(static_cast<double>(i) * a * a / (N - 1), a, p->blob_alpha, p->blob_order);
    std::vector<float2> tab(N + recon::kMaxTerms, make_float2(0.f, 0.f));
    for (int i = 0; i < N; ++i) {
        const double next = i + 1 < N ? T[i + 1] : T[i];
        tab[i] = make_float2(static_cast<float>(T[i]), static_cast<float>(next - T[i]));
    }
    for (int k = 0; k < c->g.nterms; ++k) tab[N + k] = make_float2(static_cast<float>(coef[k]), 0.f);
    e = hipMemcpyAsync(c->ws + c->L.table, tab.data(), tab.size() * sizeof(float2), hipMemcpyHostToDevice,
                       c->stream);
    if (e != hipSuccess) { delete c; return hip_fail(e, "upload blob table"); }
    // counters
    e = recon::launch_zero(reinterpret_cast<float *>(c->ws + c->L.ctr), sizeof(Counters) / sizeof(float),
                           c->stream);
    if (e != hipSuccess) { delete c; return hip_fail(e, "clear counters"); }
    const size_t nvox = static_cast<size_t>(c->g.dim) * c->g.dim * c->g.dim;
    e = recon::launch_zero(reinterpret_cast<float *>(c->G), 2 * nvox, c->stream);
    if (e == hipSuccess) e = recon::launch_zero(c->W, nvox, c->stream);
    if (e != hipSuccess) { delete c; return hip_fail(e, "zero G, W"); }
    st = upload_plan(c);   // synchronises the stream (also covers the table copy)
    if (st != RECON_OK) { delete c; return st; }
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { delete c; return hip_fail(e, "recon_init sync"); }
    *out = c;
    return RECON_OK;
}

recon_status recon_reset(recon_ctx *c)
{
    if (!c) return fail(RECON_EINVAL, "ctx is NULL");
    const size_t nvox = static_cast<size_t>(c->g.dim) * c->g.dim * c->g.dim;
    hipError_t e = recon::launch_zero(reinterpret_cast<float *>(c->G), 2 * nvox, c->stream);
    if (e == hipSuccess) e = recon::launch_zero(c->W, nvox, c->stream);
    if (e == hipSuccess)
        e = recon::launch_zero(reinterpret_cast<float *>(c->ws + c->L.ctr), sizeof(Counters) / sizeof(float),
                               c->stream);
    if (e != hipSuccess) return hip_fail(e, "recon_reset");
    return RECON_OK;
}

recon_status recon_insert_batch(recon_ctx *c, const void *d_slices, const float *d_scales, const float *d_quats,
                                int32_t count)
{
    if (!c) return fail(RECON_EINVAL, "ctx is NULL");
    if (count < 0 || count > c->p.max_batch)
        return fail(RECON_EINVAL, "count must be in [0, max_batch=%d] (got %d)", c->p.max_batch, count);
    if (count == 0) return RECON_OK;
    if (!d_slices || !d_quats) return fail(RECON_EINVAL, "slices and quaternions must be non-NULL");
    if (c->p.slice_dtype == RECON_SLICE_F16 && !d_scales)
        return fail(RECON_EINVAL, "half-precision slices need per-slice scales");
    c->g.scales = c->p.slice_dtype == RECON_SLICE_F16 ? d_scales : nullptr;
    // dynamic tuning: measure the previous step, then pick this step's configuration
    bool tuning_step = false;
    if (c->tune.active || c->tune.pending >= 0) {
        recon_status st = tune_collect(c);
        if (st != RECON_OK) return st;
        TuneState &t = c->tune;
        if (t.active) {
            const bool done = t.steps_done >= t.max_steps || t.next >= t.order.size() ||
                              (t.target > 0.0 && t.best >= 0 && t.best_ns <= t.target);
            if (done) {
                st = tune_finish(c);
                if (st != RECON_OK) return st;
            } else {
                const int idx = t.order[t.next++];
                st = apply_config(c, t.space[idx]);
                if (st != RECON_OK) return st;
                t.pending = idx;
                t.pending_count = count;
                tuning_step = true;
            }
        }
    }
    Counters *ctr = reinterpret_cast<Counters *>(c->ws + c->L.ctr);
    Orient *orient = reinterpret_cast<Orient *>(c->ws + c->L.orient);
    float4 *rem = orient_rem(c);
    const float2 *table = reinterpret_cast<const float2 *>(c->ws + c->L.table);
    const void *slices = d_slices;
    const int mode = weight_source(c->p, c->cfg.weights);
    const recon::Geom g = launch_geom(c->g, mode);
    const bool exact = recon::exact_geometry(g);
    hipError_t e = recon::launch_prep(d_quats, count, g.tscale, exact, orient, rem, ctr, &ctr->queue, c->stream);
    if (e != hipSuccess) return hip_fail(e, "prep kernel launch");
    if (c->ev_start) {
        e = hipEventRecord(c->ev_start, c->stream);
        if (e != hipSuccess) return hip_fail(e, "record start event");
    }
    if (tuning_step) {
        e = hipEventRecord(c->tune.ev0, c->stream);
        if (e != hipSuccess) return hip_fail(e, "record tuning start event");
    }
    if (c->cfg.variant == RECON_VARIANT_NAIVE) {
        e = recon::launch_insert_naive(g, mode, slices, orient, count, table,
                                       c->cfg.inner_chunk, c->cfg.waves_per_block, c->G, c->W, c->stream);
        if (e != hipSuccess) return hip_fail(e, "naive insert kernel launch");
        if (c->ev_stop) {
            e = hipEventRecord(c->ev_stop, c->stream);
            if (e != hipSuccess) return hip_fail(e, "record stop event");
        }
        if (tuning_step) {
            e = hipEventRecord(c->tune.ev1, c->stream);
            if (e != hipSuccess) return hip_fail(e, "record tuning stop event");
        }
        return RECON_OK;
    }
    const Item *items = reinterpret_cast<const Item *>(c->ws + c->L.items);
    float4 *partials = reinterpret_cast<float4 *>(c->ws + c->L.partials);
    const int nitems = static_cast<int>(c->plan.items.size());
    const int blocks = c->cfg.cu_count > 0 ? c->cfg.cu_count : c->num_cu;
    const bool slab = c->cfg.variant == RECON_VARIANT_SLAB;
    recon::JobTable jt;
    if (slab) {
        std::memset(&jt, 0, sizeof(jt));
        jt.njobs = 1;
        jt.job[0] = {g, slices, orient, rem, partials, c->G, c->W, count, 0};
        e = recon::launch_insert_slab(jt, mode, c->cfg.slab_flags & 3, exact, table, items, nitems,
                                      c->cfg.inner_chunk, c->cfg.traversal & RECON_TRAVERSAL_COLUMNS_SECOND, blocks,
                                      c->cfg.waves_per_block, ctr, c->stream);
    } else
        e = recon::launch_insert_binned(g, mode, slices, orient, count, table, items, nitems,
                                        partials, c->cfg.inner_chunk, blocks, c->cfg.waves_per_block, ctr, c->G,
                                        c->W, c->stream);
    if (e != hipSuccess) return hip_fail(e, "insert kernel launch");
    if (c->ev_stop) {
        e = hipEventRecord(c->ev_stop, c->stream);
        if (e != hipSuccess) return hip_fail(e, "record stop event");
    }
    if (c->plan.nslots > 0) {
        e = slab ? recon::launch_reduce_partials8(jt, items + nitems, static_cast<int>(c->plan.ritems.size()),
                                                  c->stream)
                 : recon::launch_reduce_partials(c->g, items, nitems, partials, c->G, c->W, c->stream);
        if (e != hipSuccess) return hip_fail(e, "partial reduction launch");
    }
    // a tuning step is timed over the whole insertion: kernel and reduction
    if (tuning_step) {
        e = hipEventRecord(c->tune.ev1, c->stream);
        if (e != hipSuccess) return hip_fail(e, "record tuning stop event");
    }
    return RECON_OK;
}

recon_status recon_finalize(recon_ctx *c, void *d_V, float w_threshold)
{
    if (!c) return fail(RECON_EINVAL, "ctx is NULL");
    if (!(w_threshold >= 0.0f) || !std::isfinite(w_threshold))
        return fail(RECON_EINVAL, "w_threshold must be finite and >= 0");
    if (d_V && (reinterpret_cast<uintptr_t>(d_V) & 7u)) return fail(RECON_EINVAL, "V must be 8-byte aligned");
    hipError_t e = recon::launch_finalize(c->g, c->G, c->W, static_cast<float2 *>(d_V), w_threshold, c->stream);
    if (e != hipSuccess) return hip_fail(e, "finalize kernel launch");
    return RECON_OK;
}

}  // extern "C"

// Fills library defaults into a configuration and checks it against the
// device's limits; no side effects.
static recon_status resolve_config(const recon_ctx *c, const recon_config *cfg, recon_config *out)
{
    recon_config d = default_config();
    recon_config n = cfg ? *cfg : d;
    if (n.variant == RECON_VARIANT_AUTO) n.variant = d.variant;
    if (n.weights < RECON_WEIGHTS_DEFAULT || n.weights > RECON_WEIGHTS_OTF)
        return fail(RECON_ECONFIG, "weights must be 0 (default), 1 (table) or 2 (on the fly)");
    if (n.weights == RECON_WEIGHTS_DEFAULT) n.weights = c->p.table_size > 0 ? RECON_WEIGHTS_TABLE : RECON_WEIGHTS_OTF;
    if (n.weights == RECON_WEIGHTS_TABLE && c->p.table_size == 0)
        return fail(RECON_ECONFIG, "table weights need table_size > 0");
    if (n.weights == RECON_WEIGHTS_OTF && c->g.nterms == 0)
        return fail(RECON_ECONFIG, "weights on the fly need at most %d polynomial terms (alpha %g, order %d)",
                    recon::kMaxTerms, c->p.blob_alpha, c->p.blob_order);
    const int mode = weight_source(c->p, n.weights);
    const bool otf = mode == recon::WEIGHT_OTF;
    const bool wide = n.variant == RECON_VARIANT_SLAB && slab_wide_ok(c->g, mode, c->max_lds);
    if (n.waves_per_block == 0) n.waves_per_block = wide ? 11 : default_waves(n.variant);
    if (n.slab_flags == 0 && (n.waves_per_block == 11 || otf)) n.slab_flags = 4;
    if (n.group == 0) n.group = d.group;
    if (n.inner_chunk == 0) n.inner_chunk = default_inner_chunk(n.variant);
    if (n.split == 0) n.split = default_split(n.variant);
    if (n.slab_flags == 0) n.slab_flags = d.slab_flags;
    if (n.slab_flags < 4 || n.slab_flags > 7) return fail(RECON_ECONFIG, "slab_flags must be 4 | bits, bits in [0, 3]");
    if (n.variant != RECON_VARIANT_NAIVE && n.variant != RECON_VARIANT_BINNED && n.variant != RECON_VARIANT_SLAB)
        return fail(RECON_ECONFIG, "unknown variant %d", n.variant);
    const int wpb = n.waves_per_block;
    if (wpb != 1 && wpb != 2 && wpb != 4 && wpb != 8 && wpb != 11 && wpb != 12 && wpb != 16)
        return fail(RECON_ECONFIG, "waves_per_block must be 1, 2, 4, 8, 11, 12 or 16");
    if (wpb == 11 && n.variant != RECON_VARIANT_SLAB)
        return fail(RECON_ECONFIG, "11 waves per work-group is a slab-kernel configuration");
    if (64 * wpb > c->max_threads) return fail(RECON_ECONFIG, "work-group of %d threads exceeds device", 64 * wpb);
    if (n.group < 1 || n.group > 16) return fail(RECON_ECONFIG, "group must be in [1, 16]");
    if (n.inner_chunk < 1 || n.inner_chunk > 256) return fail(RECON_ECONFIG, "inner_chunk must be in [1, 256]");
    if (n.split < 1 || n.split > kMaxSplit) return fail(RECON_ECONFIG, "split must be in [1, %d]", kMaxSplit);
    if (n.variant == RECON_VARIANT_BINNED && !otf &&
        static_cast<size_t>(c->p.table_size) * sizeof(float2) > c->max_lds)
        return fail(RECON_ECONFIG, "blob table of %d entries does not fit in LDS", c->p.table_size);
    if (n.variant == RECON_VARIANT_SLAB && wpb > 8 && !(wpb == 11 && wide))
        return fail(RECON_ECONFIG, "slab kernel runs at most 8 waves per work-group, or 11 for the 4x4 window "
                                   "with table interpolation");
    if (n.variant == RECON_VARIANT_SLAB && otf && (n.slab_flags & 2))
        return fail(RECON_ECONFIG, "the window-preload flag has no instance with weights on the fly");
    if (n.variant == RECON_VARIANT_SLAB && recon::slab_lds_bytes(c->g, mode, wpb) > c->max_lds)
        return fail(RECON_ECONFIG, "slab kernel needs %zu bytes of LDS with %d waves (device: %zu)",
                    recon::slab_lds_bytes(c->g, mode, wpb), wpb, c->max_lds);
    if (n.cu_count < 0 || n.cu_count > c->num_cu)
        return fail(RECON_ECONFIG, "cu_count must be in [0, %d] (got %d)", c->num_cu, n.cu_count);
    if (n.traversal < 0 || n.traversal > 3)
        return fail(RECON_ECONFIG, "traversal must be a combination of bits 1 and 2 (got %d)", n.traversal);
    if ((n.traversal & RECON_TRAVERSAL_COLUMNS_SECOND) && n.variant != RECON_VARIANT_SLAB)
        return fail(RECON_ECONFIG, "the column order of the lanes is a slab-kernel setting");
    if ((n.traversal & RECON_TRAVERSAL_SPATIAL_QUEUE) && n.variant == RECON_VARIANT_NAIVE)
        return fail(RECON_ECONFIG, "the naive kernel has no work queue to order");
    *out = n;
    return RECON_OK;
}

// Makes a resolved configuration current (re-plans and uploads the work
// plan when the tiling or the split changes; that upload synchronises).
static recon_status apply_config(recon_ctx *c, const recon_config &n)
{
    const bool replan = n.split != c->cfg.split || tile_edge(n.variant) != tile_edge(c->cfg.variant) ||
                        spatial_queue(n) != spatial_queue(c->cfg);
    c->cfg = n;
    if (replan) {
        c->plan = make_plan(c->p, n.split, tile_edge(n.variant), spatial_queue(n));
        return upload_plan(c);
    }
    return RECON_OK;
}

// The tuning space: every runnable combination of the kernel knobs.
static std::vector<recon_config> tuning_space(const recon_ctx *c)
{
    std::vector<recon_config> out;
    const int variants[3] = {RECON_VARIANT_SLAB, RECON_VARIANT_BINNED, RECON_VARIANT_NAIVE};
    for (int v : variants) {
        const bool slab = v == RECON_VARIANT_SLAB;
        std::vector<int> waves = slab ? std::vector<int>{4, 8, 11}
                                 : v == RECON_VARIANT_BINNED ? std::vector<int>{8, 16}
                                                             : std::vector<int>{4, 8, 16};
        std::vector<int> splits = v == RECON_VARIANT_NAIVE ? std::vector<int>{32} : std::vector<int>{8, 16, 32, 64};
        // traversal: both bits for the slab kernel, the queue order for the
        // binned one, none for the naive one
        std::vector<int> orders = slab ? std::vector<int>{0, 1, 2, 3}
                                  : v == RECON_VARIANT_BINNED ? std::vector<int>{0, 2} : std::vector<int>{0};
        for (int wt : {RECON_WEIGHTS_TABLE, RECON_WEIGHTS_OTF})
            for (int wpb : waves)
                for (int inner : {16, 32, 64})
                    for (int sp : splits)
                        for (int fl : (!slab ? std::vector<int>{6}
                                       : wpb == 11 ? std::vector<int>{4, 5}   // no window preload at 11 waves
                                                   : std::vector<int>{4, 5, 6, 7}))
                            for (int tv : orders) {
                                recon_config in;
                                std::memset(&in, 0, sizeof(in));
                                in.variant = v;
                                in.waves_per_block = wpb;
                                in.group = 1;
                                in.inner_chunk = inner;
                                in.split = sp;
                                in.slab_flags = fl;
                                in.weights = wt;
                                in.traversal = tv;
                                in.cu_count = c->cfg.cu_count;   // a property of the stream, not tuned
                                recon_config r;
                                const std::string keep = g_err;
                                if (resolve_config(c, &in, &r) == RECON_OK) out.push_back(r);
                                g_err = keep;
                            }
    }
    return out;
}

static recon_status tune_collect(recon_ctx *c)
{
    TuneState &t = c->tune;
    if (t.pending < 0) return RECON_OK;
    hipError_t e = hipEventSynchronize(t.ev1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.ev0, t.ev1);
    if (e != hipSuccess) return hip_fail(e, "tuning step timing");
    const double ns = 1e6 * static_cast<double>(ms) / std::max(1, t.pending_count);
    t.ns[t.pending] = ns;
    t.sum_ns += ns;
    ++t.steps_done;
    if (ns < t.best_ns) {
        t.best_ns = ns;
        t.best = t.pending;
    }
    t.pending = -1;
    return RECON_OK;
}

static recon_status tune_finish(recon_ctx *c)
{
    TuneState &t = c->tune;
    recon_status st = tune_collect(c);
    if (st != RECON_OK) return st;
    t.active = false;
    if (t.best >= 0) return apply_config(c, t.space[t.best]);
    return RECON_OK;
}

static void tune_release(recon_ctx *c)
{
    if (c->tune.ev0) (void)hipEventDestroy(c->tune.ev0);
    if (c->tune.ev1) (void)hipEventDestroy(c->tune.ev1);
    c->tune.ev0 = c->tune.ev1 = nullptr;
}

extern "C" {

recon_status recon_set_config(recon_ctx *c, const recon_config *cfg)
{
    if (!c) return fail(RECON_EINVAL, "ctx is NULL");
    recon_config n;
    recon_status st = resolve_config(c, cfg, &n);
    if (st != RECON_OK) return st;
    return apply_config(c, n);
}

recon_status recon_tune_space_size(const recon_ctx *c, int32_t *size)
{
    if (!c || !size) return fail(RECON_EINVAL, "NULL argument");
    *size = static_cast<int32_t>(tuning_space(c).size());
    return RECON_OK;
}

recon_status recon_tune_space_config(const recon_ctx *c, int32_t index, recon_config *out)
{
    if (!c || !out) return fail(RECON_EINVAL, "NULL argument");
    const std::vector<recon_config> sp = tuning_space(c);
    if (index < 0 || index >= static_cast<int32_t>(sp.size()))
        return fail(RECON_EINVAL, "index %d outside the tuning space (size %zu)", index, sp.size());
    *out = sp[index];
    return RECON_OK;
}

recon_status recon_tune_begin(recon_ctx *c, const recon_tune_opts *opts)
{
    if (!c || !opts) return fail(RECON_EINVAL, "NULL argument");
    if (opts->max_steps < 0) return fail(RECON_EINVAL, "max_steps must be >= 0");
    if (!(opts->target_ns_per_slice >= 0.0)) return fail(RECON_EINVAL, "target must be >= 0");
    recon_status st = tune_collect(c);
    if (st != RECON_OK) return st;
    TuneState &t = c->tune;
    if (!t.ev0) {
        hipError_t e = hipEventCreate(&t.ev0);
        if (e == hipSuccess) e = hipEventCreate(&t.ev1);
        if (e != hipSuccess) return hip_fail(e, "create tuning events");
    }
    std::vector<recon_config> space = tuning_space(c);
    if (space.empty()) return fail(RECON_ECONFIG, "empty tuning space on this device");
    const int n = static_cast<int>(space.size());
    std::vector<int> order;
    if (opts->order) {
        // caller's candidates, in the caller's order
        if (opts->order_count < 1 || opts->order_count > n)
            return fail(RECON_EINVAL, "order_count must be in [1, %d] (got %d)", n, opts->order_count);
        std::vector<char> seen(n, 0);
        for (int i = 0; i < opts->order_count; ++i) {
            const int k = opts->order[i];
            if (k < 0 || k >= n) return fail(RECON_EINVAL, "order[%d] = %d outside [0, %d)", i, k, n);
            if (seen[k]) return fail(RECON_EINVAL, "order[%d] = %d repeats a candidate", i, k);
            seen[k] = 1;
            order.push_back(k);
        }
    } else {
        order.resize(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        uint64_t x = opts->seed;
        for (int i = n - 1; i > 0; --i) {
            const int j = static_cast<int>(splitmix64(x) % static_cast<uint64_t>(i + 1));
            std::swap(order[i], order[j]);
        }
    }
    const int m = static_cast<int>(order.size());
    t.space = std::move(space);
    t.order = std::move(order);
    t.next = 0;
    t.max_steps = opts->max_steps == 0 ? m : std::min(opts->max_steps, m);
    t.target = opts->target_ns_per_slice;
    t.steps_done = 0;
    t.pending = -1;
    t.ns.assign(n, -1.0);
    t.best = -1;
    t.best_ns = std::numeric_limits<double>::infinity();
    t.sum_ns = 0.0;
    t.active = true;
    return RECON_OK;
}

recon_status recon_tune_get_info(recon_ctx *c, recon_tune_info *info)
{
    if (!c || !info) return fail(RECON_EINVAL, "NULL argument");
    recon_status st = tune_collect(c);
    if (st != RECON_OK) return st;
    const TuneState &t = c->tune;
    std::memset(info, 0, sizeof(*info));
    info->active = t.active ? 1 : 0;
    info->steps_done = t.steps_done;
    info->space_size = static_cast<int32_t>(t.space.empty() ? tuning_space(c).size() : t.space.size());
    info->best_index = t.best;
    info->best_ns_per_slice = t.best >= 0 ? t.best_ns : 0.0;
    info->mean_ns_per_slice = t.steps_done > 0 ? t.sum_ns / t.steps_done : 0.0;
    if (t.best >= 0) info->best = t.space[t.best];
    return RECON_OK;
}

recon_status recon_tune_end(recon_ctx *c)
{
    if (!c) return fail(RECON_EINVAL, "ctx is NULL");
    return tune_finish(c);
}

recon_status recon_tune_invocations(double rp, double s, double t_avg, double t_well, double *n)
{
    if (!n) return fail(RECON_EINVAL, "NULL argument");
    if (!(rp > 0.0 && rp < 1.0) || !(s >= 0.0) || !(t_well > 0.0) || !(t_avg >= 0.0))
        return fail(RECON_EINVAL, "need 0 < rp < 1, s >= 0, t_avg >= 0, t_well > 0");
    *n = rp * s * (t_avg / t_well - 1.0) / (1.0 - rp);
    return RECON_OK;
}

recon_status recon_tune_steps(double r, double p, double *s)
{
    if (!s) return fail(RECON_EINVAL, "NULL argument");
    if (!(r > 0.0 && r < 1.0) || !(p >= 0.0 && p < 1.0)) return fail(RECON_EINVAL, "need 0 < r < 1 and 0 <= p < 1");
    *s = std::log1p(-p) / std::log1p(-r);
    return RECON_OK;
}

recon_status recon_get_config(const recon_ctx *c, recon_config *cfg)
{
    if (!c || !cfg) return fail(RECON_EINVAL, "NULL argument");
    *cfg = c->cfg;
    return RECON_OK;
}

recon_status recon_set_stream(recon_ctx *c, void *stream)
{
    if (!c) return fail(RECON_EINVAL, "ctx is NULL");
    c->stream = static_cast<hipStream_t>(stream);
    return RECON_OK;
}

recon_status recon_set_timing_events(recon_ctx *c, void *start, void *stop)
{
    if (!c) return fail(RECON_EINVAL, "ctx is NULL");
    if ((start == nullptr) != (stop == nullptr)) return fail(RECON_EINVAL, "give both events or neither");
    c->ev_start = static_cast<hipEvent_t>(start);
    c->ev_stop = static_cast<hipEvent_t>(stop);
    return RECON_OK;
}

recon_status recon_stats(recon_ctx *c, uint64_t *inserted, uint64_t *rejected)
{
    if (!c) return fail(RECON_EINVAL, "ctx is NULL");
    Counters h;
    hipError_t e = hipMemcpyAsync(&h, c->ws + c->L.ctr, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "recon_stats");
    if (inserted) *inserted = h.inserted;
    if (rejected) *rejected = h.rejected;
    return RECON_OK;
}

}  // extern "C"

struct recon_batch {
    std::vector<recon_ctx *> ctxs;
    unsigned char *ws;
    size_t ws_bytes;
    int nitems;
    int nritems;   // split tiles, stored after the items
    size_t off_items;
    int wpb, flags, inner, lanes;   // slab launch configuration of the batch
    int mode;                       // weight source
};

// Launch configuration of a batch (the contexts share their blob): the
// first context's configuration when it is a slab-kernel one (set with
// recon_set_config or picked by its tuner; its queue-order bit does not
// apply, the batch's queue interleaves the jobs by cost), else the slab
// kernel's single-context default, 11 waves with interleaved window reads
// where that instance exists and fits, else 8 waves with preloaded reads.
struct BatchLaunch {
    int wpb, flags, inner, split, mode, lanes;
};
static BatchLaunch batch_launch(const recon_ctx *c0)
{
    if (c0->cfg.variant == RECON_VARIANT_SLAB)
        return {c0->cfg.waves_per_block, c0->cfg.slab_flags & 3, c0->cfg.inner_chunk, c0->cfg.split,
                weight_source(c0->p, c0->cfg.weights), c0->cfg.traversal & RECON_TRAVERSAL_COLUMNS_SECOND};
    const int mode = weight_source(c0->p, RECON_WEIGHTS_DEFAULT);
    if (slab_wide_ok(c0->g, mode, c0->max_lds)) return {11, 0, 64, 32, mode, 0};
    return {8, mode == recon::WEIGHT_OTF ? 0 : 2, 32, 32, mode, 0};
}

// Combined work plan of a batch: every context's slab plan (split of the
// batch's launch configuration), tagged with its job index in the tile
// field's top byte, in decreasing estimated cost across all jobs (the plans'
// own cost estimates, in slice visits).
static recon_status batch_plan(recon_ctx *const *ctxs, int32_t njobs, std::vector<Item> *items)
{
    if (!ctxs || njobs < 1 || njobs > recon::kMaxJobs)
        return fail(RECON_EINVAL, "a batch holds 1 to %d contexts", recon::kMaxJobs);
    for (int j = 0; j < njobs; ++j) {
        if (!ctxs[j]) return fail(RECON_EINVAL, "context %d is NULL", j);
        const recon_params &p = ctxs[j]->p, &q = ctxs[0]->p;
        if (p.blob_radius != q.blob_radius || p.blob_alpha != q.blob_alpha || p.blob_order != q.blob_order ||
            p.table_size != q.table_size || p.table_lerp != q.table_lerp)
            return fail(RECON_EINVAL, "batched contexts must share blob parameters (context %d differs)", j);
        if (ctxs[j]->device != ctxs[0]->device) return fail(RECON_EINVAL, "batched contexts must share a device");
        if (p.slice_dtype != q.slice_dtype)
            return fail(RECON_EINVAL, "batched contexts must share the slice storage type (context %d differs)", j);
        for (int k = 0; k < j; ++k)
            if (ctxs[k] == ctxs[j]) return fail(RECON_EINVAL, "context %d appears twice", j);
    }
    struct Tmp { Item it; double cost; };
    std::vector<Tmp> all;
    const int split = batch_launch(ctxs[0]).split;
    // Item sizes follow the cost of the whole launch, not each job's alone
    // (a larger target gives each tile at most as many parts, so every job's
    // partial-sum slots still fit its workspace); the items of all jobs are
    // then ordered by their estimated cost.
    double launch_total = 0.0;
    for (int j = 0; j < njobs; ++j)
        for (double c : make_plan(ctxs[j]->p, split, 8, false).cost) launch_total += c;
    for (int j = 0; j < njobs; ++j) {
        const Plan pl = make_plan(ctxs[j]->p, split, 8, false, launch_total);
        // slots of three planes of 512 floats in the job's workspace
        const size_t cap = (ctxs[j]->L.total - ctxs[j]->L.partials) / (384 * sizeof(float4));
        if (static_cast<size_t>(pl.nslots) > cap)
            return fail(RECON_ECONFIG, "batch plan of context %d needs %d partial-sum slots (workspace: %zu)", j,
                        pl.nslots, cap);
        for (size_t i = 0; i < pl.items.size(); ++i) {
            Item it = pl.items[i];
            if (it.tile >= (1 << 24)) return fail(RECON_EINVAL, "box too large for a batch");
            it.tile |= j << 24;
            all.push_back({it, pl.cost[i]});
        }
    }
    std::stable_sort(all.begin(), all.end(), [](const Tmp &x, const Tmp &y) { return x.cost > y.cost; });
    items->clear();
    for (const Tmp &t : all) items->push_back(t.it);
    return RECON_OK;
}

extern "C" {

recon_status recon_batch_query_size(recon_ctx *const *ctxs, int32_t njobs, size_t *ws_bytes)
{
    if (!ws_bytes) return fail(RECON_EINVAL, "ws_bytes is NULL");
    std::vector<Item> items;
    recon_status st = batch_plan(ctxs, njobs, &items);
    if (st != RECON_OK) return st;
    *ws_bytes = align_up(sizeof(Counters), 256) + align_up(2 * items.size() * sizeof(Item), 256);
    return RECON_OK;
}

recon_status recon_batch_create(recon_ctx *const *ctxs, int32_t njobs, void *d_ws, size_t ws_bytes, recon_batch **out)
{
    if (!out) return fail(RECON_EINVAL, "out is NULL");
    *out = nullptr;
    std::vector<Item> items;
    recon_status st = batch_plan(ctxs, njobs, &items);
    if (st != RECON_OK) return st;
    const size_t need = align_up(sizeof(Counters), 256) + align_up(2 * items.size() * sizeof(Item), 256);
    if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) & 255u)) return fail(RECON_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(RECON_ENOMEM, "batch workspace too small: %zu given, %zu needed", ws_bytes, need);
    const BatchLaunch bl = batch_launch(ctxs[0]);
    for (int j = 0; j < njobs; ++j)
        if (recon::slab_lds_bytes(ctxs[j]->g, bl.mode, bl.wpb) > ctxs[j]->max_lds)
            return fail(RECON_ECONFIG, "the slab kernel does not fit this device for context %d", j);
    recon_batch *b = new (std::nothrow) recon_batch();
    if (!b) return fail(RECON_ENOMEM, "host allocation failed");
    b->ctxs.assign(ctxs, ctxs + njobs);
    b->ws = static_cast<unsigned char *>(d_ws);
    b->ws_bytes = ws_bytes;
    b->nitems = static_cast<int>(items.size());
    b->off_items = align_up(sizeof(Counters), 256);
    b->wpb = bl.wpb;
    b->flags = bl.flags;
    b->inner = bl.inner;
    b->lanes = bl.lanes;
    b->mode = bl.mode;
    hipStream_t st0 = ctxs[0]->stream;
    hipError_t e = recon::launch_zero(reinterpret_cast<float *>(b->ws), sizeof(Counters) / sizeof(float), st0);
    // items, then the split tiles right after them
    const std::vector<Item> rit = split_tiles(items);
    b->nritems = static_cast<int>(rit.size());
    std::vector<Item> all(items);
    all.insert(all.end(), rit.begin(), rit.end());
    if (e == hipSuccess && !all.empty())
        e = hipMemcpyAsync(b->ws + b->off_items, all.data(), all.size() * sizeof(Item), hipMemcpyHostToDevice, st0);
    if (e == hipSuccess) e = hipStreamSynchronize(st0);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "upload batch plan");
    }
    *out = b;
    return RECON_OK;
}

recon_status recon_batch_insert(recon_batch *b, const void *const *d_slices, const float *const *d_scales,
                                const float *const *d_quats, const int32_t *counts)
{
    if (!b || !d_slices || !d_quats || !counts) return fail(RECON_EINVAL, "NULL argument");
    const int nj = static_cast<int>(b->ctxs.size());
    hipStream_t st = b->ctxs[0]->stream;
    recon::JobTable jt;
    std::memset(&jt, 0, sizeof(jt));
    jt.njobs = nj;
    for (int j = 0; j < nj; ++j) {
        recon_ctx *c = b->ctxs[j];
        if (counts[j] < 0 || counts[j] > c->p.max_batch)
            return fail(RECON_EINVAL, "counts[%d] = %d outside [0, %d]", j, counts[j], c->p.max_batch);
        if (counts[j] > 0 && (!d_slices[j] || !d_quats[j])) return fail(RECON_EINVAL, "job %d: NULL buffers", j);
        const float *sc = d_scales ? d_scales[j] : nullptr;
        if (counts[j] > 0 && c->p.slice_dtype == RECON_SLICE_F16 && !sc)
            return fail(RECON_EINVAL, "job %d: half-precision slices need scales", j);
        recon::Geom g = launch_geom(c->g, b->mode);
        g.scales = c->p.slice_dtype == RECON_SLICE_F16 ? sc : nullptr;
        jt.job[j] = {g, d_slices[j], reinterpret_cast<const Orient *>(c->ws + c->L.orient), orient_rem(c),
                     reinterpret_cast<float4 *>(c->ws + c->L.partials), c->G, c->W, counts[j], 0};
    }
    Counters *bctr = reinterpret_cast<Counters *>(b->ws);
    // one geometry mode for the whole launch: exact if any box needs it
    bool exact = false;
    for (int j = 0; j < nj; ++j) exact = exact || recon::exact_geometry(jt.job[j].g);
    for (int j = 0; j < nj; ++j) {
        recon_ctx *c = b->ctxs[j];
        if (counts[j] == 0 && j != 0) continue;
        hipError_t e = recon::launch_prep(counts[j] > 0 ? d_quats[j] : nullptr, counts[j], jt.job[j].g.tscale, exact,
                                          reinterpret_cast<Orient *>(c->ws + c->L.orient), orient_rem(c),
                                          reinterpret_cast<Counters *>(c->ws + c->L.ctr),
                                          j == 0 ? &bctr->queue : nullptr, st);
        if (e != hipSuccess) return hip_fail(e, "batch prep launch");
    }
    const Item *items = reinterpret_cast<const Item *>(b->ws + b->off_items);
    recon_ctx *c0 = b->ctxs[0];
    const float2 *table = reinterpret_cast<const float2 *>(c0->ws + c0->L.table);
    // the first context's timing events, if set, bracket the batched kernel
    if (c0->ev_start) {
        hipError_t er = hipEventRecord(c0->ev_start, st);
        if (er != hipSuccess) return hip_fail(er, "record start event");
    }
    hipError_t e = recon::launch_insert_slab(jt, b->mode, b->flags, exact, table, items, b->nitems, b->inner,
                                             b->lanes, c0->cfg.cu_count > 0 ? c0->cfg.cu_count : c0->num_cu,
                                             b->wpb, bctr, st);
    if (e == hipSuccess && c0->ev_stop) e = hipEventRecord(c0->ev_stop, st);
    if (e == hipSuccess) e = recon::launch_reduce_partials8(jt, items + b->nitems, b->nritems, st);
    if (e != hipSuccess) return hip_fail(e, "batch insert launch");
    return RECON_OK;
}

void recon_batch_destroy(recon_batch *b) { delete b; }

static recon_status mlp_check(int32_t n_in, int32_t H, int32_t C, int32_t B)
{
    if (n_in < 1 || n_in > 64 || H < 1 || H > 1024 || C < 2 || C > 4096 || B < 1 || B > 65536)
        return fail(RECON_EINVAL, "MLP sizes out of range (n_in %d, hidden %d, out %d, batch %d)", n_in, H, C, B);
    return RECON_OK;
}

recon_status recon_mlp_sizes(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t batch, size_t *param_floats,
                             size_t *ws_bytes)
{
    recon_status st = mlp_check(n_in, n_hidden, n_out, batch);
    if (st != RECON_OK) return st;
    if (param_floats) *param_floats = recon::mlp_param_count(n_in, n_hidden, n_out);
    if (ws_bytes) *ws_bytes = recon::mlp_ws_floats(n_in, n_hidden, n_out, batch) * sizeof(float);
    return RECON_OK;
}

recon_status recon_mlp_forward(const float *d_params, int32_t n_in, int32_t n_hidden, int32_t n_out, const float *d_x,
                               int32_t batch, void *d_ws, float *d_probs, void *stream)
{
    recon_status st = mlp_check(n_in, n_hidden, n_out, batch);
    if (st != RECON_OK) return st;
    if (!d_params || !d_x || !d_ws || !d_probs) return fail(RECON_EINVAL, "NULL device buffer");
    hipError_t e = recon::mlp_forward(d_params, n_in, n_hidden, n_out, d_x, batch, static_cast<float *>(d_ws), d_probs,
                                      static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "MLP forward launch");
    return RECON_OK;
}

recon_status recon_mlp_train_step(float *d_params, int32_t n_in, int32_t n_hidden, int32_t n_out, const float *d_x,
                                  const float *d_y, int32_t batch, float lr, void *d_ws, float *d_loss,
                                  float *d_grads, void *stream)
{
    recon_status st = mlp_check(n_in, n_hidden, n_out, batch);
    if (st != RECON_OK) return st;
    if (!d_params || !d_x || !d_y || !d_ws) return fail(RECON_EINVAL, "NULL device buffer");
    if (!std::isfinite(lr)) return fail(RECON_EINVAL, "learning rate must be finite");
    hipError_t e = recon::mlp_train_step(d_params, n_in, n_hidden, n_out, d_x, d_y, batch, lr,
                                         static_cast<float *>(d_ws), d_loss, d_grads, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "MLP training step launch");
    return RECON_OK;
}

void recon_destroy(recon_ctx *c)
{
    if (!c) return;
    tune_release(c);
    release_static_workspace(c->static_device);
    delete c;
}

recon_status recon_init_static(const recon_params *p, void *d_G, void *d_W, void *stream, recon_ctx **out)
{
    if (!out) return fail(RECON_EINVAL, "out is NULL");
    *out = nullptr;
    recon_status st = validate(p);
    if (st != RECON_OK) return st;
    // the size check comes before any device call
    size_t need = 0;
    recon_query_sizes(p, nullptr, nullptr, &need);
    if (need > kStaticWsBytes)
        return fail(RECON_ENOMEM, "these parameters need %zu bytes of workspace; the static workspace holds %zu "
                                  "(use recon_init with a caller buffer, or a smaller max_batch)",
                    need, kStaticWsBytes);
    int dev = -1;
    unsigned char *ws = nullptr;
    st = acquire_static_workspace(&dev, &ws);
    if (st != RECON_OK) return st;
    st = recon_init(p, d_G, d_W, ws, kStaticWsBytes, stream, out);
    if (st != RECON_OK) {
        release_static_workspace(dev);
        return st;
    }
    (*out)->static_device = dev;
    return RECON_OK;
}

}  // extern "C"
