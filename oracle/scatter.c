/*
 * Plain FP64 CPU oracle for Fourier-slice insertion (test infrastructure only:
 * it is built and called by tests, the smoke check and the benchmark's CPU
 * baseline, never by the product library).
 *
 * What it computes follows the paper's 3D reconstruction loop (Sect. 5.3.1,
 * Algorithm 1 "3D reconstruction": zero G and W, insert the samples of each
 * buffer of slice transforms into G and W, apply the weights W to G) and the
 * insertion step of Sect. 4.2 ("3D Fourier Reconstruction": 2D samples of
 * arbitrary orientation inserted into the 3D volume, with precomputed or
 * on-the-fly interpolation weights).  Readings where the paper is silent:
 *
 *   - volume B = {-h..h}^3 (h = n/2), stored [z][y][x], index = coordinate + h;
 *   - slice s is stored as the Hermitian half plane F_s[ky + h][kx],
 *     kx in [0, h]; the full-plane value is F~(k) = F(k) when kx > 0 or
 *     (kx = 0 and ky >= 0), otherwise conj F(-k);
 *   - inserted samples: the disk P = {k : kx^2 + ky^2 < r_max^2};
 *   - sample k of slice s sits at p = R_s (kx, ky, 0)^T;
 *   - every voxel v in B with |v - p|^2 <= a^2 receives
 *     G[v] += b(|v-p|^2) F~(k),  W[v] += b(|v-p|^2),  and the pair count U += 1;
 *   - b is the Kaiser-Bessel blob, exact (power series) or tabulated in d^2
 *     with linear interpolation or truncation.
 *
 * Everything is FP64.  The scatter loop runs over slices in parallel with
 * thread-private volumes that are summed in thread order at the end.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { BLOB_EXACT = 0, BLOB_TABLE_LERP = 1, BLOB_TABLE_TRUNC = 2 };

typedef struct {
    double a, a2, alpha;
    int m;
    int mode;
    const double *table;
    int N;
    double inv_im_alpha;
} blob_t;

/* I_m(x) from its power series sum_j (x/2)^(2j+m) / (j! (j+m)!). */
static double bessel_i_series(int m, double x)
{
    double half = 0.5 * x, q = half * half;
    double term = 1.0, total;
    for (int j = 1; j <= m; ++j) term *= half / j;
    total = term;
    for (int j = 1; j < 400; ++j) {
        term *= q / ((double)j * (double)(j + m));
        total += term;
        if (term <= 1e-18 * total) break;
    }
    return total;
}

static double blob_weight(const blob_t *b, double d2)
{
    if (d2 > b->a2) return 0.0;
    if (b->mode == BLOB_EXACT) {
        double s = 1.0 - d2 / b->a2;
        if (s < 0.0) s = 0.0;
        double r = sqrt(s);
        double scale = (b->m == 0) ? 1.0 : pow(s, 0.5 * b->m);
        return scale * bessel_i_series(b->m, b->alpha * r) * b->inv_im_alpha;
    } else {
        double t = d2 * (b->N - 1) / b->a2;
        long i = (long)floor(t);
        if (i > b->N - 1) i = b->N - 1;
        if (i < 0) i = 0;
        if (b->mode == BLOB_TABLE_TRUNC) return b->table[i];
        double f = t - (double)i;
        long i1 = (i + 1 < b->N) ? i + 1 : b->N - 1;
        return (1.0 - f) * b->table[i] + f * b->table[i1];
    }
}

static int blob_init(blob_t *b, double a, double alpha, int m, int mode,
                     const double *table, int N)
{
    if (!(a > 0.0) || !(alpha >= 0.0) || m < 0) return -1;
    if (mode != BLOB_EXACT && (table == NULL || N < 2)) return -1;
    b->a = a; b->a2 = a * a; b->alpha = alpha; b->m = m; b->mode = mode;
    b->table = table; b->N = N;
    b->inv_im_alpha = 1.0 / bessel_i_series(m, alpha);
    return 0;
}

/* Full-plane value F~(k) of slice Fs (complex64 interleaved, [n][h+1]). */
static void sample_full(const float *Fs, int n, int kx, int ky, double *re, double *im)
{
    int h = n / 2, w = h + 1;
    if (kx > 0 || (kx == 0 && ky >= 0)) {
        const float *p = Fs + 2 * ((size_t)(ky + h) * w + kx);
        *re = p[0]; *im = p[1];
    } else {
        const float *p = Fs + 2 * ((size_t)(-ky + h) * w + (-kx));
        *re = p[0]; *im = -(double)p[1];
    }
}

/* Scatter every sample of every slice into the full box.
 *   F : [S][n][n/2+1] complex64 (interleaved float pairs)
 *   R : [S][3][3] row-major FP64 rotation matrices
 *   G : [(n+1)^3][2] FP64 (accumulated into), W : [(n+1)^3] FP64, U : pair count,
 *   Uhalf (may be NULL) : pairs whose voxel has x >= 0
 * Returns 0, or -1 on invalid arguments, -2 when memory runs out. */
int oracle_insert(int n, int S, const float *F, const double *R,
                  double a, double alpha, int m, int mode, const double *table, int N,
                  double r_max, double *G, double *W, uint64_t *U, uint64_t *Uhalf, int nthreads)
{
    blob_t b;
    if (n < 2 || (n & 1) || S < 0 || !G || !W || !U) return -1;
    if (S > 0 && (!F || !R)) return -1;
    if (!(r_max > 0.0) || r_max > 0.5 * n) return -1;
    if (blob_init(&b, a, alpha, m, mode, table, N)) return -1;
    const int h = n / 2, dim = n + 1;
    const size_t nvox = (size_t)dim * dim * dim;
    const size_t slice_len = (size_t)n * (h + 1) * 2;
    const double r2max = r_max * r_max;
    if (nthreads < 1) nthreads = 1;
#ifndef _OPENMP
    nthreads = 1;
#endif
    double **pg = calloc((size_t)nthreads, sizeof(double *));
    double **pw = calloc((size_t)nthreads, sizeof(double *));
    uint64_t *pu = calloc((size_t)nthreads, sizeof(uint64_t));
    uint64_t *ph = calloc((size_t)nthreads, sizeof(uint64_t));
    int oom = (!pg || !pw || !pu || !ph);
    for (int t = 0; t < nthreads && !oom; ++t) {
        pg[t] = calloc(nvox * 2, sizeof(double));
        pw[t] = calloc(nvox, sizeof(double));
        if (!pg[t] || !pw[t]) oom = 1;
    }
    if (!oom) {
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static)
#endif
        for (int s = 0; s < S; ++s) {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double *g = pg[tid], *wv = pw[tid];
            uint64_t cnt = 0, cnt_half = 0;
            const float *Fs = F + (size_t)s * slice_len;
            const double *Rs = R + (size_t)s * 9;
            for (int ky = -h; ky <= h; ++ky) {
                for (int kx = -h; kx <= h; ++kx) {
                    if ((double)kx * kx + (double)ky * ky >= r2max) continue;
                    double fre, fim;
                    sample_full(Fs, n, kx, ky, &fre, &fim);
                    double px = Rs[0] * kx + Rs[1] * ky;
                    double py = Rs[3] * kx + Rs[4] * ky;
                    double pz = Rs[6] * kx + Rs[7] * ky;
                    int x0 = (int)ceil(px - a), x1 = (int)floor(px + a);
                    int y0 = (int)ceil(py - a), y1 = (int)floor(py + a);
                    int z0 = (int)ceil(pz - a), z1 = (int)floor(pz + a);
                    for (int vz = z0; vz <= z1; ++vz) {
                        if (vz < -h || vz > h) continue;
                        for (int vy = y0; vy <= y1; ++vy) {
                            if (vy < -h || vy > h) continue;
                            for (int vx = x0; vx <= x1; ++vx) {
                                if (vx < -h || vx > h) continue;
                                double dx = vx - px, dy = vy - py, dz = vz - pz;
                                double d2 = dx * dx + dy * dy + dz * dz;
                                if (d2 > b.a2) continue;
                                double wgt = blob_weight(&b, d2);
                                size_t idx = ((size_t)(vz + h) * dim + (vy + h)) * dim + (vx + h);
                                g[2 * idx] += wgt * fre;
                                g[2 * idx + 1] += wgt * fim;
                                wv[idx] += wgt;
                                ++cnt;
                                if (vx >= 0) ++cnt_half;
                            }
                        }
                    }
                }
            }
#ifdef _OPENMP
#pragma omp atomic
#endif
            pu[tid] += cnt;
            ph[tid] += cnt_half;
        }
        for (int t = 0; t < nthreads; ++t) {
            for (size_t i = 0; i < nvox; ++i) {
                G[2 * i] += pg[t][2 * i];
                G[2 * i + 1] += pg[t][2 * i + 1];
                W[i] += pw[t][i];
            }
            *U += pu[t];
            if (Uhalf) *Uhalf += ph[t];
        }
    }
    for (int t = 0; t < nthreads && pg && pw; ++t) { free(pg[t]); free(pw[t]); }
    free(pg); free(pw); free(pu); free(ph);
    return oom ? -2 : 0;
}

/* Per-voxel form of the same sum, for a list of voxels: for voxel v, every
 * slice s and every sample k in P with |v - R_s (k,0)|^2 <= a^2 contributes.
 * Candidate samples are taken from the integer square around u = R_s^T v
 * (widened by one on each side); membership is decided by the 3D distance
 * itself, so the window only bounds the search.
 *   vox : [nv][3] centered coordinates (x, y, z), each in [-h, h]
 *   Gv  : [nv][2], Wv : [nv], Uv : [nv]  (overwritten) */
int oracle_voxels(int n, int S, const float *F, const double *R,
                  double a, double alpha, int m, int mode, const double *table, int N,
                  double r_max, int nv, const int *vox, double *Gv, double *Wv, uint64_t *Uv,
                  int nthreads)
{
    blob_t b;
    if (n < 2 || (n & 1) || S < 0 || nv < 0 || !Gv || !Wv || !Uv) return -1;
    if (nv > 0 && !vox) return -1;
    if (S > 0 && (!F || !R)) return -1;
    if (!(r_max > 0.0) || r_max > 0.5 * n) return -1;
    if (blob_init(&b, a, alpha, m, mode, table, N)) return -1;
    const int h = n / 2;
    const size_t slice_len = (size_t)n * (h + 1) * 2;
    const double r2max = r_max * r_max;
    for (int i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c)
            if (vox[3 * i + c] < -h || vox[3 * i + c] > h) return -1;
    if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
#endif
    for (int i = 0; i < nv; ++i) {
        const double vx = vox[3 * i], vy = vox[3 * i + 1], vz = vox[3 * i + 2];
        double gre = 0.0, gim = 0.0, wsum = 0.0;
        uint64_t cnt = 0;
        for (int s = 0; s < S; ++s) {
            const double *Rs = R + (size_t)s * 9;
            const float *Fs = F + (size_t)s * slice_len;
            double ux = Rs[0] * vx + Rs[3] * vy + Rs[6] * vz;
            double uy = Rs[1] * vx + Rs[4] * vy + Rs[7] * vz;
            int kx0 = (int)floor(ux - a) - 1, kx1 = (int)ceil(ux + a) + 1;
            int ky0 = (int)floor(uy - a) - 1, ky1 = (int)ceil(uy + a) + 1;
            for (int ky = ky0; ky <= ky1; ++ky) {
                for (int kx = kx0; kx <= kx1; ++kx) {
                    if ((double)kx * kx + (double)ky * ky >= r2max) continue;
                    double px = Rs[0] * kx + Rs[1] * ky;
                    double py = Rs[3] * kx + Rs[4] * ky;
                    double pz = Rs[6] * kx + Rs[7] * ky;
                    double dx = vx - px, dy = vy - py, dz = vz - pz;
                    double d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 > b.a2) continue;
                    double fre, fim;
                    sample_full(Fs, n, kx, ky, &fre, &fim);
                    double wgt = blob_weight(&b, d2);
                    gre += wgt * fre;
                    gim += wgt * fim;
                    wsum += wgt;
                    ++cnt;
                }
            }
        }
        Gv[2 * i] = gre; Gv[2 * i + 1] = gim; Wv[i] = wsum; Uv[i] = cnt;
    }
    return 0;
}

/* Exact blob evaluated at an array of d^2 values (for tests of the C series). */
int oracle_blob(int count, const double *d2, double a, double alpha, int m, int mode,
                const double *table, int N, double *out)
{
    blob_t b;
    if (count < 0 || (count > 0 && (!d2 || !out))) return -1;
    if (blob_init(&b, a, alpha, m, mode, table, N)) return -1;
    for (int i = 0; i < count; ++i) out[i] = blob_weight(&b, d2[i]);
    return 0;
}

/* Sum of blob weights that each sample deposits inside the box, summed over
 * all slices and samples: sum_s sum_{k in P} sum_{v in B, |v-p|^2<=a^2} b.
 * Written as its own loop over samples (no volume), for the total-weight
 * identity sum_v W(v) = this value. */
int oracle_footprint_total(int n, int S, const double *R, double a, double alpha, int m,
                           int mode, const double *table, int N, double r_max, double *total)
{
    blob_t b;
    if (n < 2 || (n & 1) || S < 0 || !total || (S > 0 && !R)) return -1;
    if (!(r_max > 0.0) || r_max > 0.5 * n) return -1;
    if (blob_init(&b, a, alpha, m, mode, table, N)) return -1;
    const int h = n / 2;
    const double r2max = r_max * r_max;
    double acc = 0.0;
    for (int s = 0; s < S; ++s) {
        const double *Rs = R + (size_t)s * 9;
        for (int ky = -h; ky <= h; ++ky)
            for (int kx = -h; kx <= h; ++kx) {
                if ((double)kx * kx + (double)ky * ky >= r2max) continue;
                double p[3] = {Rs[0] * kx + Rs[1] * ky, Rs[3] * kx + Rs[4] * ky,
                               Rs[6] * kx + Rs[7] * ky};
                int lo[3], hi[3];
                for (int c = 0; c < 3; ++c) {
                    lo[c] = (int)ceil(p[c] - a); hi[c] = (int)floor(p[c] + a);
                    if (lo[c] < -h) lo[c] = -h;
                    if (hi[c] > h) hi[c] = h;
                }
                for (int z = lo[2]; z <= hi[2]; ++z)
                    for (int y = lo[1]; y <= hi[1]; ++y)
                        for (int x = lo[0]; x <= hi[0]; ++x) {
                            double d2 = (x - p[0]) * (x - p[0]) + (y - p[1]) * (y - p[1]) +
                                        (z - p[2]) * (z - p[2]);
                            acc += blob_weight(&b, d2);
                        }
            }
    }
    *total = acc;
    return 0;
}
