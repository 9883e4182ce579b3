/*
 * Seeded synthetic digraph generators (input side only).
 *
 * This module builds the inputs that both the sequential oracle and the GPU
 * library consume: an int32 CSR of the out-arcs and the transposed CSR of the
 * same arc multiset.  It holds none of the SCC method's arithmetic.
 *
 * Randomness is counter based: every draw is a pure function of
 * (seed, stream, index) through the SplitMix64 output function (Steele, Lea,
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), so a
 * graph does not depend on the number of threads that built it.
 *
 * Families (the paper's evaluation uses lattices, social/web graphs and k-NN
 * graphs, Section 6; the shapes below stand in for them):
 *   - lattice: rows x cols grid, optional wraparound (torus); each of the four
 *     neighbour arcs (E, W, S, N) of every vertex is kept independently with
 *     probability p.
 *   - R-MAT: recursive quadrant choice with probabilities (a, b, c, d),
 *     self-loops and duplicate arcs removed, ids relabelled by a seeded
 *     random permutation.
 *   - k-NN: points in R^3 from a mixture of isotropic Gaussians; an arc from
 *     every point to each of its k nearest other points (squared Euclidean
 *     distance in double precision, ties to the lower id), found exactly with
 *     a uniform cell grid.
 * Every adjacency list of the output is sorted ascending and duplicate free.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int64_t n;
    int64_t m;
    int32_t *off; /* n + 1 */
    int32_t *adj; /* m */
} gg_csr;

/* ---------------------------------------------------------------- RNG ---- */
static inline uint64_t sm64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
static inline uint64_t rnd(uint64_t seed, uint64_t stream, uint64_t idx) {
    return sm64(sm64(seed * 0xD1B54A32D192ED03ull + stream) ^ idx);
}
static inline double unif(uint64_t seed, uint64_t stream, uint64_t idx) {
    return (double)(rnd(seed, stream, idx) >> 11) * (1.0 / 9007199254740992.0);
}

uint64_t gg_rnd(uint64_t seed, uint64_t stream, uint64_t idx) { return rnd(seed, stream, idx); }
double gg_unif(uint64_t seed, uint64_t stream, uint64_t idx) { return unif(seed, stream, idx); }

void gg_free(gg_csr *g) {
    free(g->off);
    free(g->adj);
    g->off = NULL;
    g->adj = NULL;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void sort_small(int32_t *a, int64_t len) {
    if (len < 32) {
        for (int64_t i = 1; i < len; i++) {
            int32_t v = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; j--; }
            a[j + 1] = v;
        }
    } else {
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/* Build a CSR from per-vertex lists stored in [off, off+deg) of a scratch
 * buffer: sort each list, drop duplicates and (optionally) self loops, and
 * compact into a fresh CSR. */
static int compact_sorted(int64_t n, const int64_t *soff, int32_t *sadj, int drop_self, gg_csr *out) {
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!cnt) return -1;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; u++) {
        int32_t *a = sadj + soff[u];
        int64_t len = soff[u + 1] - soff[u];
        sort_small(a, len);
        int64_t w = 0;
        for (int64_t i = 0; i < len; i++) {
            if (drop_self && a[i] == (int32_t)u) continue;
            if (w > 0 && a[w - 1] == a[i]) continue;
            a[w++] = a[i];
        }
        cnt[u] = w;
    }
    int64_t tot = 0;
    for (int64_t u = 0; u < n; u++) { int64_t c = cnt[u]; cnt[u] = tot; tot += c; }
    cnt[n] = tot;
    if (tot >= ((int64_t)1 << 31)) { free(cnt); return -2; }
    out->n = n;
    out->m = tot;
    out->off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    out->adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    if (!out->off || !out->adj) { free(cnt); gg_free(out); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u <= n; u++) out->off[u] = (int32_t)cnt[u];
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; u++) {
        int64_t len = cnt[u + 1] - cnt[u];
        memcpy(out->adj + cnt[u], sadj + soff[u], sizeof(int32_t) * (size_t)len);
    }
    free(cnt);
    return 0;
}

/* Transposed CSR of g: in-adjacency of v = sorted list of u with arc u->v. */
int gg_transpose(const gg_csr *g, gg_csr *out) {
    int64_t n = g->n, m = g->m;
    int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    if (!cnt) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; e++) __atomic_fetch_add(&cnt[g->adj[e]], 1, __ATOMIC_RELAXED);
    int64_t tot = 0;
    for (int64_t v = 0; v < n; v++) { int64_t c = cnt[v]; cnt[v] = tot; tot += c; }
    cnt[n] = tot;
    out->n = n;
    out->m = m;
    out->off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    out->adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!out->off || !out->adj || !cur) { free(cnt); free(cur); gg_free(out); return -1; }
    memcpy(cur, cnt, sizeof(int64_t) * (size_t)(n + 1));
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; u++) {
        for (int64_t e = g->off[u]; e < g->off[u + 1]; e++) {
            int64_t pos = __atomic_fetch_add(&cur[g->adj[e]], 1, __ATOMIC_RELAXED);
            out->adj[pos] = (int32_t)u;
        }
    }
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < n; v++) sort_small(out->adj + cnt[v], cnt[v + 1] - cnt[v]);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v <= n; v++) out->off[v] = (int32_t)cnt[v];
    free(cnt);
    free(cur);
    return 0;
}

/* ------------------------------------------------------------- lattice ---- */
/* Vertex id = r * cols + c.  Direction d in {0:E, 1:W, 2:S, 3:N}; the arc to
 * that neighbour is kept iff unif(seed, 0, 4*id + d) < p. */
int gg_lattice(int64_t rows, int64_t cols, int wrap, double p, uint64_t seed, gg_csr *out) {
    int64_t n = rows * cols;
    if (rows <= 0 || cols <= 0 || n >= ((int64_t)1 << 31)) return -3;
    int64_t *soff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *sadj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * n));
    if (!soff || !sadj) { free(soff); free(sadj); return -1; }
    for (int64_t u = 0; u <= n; u++) soff[u] = 4 * u;
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; u++) {
        int64_t r = u / cols, c = u % cols, k = 0;
        for (int d = 0; d < 4; d++) {
            int64_t rr = r, cc = c;
            if (d == 0) cc = c + 1;
            else if (d == 1) cc = c - 1;
            else if (d == 2) rr = r + 1;
            else rr = r - 1;
            if (wrap) {
                rr = (rr + rows) % rows;
                cc = (cc + cols) % cols;
            } else if (rr < 0 || rr >= rows || cc < 0 || cc >= cols) {
                continue;
            }
            if (unif(seed, 0, (uint64_t)(4 * u + d)) < p) sadj[4 * u + k++] = (int32_t)(rr * cols + cc);
        }
        deg[u] = k;
    }
    /* lists are padded to 4; shrink each to its used length */
    int64_t *soff2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *sadj2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * n));
    int64_t tot = 0;
    for (int64_t u = 0; u < n; u++) { soff2[u] = tot; tot += deg[u]; }
    soff2[n] = tot;
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; u++) memcpy(sadj2 + soff2[u], sadj + 4 * u, sizeof(int32_t) * (size_t)deg[u]);
    free(soff);
    free(sadj);
    free(deg);
    int rc = compact_sorted(n, soff2, sadj2, 1, out);
    free(soff2);
    free(sadj2);
    return rc;
}

/* The paper's lattices (Section 6): a rows x cols torus (circular rows and
 * columns), vertex id = r * cols + c, every lattice edge oriented at random.
 *   mode 0 (SQR, REC): every vertex u draws, for each of its four adjacent
 *     vertices v, an orientation: u -> v with probability 1/2, else v -> u;
 *     duplicates are removed.  Each edge gets two draws (one per endpoint),
 *     so it carries both arcs with probability 1/2: 1.5 arcs per edge, the
 *     300M arcs Table 3 lists for the 10^4 x 10^4 SQR.
 *   mode 1 (SQR', REC'): each edge carries each of its two arcs
 *     independently with probability 0.3: 0.6 arcs per edge, Table 3's 120M
 *     arcs for SQR' (the text's "no edge with probability 0.4" does not fit
 *     independent arcs; this reading reproduces Table 3's arc count and its
 *     share of SCCs, 78% of the vertices).  The edge between u and its east
 *     (south) neighbour v belongs to u: u -> v is drawn at index 4u + 0
 *     (4u + 2), v -> u at 4u + 1 (4u + 3).
 * Draws: unif(seed, 2, 4u + d) for mode 0 (d in E, W, S, N order),
 * unif(seed, 3, index above) for mode 1. */
int gg_lattice_oriented(int64_t rows, int64_t cols, int mode, uint64_t seed, gg_csr *out) {
    int64_t n = rows * cols;
    if (rows <= 0 || cols <= 0 || n >= ((int64_t)1 << 31) || (mode != 0 && mode != 1)) return -3;
    int64_t *soff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *sadj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * n));
    int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!soff || !sadj || !deg) { free(soff); free(sadj); free(deg); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; u++) {
        const int64_t r = u / cols, c = u % cols;
        const int64_t nb[4] = {r * cols + (c + 1) % cols, r * cols + (c + cols - 1) % cols,
                               ((r + 1) % rows) * cols + c, ((r + rows - 1) % rows) * cols + c};
        static const int opp[4] = {1, 0, 3, 2};
        int64_t k = 0;
        for (int d = 0; d < 4; d++) {
            const int64_t v = nb[d];
            int keep;
            if (mode == 0) {
                /* u -> v if u's draw for v says so, or v's draw for u says v <- u */
                keep = unif(seed, 2, (uint64_t)(4 * u + d)) < 0.5 || unif(seed, 2, (uint64_t)(4 * v + opp[d])) >= 0.5;
            } else if (d == 0 || d == 2) {
                /* u owns the edge to its east / south neighbour: its forward arc */
                keep = unif(seed, 3, (uint64_t)(4 * u + (d == 2 ? 2 : 0))) < 0.3;
            } else {
                /* the west / north neighbour v owns the edge: its backward arc v <- u */
                keep = unif(seed, 3, (uint64_t)(4 * v + (d == 3 ? 3 : 1))) < 0.3;
            }
            if (keep) sadj[4 * u + k++] = (int32_t)v;
        }
        deg[u] = k;
    }
    int64_t tot = 0;
    for (int64_t u = 0; u < n; u++) { soff[u] = tot; tot += deg[u]; }
    soff[n] = tot;
    int32_t *sadj2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    if (!sadj2) { free(soff); free(sadj); free(deg); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; u++) memcpy(sadj2 + soff[u], sadj + 4 * u, sizeof(int32_t) * (size_t)deg[u]);
    free(sadj);
    free(deg);
    int rc = compact_sorted(n, soff, sadj2, 1, out);
    free(soff);
    free(sadj2);
    return rc;
}

/* --------------------------------------------------------------- R-MAT ---- */
/* Arc i picks, level by level from the most significant bit, one of four
 * quadrants with probabilities (a, b, c, d = 1-a-b-c).  Each level consumes a
 * 16-bit slice of rnd(seed, 1, i * ceil(scale/4) + level/4). */
int gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed, int permute, gg_csr *out) {
    if (scale < 1 || scale > 30) return -3;
    int64_t n = (int64_t)1 << scale;
    int64_t m0 = edge_factor * n;
    uint32_t ta = (uint32_t)llround(a * 65536.0);
    uint32_t tb = ta + (uint32_t)llround(b * 65536.0);
    uint32_t tc = tb + (uint32_t)llround(c * 65536.0);
    int words = (scale + 3) / 4;
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)m0);
    int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)m0);
    if (!src || !dst) { free(src); free(dst); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m0; i++) {
        uint32_t u = 0, v = 0;
        uint64_t w = 0;
        for (int l = 0; l < scale; l++) {
            if ((l & 3) == 0) w = rnd(seed, 1, (uint64_t)i * (uint64_t)words + (uint64_t)(l >> 2));
            uint32_t r16 = (uint32_t)((w >> (16 * (l & 3))) & 0xFFFFu);
            uint32_t bit = 1u << (scale - 1 - l);
            if (r16 < ta) {
            } else if (r16 < tb) {
                v |= bit;
            } else if (r16 < tc) {
                u |= bit;
            } else {
                u |= bit;
                v |= bit;
            }
        }
        src[i] = (int32_t)u;
        dst[i] = (int32_t)v;
    }
    /* optional relabel by a seeded Fisher-Yates permutation */
    int32_t *perm = NULL;
    if (permute) {
        perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
        for (int64_t i = n - 1; i > 0; i--) {
            int64_t j = (int64_t)(rnd(seed, 2, (uint64_t)i) % (uint64_t)(i + 1));
            int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m0; i++) { src[i] = perm[src[i]]; dst[i] = perm[dst[i]]; }
        free(perm);
    }
    int64_t *soff = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m0; i++) __atomic_fetch_add(&soff[src[i]], 1, __ATOMIC_RELAXED);
    int64_t tot = 0;
    for (int64_t u = 0; u < n; u++) { int64_t t = soff[u]; soff[u] = tot; tot += t; }
    soff[n] = tot;
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(cur, soff, sizeof(int64_t) * (size_t)(n + 1));
    int32_t *sadj = src; /* reuse: scatter dst into a fresh buffer */
    sadj = (int32_t *)malloc(sizeof(int32_t) * (size_t)m0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m0; i++) {
        int64_t pos = __atomic_fetch_add(&cur[src[i]], 1, __ATOMIC_RELAXED);
        sadj[pos] = dst[i];
    }
    free(src);
    free(dst);
    free(cur);
    int rc = compact_sorted(n, soff, sadj, 1, out);
    free(soff);
    free(sadj);
    return rc;
}

/* ----------------------------------------------------------------- kNN ---- */
typedef struct { uint64_t key; int32_t idx; int32_t pad; } keyidx;

static void radix_sort_keys(keyidx *a, int64_t n, int bits) {
    keyidx *tmp = (keyidx *)malloc(sizeof(keyidx) * (size_t)(n > 0 ? n : 1));
    const int D = 16;
    for (int shift = 0; shift < bits; shift += D) {
        int64_t *cnt = (int64_t *)calloc((size_t)1 << D, sizeof(int64_t));
        for (int64_t i = 0; i < n; i++) cnt[(a[i].key >> shift) & 0xFFFF]++;
        int64_t tot = 0;
        for (int64_t d = 0; d < (1 << D); d++) { int64_t t = cnt[d]; cnt[d] = tot; tot += t; }
        for (int64_t i = 0; i < n; i++) tmp[cnt[(a[i].key >> shift) & 0xFFFF]++] = a[i];
        memcpy(a, tmp, sizeof(keyidx) * (size_t)n);
        free(cnt);
    }
    free(tmp);
}

static int64_t lower_bound_key(const keyidx *a, int64_t n, uint64_t key) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid].key < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Points: centres c_j ~ U[0,1)^3 (stream 10); point i picks centre
 * floor(U * ncent) (stream 11) and adds sigma * N(0, I) by Box-Muller on
 * streams 12 and 13.  The coordinates are written to pts (3 * npts doubles)
 * when pts is non-NULL. */
int gg_knn(int64_t npts, int64_t ncent, int k, double sigma, uint64_t seed, gg_csr *out, double *pts_out) {
    if (npts <= 0 || ncent <= 0 || k <= 0 || k > 64 || npts >= ((int64_t)1 << 31)) return -3;
    double *P = (double *)malloc(sizeof(double) * (size_t)(3 * npts));
    double *C = (double *)malloc(sizeof(double) * (size_t)(3 * ncent));
    for (int64_t j = 0; j < ncent; j++)
        for (int d = 0; d < 3; d++) C[3 * j + d] = unif(seed, 10, (uint64_t)(3 * j + d));
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; i++) {
        int64_t cj = (int64_t)(unif(seed, 11, (uint64_t)i) * (double)ncent);
        if (cj >= ncent) cj = ncent - 1;
        double a1 = 1.0 - unif(seed, 12, (uint64_t)(3 * i));
        double b1 = unif(seed, 12, (uint64_t)(3 * i + 1));
        double a2 = 1.0 - unif(seed, 12, (uint64_t)(3 * i + 2));
        double b2 = unif(seed, 13, (uint64_t)i);
        double r1 = sqrt(-2.0 * log(a1)), r2 = sqrt(-2.0 * log(a2));
        P[3 * i + 0] = C[3 * cj + 0] + sigma * r1 * cos(two_pi * b1);
        P[3 * i + 1] = C[3 * cj + 1] + sigma * r1 * sin(two_pi * b1);
        P[3 * i + 2] = C[3 * cj + 2] + sigma * r2 * cos(two_pi * b2);
    }
    free(C);
    double lo[3], hi[3];
    for (int d = 0; d < 3; d++) { lo[d] = P[d]; hi[d] = P[d]; }
    for (int64_t i = 0; i < npts; i++)
        for (int d = 0; d < 3; d++) {
            if (P[3 * i + d] < lo[d]) lo[d] = P[3 * i + d];
            if (P[3 * i + d] > hi[d]) hi[d] = P[3 * i + d];
        }
    /* cell edge: about 8 points per cell at a cluster's core density */
    double per = (double)npts / (double)ncent;
    double rho = per / (pow(two_pi, 1.5) * sigma * sigma * sigma);
    double h = cbrt(8.0 / rho);
    double ext = 0.0;
    for (int d = 0; d < 3; d++) if (hi[d] - lo[d] > ext) ext = hi[d] - lo[d];
    if (h < ext / 2000.0) h = ext / 2000.0; /* bounds the key width */
    if (h <= 0.0) h = 1.0;
    int64_t dim[3];
    for (int d = 0; d < 3; d++) dim[d] = (int64_t)floor((hi[d] - lo[d]) / h) + 1;
    keyidx *cells = (keyidx *)malloc(sizeof(keyidx) * (size_t)npts);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; i++) {
        int64_t cx = (int64_t)floor((P[3 * i] - lo[0]) / h);
        int64_t cy = (int64_t)floor((P[3 * i + 1] - lo[1]) / h);
        int64_t cz = (int64_t)floor((P[3 * i + 2] - lo[2]) / h);
        if (cx >= dim[0]) cx = dim[0] - 1;
        if (cy >= dim[1]) cy = dim[1] - 1;
        if (cz >= dim[2]) cz = dim[2] - 1;
        cells[i].key = (uint64_t)((cx * dim[1] + cy) * dim[2] + cz);
        cells[i].idx = (int32_t)i;
        cells[i].pad = 0;
    }
    int bits = 0;
    while (bits < 64 && ((uint64_t)1 << bits) <= (uint64_t)(dim[0] * dim[1] * dim[2])) bits++;
    radix_sort_keys(cells, npts, bits);
    int kk = (int)((npts - 1 < k) ? npts - 1 : k);
    int64_t *soff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npts + 1));
    for (int64_t i = 0; i <= npts; i++) soff[i] = i * kk;
    int32_t *sadj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(npts * (kk > 0 ? kk : 1)));
    int64_t maxdim = dim[0];
    if (dim[1] > maxdim) maxdim = dim[1];
    if (dim[2] > maxdim) maxdim = dim[2];
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < npts; i++) {
        if (kk == 0) continue;
        double bd[64];
        int32_t bi[64];
        int cnt = 0;
        double qx = P[3 * i], qy = P[3 * i + 1], qz = P[3 * i + 2];
        int64_t cx = (int64_t)floor((qx - lo[0]) / h), cy = (int64_t)floor((qy - lo[1]) / h),
                cz = (int64_t)floor((qz - lo[2]) / h);
        if (cx >= dim[0]) cx = dim[0] - 1;
        if (cy >= dim[1]) cy = dim[1] - 1;
        if (cz >= dim[2]) cz = dim[2] - 1;
        for (int64_t s = 0; s <= maxdim; s++) {
            for (int64_t dx = -s; dx <= s; dx++) {
                int64_t x = cx + dx;
                if (x < 0 || x >= dim[0]) continue;
                for (int64_t dy = -s; dy <= s; dy++) {
                    int64_t y = cy + dy;
                    if (y < 0 || y >= dim[1]) continue;
                    int surface_xy = (dx == -s || dx == s || dy == -s || dy == s);
                    for (int64_t dz = -s; dz <= s; dz += (surface_xy ? 1 : (s > 0 ? 2 * s : 1))) {
                        int64_t z = cz + dz;
                        if (z >= 0 && z < dim[2]) {
                            uint64_t key = (uint64_t)((x * dim[1] + y) * dim[2] + z);
                            int64_t p0 = lower_bound_key(cells, npts, key);
                            for (int64_t q = p0; q < npts && cells[q].key == key; q++) {
                                int32_t j = cells[q].idx;
                                if (j == (int32_t)i) continue;
                                double ex = P[3 * (int64_t)j] - qx, ey = P[3 * (int64_t)j + 1] - qy,
                                       ez = P[3 * (int64_t)j + 2] - qz;
                                double d2 = ex * ex + ey * ey + ez * ez;
                                if (cnt == kk && (d2 > bd[kk - 1] || (d2 == bd[kk - 1] && j > bi[kk - 1]))) continue;
                                int pos = (cnt < kk) ? cnt++ : kk - 1;
                                while (pos > 0 && (bd[pos - 1] > d2 || (bd[pos - 1] == d2 && bi[pos - 1] > j))) {
                                    bd[pos] = bd[pos - 1];
                                    bi[pos] = bi[pos - 1];
                                    pos--;
                                }
                                bd[pos] = d2;
                                bi[pos] = j;
                            }
                        }
                        if (s == 0) break;
                    }
                }
            }
            /* every point not yet examined is at distance >= s * h */
            double bound = (double)s * h * (1.0 - 1e-9);
            if (cnt == kk && bd[kk - 1] < bound * bound) break;
        }
        for (int t = 0; t < kk; t++) sadj[i * kk + t] = bi[t];
    }
    free(cells);
    if (pts_out) memcpy(pts_out, P, sizeof(double) * (size_t)(3 * npts));
    free(P);
    int rc = compact_sorted(npts, soff, sadj, 1, out);
    free(soff);
    free(sadj);
    return rc;
}

/* Build a CSR from an arc list (src[i] -> dst[i]); keeps duplicates and self
 * loops unless asked to drop them.  Lists come out sorted. */
int gg_from_arcs(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int dedup, gg_csr *out) {
    int64_t *soff = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    for (int64_t i = 0; i < m; i++) soff[src[i]]++;
    int64_t tot = 0;
    for (int64_t u = 0; u < n; u++) { int64_t t = soff[u]; soff[u] = tot; tot += t; }
    soff[n] = tot;
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(cur, soff, sizeof(int64_t) * (size_t)(n + 1));
    int32_t *sadj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t i = 0; i < m; i++) sadj[cur[src[i]]++] = dst[i];
    free(cur);
    int rc;
    if (dedup) {
        rc = compact_sorted(n, soff, sadj, 1, out);
    } else {
        for (int64_t u = 0; u < n; u++) sort_small(sadj + soff[u], soff[u + 1] - soff[u]);
        out->n = n;
        out->m = m;
        out->off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
        for (int64_t u = 0; u <= n; u++) out->off[u] = (int32_t)soff[u];
        out->adj = sadj;
        sadj = NULL;
        rc = 0;
    }
    free(soff);
    free(sadj);
    return rc;
}

int gg_num_threads(void) { return omp_get_max_threads(); }
