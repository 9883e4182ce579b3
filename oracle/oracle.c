/*
 * Sequential CPU oracle for strongly connected components and reachability.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * loads this file; only the tests, the smoke check and the CPU baseline of the
 * benchmark do.  It shares no code with the GPU path.
 *
 * What it computes, each by its plain definition:
 *   or_tarjan          SCC partition of a digraph (the SCC definition of
 *                      Section 2, computed by Tarjan's sequential algorithm,
 *                      which the paper uses as its exact baseline "SEQ",
 *                      Section 6), written out as the canonical label
 *                      "minimum vertex id of the vertex's SCC".
 *   or_reach_pairs     the reachability pairs {(v, j) : s_j ~> v} of a source
 *                      set (Section 2, "Reachability Search"), restricted, as
 *                      the multi-reachability search of Algorithm 1 is, to
 *                      arcs (u, w) whose endpoints carry the same label; here
 *                      labels < 0 mark excluded vertices.  One plain BFS per
 *                      source.
 *   or_check_partition an implementation-free certificate that a labelling is
 *                      the SCC partition: (i) inside every class, the minimum
 *                      member reaches and is reached by every member using
 *                      only arcs inside the class; (ii) the graph of classes
 *                      is acyclic; (iii) every label is the minimum id of its
 *                      class.  (i) says classes are strongly connected,
 *                      (ii) that no two classes can merge, so together they
 *                      characterise the SCCs.
 *
 * Error codes: 0 ok; -1 invalid argument; -2 out of memory; -3 capacity
 * exceeded (or_reach_pairs: *count still holds the full size).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Tarjan's algorithm, iterative: an explicit frame stack of (vertex, next arc)
 * replaces the recursion so that graphs with 1e8 vertices do not overflow the
 * call stack. labels[v] <- min id of v's SCC. */
int or_tarjan(int64_t n, const int32_t *off, const int32_t *adj, int32_t *labels) {
    if (n < 0) return -1;
    if (n == 0) return 0;
    int32_t *index = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *low = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *onstack = (uint8_t *)calloc((size_t)n, 1);
    int32_t *sstack = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *fv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *fpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!index || !low || !onstack || !sstack || !fv || !fpos) {
        free(index); free(low); free(onstack); free(sstack); free(fv); free(fpos);
        return -2;
    }
    for (int64_t v = 0; v < n; v++) index[v] = -1;
    int32_t counter = 0;
    int64_t sp = 0; /* SCC stack size */
    for (int64_t root = 0; root < n; root++) {
        if (index[root] != -1) continue;
        int64_t fp = 0; /* frame stack size */
        fv[0] = (int32_t)root;
        fpos[0] = off[root];
        index[root] = low[root] = counter++;
        sstack[sp++] = (int32_t)root;
        onstack[root] = 1;
        fp = 1;
        while (fp > 0) {
            int32_t v = fv[fp - 1];
            if (fpos[fp - 1] < off[v + 1]) {
                int32_t w = adj[fpos[fp - 1]++];
                if (index[w] == -1) {
                    index[w] = low[w] = counter++;
                    sstack[sp++] = w;
                    onstack[w] = 1;
                    fv[fp] = w;
                    fpos[fp] = off[w];
                    fp++;
                } else if (onstack[w] && index[w] < low[v]) {
                    low[v] = index[w];
                }
            } else {
                fp--;
                if (low[v] == index[v]) {
                    /* v roots an SCC: the members are on top of the stack */
                    int64_t top = sp;
                    int32_t mn = v;
                    do {
                        sp--;
                        if (sstack[sp] < mn) mn = sstack[sp];
                    } while (sstack[sp] != v);
                    for (int64_t i = sp; i < top; i++) {
                        labels[sstack[i]] = mn;
                        onstack[sstack[i]] = 0;
                    }
                }
                if (fp > 0) {
                    int32_t p = fv[fp - 1];
                    if (low[v] < low[p]) low[p] = low[v];
                }
            }
        }
    }
    free(index); free(low); free(onstack); free(sstack); free(fv); free(fpos);
    return 0;
}

/* One BFS per source over arcs (u, w) with labels[u] == labels[w] >= 0.
 * Output pairs (vertex, source index) sorted by (source index, vertex) into
 * pairs[2*i], pairs[2*i+1]; *count receives the total even when it exceeds
 * cap (then -3 is returned and only the first cap pairs are written).
 * Sources must be distinct, in range and not excluded (labels >= 0). */
int or_reach_pairs(int64_t n, const int32_t *off, const int32_t *adj, const int32_t *labels, int64_t k,
                   const int32_t *sources, int32_t *pairs, int64_t cap, int64_t *count) {
    if (n < 0 || k < 0 || (k > 0 && !sources) || !count) return -1;
    *count = 0;
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *mark = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!seen || !queue || !mark) { free(seen); free(queue); free(mark); return -2; }
    for (int64_t j = 0; j < k; j++) {
        int32_t s = sources[j];
        if (s < 0 || s >= n || labels[s] < 0 || mark[s]) { free(seen); free(queue); free(mark); return -1; }
        mark[s] = 1;
    }
    for (int64_t v = 0; v < n; v++) seen[v] = -1;
    int64_t total = 0;
    for (int64_t j = 0; j < k; j++) {
        int32_t s = sources[j];
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        seen[s] = (int32_t)j;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int64_t e = off[u]; e < off[u + 1]; e++) {
                int32_t w = adj[e];
                if (labels[w] != labels[u] || seen[w] == (int32_t)j) continue;
                seen[w] = (int32_t)j;
                queue[tail++] = w;
            }
        }
        /* the visited set, ascending by vertex */
        qsort(queue, (size_t)tail, sizeof(int32_t), cmp_i32);
        for (int64_t a = 0; a < tail; a++) {
            if (total < cap) {
                pairs[2 * total] = queue[a];
                pairs[2 * total + 1] = (int32_t)j;
            }
            total++;
        }
    }
    free(seen); free(queue); free(mark);
    *count = total;
    return total > cap ? -3 : 0;
}

/* Certificate check.  Returns 0 when labels is the canonical SCC labelling,
 * 1 if a class is not strongly connected through its own arcs, 2 if the class
 * graph has a cycle, 3 if a label is not the minimum id of its class (or out
 * of range).  *bad receives an offending vertex (or -1). */
int or_check_partition(int64_t n, const int32_t *out_off, const int32_t *out_adj, const int32_t *in_off,
                       const int32_t *in_adj, const int32_t *labels, int64_t *bad) {
    *bad = -1;
    if (n < 0) return -1;
    if (n == 0) return 0;
    /* (iii) labels are the minimum member: label in range, label <= v and
     * the representative labels itself */
    for (int64_t v = 0; v < n; v++) {
        int32_t l = labels[v];
        if (l < 0 || l >= n || l > v || labels[l] != l) { *bad = v; return 3; }
    }
    /* group members by class */
    int64_t *start = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int32_t *memb = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!start || !memb || !seen || !queue) { free(start); free(memb); free(seen); free(queue); return -2; }
    for (int64_t v = 0; v < n; v++) start[labels[v] + 1]++;
    for (int64_t c = 0; c < n; c++) start[c + 1] += start[c];
    {
        int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        memcpy(cur, start, sizeof(int64_t) * (size_t)n);
        for (int64_t v = 0; v < n; v++) memb[cur[labels[v]]++] = (int32_t)v;
        free(cur);
    }
    /* (i) mutual reachability inside each class, both directions */
    for (int dir = 0; dir < 2; dir++) {
        const int32_t *off = dir ? in_off : out_off;
        const int32_t *adj = dir ? in_adj : out_adj;
        for (int64_t v = 0; v < n; v++) seen[v] = -1;
        for (int64_t c = 0; c < n; c++) {
            int64_t size = start[c + 1] - start[c];
            if (size == 0) continue;
            int64_t head = 0, tail = 0;
            queue[tail++] = (int32_t)c;
            seen[c] = (int32_t)c;
            while (head < tail) {
                int32_t u = queue[head++];
                for (int64_t e = off[u]; e < off[u + 1]; e++) {
                    int32_t w = adj[e];
                    if (labels[w] != (int32_t)c || seen[w] == (int32_t)c) continue;
                    seen[w] = (int32_t)c;
                    queue[tail++] = w;
                }
            }
            if (tail != size) {
                for (int64_t i = start[c]; i < start[c + 1]; i++)
                    if (seen[memb[i]] != (int32_t)c) { *bad = memb[i]; break; }
                free(start); free(memb); free(seen); free(queue);
                return 1;
            }
        }
    }
    /* (ii) Kahn's topological sort of the class graph (parallel arcs are
     * counted with multiplicity, which Kahn's algorithm tolerates) */
    int64_t *indeg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t nclass = 0;
    for (int64_t c = 0; c < n; c++) nclass += (start[c + 1] > start[c]);
    for (int64_t u = 0; u < n; u++)
        for (int64_t e = out_off[u]; e < out_off[u + 1]; e++) {
            int32_t w = out_adj[e];
            if (labels[w] != labels[u]) indeg[labels[w]]++;
        }
    int64_t head = 0, tail = 0, done = 0;
    for (int64_t c = 0; c < n; c++)
        if (start[c + 1] > start[c] && indeg[c] == 0) queue[tail++] = (int32_t)c;
    while (head < tail) {
        int32_t c = queue[head++];
        done++;
        for (int64_t i = start[c]; i < start[c + 1]; i++) {
            int32_t u = memb[i];
            for (int64_t e = out_off[u]; e < out_off[u + 1]; e++) {
                int32_t w = out_adj[e];
                int32_t d = labels[w];
                if (d != c && --indeg[d] == 0) queue[tail++] = d;
            }
        }
    }
    int rc = 0;
    if (done != nclass) {
        for (int64_t c = 0; c < n; c++)
            if (indeg[c] > 0) { *bad = c; break; }
        rc = 2;
    }
    free(indeg); free(start); free(memb); free(seen); free(queue);
    return rc;
}

/* BFS depth of each source's label-restricted reach (Section 2, "Reachability
 * Search"; Algorithm 2 runs one frontier round per BFS level).  ecc[j] = the
 * largest distance from sources[j] to a vertex it reaches over arcs (u, w)
 * with labels[u] == labels[w] >= 0 (0 when it reaches only itself).  Same
 * argument rules as or_reach_pairs. */
int or_bfs_depths(int64_t n, const int32_t *off, const int32_t *adj, const int32_t *labels, int64_t k,
                  const int32_t *sources, int32_t *ecc) {
    if (n < 0 || k < 0 || (k > 0 && (!sources || !ecc))) return -1;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!dist || !seen || !queue) { free(dist); free(seen); free(queue); return -2; }
    for (int64_t v = 0; v < n; v++) seen[v] = -1;
    for (int64_t j = 0; j < k; j++) {
        int32_t s = sources[j];
        if (s < 0 || s >= n || labels[s] < 0) { free(dist); free(seen); free(queue); return -1; }
        int64_t head = 0, tail = 0;
        int32_t far = 0;
        queue[tail++] = s;
        seen[s] = (int32_t)j;
        dist[s] = 0;
        while (head < tail) {
            int32_t u = queue[head++];
            if (dist[u] > far) far = dist[u];
            for (int64_t e = off[u]; e < off[u + 1]; e++) {
                int32_t w = adj[e];
                if (labels[w] != labels[u] || seen[w] == (int32_t)j) continue;
                seen[w] = (int32_t)j;
                dist[w] = dist[u] + 1;
                queue[tail++] = w;
            }
        }
        ecc[j] = far;
    }
    free(dist); free(seen); free(queue);
    return 0;
}

/* ------------------------------------------------------------------------
 * Sequential model of the parallel hash bag of Section 3.3 (Figure 5 and the
 * text around it), with one inserting processor (P = 1, the sequential case
 * of the proof of Theorem 1 in Appendix A).
 *
 * Layout: chunk 0 is [0, lambda), chunk i >= 1 is [lambda 2^(i-1),
 * lambda 2^i) (the doubling tails of Figure 5: tail[0] = lambda, tail[i] =
 * 2 tail[i-1]); the array holds chunks 0..C-1 with lambda 2^(C-1) >= (s_max +
 * lambda) / alpha, s_max the largest round.  Insert(k): with r' the current
 * chunk, the element is sampled with probability sigma / (alpha |chunk r'|);
 * a sample increments sample[r'] and, once sample[r'] reaches sigma, moves r
 * from r' to r' + 1 and inserts k again.  Otherwise k goes to a uniformly
 * random slot of chunk r' and probes linearly (wrapping inside the chunk);
 * more than kappa probes also move r forward and insert k again.  The last
 * chunk never moves r.  ExtractAll lists the non-empty slots of [0,
 * tail[r]) in index order, empties them and resets r and the samples.
 *
 * Randomness: SplitMix64 (Steele, Lea, Flood 2014) of a running counter
 * seeded by `seed`, written here for this model.
 *
 * keys[0..n) are inserted round by round: round q holds keys
 * [round_start[q], round_start[q+1]).  Outputs:
 *   out[n]            the extracted keys, round after round;
 *   prefix[q]         tail[r] when round q was extracted (the used prefix);
 *   adv_chunk/adv_load/adv_cause[adv_cap]  one row per move of r: the chunk
 *                     left, its load (occupied / size) at that moment, and
 *                     the cause (0 sample count reached sigma, 1 probe limit);
 *   *n_adv            the number of moves (rows beyond adv_cap dropped).
 * Returns 0, -1 bad argument, -2 out of memory, -4 the last chunk filled. */
static uint64_t bag_sm64(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int or_hashbag_sim(int64_t n, const int64_t *keys, int64_t rounds, const int64_t *round_start, int32_t lam_log2,
                   int32_t sigma, double alpha, int32_t kappa, uint64_t seed, int64_t *out, int64_t *prefix,
                   int32_t *adv_chunk, double *adv_load, int32_t *adv_cause, int64_t adv_cap, int64_t *n_adv) {
    if (n < 0 || rounds < 0 || lam_log2 < 0 || lam_log2 > 40 || sigma < 1 || !(alpha > 0.0 && alpha < 1.0) ||
        kappa < 0 || !n_adv || (rounds > 0 && (!round_start || !prefix)) || (n > 0 && (!keys || !out)))
        return -1;
    *n_adv = 0;
    int64_t smax = 0;
    for (int64_t q = 0; q < rounds; q++) {
        int64_t s = round_start[q + 1] - round_start[q];
        if (s < 0 || round_start[q + 1] > n) return -1;
        if (s > smax) smax = s;
    }
    const uint64_t lam = 1ull << lam_log2;
    int nchunks = 1;
    while ((double)(lam << (nchunks - 1)) < ((double)smax + (double)lam) / alpha) nchunks++;
    const uint64_t cap = lam << (nchunks - 1);
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * cap);
    uint8_t *used = (uint8_t *)calloc(cap, 1);
    int64_t *fill = (int64_t *)calloc((size_t)nchunks, sizeof(int64_t));
    int64_t *sample = (int64_t *)calloc((size_t)nchunks, sizeof(int64_t));
    if (!slot || !used || !fill || !sample) { free(slot); free(used); free(fill); free(sample); return -2; }
    uint64_t rng = seed;
    int64_t w = 0;
    int rc = 0;
    for (int64_t q = 0; q < rounds && rc == 0; q++) {
        int r = 0;
        for (int64_t i = round_start[q]; i < round_start[q + 1] && rc == 0; i++) {
            const int64_t key = keys[i];
            for (;;) {
                const int rr = r;
                const uint64_t lo = rr == 0 ? 0 : (lam << (rr - 1)), hi = lam << rr;
                const uint64_t size = hi - lo;
                const int last = rr == nchunks - 1;
                int moved = 0;
                if (!last) {
                    /* sampled with probability sigma / (alpha * size) */
                    const double u = (double)(bag_sm64(&rng) >> 11) * (1.0 / 9007199254740992.0);
                    if (u * alpha * (double)size < (double)sigma) {
                        if (++sample[rr] >= sigma) {
                            if (*n_adv < adv_cap) {
                                adv_chunk[*n_adv] = rr;
                                adv_load[*n_adv] = (double)fill[rr] / (double)size;
                                adv_cause[*n_adv] = 0;
                            }
                            (*n_adv)++;
                            r = rr + 1;
                            moved = 1;
                        }
                    }
                }
                if (moved) continue;
                uint64_t pos = lo + bag_sm64(&rng) % size;
                int64_t probes = 0;
                while (used[pos]) {
                    pos = pos + 1 == hi ? lo : pos + 1;
                    probes++;
                    if (!last && probes > kappa) break;
                    if (last && (uint64_t)probes >= size) break;
                }
                if (used[pos]) {
                    if (last) { rc = -4; break; }
                    if (*n_adv < adv_cap) {
                        adv_chunk[*n_adv] = rr;
                        adv_load[*n_adv] = (double)fill[rr] / (double)size;
                        adv_cause[*n_adv] = 1;
                    }
                    (*n_adv)++;
                    r = rr + 1;
                    continue;
                }
                used[pos] = 1;
                slot[pos] = key;
                fill[rr]++;
                break;
            }
        }
        /* ExtractAll: the used prefix [0, tail[r]) in index order, cleared */
        const uint64_t tail = lam << r;
        prefix[q] = (int64_t)tail;
        for (uint64_t p = 0; p < tail; p++) {
            if (!used[p]) continue;
            out[w++] = slot[p];
            used[p] = 0;
        }
        for (int c = 0; c < nchunks; c++) { fill[c] = 0; sample[c] = 0; }
    }
    free(slot); free(used); free(fill); free(sample);
    return rc;
}

/* Weakly connected components (the connected components of the undirected
 * graph underlying the arcs; for a symmetric digraph these are the connected
 * components Algorithm 4 computes): a sequential union-find over the arcs,
 * union by size with path compression (Tarjan 1975), then labels[v] = the
 * smallest vertex id of v's component. */
static int64_t wcc_find(int64_t *parent, int64_t x) {
    int64_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) {
        int64_t nx = parent[x];
        parent[x] = r;
        x = nx;
    }
    return r;
}

int or_wcc(int64_t n, const int32_t *off, const int32_t *adj, int32_t *labels) {
    if (n < 0) return -1;
    if (n == 0) return 0;
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *size = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *mn = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!parent || !size || !mn) { free(parent); free(size); free(mn); return -2; }
    for (int64_t v = 0; v < n; v++) { parent[v] = v; size[v] = 1; }
    for (int64_t u = 0; u < n; u++)
        for (int64_t e = off[u]; e < off[u + 1]; e++) {
            int64_t a = wcc_find(parent, u), b = wcc_find(parent, adj[e]);
            if (a == b) continue;
            if (size[a] < size[b]) { int64_t t = a; a = b; b = t; }
            parent[b] = a;
            size[a] += size[b];
        }
    for (int64_t v = 0; v < n; v++) mn[v] = (int32_t)n;
    for (int64_t v = 0; v < n; v++) {
        int64_t r = wcc_find(parent, v);
        if ((int32_t)v < mn[r]) mn[r] = (int32_t)v;
    }
    for (int64_t v = 0; v < n; v++) labels[v] = mn[wcc_find(parent, v)];
    free(parent); free(size); free(mn);
    return 0;
}

/* Least-element lists (Section 5.2): with the vertices in the total order
 * order[0..n), the list of u holds every s with d(s, u) < d(k, u) for all k
 * before s in the order (d along arcs from s to u; on a symmetric digraph,
 * the undirected distance the paper uses).  Computed source by source in
 * order: a BFS from s that only enters a vertex u while d(s, u) < delta(u),
 * the smallest distance to u from any earlier source; every vertex it enters
 * gets (s, d) appended and delta(u) = d (Cohen's sequential construction,
 * which Algorithm 5 batches).  Output CSR: entries of u at
 * [off[u], off[u+1]) in order of the sources' positions, i.e. decreasing
 * distance; src/dist hold at most cap entries, *count the total.  Returns 0,
 * -1 bad argument, -2 out of memory, -3 cap exceeded (off still complete). */
int or_le_lists(int64_t n, const int32_t *off, const int32_t *adj, const int32_t *order, int64_t *loff,
                int32_t *src, int32_t *dist, int64_t cap, int64_t *count) {
    if (n < 0 || !count || (n > 0 && (!order || !loff))) return -1;
    *count = 0;
    if (n == 0) { if (loff) loff[0] = 0; return 0; }
    int32_t *delta = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    /* entries are produced source by source; keep them as (u, s, d) rows */
    int64_t rcap = 4 * n + 16, rows = 0;
    int32_t *ru = (int32_t *)malloc(sizeof(int32_t) * (size_t)rcap);
    int32_t *rs = (int32_t *)malloc(sizeof(int32_t) * (size_t)rcap);
    int32_t *rd = (int32_t *)malloc(sizeof(int32_t) * (size_t)rcap);
    uint8_t *used = (uint8_t *)calloc((size_t)n, 1);
    if (!delta || !d || !seen || !queue || !ru || !rs || !rd || !used) {
        free(delta); free(d); free(seen); free(queue); free(ru); free(rs); free(rd); free(used);
        return -2;
    }
    int rc = 0;
    for (int64_t v = 0; v < n; v++) { delta[v] = INT32_MAX; seen[v] = -1; }
    for (int64_t p = 0; p < n && rc == 0; p++) {
        const int32_t s = order[p];
        if (s < 0 || s >= n || used[s]) { rc = -1; break; }
        used[s] = 1;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        seen[s] = (int32_t)p;
        d[s] = 0;
        while (head < tail) {
            const int32_t u = queue[head++];
            /* u is entered only while it improves on delta(u) */
            if (rows == rcap) {
                rcap *= 2;
                int32_t *a = (int32_t *)realloc(ru, sizeof(int32_t) * (size_t)rcap);
                int32_t *b = a ? (int32_t *)realloc(rs, sizeof(int32_t) * (size_t)rcap) : NULL;
                int32_t *c = b ? (int32_t *)realloc(rd, sizeof(int32_t) * (size_t)rcap) : NULL;
                if (a) ru = a;
                if (b) rs = b;
                if (c) rd = c;
                if (!a || !b || !c) { rc = -2; break; }
            }
            ru[rows] = u; rs[rows] = s; rd[rows] = d[u]; rows++;
            delta[u] = d[u];
            for (int64_t e = off[u]; e < off[u + 1]; e++) {
                const int32_t w = adj[e];
                if (seen[w] == (int32_t)p) continue;
                if (d[u] + 1 >= delta[w]) continue;
                seen[w] = (int32_t)p;
                d[w] = d[u] + 1;
                queue[tail++] = w;
            }
        }
    }
    if (rc == 0) {
        /* counting sort of the rows by u; within u they are already in
         * source order (rows were produced source by source) */
        for (int64_t v = 0; v <= n; v++) loff[v] = 0;
        for (int64_t i = 0; i < rows; i++) loff[ru[i] + 1]++;
        for (int64_t v = 0; v < n; v++) loff[v + 1] += loff[v];
        *count = rows;
        if (rows > cap) {
            rc = -3;
        } else {
            int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
            if (!cur) {
                rc = -2;
            } else {
                memcpy(cur, loff, sizeof(int64_t) * (size_t)n);
                for (int64_t i = 0; i < rows; i++) {
                    const int64_t at = cur[ru[i]]++;
                    src[at] = rs[i];
                    dist[at] = rd[i];
                }
                free(cur);
            }
        }
    }
    free(delta); free(d); free(seen); free(queue); free(ru); free(rs); free(rd); free(used);
    return rc;
}
