/*
 * vc_oracle.c -- sequential CPU oracle for minimum vertex cover (MVC) and
 * parameterized vertex cover (PVC).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the solver library links, includes or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it (through oracle/__init__.py).  It shares no code,
 * header or table with the GPU path.
 *
 * What it computes (Sec. II-A): MVC(G) = min |C| over vertex covers C of the
 * simple undirected graph G, plus one cover attaining it; PVC(G, k) = whether
 * MVC(G) <= k, plus a cover of size <= k when it is.
 *
 * How: a plain, slow, one-thread branch-and-reduce that takes the steps of the
 * component-aware algorithm (Alg. 2) in the paper's order:
 *   - the initial bound is an attained approximate cover from a max-degree
 *     greedy (Sec. II-B, initial invocation of Alg. 1);
 *   - the reduction rules are degree-one, degree-two triangle and high-degree
 *     (Sec. II-B), applied sequentially in increasing vertex id until none
 *     fires;
 *   - the stopping test is |S| >= best or |E| > (best-|S|-1)^2 (Alg. 1/2);
 *   - a graph with no edges is a new best (Alg. 2);
 *   - components are found by breadth-first search from the lowest-id vertex
 *     of non-zero degree (Sec. III-B); a single component branches on a
 *     lowest-id vertex of maximum degree (v, then N(v)); several components
 *     are solved one after the other with best_i = min(best - sum, |V_i|-1)
 *     and summed (Alg. 2);
 *   - components that are cliques or chordless cycles are solved by the
 *     component rules (Sec. III-D): |C|-1 and ceil(|C|/2);
 *   - the rules are first run to a fixpoint on the whole graph and the search
 *     then runs on the subgraph induced by the remaining vertices
 *     (Sec. IV-B); crown reduction is not applied.
 * PVC runs the same search with best = k + 1 (Sec. II-B: rules and stopping
 * test use k instead of best) and answers yes iff a cover of size <= k is
 * found; a greedy cover already within k answers yes at once.
 *
 * Readings of the paper taken here (each listed in the design notes):
 *   - the stopping bound uses (best - |S| - 1)^2 as in the algorithm
 *     listings; the prose has the operands of the difference swapped;
 *   - the high-degree rule fires when d(v) > best - |S| - 1;
 *   - an isolated vertex is not a component; an edge is (a clique of two);
 *   - the component rules are applied to every component, including a
 *     single remaining one;
 *   - a component whose bound |V_i|-1 is never improved contributes the
 *     cover V_i minus its highest-id vertex.
 *
 * Tree nodes are counted as calls of the recursive solve (Table III's
 * "tree nodes visited").
 *
 * Pins (tests/test_oracle_pins.py): brute-force subset enumeration, an
 * independent bitset maximum-independent-set search, Koenig's theorem through
 * a library bipartite matching, a tree dynamic program, and the closed forms
 * P_n, C_n, K_n, K_{a,b}, star, Petersen and disjoint unions.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IN_COVER (-1)

typedef struct {
    uint32_t n;
    const uint32_t *off; /* n + 1 */
    const uint32_t *col; /* off[n] */
} graph_t;

typedef struct {
    graph_t g;
    uint64_t nodes;
    uint64_t node_limit; /* 0: unlimited */
    int aborted;
    uint8_t *seen; /* scratch for the component search, sized n */
} ctx_t;

/* ------------------------------------------------------------ basic moves */

/* Put v into the cover: v and its edges leave the graph. */
static void take(const graph_t *g, int32_t *deg, uint32_t v)
{
    for (uint32_t e = g->off[v]; e < g->off[v + 1]; ++e) {
        uint32_t w = g->col[e];
        if (deg[w] > 0)
            deg[w]--;
    }
    deg[v] = IN_COVER;
}

/* The live neighbours of v (those of non-zero degree), up to max of them. */
static int live_neighbours(const graph_t *g, const int32_t *deg, uint32_t v,
                           uint32_t *out, int max)
{
    int c = 0;
    for (uint32_t e = g->off[v]; e < g->off[v + 1]; ++e) {
        uint32_t w = g->col[e];
        if (deg[w] > 0) {
            if (c < max)
                out[c] = w;
            c++;
        }
    }
    return c;
}

static int adjacent(const graph_t *g, uint32_t u, uint32_t w)
{
    for (uint32_t e = g->off[u]; e < g->off[u + 1]; ++e)
        if (g->col[e] == w)
            return 1;
    return 0;
}

/* --------------------------------------------------------- reduction rules */

/* v has degree two and its two live neighbours (left in nb) are adjacent. */
static int in_triangle(const graph_t *g, const int32_t *deg, uint32_t v,
                       uint32_t *nb)
{
    live_neighbours(g, deg, v, nb, 2);
    return adjacent(g, nb[0], nb[1]);
}

/*
 * Sec. II-B rules, one vertex at a time in increasing id order (the vertex
 * list vl is ascending), repeated until a full pass changes nothing.
 * Stops early once |S| >= best, where the node is pruned anyway.
 */
static void reduce(const graph_t *g, int32_t *deg, const uint32_t *vl,
                   uint32_t nv, int64_t *s, int64_t best)
{
    int changed = 1;
    uint32_t nb[2];
    while (changed) {
        changed = 0;
        for (uint32_t i = 0; i < nv; ++i) {
            if (*s >= best)
                return;
            uint32_t v = vl[i];
            int32_t d = deg[v];
            if (d <= 0)
                continue;
            if (d == 1) {
                /* degree-one: the neighbour covers the same edge and more */
                live_neighbours(g, deg, v, nb, 1);
                take(g, deg, nb[0]);
                *s += 1;
                changed = 1;
            } else if (d == 2 && in_triangle(g, deg, v, nb)) {
                /* degree-two triangle: take both neighbours */
                take(g, deg, nb[0]);
                take(g, deg, nb[1]);
                *s += 2;
                changed = 1;
            } else if ((int64_t)d > best - *s - 1) {
                /* high-degree: leaving v out needs d(v) more vertices */
                take(g, deg, v);
                *s += 1;
                changed = 1;
            }
        }
    }
}

/* ------------------------------------------------------------------ search */

static void solve(ctx_t *cx, int32_t *deg, const uint32_t *vl, uint32_t nv,
                  int64_t s, int64_t *best, uint8_t *bestcov);

/* Cover of a chordless cycle: walk it from cv[0], take every second vertex
 * (and the last one when the length is odd).  cv holds the cycle's vertices. */
static void cycle_cover(const graph_t *g, const int32_t *deg, const uint32_t *cv,
                        uint32_t len, uint8_t *mark)
{
    uint32_t start = cv[0], prev = UINT32_MAX, cur = start;
    for (uint32_t i = 0; i < len; ++i) {
        if ((i & 1u) || (i == len - 1 && (len & 1u)))
            mark[cur] = 1;
        uint32_t next = UINT32_MAX;
        for (uint32_t e = g->off[cur]; e < g->off[cur + 1]; ++e) {
            uint32_t w = g->col[e];
            if (deg[w] > 0 && w != prev) {
                next = w;
                break;
            }
        }
        prev = cur;
        cur = next;
    }
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

static void solve(ctx_t *cx, int32_t *deg, const uint32_t *vl, uint32_t nv,
                  int64_t s, int64_t *best, uint8_t *bestcov)
{
    const graph_t *g = &cx->g;
    if (cx->aborted)
        return;
    cx->nodes++;
    if (cx->node_limit && cx->nodes > cx->node_limit) {
        cx->aborted = 1;
        return;
    }

    reduce(g, deg, vl, nv, &s, *best);

    /* stopping condition */
    if (s >= *best)
        return;
    int64_t E2 = 0;
    for (uint32_t i = 0; i < nv; ++i)
        if (deg[vl[i]] > 0)
            E2 += deg[vl[i]];
    int64_t E = E2 / 2, b = *best - s - 1;
    if (E > b * b)
        return;

    /* no edges left: a new best */
    if (E == 0) {
        *best = s;
        for (uint32_t i = 0; i < nv; ++i)
            bestcov[vl[i]] = (deg[vl[i]] == IN_COVER);
        return;
    }

    /* find components: BFS from each not-yet-seen vertex of non-zero degree,
     * taken in increasing id order */
    uint32_t n = g->n;
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (nv ? nv : 1));
    uint32_t *cstart = (uint32_t *)malloc(sizeof(uint32_t) * (nv + 1));
    uint32_t ncomp = 0, filled = 0;
    for (uint32_t i = 0; i < nv; ++i)
        cx->seen[vl[i]] = 0;
    for (uint32_t i = 0; i < nv; ++i) {
        uint32_t r = vl[i];
        if (deg[r] <= 0 || cx->seen[r])
            continue;
        cstart[ncomp++] = filled;
        uint32_t head = filled;
        order[filled++] = r;
        cx->seen[r] = 1;
        while (head < filled) {
            uint32_t x = order[head++];
            for (uint32_t e = g->off[x]; e < g->off[x + 1]; ++e) {
                uint32_t w = g->col[e];
                if (deg[w] > 0 && !cx->seen[w]) {
                    cx->seen[w] = 1;
                    order[filled++] = w;
                }
            }
        }
    }
    cstart[ncomp] = filled;

    /* component rules; a lone component that is neither branches on v_max */
    if (ncomp == 1) {
        uint32_t len = filled;
        int clique = 1, cyc = 1;
        for (uint32_t i = 0; i < len; ++i) {
            int32_t d = deg[order[i]];
            if ((uint32_t)d != len - 1)
                clique = 0;
            if (d != 2)
                cyc = 0;
        }
        if (clique || cyc) {
            int64_t c = clique ? (int64_t)len - 1 : ((int64_t)len + 1) / 2;
            if (s + c < *best) {
                *best = s + c;
                for (uint32_t i = 0; i < nv; ++i)
                    bestcov[vl[i]] = (deg[vl[i]] == IN_COVER);
                if (clique) {
                    uint32_t hi = 0;
                    for (uint32_t i = 0; i < len; ++i)
                        if (order[i] > hi)
                            hi = order[i];
                    for (uint32_t i = 0; i < len; ++i)
                        if (order[i] != hi)
                            bestcov[order[i]] = 1;
                } else {
                    cycle_cover(g, deg, order, len, bestcov);
                }
            }
            free(order);
            free(cstart);
            return;
        }
        free(order);
        free(cstart);

        /* branch on a vertex of maximum degree (lowest id on ties) */
        uint32_t vmax = UINT32_MAX;
        int32_t dmax = 0;
        for (uint32_t i = 0; i < nv; ++i) {
            uint32_t v = vl[i];
            if (deg[v] > dmax) {
                dmax = deg[v];
                vmax = v;
            }
        }
        int32_t *child = (int32_t *)malloc(sizeof(int32_t) * n);
        memcpy(child, deg, sizeof(int32_t) * n);
        take(g, child, vmax);
        solve(cx, child, vl, nv, s + 1, best, bestcov);

        memcpy(child, deg, sizeof(int32_t) * n);
        int64_t t = 0;
        for (uint32_t e = g->off[vmax]; e < g->off[vmax + 1]; ++e) {
            uint32_t w = g->col[e];
            if (deg[w] > 0) { /* neighbour live in the parent graph */
                take(g, child, w);
                t++;
            }
        }
        solve(cx, child, vl, nv, s + t, best, bestcov);
        free(child);
        return;
    }

    /* several components: solve each with its own bound, then combine */
    int64_t sum = s;
    uint8_t *cov = (uint8_t *)calloc(n, 1);  /* union of component covers */
    uint8_t *ccov = (uint8_t *)calloc(n, 1); /* one component's cover */
    int32_t *child = (int32_t *)malloc(sizeof(int32_t) * n);
    uint32_t *cvl = (uint32_t *)malloc(sizeof(uint32_t) * (filled ? filled : 1));
    for (uint32_t c = 0; c < ncomp && sum < *best && !cx->aborted; ++c) {
        uint32_t *cv = order + cstart[c];
        uint32_t len = cstart[c + 1] - cstart[c];
        int clique = 1, cyc = 1;
        for (uint32_t i = 0; i < len; ++i) {
            int32_t d = deg[cv[i]];
            if ((uint32_t)d != len - 1)
                clique = 0;
            if (d != 2)
                cyc = 0;
        }
        uint32_t hi = 0;
        for (uint32_t i = 0; i < len; ++i)
            if (cv[i] > hi)
                hi = cv[i];
        if (clique) {
            for (uint32_t i = 0; i < len; ++i)
                if (cv[i] != hi)
                    cov[cv[i]] = 1;
            sum += (int64_t)len - 1;
            continue;
        }
        if (cyc) {
            cycle_cover(g, deg, cv, len, cov);
            sum += ((int64_t)len + 1) / 2;
            continue;
        }
        /* best_i = min(best - sum, |V_i| - 1) */
        int64_t bi = *best - sum;
        if ((int64_t)len - 1 < bi)
            bi = (int64_t)len - 1;
        memset(child, 0, sizeof(int32_t) * n);
        for (uint32_t i = 0; i < len; ++i) {
            child[cv[i]] = deg[cv[i]];
            ccov[cv[i]] = (cv[i] != hi); /* |V_i|-1: all but one vertex */
        }
        memcpy(cvl, cv, sizeof(uint32_t) * len);
        qsort(cvl, len, sizeof(uint32_t), cmp_u32);
        solve(cx, child, cvl, len, 0, &bi, ccov);
        for (uint32_t i = 0; i < len; ++i) {
            if (ccov[cv[i]])
                cov[cv[i]] = 1;
            ccov[cv[i]] = 0;
        }
        sum += bi;
    }
    if (!cx->aborted && sum < *best) {
        *best = sum;
        for (uint32_t i = 0; i < nv; ++i)
            bestcov[vl[i]] = (deg[vl[i]] == IN_COVER) || cov[vl[i]];
    }
    free(cvl);
    free(child);
    free(ccov);
    free(cov);
    free(order);
    free(cstart);
}

/* ----------------------------------------------------------- greedy bound */

/* Max-degree greedy (lowest id on ties), lazy binary max-heap of
 * (degree, -id).  Returns |C_g| and marks C_g in cov. */
typedef struct { int32_t d; uint32_t v; } hitem;

static int hless(hitem a, hitem b) /* a below b in the max-heap */
{
    if (a.d != b.d)
        return a.d < b.d;
    return a.v > b.v;
}

static int64_t greedy_cover(const graph_t *g, uint8_t *cov)
{
    uint32_t n = g->n;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    hitem *h = (hitem *)malloc(sizeof(hitem) * (n ? n : 1));
    uint32_t hn = 0;
    for (uint32_t v = 0; v < n; ++v) {
        deg[v] = (int32_t)(g->off[v + 1] - g->off[v]);
        cov[v] = 0;
    }
    for (uint32_t v = 0; v < n; ++v) {
        if (deg[v] <= 0)
            continue;
        hitem it = {deg[v], v};
        uint32_t i = hn++;
        while (i > 0 && hless(h[(i - 1) / 2], it)) {
            h[i] = h[(i - 1) / 2];
            i = (i - 1) / 2;
        }
        h[i] = it;
    }
    int64_t size = 0;
    while (hn > 0) {
        hitem top = h[0];
        hitem last = h[--hn];
        uint32_t i = 0;
        for (;;) {
            uint32_t c = 2 * i + 1;
            if (c >= hn)
                break;
            if (c + 1 < hn && hless(h[c], h[c + 1]))
                c++;
            if (!hless(last, h[c]))
                break;
            h[i] = h[c];
            i = c;
        }
        if (hn > 0)
            h[i] = last;
        int32_t d = deg[top.v];
        if (d <= 0)
            continue;
        if (d != top.d) { /* stale key: re-insert with the current degree */
            hitem it = {d, top.v};
            uint32_t j = hn++;
            while (j > 0 && hless(h[(j - 1) / 2], it)) {
                h[j] = h[(j - 1) / 2];
                j = (j - 1) / 2;
            }
            h[j] = it;
            continue;
        }
        take(g, deg, top.v);
        cov[top.v] = 1;
        size++;
    }
    free(h);
    free(deg);
    return size;
}

/* ---------------------------------------------------------------- driver */

/*
 * Solve with initial bound best0 whose attained cover is cov0 (may be NULL
 * when best0 is only a bound, as k + 1 in PVC).  On return *best holds the
 * final value and cover[] marks a cover of that size if it was attained.
 * Returns 0, or -2 when the node limit was hit.
 */
static int run(const graph_t *g, int64_t best0, const uint8_t *cov0,
               uint64_t node_limit, int64_t *best_out, uint8_t *cover,
               uint64_t *nodes_out, uint32_t *kernel_n_out)
{
    uint32_t n = g->n;
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    uint32_t *all = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    for (uint32_t v = 0; v < n; ++v) {
        deg[v] = (int32_t)(g->off[v + 1] - g->off[v]);
        all[v] = v;
    }
    /* root: rules to a fixpoint on the whole graph (Sec. IV-B) */
    int64_t s = 0;
    reduce(g, deg, all, n, &s, best0);

    /* induce the subgraph on the vertices that still have edges */
    uint32_t *newid = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint32_t np = 0;
    for (uint32_t v = 0; v < n; ++v)
        newid[v] = deg[v] > 0 ? np++ : UINT32_MAX;
    uint32_t *oldid = (uint32_t *)malloc(sizeof(uint32_t) * (np ? np : 1));
    uint32_t *noff = (uint32_t *)malloc(sizeof(uint32_t) * (np + 1));
    uint64_t nnz = 0;
    for (uint32_t v = 0; v < n; ++v)
        if (newid[v] != UINT32_MAX) {
            oldid[newid[v]] = v;
            nnz += (uint64_t)deg[v];
        }
    uint32_t *ncol = (uint32_t *)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
    noff[0] = 0;
    uint64_t at = 0;
    for (uint32_t i = 0; i < np; ++i) {
        uint32_t v = oldid[i];
        for (uint32_t e = g->off[v]; e < g->off[v + 1]; ++e) {
            uint32_t w = g->col[e];
            if (deg[w] > 0)
                ncol[at++] = newid[w];
        }
        noff[i + 1] = (uint32_t)at;
    }
    if (kernel_n_out)
        *kernel_n_out = np;

    ctx_t cx;
    memset(&cx, 0, sizeof cx);
    cx.g.n = np;
    cx.g.off = noff;
    cx.g.col = ncol;
    cx.node_limit = node_limit;
    cx.seen = (uint8_t *)calloc(np ? np : 1, 1);
    int32_t *kdeg = (int32_t *)malloc(sizeof(int32_t) * (np ? np : 1));
    uint32_t *kvl = (uint32_t *)malloc(sizeof(uint32_t) * (np ? np : 1));
    uint8_t *kcov = (uint8_t *)calloc(np ? np : 1, 1);
    for (uint32_t i = 0; i < np; ++i) {
        kdeg[i] = (int32_t)(noff[i + 1] - noff[i]);
        kvl[i] = i;
    }
    int64_t kbest = best0 - s; /* what the kernel must beat */
    int64_t kbest0 = kbest;
    int rc = 0;
    if (kbest > 0)
        solve(&cx, kdeg, kvl, np, 0, &kbest, kcov);
    if (cx.aborted)
        rc = -2;
    if (nodes_out)
        *nodes_out = cx.nodes;

    if (kbest < kbest0) {
        /* improved: root-forced vertices plus the kernel's cover */
        *best_out = s + kbest;
        for (uint32_t v = 0; v < n; ++v)
            cover[v] = (deg[v] == IN_COVER);
        for (uint32_t i = 0; i < np; ++i)
            if (kcov[i])
                cover[oldid[i]] = 1;
    } else {
        *best_out = best0;
        if (cov0)
            memcpy(cover, cov0, n);
        else
            memset(cover, 0, n);
    }
    free(kcov);
    free(kvl);
    free(kdeg);
    free(cx.seen);
    free(ncol);
    free(noff);
    free(oldid);
    free(newid);
    free(all);
    free(deg);
    return rc;
}

/* ------------------------------------------------------------ public API */

/*
 * oracle_mvc: minimum vertex cover.  off[n+1], col[off[n]] is a symmetric
 * simple CSR with 32-bit column ids.  Writes the cover's vertex ids in
 * ascending order to cover_out (capacity n) and its length to *cover_len.
 * Returns the MVC size, -2 when node_limit (0 = none) was exceeded, -1 on
 * allocation failure.
 */
int64_t oracle_mvc(uint32_t n, const uint32_t *off, const uint32_t *col,
                   uint64_t node_limit, uint32_t *cover_out,
                   uint32_t *cover_len, uint64_t *nodes, uint32_t *kernel_n)
{
    graph_t g = {n, off, col};
    uint8_t *cg = (uint8_t *)calloc(n ? n : 1, 1);
    uint8_t *cov = (uint8_t *)calloc(n ? n : 1, 1);
    if (!cg || !cov)
        return -1;
    int64_t best0 = greedy_cover(&g, cg);
    int64_t best = best0;
    int rc = run(&g, best0, cg, node_limit, &best, cov, nodes, kernel_n);
    uint32_t c = 0;
    for (uint32_t v = 0; v < n; ++v)
        if (cov[v])
            cover_out[c++] = v;
    *cover_len = c;
    free(cg);
    free(cov);
    return rc ? rc : best;
}

/*
 * oracle_pvc: is there a vertex cover of size <= k?  Returns 1 (yes, cover
 * written), 0 (no, *cover_len = 0), -2 when node_limit was exceeded.
 */
int oracle_pvc(uint32_t n, const uint32_t *off, const uint32_t *col,
               uint32_t k, uint64_t node_limit, uint32_t *cover_out,
               uint32_t *cover_len, uint64_t *nodes, uint32_t *kernel_n)
{
    graph_t g = {n, off, col};
    uint8_t *cg = (uint8_t *)calloc(n ? n : 1, 1);
    uint8_t *cov = (uint8_t *)calloc(n ? n : 1, 1);
    if (!cg || !cov)
        return -1;
    int64_t gsize = greedy_cover(&g, cg);
    int yes;
    int rc = 0;
    if (gsize <= (int64_t)k) {
        memcpy(cov, cg, n);
        yes = 1;
        if (nodes)
            *nodes = 0;
        if (kernel_n)
            *kernel_n = 0;
    } else {
        int64_t best = (int64_t)k + 1;
        rc = run(&g, (int64_t)k + 1, NULL, node_limit, &best, cov, nodes,
                 kernel_n);
        yes = best <= (int64_t)k;
    }
    uint32_t c = 0;
    if (yes)
        for (uint32_t v = 0; v < n; ++v)
            if (cov[v])
                cover_out[c++] = v;
    *cover_len = c;
    free(cg);
    free(cov);
    return rc ? rc : yes;
}

/* oracle_greedy: the max-degree greedy cover used as the initial bound. */
int64_t oracle_greedy(uint32_t n, const uint32_t *off, const uint32_t *col,
                      uint32_t *cover_out, uint32_t *cover_len)
{
    graph_t g = {n, off, col};
    uint8_t *cg = (uint8_t *)calloc(n ? n : 1, 1);
    if (!cg)
        return -1;
    int64_t s = greedy_cover(&g, cg);
    uint32_t c = 0;
    for (uint32_t v = 0; v < n; ++v)
        if (cg[v])
            cover_out[c++] = v;
    *cover_len = c;
    free(cg);
    return s;
}

/* ------------------------------------------------------------------------
 * Enumeration of the minimal vertex covers of size <= k (the PVC variant
 * that Sec. III-E describes but the paper does not build).  Reading taken:
 * "all covers of size <= k" is represented by its minimal members; every
 * cover of size <= k contains one of them.  A cover C is minimal when every
 * vertex of C has a neighbour outside C.
 *
 * Plain enumeration from that definition: take the lowest-id vertex u with an
 * edge to a vertex outside C (an uncovered edge {u, w}); either u joins C, or
 * u stays out for good and all of N(u) joins C (a branch that would put an
 * excluded vertex into C is dropped).  Every assignment reached is
 * consistent, so no set is reached twice, and following a minimal cover C*
 * (u in C* or not) reaches C* itself; a leaf (no uncovered edge) is kept
 * when it is minimal.  Branches with |C| > k are cut.
 * ------------------------------------------------------------------------ */

typedef struct {
    const graph_t *g;
    uint32_t k;
    uint8_t *in;  /* 1: in C */
    uint8_t *out; /* 1: kept out of C */
    uint32_t size;
    uint64_t found, cap; /* covers found; covers that fit in ids/offs */
    uint32_t *ids;       /* cap * k ids */
    uint32_t *lens;      /* cap lengths */
    uint64_t nodes, node_limit;
    int over; /* node limit reached */
} enum_t;

static int enum_minimal_leaf(const enum_t *e)
{
    const graph_t *g = e->g;
    for (uint32_t v = 0; v < g->n; ++v) {
        if (!e->in[v])
            continue;
        int has_out = 0;
        for (uint32_t i = g->off[v]; i < g->off[v + 1]; ++i)
            if (!e->in[g->col[i]]) {
                has_out = 1;
                break;
            }
        if (!has_out)
            return 0;
    }
    return 1;
}

static void enum_rec(enum_t *e)
{
    const graph_t *g = e->g;
    if (e->over)
        return;
    if (e->node_limit && ++e->nodes > e->node_limit) {
        e->over = 1;
        return;
    }
    if (e->size > e->k)
        return;
    /* lowest u with an uncovered edge */
    uint32_t u = g->n;
    for (uint32_t v = 0; v < g->n && u == g->n; ++v) {
        if (e->in[v])
            continue;
        for (uint32_t i = g->off[v]; i < g->off[v + 1]; ++i)
            if (!e->in[g->col[i]]) {
                u = v;
                break;
            }
    }
    if (u == g->n) {
        if (enum_minimal_leaf(e)) {
            if (e->found < e->cap) {
                uint32_t c = 0;
                for (uint32_t v = 0; v < g->n; ++v)
                    if (e->in[v])
                        e->ids[e->found * e->k + c++] = v;
                e->lens[e->found] = c;
            }
            ++e->found;
        }
        return;
    }
    /* u joins C */
    e->in[u] = 1;
    ++e->size;
    enum_rec(e);
    e->in[u] = 0;
    --e->size;
    /* u stays out: N(u) joins C, unless one of them was kept out */
    for (uint32_t i = g->off[u]; i < g->off[u + 1]; ++i)
        if (e->out[g->col[i]])
            return;
    uint32_t added = 0;
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (g->off[u + 1] - g->off[u] + 1));
    if (!list) {
        e->over = 2;
        return;
    }
    for (uint32_t i = g->off[u]; i < g->off[u + 1]; ++i) {
        uint32_t w = g->col[i];
        if (!e->in[w]) {
            e->in[w] = 1;
            list[added++] = w;
        }
    }
    e->out[u] = 1;
    e->size += added;
    enum_rec(e);
    e->size -= added;
    e->out[u] = 0;
    for (uint32_t i = 0; i < added; ++i)
        e->in[list[i]] = 0;
    free(list);
}

/* oracle_enum_minimal: number of minimal covers of size <= k (-2: node limit,
 * -1: allocation); the first `cap` of them go to ids[c*k ..] (ascending) and
 * lens[c]. */
int64_t oracle_enum_minimal(uint32_t n, const uint32_t *off, const uint32_t *col, uint32_t k,
                            uint64_t cap, uint32_t *ids, uint32_t *lens, uint64_t node_limit)
{
    graph_t g = {n, off, col};
    enum_t e;
    memset(&e, 0, sizeof e);
    e.g = &g;
    e.k = k;
    e.cap = cap;
    e.ids = ids;
    e.lens = lens;
    e.node_limit = node_limit;
    e.in = (uint8_t *)calloc(n ? n : 1, 1);
    e.out = (uint8_t *)calloc(n ? n : 1, 1);
    if (!e.in || !e.out) {
        free(e.in);
        free(e.out);
        return -1;
    }
    enum_rec(&e);
    free(e.in);
    free(e.out);
    if (e.over == 2)
        return -1;
    if (e.over)
        return -2;
    return (int64_t)e.found;
}
