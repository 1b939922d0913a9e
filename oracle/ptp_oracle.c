/*
 * CPU FP64 oracle for Parallel Toplesets Propagation (PTP), written from the
 * paper (Romero Calla, Fuentes Perez, Montenegro, "A minimalistic approach for
 * fast computation of geodesic distances on triangular meshes").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library: it is a plain, slow, sequential restatement of the method.
 *
 * Contents
 *   ptpo_toplesets      topological level sets by BFS (Sec. 4.1, Definition of
 *                       V_r) and their canonical order (Sec. 4.3 reorder; the
 *                       order inside a topleset is ascending vertex id).
 *   ptpo_local_update   the planar (Kimmel-Sethian) update of a vertex from one
 *                       incident triangle, in the matrix form with the
 *                       monotonicity test Q X^T n < 0 (Sec. 3.2).
 *   ptpo_run            the PTP iteration: Jacobi update of the band
 *                       B_{i_k}^{j_k} (Sec. 4.2), band ends from Eq. upper_band
 *                       and Eq. lower_band; optionally the fixed half band of
 *                       the complexity analysis (Sec. 6).
 *   ptpo_run_replay     the same iteration under a given retirement schedule
 *                       (the arithmetic compared under another run's band).
 *   ptpo_run_warm       the same iteration started from a caller's upper
 *                       bound instead of +inf, certified first or taken as a
 *                       known supersolution (an extension of the method, not
 *                       in the paper; farthest point sampling restarts from
 *                       the previous map this way).
 *   ptpo_fixed_point    plain Jacobi over all vertices until nothing changes:
 *                       the fixed point d* that PTP approximates.
 *   ptpo_labels_from_map  Voronoi labels (Sec. 5.3) of a distance map: each
 *                       vertex takes the source at the root of its chain of
 *                       parents (the input its value comes from).
 *   ptpo_fast_marching  sequential Fast Marching (Sec. 3.2) with the same
 *                       local update and accepted-only inputs.
 *
 * Precision: all arithmetic in double.  Coordinates arrive as doubles that
 * the caller promoted exactly from the float32 mesh.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - V_0 = S is converged from the start; the band starts at i = 1.
 *   - a value that was still infinite at the previous iteration is not
 *     converged; an unchanged value counts as converged (avoids 0/0).
 *   - the band of iteration k is [i_{k-1}, j_k]; V_{i_{k-1}} is then tested
 *     to obtain i_k; at most one topleset retires per iteration.
 *   - new value = min(old value, min over incident triangles of the update).
 *   - unreachable vertices keep +inf and label -1 and are ordered last.
 *   - degenerate triangle (det G <= 1e-12 a c): edge updates only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PTPO_OK 0
#define PTPO_EINVAL (-1)
#define PTPO_ENOMEM (-2)
#define PTPO_ENOCONV (-4)

/* ------------------------------------------------------------------ */
/* vertex -> incident faces                                           */
/* ------------------------------------------------------------------ */

typedef struct {
    int n, nf;
    int *start; /* n + 1 */
    int *face;  /* 3 nf */
} incidence;

static int build_incidence(int n, int nf, const int *F, incidence *inc)
{
    inc->n = n;
    inc->nf = nf;
    inc->start = (int *)calloc((size_t)n + 1, sizeof(int));
    inc->face = (int *)malloc(sizeof(int) * (size_t)(3 * (size_t)nf + 1));
    int *fill = (int *)calloc((size_t)n + 1, sizeof(int));
    if (!inc->start || !inc->face || !fill) {
        free(inc->start); free(inc->face); free(fill);
        return PTPO_ENOMEM;
    }
    for (size_t t = 0; t < 3 * (size_t)nf; ++t)
        inc->start[F[t] + 1] += 1;
    for (int v = 0; v < n; ++v)
        inc->start[v + 1] += inc->start[v];
    for (int t = 0; t < nf; ++t)
        for (int c = 0; c < 3; ++c) {
            int v = F[3 * t + c];
            inc->face[inc->start[v] + fill[v]++] = t;
        }
    free(fill);
    return PTPO_OK;
}

static void free_incidence(incidence *inc)
{
    free(inc->start);
    free(inc->face);
}

static int check_mesh(int n, int nf, const int *F, int m, const int *S)
{
    if (n <= 0 || nf < 0 || m <= 0) return PTPO_EINVAL;
    for (size_t t = 0; t < 3 * (size_t)nf; ++t)
        if (F[t] < 0 || F[t] >= n) return PTPO_EINVAL;
    for (int a = 0; a < m; ++a) {
        if (S[a] < 0 || S[a] >= n) return PTPO_EINVAL;
        for (int b = 0; b < a; ++b)
            if (S[a] == S[b]) return PTPO_EINVAL;
    }
    return PTPO_OK;
}

/* ------------------------------------------------------------------ */
/* toplesets: BFS hop distance from S over the edges of the faces      */
/* ------------------------------------------------------------------ */

static int toplesets_with(const incidence *inc, const int *F, int m, const int *S,
                          int *level, int *order, int *offsets, int *rho_out)
{
    int n = inc->n;
    int *queue = (int *)malloc(sizeof(int) * (size_t)n);
    if (!queue) return PTPO_ENOMEM;
    for (int v = 0; v < n; ++v) level[v] = -1;
    int head = 0, tail = 0;
    for (int a = 0; a < m; ++a) {
        level[S[a]] = 0;
        queue[tail++] = S[a];
    }
    int maxlev = 0;
    while (head < tail) {
        int v = queue[head++];
        for (int e = inc->start[v]; e < inc->start[v + 1]; ++e) {
            const int *f = F + 3 * inc->face[e];
            for (int c = 0; c < 3; ++c) {
                int u = f[c];
                if (level[u] < 0) {
                    level[u] = level[v] + 1;
                    if (level[u] > maxlev) maxlev = level[u];
                    queue[tail++] = u;
                }
            }
        }
    }
    free(queue);
    int rho = maxlev + 1;
    /* canonical order: by level, ascending id inside a level; unreachable last */
    int *count = (int *)calloc((size_t)rho + 2, sizeof(int));
    if (!count) return PTPO_ENOMEM;
    for (int v = 0; v < n; ++v) {
        int b = level[v] < 0 ? rho : level[v];
        count[b + 1] += 1;
    }
    for (int r = 0; r <= rho; ++r) count[r + 1] += count[r];
    if (offsets)
        for (int r = 0; r <= rho; ++r) offsets[r] = count[r];
    for (int v = 0; v < n; ++v) {
        int b = level[v] < 0 ? rho : level[v];
        order[count[b]++] = v;
    }
    free(count);
    *rho_out = rho;
    return PTPO_OK;
}

/* level[n]: hop distance (-1 unreachable); order[n]: vertex ids sorted by
 * (level, id) with unreachable vertices last; offsets[rho + 1]: V_r is
 * order[offsets[r] .. offsets[r+1]); caller sizes offsets for n + 1.     */
int ptpo_toplesets(int n, int nf, const int *F, int m, const int *S,
                   int *level, int *order, int *offsets, int *rho)
{
    int rc = check_mesh(n, nf, F, m, S);
    if (rc) return rc;
    incidence inc;
    rc = build_incidence(n, nf, F, &inc);
    if (rc) return rc;
    rc = toplesets_with(&inc, F, m, S, level, order, offsets, rho);
    free_incidence(&inc);
    return rc;
}

/* ------------------------------------------------------------------ */
/* local update (Sec. 3.2, update_step)                                */
/* ------------------------------------------------------------------ */

/* The distance is modelled on the triangle (x0, x1, x2) as a plane front
 * phi(x) = n . x + c with |n| = 1 and n in the triangle's plane, through
 * (x1, d1) and (x2, d2).  With X = [x1 - x0, x2 - x0], Q = (X^T X)^{-1} and
 * t = (d1, d2) the unknown p = phi(x0) satisfies
 *     (t - p 1)^T Q (t - p 1) = 1,
 * a quadratic in p whose larger root is taken.  The solution is accepted only
 * when Q X^T n = Q (t - p 1) < 0 in both components (the monotonicity
 * condition); otherwise, and when either input is missing, the update comes
 * from the edges, min_i (d_i + |x_i - x0|).
 *
 * *lab_out names where the value comes from: an edge update gives the tag
 * (l1 or l2) of its vertex, a planar value that of its smaller input; equal
 * candidates give the smaller tag.  With vertex ids as tags this is the
 * vertex the value comes from (the parent of the Voronoi labels below). */
static double local_update(const double *x0, const double *x1, const double *x2,
                           double d1, double d2, int l1, int l2, int *lab_out)
{
    double e1[3], e2[3];
    for (int c = 0; c < 3; ++c) {
        e1[c] = x1[c] - x0[c];
        e2[c] = x2[c] - x0[c];
    }
    double a = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    double b = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    double c = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    int f1 = isfinite(d1), f2 = isfinite(d2);
    if (!f1 && !f2) {
        *lab_out = -1;
        return INFINITY;
    }
    if (!f2) {
        *lab_out = l1;
        return d1 + sqrt(a);
    }
    if (!f1) {
        *lab_out = l2;
        return d2 + sqrt(c);
    }
    double p1 = d1 + sqrt(a), p2 = d2 + sqrt(c);
    double pedge;
    int ledge;
    if (p1 < p2) { pedge = p1; ledge = l1; }
    else if (p2 < p1) { pedge = p2; ledge = l2; }
    else { pedge = p1; ledge = l1 < l2 ? l1 : l2; }

    double det = a * c - b * b;
    if (!(det > 1e-12 * a * c)) {
        *lab_out = ledge;
        return pedge;
    }
    /* Q = G^{-1} = [[c, -b], [-b, a]] / det */
    double q11 = c / det, q12 = -b / det, q22 = a / det;
    double s11 = q11 + 2.0 * q12 + q22;                    /* 1^T Q 1 */
    double s1t = (q11 + q12) * d1 + (q12 + q22) * d2;      /* 1^T Q t */
    double stt = q11 * d1 * d1 + 2.0 * q12 * d1 * d2 + q22 * d2 * d2; /* t^T Q t */
    double disc = s1t * s1t - s11 * (stt - 1.0);
    if (disc < 0.0) {
        *lab_out = ledge;
        return pedge;
    }
    double p = (s1t + sqrt(disc)) / s11;
    double r1 = d1 - p, r2 = d2 - p;                       /* t - p 1 = X^T n */
    double al1 = q11 * r1 + q12 * r2;
    double al2 = q12 * r1 + q22 * r2;
    if (al1 < 0.0 && al2 < 0.0) {
        if (d1 < d2) *lab_out = l1;
        else if (d2 < d1) *lab_out = l2;
        else *lab_out = l1 < l2 ? l1 : l2;
        return p;
    }
    *lab_out = ledge;
    return pedge;
}

double ptpo_local_update(const double *x0, const double *x1, const double *x2,
                         double d1, double d2, int *lab_out)
{
    int lab;
    double p = local_update(x0, x1, x2, d1, d2, 1, 2, &lab);
    if (lab_out) *lab_out = lab;
    return p;
}

/* Best update of vertex v over its incident triangles, reading dist; with
 * `usable`, an input not marked usable counts as +inf. */
static double best_update(int v, const incidence *inc, const int *F, const double *X,
                          const double *dist, const unsigned char *usable)
{
    double bu = INFINITY;
    for (int e = inc->start[v]; e < inc->start[v + 1]; ++e) {
        const int *f = F + 3 * inc->face[e];
        int a, b;
        if (f[0] == v) { a = f[1]; b = f[2]; }
        else if (f[1] == v) { a = f[2]; b = f[0]; }
        else { a = f[0]; b = f[1]; }
        double da = dist[a], db = dist[b];
        if (usable) {
            if (!usable[a]) da = INFINITY;
            if (!usable[b]) db = INFINITY;
        }
        int l;
        double u = local_update(X + 3 * (size_t)v, X + 3 * (size_t)a, X + 3 * (size_t)b,
                                da, db, a, b, &l);
        if (u < bu) bu = u;
    }
    return bu;
}

/* ------------------------------------------------------------------ */
/* Voronoi labels from the final map                                   */
/* ------------------------------------------------------------------ */

/* The paper splits the mesh into the regions of the sources (Sec. 5.3)
 * without saying how a vertex is assigned to one; the reading here makes
 * the label a function of the final distance map.  The parent of a
 * reachable vertex v that is not a source is the vertex its value comes
 * from under its best triangle: over the incident triangles the smallest
 * (update, giver id), where the giver of a planar value is its smaller
 * input (equal inputs: the smaller id) and that of an edge update the
 * edge's other end (equal updates: the smaller id).  Only givers that come
 * before v in (distance, id) order count, so the parents form a forest
 * whose roots are the sources.  A vertex takes the index in S of its root;
 * unreachable vertices, and a vertex with no giver before it (possible only
 * on degenerate input), get -1.  Vertices are labelled in (distance, id)
 * order, so a parent is labelled before its children. */
typedef struct {
    double d;
    int v;
} dist_id;

static int cmp_dist_id(const void *pa, const void *pb)
{
    const dist_id *a = (const dist_id *)pa, *b = (const dist_id *)pb;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    return (a->v > b->v) - (a->v < b->v);
}

static int label_from_map(int n, const incidence *inc, const int *F, const double *X, int m,
                          const int *S, const double *dist, int *label, int *parent)
{
    dist_id *ord = (dist_id *)malloc(sizeof(dist_id) * ((size_t)n + 1));
    if (!ord) return PTPO_ENOMEM;
    int cnt = 0;
    for (int v = 0; v < n; ++v) {
        label[v] = -1;
        if (parent) parent[v] = -1;
        if (isfinite(dist[v])) {
            ord[cnt].d = dist[v];
            ord[cnt].v = v;
            cnt++;
        }
    }
    for (int a = 0; a < m; ++a) {
        label[S[a]] = a;
        if (parent) parent[S[a]] = S[a];
    }
    qsort(ord, (size_t)cnt, sizeof(dist_id), cmp_dist_id);
    for (int q = 0; q < cnt; ++q) {
        const int v = ord[q].v;
        if (label[v] >= 0) continue;                     /* a source */
        double bu = INFINITY;
        int bg = -1;
        for (int e = inc->start[v]; e < inc->start[v + 1]; ++e) {
            const int *f = F + 3 * inc->face[e];
            int a, b;
            if (f[0] == v) { a = f[1]; b = f[2]; }
            else if (f[1] == v) { a = f[2]; b = f[0]; }
            else { a = f[0]; b = f[1]; }
            int g;
            double u = local_update(X + 3 * (size_t)v, X + 3 * (size_t)a, X + 3 * (size_t)b,
                                    dist[a], dist[b], a, b, &g);
            if (!isfinite(u)) continue;
            if (!(dist[g] < dist[v] || (dist[g] == dist[v] && g < v))) continue;
            if (u < bu || (u == bu && g < bg)) {
                bu = u;
                bg = g;
            }
        }
        if (parent) parent[v] = bg;
        label[v] = bg >= 0 ? label[bg] : -1;
    }
    free(ord);
    return PTPO_OK;
}

int ptpo_labels_from_map(int n, int nf, const double *X, const int *F, int m, const int *S,
                         const double *dist, int *label, int *parent)
{
    int rc = check_mesh(n, nf, F, m, S);
    if (rc) return rc;
    incidence inc;
    rc = build_incidence(n, nf, F, &inc);
    if (rc) return rc;
    rc = label_from_map(n, &inc, F, X, m, S, dist, label, parent);
    free_incidence(&inc);
    return rc;
}

/* ------------------------------------------------------------------ */
/* PTP iteration (Sec. 4.2)                                            */
/* ------------------------------------------------------------------ */

typedef struct {
    double tol;       /* epsilon of Eq. lower_band, > 0                     */
    int max_iters;    /* iteration cap K_max; 0 -> 4 rho + 16               */
    int band_rule;    /* 0: relative change (Eq. lower_band)                */
                      /* 1: fixed half band [floor((k+1)/2), k] of the      */
                      /*    complexity analysis (Sec. 6), stop after        */
                      /*    2 rho - 3 iterations                            */
    int window;       /* > 0: band holds at most `window` toplesets; the    */
                      /* ones pushed out below it retire.  0: unbounded     */
} ptpo_options;

typedef struct {
    int iterations;       /* K                                             */
    int rho;              /* number of toplesets                           */
    int reachable;        /* vertices with finite distance                 */
    long long updates;    /* U = sum_k |B_k| (vertex updates)              */
} ptpo_stats;

/* How the lower end of the band is chosen.  Exactly one mode per run. */
typedef struct {
    const double *upper;      /* warm start (caller order), or NULL: start from +inf */
    int certify;              /* warm start: certify the bound first (1) or take it  */
                              /* as a known supersolution (0)                       */
    const int *replay;        /* replay: retire[r] of a given run (the last          */
                              /* iteration that updated V_r, -1 never) and the      */
    int replay_K;             /* iteration count K of that run; or NULL             */
} run_mode;

/*
 * dist[n], label[n] (may be NULL): results in the caller's vertex order.
 * retire_k[n] (may be NULL): the last iteration that updated V_r (V_0: 0;
 *   never retired: -1).
 * trace_lo[max_iters + 1], trace_maxrel[max_iters + 1] (may be NULL): for
 *   each k, the first topleset of the band and the largest relative change
 *   over V_{i_{k-1}} (inf when some value was still infinite).
 * Returns PTPO_OK, PTPO_ENOCONV (cap reached; results so far written) or an
 * error.
 */
static int run_core(int n, int nf, const double *X, const int *F, int m, const int *S,
                    const ptpo_options *opt, const run_mode *mode, double *dist, int *label,
                    ptpo_stats *st, int *retire_k, int *trace_lo, double *trace_maxrel,
                    int trace_len, int *rejected_out, double *certified_out)
{
    int rc = check_mesh(n, nf, F, m, S);
    if (rc) return rc;
    if (!(opt->tol > 0.0) || opt->window < 0 || opt->max_iters < 0 || opt->band_rule < 0 ||
        opt->band_rule > 1)
        return PTPO_EINVAL;
    const double *upper = mode ? mode->upper : NULL;
    const int *replay = mode ? mode->replay : NULL;
    incidence inc;
    rc = build_incidence(n, nf, F, &inc);
    if (rc) return rc;
    int *level = (int *)malloc(sizeof(int) * (size_t)n);
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    int *offsets = (int *)malloc(sizeof(int) * ((size_t)n + 2));
    double *dold = (double *)malloc(sizeof(double) * (size_t)n);
    double *dnew = (double *)malloc(sizeof(double) * (size_t)n);
    if (!level || !order || !offsets || !dold || !dnew) {
        rc = PTPO_ENOMEM;
        goto out;
    }
    int rho;
    rc = toplesets_with(&inc, F, m, S, level, order, offsets, &rho);
    if (rc) goto out;

    for (int v = 0; v < n; ++v) dold[v] = INFINITY;
    for (int a = 0; a < m; ++a) dold[S[a]] = 0.0;
    if (upper) {
        /* Warm start.  Every reachable non-source vertex starts from the
         * caller's bound (negative or NaN: no bound).  Certification: a vertex
         * whose bound is below the best planar update from its neighbours'
         * bounds, w(v) < U(w)(v), loses it (+inf); repeated until nothing
         * changes.  What remains obeys w >= U(w) with w = 0 on S.  Without
         * certification the caller vouches for that property (a distance map
         * of a subset of S computed by this iteration has it: each value was
         * set to U of an earlier, pointwise larger map). */
        for (int v = 0; v < n; ++v)
            if (level[v] > 0) dold[v] = upper[v] >= 0.0 ? upper[v] : INFINITY;
        int rejected = 0, changed = mode->certify;
        while (changed) {
            changed = 0;
            for (int q = 0; q < n; ++q) {
                int v = order[q];
                if (level[v] <= 0 || !isfinite(dold[v])) continue;
                const double bu = best_update(v, &inc, F, X, dold, NULL);
                if (dold[v] < bu) {
                    dold[v] = INFINITY;
                    rejected++;
                    changed = 1;
                }
            }
        }
        if (rejected_out) *rejected_out = rejected;
        if (certified_out) memcpy(certified_out, dold, sizeof(double) * (size_t)n);
    }
    if (retire_k) {
        for (int r = 0; r < n; ++r) retire_k[r] = -1;
        retire_k[0] = 0;
    }
    int kmax = opt->max_iters > 0 ? opt->max_iters : 4 * rho + 16;
    /* the fixed band finalises V_r by iteration 2r - 1 (Sec. 6 lemma for
     * regular meshes), so the last topleset is done after 2 rho - 3 */
    const int kfix = 2 * rho - 3 > 1 ? 2 * rho - 3 : 1;
    if (replay) {
        kmax = mode->replay_K;
        if (kmax < 0 || replay[0] != 0) {
            rc = PTPO_EINVAL;
            goto out;
        }
    }
    int i = 1, k = 0;
    long long U = 0;
    memcpy(dnew, dold, sizeof(double) * (size_t)n);
    while (i < rho && k < kmax) {
        k += 1;
        int j = k < rho ? k : rho - 1;                   /* Eq. upper_band */
        int lo;
        if (replay) {
            /* the band holds every topleset the given run had not retired
             * before iteration k */
            lo = i;
            while (lo < rho && replay[lo] >= 0 && replay[lo] < k) lo++;
            if (lo > j) {
                rc = PTPO_EINVAL;
                goto out;
            }
        } else if (opt->band_rule == 1) {
            lo = (k + 1) / 2;                            /* fixed half band */
            if (lo < 1) lo = 1;
        } else {
            lo = i;
        }
        if (opt->window > 0 && !replay && j - opt->window + 1 > lo) {
            lo = j - opt->window + 1;
            /* toplesets pushed below the window are no longer updated */
        }
        if (retire_k)
            for (int r = i; r < lo; ++r) retire_k[r] = k - 1;
        /* Jacobi update of the band: d_k on B from d_{k-1}; d_k = d_{k-1}
         * everywhere else.  The vertices are independent (each reads the
         * previous map only), so the loop may run on several threads. */
        const int qb = offsets[lo], qe = offsets[j + 1];
#pragma omp parallel for schedule(static)
        for (int q = qb; q < qe; ++q) {
            int v = order[q];
            const double bu = best_update(v, &inc, F, X, dold, NULL);
            dnew[v] = bu < dold[v] ? bu : dold[v];
        }
        U += qe - qb;
        if (trace_lo && k < trace_len) trace_lo[k] = lo;
        int inew;
        if (replay) {
            inew = lo;
            while (inew < rho && replay[inew] >= 0 && replay[inew] <= k) inew++;
            if (retire_k)
                for (int r = lo; r < inew; ++r) retire_k[r] = k;
        } else if (opt->band_rule == 1) {
            /* the toplesets below the next iteration's band are final; after
             * the last iteration every topleset is */
            inew = k >= kfix ? rho : (k + 2) / 2;
            if (inew < lo) inew = lo;
            if (retire_k)
                for (int r = lo; r < inew && r < rho; ++r) retire_k[r] = k;
        } else {
            /* Eq. lower_band: V_lo retires when every value in it was finite
             * and changed by a relative amount below tol, and not before its
             * second update (k > lo).  From +inf a value is first finite after
             * the iteration that reached its topleset, so the second condition
             * only binds for a warm start.  At most one topleset per
             * iteration. */
            inew = lo;
            if (lo < rho && lo <= j && k > lo) {
                double worst = 0.0;
                int ok = 1;
                for (int q = offsets[lo]; q < offsets[lo + 1]; ++q) {
                    int v = order[q];
                    if (!isfinite(dold[v])) {
                        ok = 0;
                        worst = INFINITY;
                        break;
                    }
                    if (dnew[v] == dold[v]) continue;
                    double rel = fabs(dnew[v] - dold[v]) / dold[v];
                    if (rel > worst) worst = rel;
                    if (!(rel < opt->tol)) ok = 0;
                }
                if (trace_maxrel && k < trace_len) trace_maxrel[k] = worst;
                if (ok) {
                    if (retire_k) retire_k[lo] = k;
                    inew = lo + 1;
                }
            } else if (trace_maxrel && k < trace_len) {
                trace_maxrel[k] = INFINITY;
            }
        }
        i = inew;
        /* d_{k-1} <- d_k */
        for (int q = qb; q < qe; ++q) {
            int v = order[q];
            dold[v] = dnew[v];
        }
    }
    if (i < rho) rc = PTPO_ENOCONV;
    int reach = 0;
    for (int v = 0; v < n; ++v) {
        dist[v] = dold[v];
        if (isfinite(dold[v])) reach++;
    }
    if (label) {
        const int lrc = label_from_map(n, &inc, F, X, m, S, dist, label, NULL);
        if (lrc) rc = lrc;
    }
    if (st) {
        st->iterations = k;
        st->rho = rho;
        st->reachable = reach;
        st->updates = U;
    }
out:
    free(level); free(order); free(offsets);
    free(dold); free(dnew);
    free_incidence(&inc);
    return rc;
}

int ptpo_run(int n, int nf, const double *X, const int *F, int m, const int *S,
             const ptpo_options *opt, double *dist, int *label, ptpo_stats *st,
             int *retire_k, int *trace_lo, double *trace_maxrel, int trace_len)
{
    return run_core(n, nf, X, F, m, S, opt, NULL, dist, label, st, retire_k, trace_lo,
                    trace_maxrel, trace_len, NULL, NULL);
}

/* Replay: the same iteration, but the band's lower end follows a given
 * schedule (retire_in[rho], K) instead of the relative-change test, so that
 * the arithmetic can be compared under another run's schedule.  Returns
 * PTPO_EINVAL when the schedule is not one the iteration could produce. */
int ptpo_run_replay(int n, int nf, const double *X, const int *F, int m, const int *S,
                    const ptpo_options *opt, const int *retire_in, int K, double *dist,
                    int *label, ptpo_stats *st, int *retire_k)
{
    if (!retire_in) return PTPO_EINVAL;
    run_mode md = {NULL, 0, retire_in, K};
    return run_core(n, nf, X, F, m, S, opt, &md, dist, label, st, retire_k, NULL, NULL, 0,
                    NULL, NULL);
}

/* upper[n]: the warm start in the caller's vertex order.  certify: 1 to
 * certify it first, 0 to take it as a supersolution.  rejected_out (may be
 * NULL): number of bounds the certification withdrew; certified[n] (may be
 * NULL): the start after certification, caller order. */
int ptpo_run_warm(int n, int nf, const double *X, const int *F, int m, const int *S,
                  const ptpo_options *opt, const double *upper, int certify, double *dist,
                  int *label, ptpo_stats *st, int *retire_k, int *rejected_out, double *certified)
{
    if (!upper) return PTPO_EINVAL;
    run_mode md = {upper, certify ? 1 : 0, NULL, 0};
    return run_core(n, nf, X, F, m, S, opt, &md, dist, label, st, retire_k, NULL, NULL, 0,
                    rejected_out, certified);
}

/* ------------------------------------------------------------------ */
/* fixed point d* = min(d*, U(d*)), d*(S) = 0, by Jacobi from +inf       */
/* ------------------------------------------------------------------ */

int ptpo_fixed_point(int n, int nf, const double *X, const int *F, int m, const int *S,
                     int max_sweeps, double *dist, int *label, int *sweeps_out)
{
    int rc = check_mesh(n, nf, F, m, S);
    if (rc) return rc;
    incidence inc;
    rc = build_incidence(n, nf, F, &inc);
    if (rc) return rc;
    double *dold = (double *)malloc(sizeof(double) * (size_t)n);
    unsigned char *is_src = (unsigned char *)calloc((size_t)n, 1);
    if (!dold || !is_src) {
        rc = PTPO_ENOMEM;
        goto out;
    }
    for (int v = 0; v < n; ++v) dist[v] = INFINITY;
    for (int a = 0; a < m; ++a) {
        dist[S[a]] = 0.0;
        is_src[S[a]] = 1;
    }
    int sweeps = 0;
    rc = PTPO_ENOCONV;
    while (sweeps < max_sweeps) {
        sweeps++;
        memcpy(dold, dist, sizeof(double) * (size_t)n);
        int changed = 0;
        for (int v = 0; v < n; ++v) {
            if (is_src[v]) continue;
            const double bu = best_update(v, &inc, F, X, dold, NULL);
            if (bu < dold[v]) {
                dist[v] = bu;
                changed = 1;
            }
        }
        if (!changed) {
            rc = PTPO_OK;
            break;
        }
    }
    if (sweeps_out) *sweeps_out = sweeps;
    if (label) {
        const int lrc = label_from_map(n, &inc, F, X, m, S, dist, label, NULL);
        if (lrc) rc = lrc;
    }
out:
    free(dold); free(is_src);
    free_incidence(&inc);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Fast Marching (Sec. 3.2): accept the smallest trial vertex, then     */
/* update every triangle around each of its neighbours from accepted    */
/* values only.                                                        */
/* ------------------------------------------------------------------ */

typedef struct { double key; int v; } heap_item;

static void heap_push(heap_item *h, int *size, double key, int v)
{
    int i = (*size)++;
    h[i].key = key;
    h[i].v = v;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (h[p].key <= h[i].key) break;
        heap_item t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static heap_item heap_pop(heap_item *h, int *size)
{
    heap_item top = h[0];
    h[0] = h[--(*size)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, s = i;
        if (l < *size && h[l].key < h[s].key) s = l;
        if (r < *size && h[r].key < h[s].key) s = r;
        if (s == i) break;
        heap_item t = h[s]; h[s] = h[i]; h[i] = t;
        i = s;
    }
    return top;
}

int ptpo_fast_marching(int n, int nf, const double *X, const int *F, int m, const int *S,
                       double *dist)
{
    int rc = check_mesh(n, nf, F, m, S);
    if (rc) return rc;
    incidence inc;
    rc = build_incidence(n, nf, F, &inc);
    if (rc) return rc;
    size_t cap = (size_t)n + 6 * (size_t)nf + 16;
    heap_item *h = (heap_item *)malloc(sizeof(heap_item) * cap);
    unsigned char *acc = (unsigned char *)calloc((size_t)n, 1);
    if (!h || !acc) {
        rc = PTPO_ENOMEM;
        goto out;
    }
    for (int v = 0; v < n; ++v) dist[v] = INFINITY;
    int size = 0;
    for (int a = 0; a < m; ++a) {
        dist[S[a]] = 0.0;
        heap_push(h, &size, 0.0, S[a]);
    }
    while (size > 0) {
        heap_item it = heap_pop(h, &size);
        int v = it.v;
        if (acc[v] || it.key > dist[v]) continue;
        acc[v] = 1;
        for (int e = inc.start[v]; e < inc.start[v + 1]; ++e) {
            const int *f = F + 3 * inc.face[e];
            for (int c = 0; c < 3; ++c) {
                int u = f[c];
                if (acc[u]) continue;
                const double bu = best_update(u, &inc, F, X, dist, acc);
                if (bu < dist[u]) {
                    dist[u] = bu;
                    if ((size_t)size >= cap) { rc = PTPO_ENOMEM; goto out; }
                    heap_push(h, &size, bu, u);
                }
            }
        }
    }
out:
    free(h); free(acc);
    free_incidence(&inc);
    return rc;
}
