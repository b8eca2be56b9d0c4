/*
 * CPU ORACLE for point-to-plane ICP and its neighbour search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU library.
 *
 * It is written to be checked by eye against the method, not to be fast:
 *   - k nearest neighbours: the definition (Section 3, "Core operations":
 *     k-NN queries), i.e. every reference point is ranked by a float32
 *     squared distance and the k smallest (distance, index) pairs are kept,
 *     ties going to the lower index.  A textbook kd-tree (Friedman, Bentley
 *     and Finkel 1977) is offered as an accelerator with the same result;
 *     the tests hold it bit-equal to the brute-force definition.
 *   - normals and curvature: principal component analysis of each point's k
 *     nearest neighbours (Section 3, "Core operations": normal and curvature
 *     estimation, PCA), the eigenvector of the smallest eigenvalue of the
 *     neighbourhood covariance, oriented toward a viewpoint (Section 4, the
 *     normal-estimation benchmark enforces viewpoint-consistent normals).
 *     Eigen-decomposition by cyclic Jacobi rotations (textbook).
 *   - point-to-plane ICP: the loop of Section 3 ("Iterative geometric
 *     registration": alternate correspondence search and transform
 *     estimation) with nearest-neighbour correspondences and a rejection
 *     distance, as in the Section 4 ICP benchmark, and the linear
 *     least-squares point-to-plane estimator the paper cites (Low 2004):
 *     small-angle linearisation of the rotation, 6x6 normal equations solved
 *     by Cholesky, exact rotation Rz(gamma) Ry(beta) Rx(alpha) applied on
 *     the left of the running pose.
 * Everything is float64 (the paper benchmarks in double precision,
 * Section 4) except the kNN ranking key, which is defined in float32 so that
 * a float32 implementation can reproduce neighbour lists bit for bit:
 *     dx = r.x - q.x, dy = ..., dz = ...   (float32 subtractions)
 *     key = fmaf(dz, dz, fmaf(dy, dy, dx * dx))
 * Build with -ffp-contract=off so that no other contraction happens.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* float32 ranking key of the k-NN definition                                */
/* ------------------------------------------------------------------------ */

static float knn_key(const float *r, const float *q)
{
    float dx = r[0] - q[0];
    float dy = r[1] - q[1];
    float dz = r[2] - q[2];
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* (key, index) lexicographic order */
static int pair_less(float ka, int64_t ia, float kb, int64_t ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

/* keep the k best pairs in ascending order; returns nothing */
static void topk_insert(float *kd, int32_t *ki, int k, int *filled, float key, int32_t idx)
{
    int n = *filled;
    if (n == k) {
        if (!pair_less(key, idx, kd[k - 1], ki[k - 1])) return;
        n = k - 1;               /* drop the current worst */
    }
    int pos = n;
    while (pos > 0 && pair_less(key, idx, kd[pos - 1], ki[pos - 1])) {
        kd[pos] = kd[pos - 1];
        ki[pos] = ki[pos - 1];
        pos--;
    }
    kd[pos] = key;
    ki[pos] = idx;
    if (*filled < k) (*filled)++;
}

/* ------------------------------------------------------------------------ */
/* brute-force k-NN: the definition                                          */
/* ------------------------------------------------------------------------ */

int oracle_knn_brute(const float *ref, int64_t n_ref, const float *qry, int64_t n_qry,
                     int k, int32_t *out_idx, float *out_d2)
{
    if (k < 1 || k > n_ref) return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_qry; i++) {
        float kd[64];
        int32_t ki[64];
        int filled = 0;
        for (int64_t j = 0; j < n_ref; j++)
            topk_insert(kd, ki, k, &filled, knn_key(ref + 3 * j, qry + 3 * i), (int32_t)j);
        for (int s = 0; s < k; s++) {
            out_idx[i * k + s] = ki[s];
            if (out_d2) out_d2[i * k + s] = kd[s];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* textbook kd-tree                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t lo, hi;       /* range of perm[] owned by the node              */
    int32_t left, right;  /* children, -1 for a leaf                        */
    int32_t axis;
    float split;          /* left: coord <= split, right: coord >= split    */
} kd_node;

typedef struct {
    const float *pts;
    int64_t n;
    int32_t *perm;
    kd_node *nodes;
    int64_t n_nodes, cap;
} kd_tree;

enum { KD_LEAF = 8 };

static float kd_coord(const kd_tree *t, int32_t p, int axis)
{
    return t->pts[3 * (int64_t)p + axis];
}

/* Quickselect (three-way partition, median-of-three pivot): afterwards
   perm[kth] holds the kth smallest coordinate of perm[lo, hi) on ``axis``,
   everything before it is <= and everything after it is >=. */
static void kd_select(kd_tree *t, int32_t lo, int32_t hi, int32_t kth, int axis)
{
    int32_t *pm = t->perm;
    while (hi - lo > 1) {
        float a = kd_coord(t, pm[lo], axis), b = kd_coord(t, pm[lo + (hi - lo) / 2], axis);
        float c = kd_coord(t, pm[hi - 1], axis);
        float pv = (a < b) ? ((b < c) ? b : ((a < c) ? c : a)) : ((a < c) ? a : ((b < c) ? c : b));
        int32_t lt = lo, i = lo, gt = hi;
        while (i < gt) {
            float v = kd_coord(t, pm[i], axis);
            if (v < pv) { int32_t tmp = pm[lt]; pm[lt] = pm[i]; pm[i] = tmp; lt++; i++; }
            else if (v > pv) { gt--; int32_t tmp = pm[gt]; pm[gt] = pm[i]; pm[i] = tmp; }
            else i++;
        }
        if (kth < lt) hi = lt;
        else if (kth >= gt) lo = gt;
        else return;
    }
}

static int32_t kd_build_rec(kd_tree *t, int32_t lo, int32_t hi)
{
    int32_t id = (int32_t)t->n_nodes++;
    kd_node *nd = &t->nodes[id];
    nd->lo = lo; nd->hi = hi; nd->left = nd->right = -1; nd->axis = 0; nd->split = 0.f;
    if (hi - lo <= KD_LEAF) return id;
    /* split on the axis of widest spread, at the median */
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = lo; i < hi; i++)
        for (int a = 0; a < 3; a++) {
            float v = t->pts[3 * (int64_t)t->perm[i] + a];
            if (v < mn[a]) mn[a] = v;
            if (v > mx[a]) mx[a] = v;
        }
    int axis = 0;
    for (int a = 1; a < 3; a++)
        if (mx[a] - mn[a] > mx[axis] - mn[axis]) axis = a;
    if (!(mx[axis] > mn[axis])) return id;       /* all points coincide: leaf */
    int32_t mid = lo + (hi - lo) / 2;
    kd_select(t, lo, hi, mid, axis);
    float split = kd_coord(t, t->perm[mid], axis);
    /* left holds perm[lo, mid) whose coords are <= split, right holds
       perm[mid, hi) whose coords are >= split (the selection guarantees it) */
    t->nodes[id].axis = axis;
    t->nodes[id].split = split;
    int32_t l = kd_build_rec(t, lo, mid);
    int32_t r = kd_build_rec(t, mid, hi);
    t->nodes[id].left = l;
    t->nodes[id].right = r;
    return id;
}

static int kd_build(kd_tree *t, const float *pts, int64_t n)
{
    t->pts = pts;
    t->n = n;
    t->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    t->cap = 2 * (n / (KD_LEAF / 2) + 2);
    t->nodes = (kd_node *)malloc(sizeof(kd_node) * (size_t)t->cap);
    t->n_nodes = 0;
    if (!t->perm || !t->nodes) return 1;
    for (int64_t i = 0; i < n; i++) t->perm[i] = (int32_t)i;
    if (n > 0) kd_build_rec(t, 0, (int32_t)n);
    return 0;
}

static void kd_free(kd_tree *t)
{
    free(t->perm);
    free(t->nodes);
}

/* k-NN under the float32 key.  A subtree beyond a splitting plane at axis
   distance a holds only points whose float32 key is at least
   a^2 * (1 - 6e-7) (five roundings of relative size 2^-24 at most), so it
   is skipped only when a^2 * (1 - 1e-6) > current k-th key. */
static void kd_knn_rec(const kd_tree *t, int32_t id, const float *q, int k,
                       float *kd, int32_t *ki, int *filled)
{
    const kd_node *nd = &t->nodes[id];
    if (nd->left < 0) {
        for (int32_t i = nd->lo; i < nd->hi; i++) {
            int32_t j = t->perm[i];
            topk_insert(kd, ki, k, filled, knn_key(t->pts + 3 * (int64_t)j, q), j);
        }
        return;
    }
    double diff = (double)q[nd->axis] - (double)nd->split;
    int32_t near = diff <= 0 ? nd->left : nd->right;
    int32_t far = diff <= 0 ? nd->right : nd->left;
    kd_knn_rec(t, near, q, k, kd, ki, filled);
    if (*filled < k || diff * diff * (1.0 - 1e-6) <= (double)kd[k - 1])
        kd_knn_rec(t, far, q, k, kd, ki, filled);
}

int oracle_knn_kdtree(const float *ref, int64_t n_ref, const float *qry, int64_t n_qry,
                      int k, int32_t *out_idx, float *out_d2)
{
    if (k < 1 || k > n_ref || k > 64) return 1;
    kd_tree t;
    if (kd_build(&t, ref, n_ref)) { kd_free(&t); return 2; }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n_qry; i++) {
        float kd[64];
        int32_t ki[64];
        int filled = 0;
        kd_knn_rec(&t, 0, qry + 3 * i, k, kd, ki, &filled);
        for (int s = 0; s < k; s++) {
            out_idx[i * k + s] = ki[s];
            if (out_d2) out_d2[i * k + s] = kd[s];
        }
    }
    kd_free(&t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3x3 symmetric eigen-decomposition by cyclic Jacobi rotations              */
/* ------------------------------------------------------------------------ */

/* a: symmetric 3x3 (row-major), destroyed.  On return w[0] <= w[1] <= w[2]
   and column c of v (v[r*3+c]) is the unit eigenvector of w[c]. */
void oracle_jacobi3(double a[9], double w[3], double v[9])
{
    for (int i = 0; i < 9; i++) v[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; sweep++) {
        double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        if (off == 0.0) break;
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                double apq = a[p * 3 + q];
                if (apq == 0.0) continue;
                double app = a[p * 3 + p], aqq = a[q * 3 + q];
                double theta = (aqq - app) / (2.0 * apq);
                double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
                /* A <- J^T A J with J the rotation in the (p,q) plane */
                for (int r = 0; r < 3; r++) {
                    double arp = a[r * 3 + p], arq = a[r * 3 + q];
                    a[r * 3 + p] = c * arp - s * arq;
                    a[r * 3 + q] = s * arp + c * arq;
                }
                for (int r = 0; r < 3; r++) {
                    double apr = a[p * 3 + r], aqr = a[q * 3 + r];
                    a[p * 3 + r] = c * apr - s * aqr;
                    a[q * 3 + r] = s * apr + c * aqr;
                }
                a[p * 3 + q] = a[q * 3 + p] = 0.0;
                for (int r = 0; r < 3; r++) {
                    double vrp = v[r * 3 + p], vrq = v[r * 3 + q];
                    v[r * 3 + p] = c * vrp - s * vrq;
                    v[r * 3 + q] = s * vrp + c * vrq;
                }
            }
        /* stop once the off-diagonal part is negligible next to the diagonal */
        double diag = fabs(a[0]) + fabs(a[4]) + fabs(a[8]);
        double off2 = fabs(a[1]) + fabs(a[2]) + fabs(a[5]);
        if (off2 <= 1e-300 || off2 < 1e-18 * diag) {
            a[1] = a[2] = a[5] = a[3] = a[6] = a[7] = 0.0;
            break;
        }
    }
    double d[3] = {a[0], a[4], a[8]};
    int ord[3] = {0, 1, 2};
    for (int i = 0; i < 3; i++)
        for (int j = i + 1; j < 3; j++)
            if (d[ord[j]] < d[ord[i]]) { int tmp = ord[i]; ord[i] = ord[j]; ord[j] = tmp; }
    double vs[9];
    memcpy(vs, v, sizeof vs);
    for (int c = 0; c < 3; c++) {
        w[c] = d[ord[c]];
        for (int r = 0; r < 3; r++) v[r * 3 + c] = vs[r * 3 + ord[c]];
    }
}

/* ------------------------------------------------------------------------ */
/* normals and curvature                                                     */
/* ------------------------------------------------------------------------ */

/* Neighbourhoods N(i) = the k nearest points of i in its own cloud (i itself
   included).  Covariance C = (1/k) sum (x - mu)(x - mu)^T in float64.  The
   normal is the unit eigenvector of the smallest eigenvalue, flipped so that
   n . (viewpoint - p) >= 0; when that product is exactly zero, the first
   nonzero component is made positive.  Curvature (surface variation) is
   l0 / (l0 + l1 + l2), 0 when the trace is 0.  A neighbourhood whose
   covariance is all zeros has normal (0,0,0).
   out_evals (nullable) receives the ascending eigenvalues. */
int oracle_normals(const float *xyz, int64_t n, int k, const double viewpoint[3],
                   int use_kdtree, double *out_normals, double *out_curv, double *out_evals)
{
    if (k < 1 || k > n || k > 64) return 1;
    int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)k);
    if (!nbr) return 2;
    int rc = use_kdtree ? oracle_knn_kdtree(xyz, n, xyz, n, k, nbr, NULL)
                        : oracle_knn_brute(xyz, n, xyz, n, k, nbr, NULL);
    if (rc) { free(nbr); return rc; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        /* covariance is translation invariant: use offsets from p_i, which
           are exact in float64 (differences of float32 values), so a
           neighbourhood of coincident points gives exactly zero */
        double mu[3] = {0, 0, 0};
        for (int s = 0; s < k; s++)
            for (int a = 0; a < 3; a++)
                mu[a] += (double)xyz[3 * (int64_t)nbr[i * k + s] + a] - (double)xyz[3 * i + a];
        for (int a = 0; a < 3; a++) mu[a] /= k;
        double c[9] = {0};
        for (int s = 0; s < k; s++) {
            double e[3];
            for (int a = 0; a < 3; a++)
                e[a] = ((double)xyz[3 * (int64_t)nbr[i * k + s] + a] - (double)xyz[3 * i + a]) - mu[a];
            for (int r = 0; r < 3; r++)
                for (int cc = 0; cc < 3; cc++) c[r * 3 + cc] += e[r] * e[cc];
        }
        for (int r = 0; r < 9; r++) c[r] /= k;
        double w[3], v[9];
        int zero = 1;
        for (int r = 0; r < 9; r++) if (c[r] != 0.0) zero = 0;
        double nn[3] = {0, 0, 0};
        if (zero) {
            w[0] = w[1] = w[2] = 0.0;
        } else {
            oracle_jacobi3(c, w, v);
            for (int a = 0; a < 3; a++) nn[a] = v[a * 3 + 0];
            double nrm = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
            for (int a = 0; a < 3; a++) nn[a] /= nrm;
            double dot = 0;
            for (int a = 0; a < 3; a++) dot += nn[a] * (viewpoint[a] - (double)xyz[3 * i + a]);
            int flip = dot < 0;
            if (dot == 0) {
                for (int a = 0; a < 3; a++)
                    if (nn[a] != 0) { flip = nn[a] < 0; break; }
            }
            if (flip) for (int a = 0; a < 3; a++) nn[a] = -nn[a];
        }
        for (int a = 0; a < 3; a++) out_normals[3 * i + a] = nn[a];
        double tr = w[0] + w[1] + w[2];
        if (out_curv) out_curv[i] = tr > 0 ? w[0] / tr : 0.0;
        if (out_evals) for (int a = 0; a < 3; a++) out_evals[3 * i + a] = w[a];
    }
    free(nbr);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* point-to-plane ICP                                                        */
/* ------------------------------------------------------------------------ */

/* Nearest target point of p within the rejection ball, in float64: the j
   with the smallest |p - q_j|^2 among those with |p - q_j|^2 <= *best on
   entry (d_max^2), ties to the lower j; *bj stays -1 when the ball is empty.
   This is the nearest neighbour followed by the rejection test, with the
   search confined to where an accepted answer can lie.  The far side of a
   splitting plane at distance a is skipped only when a^2 (1 - 1e-12) > best,
   so no point that could tie is ever skipped. */
static int nn64_better(double d2, int32_t j, double best, int32_t bj)
{
    return d2 < best || (d2 == best && (bj < 0 || j < bj));
}

static void kd_nn64_rec(const kd_tree *t, int32_t id, const double p[3], double *best, int32_t *bj)
{
    const kd_node *nd = &t->nodes[id];
    if (nd->left < 0) {
        for (int32_t i = nd->lo; i < nd->hi; i++) {
            int32_t j = t->perm[i];
            const float *q = t->pts + 3 * (int64_t)j;
            double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (nn64_better(d2, j, *best, *bj)) { *best = d2; *bj = j; }
        }
        return;
    }
    double diff = p[nd->axis] - (double)nd->split;
    int32_t near = diff <= 0 ? nd->left : nd->right;
    int32_t far = diff <= 0 ? nd->right : nd->left;
    kd_nn64_rec(t, near, p, best, bj);
    if (diff * diff * (1.0 - 1e-12) <= *best) kd_nn64_rec(t, far, p, best, bj);
}

static void nn64_brute(const float *tgt, int64_t nt, const double p[3], double *best, int32_t *bj)
{
    for (int64_t j = 0; j < nt; j++) {
        const float *q = tgt + 3 * j;
        double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        double d2 = dx * dx + dy * dy + dz * dz;
        if (nn64_better(d2, (int32_t)j, *best, *bj)) { *best = d2; *bj = (int32_t)j; }
    }
}

/* The linearised point-to-plane system at pose T (row-major 4x4) for the
   correspondences found at that pose:
     p'_i = R p_i + t,   j(i) = nearest target point,
     inlier iff |p'_i - q_j|^2 <= d_max^2 and n_j != 0,
     r_i = (p'_i - q_j) . n_j,   J_i = [p'_i x n_j, n_j],
     A = sum J_i^T J_i,  b = sum J_i^T r_i,  also sum r_i^2 and the count.
   Sums run over source points in index order (deterministic).
   corr (nullable) receives j(i) or -1 for rejected points. */
static int p2plane_system(const float *src, int64_t ns, const float *tgt, const float *nrm, int64_t nt,
                          const kd_tree *tree, const double T[16], double d_max,
                          double A[36], double b[6], int64_t *inliers, double *sum_r2, int32_t *corr)
{
    double *rows = (double *)malloc(sizeof(double) * 7 * (size_t)(ns > 0 ? ns : 1));
    int32_t *jj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ns > 0 ? ns : 1));
    if (!rows || !jj) { free(rows); free(jj); return 2; }
    double dmax2 = d_max * d_max;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < ns; i++) {
        const float *ps = src + 3 * i;
        double p[3];
        for (int a = 0; a < 3; a++)
            p[a] = T[a * 4 + 0] * ps[0] + T[a * 4 + 1] * ps[1] + T[a * 4 + 2] * ps[2] + T[a * 4 + 3];
        double best = dmax2;
        int32_t bj = -1;
        if (tree) kd_nn64_rec(tree, 0, p, &best, &bj);
        else nn64_brute(tgt, nt, p, &best, &bj);
        int ok = bj >= 0;
        const float *q = tgt + 3 * (int64_t)(ok ? bj : 0);
        const float *nq = nrm + 3 * (int64_t)(ok ? bj : 0);
        ok = ok && (nq[0] != 0.f || nq[1] != 0.f || nq[2] != 0.f);
        jj[i] = ok ? bj : -1;
        if (ok) {
            double n[3] = {nq[0], nq[1], nq[2]};
            double r = (p[0] - q[0]) * n[0] + (p[1] - q[1]) * n[1] + (p[2] - q[2]) * n[2];
            double *J = rows + 7 * i;
            J[0] = p[1] * n[2] - p[2] * n[1];
            J[1] = p[2] * n[0] - p[0] * n[2];
            J[2] = p[0] * n[1] - p[1] * n[0];
            J[3] = n[0]; J[4] = n[1]; J[5] = n[2];
            J[6] = r;
        }
    }
    for (int i = 0; i < 36; i++) A[i] = 0;
    for (int i = 0; i < 6; i++) b[i] = 0;
    int64_t cnt = 0;
    double s2 = 0;
    for (int64_t i = 0; i < ns; i++) {
        if (corr) corr[i] = jj[i];
        if (jj[i] < 0) continue;
        const double *J = rows + 7 * i;
        for (int r = 0; r < 6; r++) {
            for (int c = 0; c < 6; c++) A[r * 6 + c] += J[r] * J[c];
            b[r] += J[r] * J[6];
        }
        s2 += J[6] * J[6];
        cnt++;
    }
    free(rows);
    free(jj);
    *inliers = cnt;
    *sum_r2 = s2;
    return 0;
}

int oracle_p2plane_system(const float *src, int64_t ns, const float *tgt, const float *nrm, int64_t nt,
                          const double T[16], double d_max, int use_kdtree,
                          double A[36], double b[6], int64_t *inliers, double *sum_r2, int32_t *corr)
{
    kd_tree t;
    int rc;
    if (use_kdtree) {
        if (kd_build(&t, tgt, nt)) { kd_free(&t); return 2; }
        rc = p2plane_system(src, ns, tgt, nrm, nt, &t, T, d_max, A, b, inliers, sum_r2, corr);
        kd_free(&t);
    } else {
        rc = p2plane_system(src, ns, tgt, nrm, nt, NULL, T, d_max, A, b, inliers, sum_r2, corr);
    }
    return rc;
}

/* Cholesky A = L L^T of a 6x6 SPD matrix.  Fails (returns 1) when a pivot is
   not above 1e-14 times the largest diagonal entry. */
int oracle_cholesky6(const double A[36], double L[36])
{
    double dmax = 0;
    for (int i = 0; i < 6; i++) if (A[i * 7] > dmax) dmax = A[i * 7];
    for (int i = 0; i < 36; i++) L[i] = 0;
    for (int j = 0; j < 6; j++) {
        double s = A[j * 6 + j];
        for (int k = 0; k < j; k++) s -= L[j * 6 + k] * L[j * 6 + k];
        if (!(s > 1e-14 * dmax)) return 1;
        L[j * 6 + j] = sqrt(s);
        for (int i = j + 1; i < 6; i++) {
            double t = A[i * 6 + j];
            for (int k = 0; k < j; k++) t -= L[i * 6 + k] * L[j * 6 + k];
            L[i * 6 + j] = t / L[j * 6 + j];
        }
    }
    return 0;
}

/* x = -A^{-1} b via the Cholesky factor */
static void chol_solve6(const double L[36], const double b[6], double x[6])
{
    double y[6];
    for (int i = 0; i < 6; i++) {
        double s = -b[i];
        for (int k = 0; k < i; k++) s -= L[i * 6 + k] * y[k];
        y[i] = s / L[i * 6 + i];
    }
    for (int i = 5; i >= 0; i--) {
        double s = y[i];
        for (int k = i + 1; k < 6; k++) s -= L[k * 6 + i] * x[k];
        x[i] = s / L[i * 6 + i];
    }
}

/* R = Rz(gamma) Ry(beta) Rx(alpha), row-major 3x3 */
void oracle_euler_zyx(double alpha, double beta, double gamma, double R[9])
{
    double ca = cos(alpha), sa = sin(alpha), cb = cos(beta), sb = sin(beta);
    double cg = cos(gamma), sg = sin(gamma);
    double Rx[9] = {1, 0, 0, 0, ca, -sa, 0, sa, ca};
    double Ry[9] = {cb, 0, sb, 0, 1, 0, -sb, 0, cb};
    double Rz[9] = {cg, -sg, 0, sg, cg, 0, 0, 0, 1};
    double Ryx[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += Ry[r * 3 + k] * Rx[k * 3 + c];
            Ryx[r * 3 + c] = s;
        }
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += Rz[r * 3 + k] * Ryx[k * 3 + c];
            R[r * 3 + c] = s;
        }
}

enum { ICP_CONVERGED = 0, ICP_MAXITER = 1, ICP_DEGENERATE = 2, ICP_NO_INLIERS = 3 };

/* Point-to-plane ICP.
   T_init (nullable: identity) and T_out are row-major 4x4 maps source ->
   target.  Each iteration: correspondences at the current pose, system,
   x = -A^{-1} b = (alpha, beta, gamma, tau), dR = Rz Ry Rx,
   R <- dR R, t <- dR t + tau.  Stops early on a degenerate system (fewer than
   6 inliers or a failed Cholesky; the pose is kept) or, when conv_tol > 0,
   once max |x_i| < conv_tol.  A final correspondence pass at the returned
   pose gives the inlier count and rms = sqrt(sum r^2 / inliers).
   stats_i: [status, iterations_run], stats_i64: [inliers], stats_d: [rms].
   x_hist (nullable): max_iters*6 increments, as they were applied. */
int oracle_icp(const float *src, int64_t ns, const float *tgt, const float *nrm, int64_t nt,
               const double *T_init, double d_max, int max_iters, double conv_tol, int use_kdtree,
               double T_out[16], int32_t stats_i[2], int64_t stats_i64[1], double stats_d[1],
               double *x_hist)
{
    double T[16];
    for (int i = 0; i < 16; i++) T[i] = T_init ? T_init[i] : ((i % 5 == 0) ? 1.0 : 0.0);
    kd_tree tree;
    int have_tree = 0;
    if (use_kdtree) {
        if (kd_build(&tree, tgt, nt)) { kd_free(&tree); return 2; }
        have_tree = 1;
    }
    int status = ICP_MAXITER, it = 0;
    double A[36], b[6], L[36], x[6];
    int64_t inl;
    double s2;
    for (it = 0; it < max_iters; it++) {
        int rc = p2plane_system(src, ns, tgt, nrm, nt, have_tree ? &tree : NULL, T, d_max, A, b, &inl, &s2, NULL);
        if (rc) { if (have_tree) kd_free(&tree); return rc; }
        if (inl == 0) { status = ICP_NO_INLIERS; break; }
        if (inl < 6 || oracle_cholesky6(A, L)) { status = ICP_DEGENERATE; break; }
        chol_solve6(L, b, x);
        if (x_hist) for (int a = 0; a < 6; a++) x_hist[it * 6 + a] = x[a];
        double dR[9];
        oracle_euler_zyx(x[0], x[1], x[2], dR);
        double R[9], t[3], Rn[9], tn[3];
        for (int r = 0; r < 3; r++) {
            for (int c = 0; c < 3; c++) R[r * 3 + c] = T[r * 4 + c];
            t[r] = T[r * 4 + 3];
        }
        for (int r = 0; r < 3; r++) {
            for (int c = 0; c < 3; c++) {
                double s = 0;
                for (int k = 0; k < 3; k++) s += dR[r * 3 + k] * R[k * 3 + c];
                Rn[r * 3 + c] = s;
            }
            double s = 0;
            for (int k = 0; k < 3; k++) s += dR[r * 3 + k] * t[k];
            tn[r] = s + x[3 + r];
        }
        for (int r = 0; r < 3; r++) {
            for (int c = 0; c < 3; c++) T[r * 4 + c] = Rn[r * 3 + c];
            T[r * 4 + 3] = tn[r];
        }
        T[12] = T[13] = T[14] = 0.0;
        T[15] = 1.0;
        if (conv_tol > 0) {
            double m = 0;
            for (int a = 0; a < 6; a++) if (fabs(x[a]) > m) m = fabs(x[a]);
            if (m < conv_tol) { status = ICP_CONVERGED; it++; break; }
        }
    }
    int rc = p2plane_system(src, ns, tgt, nrm, nt, have_tree ? &tree : NULL, T, d_max, A, b, &inl, &s2, NULL);
    if (have_tree) kd_free(&tree);
    if (rc) return rc;
    memcpy(T_out, T, sizeof T);
    stats_i[0] = status;
    stats_i[1] = it;
    stats_i64[0] = inl;
    stats_d[0] = inl > 0 ? sqrt(s2 / (double)inl) : 0.0;
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* point-to-point rigid fit (closed form) and the metric variants of ICP     */
/* (Section 3, "Iterative geometric registration": optimizers for the       */
/* point-to-point and point-to-plane metrics and weighted combinations)      */
/* ------------------------------------------------------------------------ */

/* Singular value decomposition of a 3x3 matrix by one-sided Jacobi
   rotations (Hestenes 1958): the columns of W = A V are made orthogonal by
   plane rotations applied on the right.  Then s[c] = |W col c| in descending
   order, u col c = W col c / s[c] (completed to a right-handed orthonormal
   basis where s[c] is 0), a = u diag(s) v^T; u, v row-major. */
static void svd3(const double a[9], double u[9], double s[3], double v[9])
{
    double w[9];
    memcpy(w, a, sizeof w);
    for (int i = 0; i < 9; i++) v[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; sweep++) {
        int rotated = 0;
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                double alpha = 0, beta = 0, gamma = 0;
                for (int r = 0; r < 3; r++) {
                    alpha += w[r * 3 + p] * w[r * 3 + p];
                    beta += w[r * 3 + q] * w[r * 3 + q];
                    gamma += w[r * 3 + p] * w[r * 3 + q];
                }
                if (gamma == 0.0 || fabs(gamma) <= 1e-17 * sqrt(alpha * beta)) continue;
                rotated = 1;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
                for (int r = 0; r < 3; r++) {
                    double wp = w[r * 3 + p], wq = w[r * 3 + q];
                    w[r * 3 + p] = c * wp - sn * wq;
                    w[r * 3 + q] = sn * wp + c * wq;
                    double vp = v[r * 3 + p], vq = v[r * 3 + q];
                    v[r * 3 + p] = c * vp - sn * vq;
                    v[r * 3 + q] = sn * vp + c * vq;
                }
            }
        if (!rotated) break;
    }
    double nrm[3];
    for (int c = 0; c < 3; c++) nrm[c] = sqrt(w[c] * w[c] + w[3 + c] * w[3 + c] + w[6 + c] * w[6 + c]);
    int ord[3] = {0, 1, 2};
    for (int i = 0; i < 3; i++)
        for (int j = i + 1; j < 3; j++)
            if (nrm[ord[j]] > nrm[ord[i]]) { int tmp = ord[i]; ord[i] = ord[j]; ord[j] = tmp; }
    double vs[9];
    memcpy(vs, v, sizeof vs);
    for (int c = 0; c < 3; c++) {
        s[c] = nrm[ord[c]];
        for (int r = 0; r < 3; r++) {
            v[r * 3 + c] = vs[r * 3 + ord[c]];
            u[r * 3 + c] = s[c] > 0 ? w[r * 3 + ord[c]] / s[c] : 0.0;
        }
    }
    /* complete u where columns vanished: u2 = u0 x u1, and if needed
       u1 = any unit vector orthogonal to u0 */
    if (!(s[1] > 0)) {
        double a0 = fabs(u[0]), a1 = fabs(u[3]), a2 = fabs(u[6]);
        double e[3] = {0, 0, 0};
        e[(a0 <= a1 && a0 <= a2) ? 0 : (a1 <= a2 ? 1 : 2)] = 1.0;
        if (!(s[0] > 0)) { u[0] = 1; u[3] = 0; u[6] = 0; e[0] = 0; e[1] = 1; e[2] = 0; }
        double x[3] = {u[3] * e[2] - u[6] * e[1], u[6] * e[0] - u[0] * e[2], u[0] * e[1] - u[3] * e[0]};
        double xn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        for (int r = 0; r < 3; r++) u[r * 3 + 1] = x[r] / xn;
    }
    if (!(s[2] > 0)) {
        u[2] = u[3] * u[7] - u[6] * u[4];
        u[5] = u[6] * u[1] - u[0] * u[7];
        u[8] = u[0] * u[4] - u[3] * u[1];
    }
}

static double det3(const double m[9])
{
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
}

/* Least-squares rigid motion between corresponding point sets p_i -> q_i
   (Arun, Huang and Blostein 1987; the reflection case as in Umeyama 1991):
   H = sum (p - pbar)(q - qbar)^T = U S V^T, R = V diag(1, 1, d) U^T with
   d = sign det(V U^T), t = qbar - R pbar.  *top = s0 + s1 + d s2 and
   *gap = 2 (s1 + d s2) are the largest eigenvalue of Horn's (1987) 4x4
   quaternion matrix and its distance to the next one: the rotation is
   unique when the gap is positive.  Returns 1 when n < 1. */
int oracle_rigid_fit(const double *p, const double *q, int64_t n, double R[9], double t[3], double *top,
                     double *gap)
{
    if (n < 1) return 1;
    double pb[3] = {0, 0, 0}, qb[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            pb[a] += p[3 * i + a];
            qb[a] += q[3 * i + a];
        }
    for (int a = 0; a < 3; a++) {
        pb[a] /= (double)n;
        qb[a] /= (double)n;
    }
    double H[9] = {0};
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) H[a * 3 + b] += (p[3 * i + a] - pb[a]) * (q[3 * i + b] - qb[b]);
    double U[9], S[3], V[9], VUt[9];
    svd3(H, U, S, V);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += V[r * 3 + k] * U[c * 3 + k];
            VUt[r * 3 + c] = acc;
        }
    double d = det3(VUt) < 0 ? -1.0 : 1.0;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            R[r * 3 + c] = V[r * 3 + 0] * U[c * 3 + 0] + V[r * 3 + 1] * U[c * 3 + 1] + d * V[r * 3 + 2] * U[c * 3 + 2];
    for (int r = 0; r < 3; r++) t[r] = qb[r] - (R[r * 3] * pb[0] + R[r * 3 + 1] * pb[1] + R[r * 3 + 2] * pb[2]);
    if (top) *top = S[0] + S[1] + d * S[2];
    if (gap) *gap = 2.0 * (S[1] + d * S[2]);
    return 0;
}

/* transformed source point p' = R p + t (float64, from the float32 source) */
static void transform_point(const double T[16], const float *ps, double p[3])
{
    for (int a = 0; a < 3; a++) p[a] = T[a * 4 + 0] * ps[0] + T[a * 4 + 1] * ps[1] + T[a * 4 + 2] * ps[2] + T[a * 4 + 3];
}

/* nearest target point within d_max (index or -1), as in p2plane_system */
static int32_t nearest_within(const float *tgt, int64_t nt, const kd_tree *tree, const double p[3], double dmax2)
{
    double best = dmax2;
    int32_t bj = -1;
    if (tree) kd_nn64_rec(tree, 0, p, &best, &bj);
    else nn64_brute(tgt, nt, p, &best, &bj);
    return bj;
}

/* left-compose the increment (dR, dt) onto T */
static void compose_left(double T[16], const double dR[9], const double dt[3])
{
    double R[9], t[3];
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) R[r * 3 + c] = T[r * 4 + c];
        t[r] = T[r * 4 + 3];
    }
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += dR[r * 3 + k] * R[k * 3 + c];
            T[r * 4 + c] = acc;
        }
        double acc = 0;
        for (int k = 0; k < 3; k++) acc += dR[r * 3 + k] * t[k];
        T[r * 4 + 3] = acc + dt[r];
    }
    T[12] = T[13] = T[14] = 0.0;
    T[15] = 1.0;
}

/* Point-to-point ICP (Besl and McKay 1992).  Correspondences as in
   oracle_icp: the nearest target point by float64 distance, ties to the
   lower index, kept when |p' - q|^2 <= d_max^2 (normals are not used).
   Each iteration fits the closed-form rigid motion (oracle_rigid_fit) of the
   inlier pairs (p'_i, q_j(i)) and composes it on the left of the pose.
   Fewer than 3 inliers, or gap <= 1e-6 top: DEGENERATE (pose kept): a
   rotation fixed only to that relative level (nearly collinear pairs; float32
   inputs are collinear only to ~1e-8) is taken as undetermined.
   Converged when max(|dR - I|, |dt|) < conv_tol (conv_tol > 0).  The final
   pass gives the inliers and rms = sqrt(sum |p' - q|^2 / inliers). */
int oracle_icp_p2p(const float *src, int64_t ns, const float *tgt, int64_t nt, const double *T_init, double d_max,
                   int max_iters, double conv_tol, int use_kdtree, double T_out[16], int32_t stats_i[2],
                   int64_t stats_i64[1], double stats_d[1])
{
    double T[16];
    for (int i = 0; i < 16; i++) T[i] = T_init ? T_init[i] : ((i % 5 == 0) ? 1.0 : 0.0);
    kd_tree tree;
    int have_tree = 0;
    if (use_kdtree) {
        if (kd_build(&tree, tgt, nt)) { kd_free(&tree); return 2; }
        have_tree = 1;
    }
    double *P = (double *)malloc(sizeof(double) * 3 * (size_t)(ns > 0 ? ns : 1));
    double *Q = (double *)malloc(sizeof(double) * 3 * (size_t)(ns > 0 ? ns : 1));
    int32_t *jj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ns > 0 ? ns : 1));
    if (!P || !Q || !jj) { free(P); free(Q); free(jj); if (have_tree) kd_free(&tree); return 2; }
    double dmax2 = d_max * d_max;
    int status = ICP_MAXITER, it = 0;
    int64_t inl = 0;
    double s2 = 0;
    for (int pass = 0;; pass++) {
        int last = pass == max_iters;
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < ns; i++) {
            double p[3];
            transform_point(T, src + 3 * i, p);
            jj[i] = nearest_within(tgt, nt, have_tree ? &tree : NULL, p, dmax2);
            for (int a = 0; a < 3; a++) P[3 * i + a] = p[a];
        }
        inl = 0;
        s2 = 0;
        for (int64_t i = 0; i < ns; i++) {
            if (jj[i] < 0) continue;
            const float *q = tgt + 3 * (int64_t)jj[i];
            double e = 0;
            for (int a = 0; a < 3; a++) {
                double d = P[3 * i + a] - q[a];
                e += d * d;
                P[3 * inl + a] = P[3 * i + a];
                Q[3 * inl + a] = q[a];
            }
            s2 += e;
            inl++;
        }
        if (last) break;
        /* stopping keeps the pose, so this pass's sums are the final ones */
        if (inl == 0) { status = ICP_NO_INLIERS; break; }
        double dR[9], dt[3], top, gap;
        oracle_rigid_fit(P, Q, inl, dR, dt, &top, &gap);
        if (inl < 3 || !(gap > 1e-6 * top)) { status = ICP_DEGENERATE; break; }
        compose_left(T, dR, dt);
        it++;
        if (conv_tol > 0) {
            double m = 0;
            for (int r = 0; r < 3; r++) {
                for (int c = 0; c < 3; c++) m = fmax(m, fabs(dR[r * 3 + c] - (r == c ? 1.0 : 0.0)));
                m = fmax(m, fabs(dt[r]));
            }
            if (m < conv_tol) { status = ICP_CONVERGED; max_iters = pass + 1; }
        }
    }
    free(P);
    free(Q);
    free(jj);
    if (have_tree) kd_free(&tree);
    memcpy(T_out, T, sizeof T);
    stats_i[0] = status;
    stats_i[1] = it;
    stats_i64[0] = inl;
    stats_d[0] = inl > 0 ? sqrt(s2 / (double)inl) : 0.0;
    return 0;
}

/* The linearised system of the combined metric at pose T:
       w_plane * sum ((p' - q) . n)^2 + w_point * sum |p' - q|^2
   with the motion p' -> p' + omega x p' + tau, x = (omega, tau):
       J_plane = [p' x n, n]              (1 x 6), r_plane = (p' - q) . n
       J_point = [-[p']_x, I]             (3 x 6), r_point = p' - q
   where [a]_x b = a x b;  A = w_plane J_plane^T J_plane + w_point J_point^T J_point,
   b = w_plane J_plane^T r_plane + w_point J_point^T r_point, and the weighted
   residual sum w_plane r_plane^2 + w_point |r_point|^2.  Inliers as in
   p2plane_system (n != 0 required only when w_plane > 0); sums in source
   order. */
static int combined_system(const float *src, int64_t ns, const float *tgt, const float *nrm, int64_t nt,
                           const kd_tree *tree, const double T[16], double d_max, double w_point, double w_plane,
                           double A[36], double b[6], int64_t *inliers, double *sum_r2)
{
    double *rows = (double *)malloc(sizeof(double) * 43 * (size_t)(ns > 0 ? ns : 1));
    int32_t *jj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ns > 0 ? ns : 1));
    if (!rows || !jj) { free(rows); free(jj); return 2; }
    double dmax2 = d_max * d_max;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < ns; i++) {
        double p[3];
        transform_point(T, src + 3 * i, p);
        int32_t bj = nearest_within(tgt, nt, tree, p, dmax2);
        int ok = bj >= 0;
        const float *q = tgt + 3 * (int64_t)(ok ? bj : 0);
        if (ok && w_plane > 0) {
            const float *nq = nrm + 3 * (int64_t)bj;
            ok = nq[0] != 0.f || nq[1] != 0.f || nq[2] != 0.f;
        }
        jj[i] = ok ? bj : -1;
        if (!ok) continue;
        /* rows: [0..5] J_plane, [6] r_plane, [7..24] J_point (3 x 6),
           [25..27] r_point */
        double *R = rows + 43 * i;
        double n[3] = {0, 0, 0};
        if (w_plane > 0) {
            const float *nq = nrm + 3 * (int64_t)bj;
            n[0] = nq[0]; n[1] = nq[1]; n[2] = nq[2];
        }
        R[0] = p[1] * n[2] - p[2] * n[1];
        R[1] = p[2] * n[0] - p[0] * n[2];
        R[2] = p[0] * n[1] - p[1] * n[0];
        R[3] = n[0]; R[4] = n[1]; R[5] = n[2];
        R[6] = (p[0] - q[0]) * n[0] + (p[1] - q[1]) * n[1] + (p[2] - q[2]) * n[2];
        double skew[9] = {0, -p[2], p[1], p[2], 0, -p[0], -p[1], p[0], 0};   /* [p']_x */
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 6; c++)
                R[7 + r * 6 + c] = c < 3 ? -skew[r * 3 + c] : (c - 3 == r ? 1.0 : 0.0);
        for (int a = 0; a < 3; a++) R[25 + a] = p[a] - q[a];
    }
    for (int i = 0; i < 36; i++) A[i] = 0;
    for (int i = 0; i < 6; i++) b[i] = 0;
    int64_t cnt = 0;
    double s2 = 0;
    for (int64_t i = 0; i < ns; i++) {
        if (jj[i] < 0) continue;
        const double *R = rows + 43 * i;
        const double *Jpl = R, *Jpt = R + 7, *rpt = R + 25;
        for (int r = 0; r < 6; r++) {
            for (int c = 0; c < 6; c++) {
                double pt = 0;
                for (int k = 0; k < 3; k++) pt += Jpt[k * 6 + r] * Jpt[k * 6 + c];
                A[r * 6 + c] += w_plane * Jpl[r] * Jpl[c] + w_point * pt;
            }
            double bpt = 0;
            for (int k = 0; k < 3; k++) bpt += Jpt[k * 6 + r] * rpt[k];
            b[r] += w_plane * Jpl[r] * R[6] + w_point * bpt;
        }
        s2 += w_plane * R[6] * R[6] + w_point * (rpt[0] * rpt[0] + rpt[1] * rpt[1] + rpt[2] * rpt[2]);
        cnt++;
    }
    free(rows);
    free(jj);
    *inliers = cnt;
    *sum_r2 = s2;
    return 0;
}

int oracle_combined_system(const float *src, int64_t ns, const float *tgt, const float *nrm, int64_t nt,
                           const double T[16], double d_max, double w_point, double w_plane, double A[36],
                           double b[6], int64_t *inliers, double *sum_r2)
{
    return combined_system(src, ns, tgt, nrm, nt, NULL, T, d_max, w_point, w_plane, A, b, inliers, sum_r2);
}

/* ICP with the combined metric: as oracle_icp with combined_system in place
   of the point-to-plane system (Cholesky solve, Rz(gamma) Ry(beta) Rx(alpha)
   applied on the left, fewer than 6 inliers or a failed pivot:
   DEGENERATE); rms = sqrt(weighted residual sum / inliers). */
int oracle_icp_combined(const float *src, int64_t ns, const float *tgt, const float *nrm, int64_t nt,
                        const double *T_init, double w_point, double w_plane, double d_max, int max_iters,
                        double conv_tol, int use_kdtree, double T_out[16], int32_t stats_i[2],
                        int64_t stats_i64[1], double stats_d[1])
{
    double T[16];
    for (int i = 0; i < 16; i++) T[i] = T_init ? T_init[i] : ((i % 5 == 0) ? 1.0 : 0.0);
    kd_tree tree;
    int have_tree = 0;
    if (use_kdtree) {
        if (kd_build(&tree, tgt, nt)) { kd_free(&tree); return 2; }
        have_tree = 1;
    }
    int status = ICP_MAXITER, it = 0;
    double A[36], b[6], L[36], x[6];
    int64_t inl;
    double s2;
    for (it = 0; it < max_iters; it++) {
        int rc = combined_system(src, ns, tgt, nrm, nt, have_tree ? &tree : NULL, T, d_max, w_point, w_plane, A, b,
                                 &inl, &s2);
        if (rc) { if (have_tree) kd_free(&tree); return rc; }
        if (inl == 0) { status = ICP_NO_INLIERS; break; }
        if (inl < 6 || oracle_cholesky6(A, L)) { status = ICP_DEGENERATE; break; }
        chol_solve6(L, b, x);
        double dR[9];
        oracle_euler_zyx(x[0], x[1], x[2], dR);
        compose_left(T, dR, x + 3);
        if (conv_tol > 0) {
            double m = 0;
            for (int a = 0; a < 6; a++) if (fabs(x[a]) > m) m = fabs(x[a]);
            if (m < conv_tol) { status = ICP_CONVERGED; it++; break; }
        }
    }
    int rc = combined_system(src, ns, tgt, nrm, nt, have_tree ? &tree : NULL, T, d_max, w_point, w_plane, A, b,
                             &inl, &s2);
    if (have_tree) kd_free(&tree);
    if (rc) return rc;
    memcpy(T_out, T, sizeof T);
    stats_i[0] = status;
    stats_i[1] = it;
    stats_i64[0] = inl;
    stats_d[0] = inl > 0 ? sqrt(s2 / (double)inl) : 0.0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* projective data association (Section 3, "Iterative geometric             */
/* registration": correspondences by projective data association in 3D)    */
/* ------------------------------------------------------------------------ */

/* The target is an organized image: width x height pixels in raster order
   from a pinhole camera at the target frame's origin looking along +z, with
   intrinsics K = (fx, fy, cx, cy).  A pixel is valid when its point is
   finite with z > 0.  The candidate of a transformed source point p' is the
   pixel it projects to:
       u = fx * p'x / p'z + cx,  v = fy * p'y / p'z + cy   (float64, this order)
       iu = floor(u + 0.5),  iv = floor(v + 0.5)
   when p'z > 0 and (iu, iv) lies in the image; -1 otherwise. */
static int64_t project_pixel(const double p[3], int W, int H, const double K[4])
{
    if (!(p[2] > 0.0)) return -1;
    double u = K[0] * p[0] / p[2] + K[2];
    double v = K[1] * p[1] / p[2] + K[3];
    double fu = floor(u + 0.5), fv = floor(v + 0.5);
    if (!(fu >= 0.0 && fu < (double)W && fv >= 0.0 && fv < (double)H)) return -1;
    return (int64_t)fv * W + (int64_t)fu;
}

static int pixel_valid(const float *q)
{
    return isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && q[2] > 0.f;
}

/* Candidate pixel of every source point at pose T (for the pins). */
int oracle_projective_pixels(const float *src, int64_t ns, int W, int H, const double K[4], const double T[16],
                             int64_t *pix)
{
    for (int64_t i = 0; i < ns; i++) {
        double p[3];
        transform_point(T, src + 3 * i, p);
        pix[i] = project_pixel(p, W, H, K);
    }
    return 0;
}

/* The point-to-plane system of p2plane_system with projective
   correspondences: the candidate pixel's point q and normal n, kept when the
   pixel is valid, n != 0 and |p' - q|^2 <= d_max^2. */
static void projective_system(const float *src, int64_t ns, const float *tgt, const float *nrm, int W, int H,
                              const double K[4], const double T[16], double d_max, double A[36], double b[6],
                              int64_t *inliers, double *sum_r2)
{
    double dmax2 = d_max * d_max;
    for (int i = 0; i < 36; i++) A[i] = 0;
    for (int i = 0; i < 6; i++) b[i] = 0;
    int64_t cnt = 0;
    double s2 = 0;
    for (int64_t i = 0; i < ns; i++) {
        double p[3];
        transform_point(T, src + 3 * i, p);
        int64_t k = project_pixel(p, W, H, K);
        if (k < 0) continue;
        const float *q = tgt + 3 * k, *nq = nrm + 3 * k;
        if (!pixel_valid(q) || !(nq[0] != 0.f || nq[1] != 0.f || nq[2] != 0.f)) continue;
        double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
        if (dx * dx + dy * dy + dz * dz > dmax2) continue;
        double n[3] = {nq[0], nq[1], nq[2]};
        double J[6] = {p[1] * n[2] - p[2] * n[1], p[2] * n[0] - p[0] * n[2], p[0] * n[1] - p[1] * n[0],
                       n[0], n[1], n[2]};
        double r = dx * n[0] + dy * n[1] + dz * n[2];
        for (int rr = 0; rr < 6; rr++) {
            for (int c = 0; c < 6; c++) A[rr * 6 + c] += J[rr] * J[c];
            b[rr] += J[rr] * r;
        }
        s2 += r * r;
        cnt++;
    }
    *inliers = cnt;
    *sum_r2 = s2;
}

/* Point-to-plane ICP with projective correspondences: the loop of oracle_icp
   (Cholesky, Rz Ry Rx on the left, same stopping rules and statistics). */
int oracle_icp_projective(const float *src, int64_t ns, const float *tgt, const float *nrm, int W, int H,
                          const double K[4], const double *T_init, double d_max, int max_iters, double conv_tol,
                          double T_out[16], int32_t stats_i[2], int64_t stats_i64[1], double stats_d[1])
{
    double T[16];
    for (int i = 0; i < 16; i++) T[i] = T_init ? T_init[i] : ((i % 5 == 0) ? 1.0 : 0.0);
    int status = ICP_MAXITER, it = 0;
    double A[36], b[6], L[36], x[6];
    int64_t inl;
    double s2;
    for (it = 0; it < max_iters; it++) {
        projective_system(src, ns, tgt, nrm, W, H, K, T, d_max, A, b, &inl, &s2);
        if (inl == 0) { status = ICP_NO_INLIERS; break; }
        if (inl < 6 || oracle_cholesky6(A, L)) { status = ICP_DEGENERATE; break; }
        chol_solve6(L, b, x);
        double dR[9];
        oracle_euler_zyx(x[0], x[1], x[2], dR);
        compose_left(T, dR, x + 3);
        if (conv_tol > 0) {
            double m = 0;
            for (int a = 0; a < 6; a++) if (fabs(x[a]) > m) m = fabs(x[a]);
            if (m < conv_tol) { status = ICP_CONVERGED; it++; break; }
        }
    }
    projective_system(src, ns, tgt, nrm, W, H, K, T, d_max, A, b, &inl, &s2);
    memcpy(T_out, T, sizeof T);
    stats_i[0] = status;
    stats_i[1] = it;
    stats_i64[0] = inl;
    stats_d[0] = inl > 0 ? sqrt(s2 / (double)inl) : 0.0;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* radius and hybrid neighbourhoods for normals (Section 3, "Core           */
/* operations": radius and hybrid queries; Section 4: normals from a 1 cm    */
/* radius neighbourhood)                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t *idx;
    int64_t n, cap;
} idx_list;

static int list_push(idx_list *l, int32_t j)
{
    if (l->n == l->cap) {
        int64_t cap = l->cap ? 2 * l->cap : 64;
        int32_t *p = (int32_t *)realloc(l->idx, sizeof(int32_t) * (size_t)cap);
        if (!p) return 1;
        l->idx = p;
        l->cap = cap;
    }
    l->idx[l->n++] = j;
    return 0;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* every reference point with float32 key <= r2 (the kNN key of the
   definition), pruned like kd_knn_rec */
static void kd_radius_rec(const kd_tree *t, int32_t id, const float *q, float r2, idx_list *out)
{
    const kd_node *nd = &t->nodes[id];
    if (nd->left < 0) {
        for (int32_t i = nd->lo; i < nd->hi; i++) {
            int32_t j = t->perm[i];
            if (knn_key(t->pts + 3 * (int64_t)j, q) <= r2) list_push(out, j);
        }
        return;
    }
    double diff = (double)q[nd->axis] - (double)nd->split;
    int32_t near = diff <= 0 ? nd->left : nd->right;
    int32_t far = diff <= 0 ? nd->right : nd->left;
    kd_radius_rec(t, near, q, r2, out);
    if (diff * diff * (1.0 - 1e-6) <= (double)r2) kd_radius_rec(t, far, q, r2, out);
}

/* PCA normal of point i from the neighbour set idx[0..m) (as oracle_normals:
   mean-centred covariance of the offsets from p_i, 1/m, cyclic Jacobi,
   viewpoint orientation, curvature); m < 3 gives normal 0 and curvature 0
   (fewer than three points do not fix a plane). */
static void pca_normal(const float *xyz, int64_t i, const int32_t *idx, int64_t m, const double vp[3],
                       double nn[3], double *curv, double ev[3])
{
    nn[0] = nn[1] = nn[2] = 0.0;
    double w[3] = {0.0, 0.0, 0.0};
    if (m >= 3) {
        double mu[3] = {0, 0, 0};
        for (int64_t s = 0; s < m; s++)
            for (int a = 0; a < 3; a++) mu[a] += (double)xyz[3 * (int64_t)idx[s] + a] - (double)xyz[3 * i + a];
        for (int a = 0; a < 3; a++) mu[a] /= (double)m;
        double c[9] = {0};
        for (int64_t s = 0; s < m; s++) {
            double e[3];
            for (int a = 0; a < 3; a++) e[a] = ((double)xyz[3 * (int64_t)idx[s] + a] - (double)xyz[3 * i + a]) - mu[a];
            for (int r = 0; r < 3; r++)
                for (int cc = 0; cc < 3; cc++) c[r * 3 + cc] += e[r] * e[cc];
        }
        for (int r = 0; r < 9; r++) c[r] /= (double)m;
        int zero = 1;
        for (int r = 0; r < 9; r++) if (c[r] != 0.0) zero = 0;
        if (!zero) {
            double v[9];
            oracle_jacobi3(c, w, v);
            for (int a = 0; a < 3; a++) nn[a] = v[a * 3 + 0];
            double nrm = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
            for (int a = 0; a < 3; a++) nn[a] /= nrm;
            double dot = 0;
            for (int a = 0; a < 3; a++) dot += nn[a] * (vp[a] - (double)xyz[3 * i + a]);
            int flip = dot < 0;
            if (dot == 0) {
                for (int a = 0; a < 3; a++)
                    if (nn[a] != 0) { flip = nn[a] < 0; break; }
            }
            if (flip) for (int a = 0; a < 3; a++) nn[a] = -nn[a];
        }
    }
    double tr = w[0] + w[1] + w[2];
    *curv = tr > 0 ? w[0] / tr : 0.0;
    for (int a = 0; a < 3; a++) ev[a] = w[a];
}

/* Normals from radius neighbourhoods N(i) = {j : key(p_j, p_i) <= r2}
   (k == 0), or hybrid ones: the k nearest points of i that have
   key <= r2 (k > 0; the k nearest by the kNN definition, then those within
   the radius).  r2 is the float32 square of the radius, as the GPU takes it.
   out_count (nullable) receives |N(i)|. */
int oracle_normals_radius(const float *xyz, int64_t n, float radius, int k, const double viewpoint[3],
                          int use_kdtree, double *out_normals, double *out_curv, double *out_evals,
                          int32_t *out_count)
{
    if (!(radius > 0.f) || k < 0 || k > 64 || (k > 0 && k > n)) return 1;
    const float r2 = radius * radius;
    int32_t *nbr = NULL;
    float *nd2 = NULL;
    if (k > 0) {
        nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1) * (size_t)k);
        nd2 = (float *)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1) * (size_t)k);
        if (!nbr || !nd2) { free(nbr); free(nd2); return 2; }
        int rc = use_kdtree ? oracle_knn_kdtree(xyz, n, xyz, n, k, nbr, nd2)
                            : oracle_knn_brute(xyz, n, xyz, n, k, nbr, nd2);
        if (rc) { free(nbr); free(nd2); return rc; }
    }
    kd_tree t;
    int have_tree = 0;
    if (k == 0 && use_kdtree) {
        if (kd_build(&t, xyz, n)) { kd_free(&t); return 2; }
        have_tree = 1;
    }
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++) {
        idx_list l = {NULL, 0, 0};
        if (k > 0) {
            for (int s = 0; s < k; s++)
                if (nd2[i * k + s] <= r2) list_push(&l, nbr[i * k + s]);
        } else if (have_tree) {
            kd_radius_rec(&t, 0, xyz + 3 * i, r2, &l);
        } else {
            for (int64_t j = 0; j < n; j++)
                if (knn_key(xyz + 3 * j, xyz + 3 * i) <= r2) list_push(&l, (int32_t)j);
        }
        if (l.n > 0 && !l.idx) failed = 1;
        /* one summation order whatever found the set: ascending index */
        if (l.n > 1) qsort(l.idx, (size_t)l.n, sizeof(int32_t), cmp_i32);
        double nn[3], curv, ev[3];
        pca_normal(xyz, i, l.idx, l.n, viewpoint, nn, &curv, ev);
        for (int a = 0; a < 3; a++) out_normals[3 * i + a] = nn[a];
        if (out_curv) out_curv[i] = curv;
        if (out_evals) for (int a = 0; a < 3; a++) out_evals[3 * i + a] = ev[a];
        if (out_count) out_count[i] = (int32_t)l.n;
        free(l.idx);
    }
    if (have_tree) kd_free(&t);
    free(nbr);
    free(nd2);
    return failed ? 2 : 0;
}
