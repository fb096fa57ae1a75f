/*
 * am_oracle.c -- plain FP64 CPU oracle for analytic marching.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header or constant with the GPU
 * path.
 *
 * What it computes (paper: Lei, Jia, Ma, "Learning and Meshing from Deep
 * Implicit Surface Networks Using an Efficient Implementation of Analytic
 * Marching"):
 *   - forward pass and activation code: Sec. 2.2, Eqns (NeuronState),
 *     (LayerState), (MLPState); a unit is "on" iff its pre-activation is > 0.
 *   - the per-cell affine chain: Lemma 1 (RegionMapping) and Corollary 1
 *     (RegionAssociatedNeuronMapping, SDFPlaneFunctional), with the shortcut
 *     blocks of Sec. 5.1 and the max-pooled heads of Sec. 5.2; biases enter
 *     through the homogeneous coordinate.
 *   - the analytic face: Eqns (AnalyticCellSystem) and (AnalyticFace), plus
 *     the sub-cell rows of Eqn (AnalyticCellSystemMaxPooling), clipped to the
 *     domain box [-1,1]^3.  The polygon is built by clipping the zero plane by
 *     every oriented constraint in turn (box, hidden units in code order, then
 *     the max-pool comparison rows).
 *   - vertices: the 3x3 system of Eqn (VertexEquationSystem) for each pair of
 *     consecutive edges, solved by Gaussian elimination with partial pivoting.
 *   - marching: Algorithm 1 (Analytic Marching) with a FIFO active set, new
 *     states checked against every state seen so far; the neighbour across
 *     an edge on unit k has code s XOR e_k (Sec. 3.1, Fig. 2), the neighbour
 *     across a max-pool comparison edge i has the same sub-codes and argmax i
 *     (Eqn (StateFuntionalMaxPoolingOperation)).
 *   - pivoting enumeration of one face (Sec. 4.2.1, Alg. 2): a second,
 *     independent face routine, used to cross-check the clipping one.
 *   - seeding: dichotomy along a ray (Sec. 4.3.2), stopped once both ends of
 *     the bracket share one code, then the linear root inside that cell.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - a vertex is ON a line when |c.[v;1]| <= TAU*(|(cu,cv)|(1+|v|) + |cw|),
 *     TAU = 2^-40; a line cuts only if some vertex is strictly above that;
 *   - only constraints that carry an edge of positive length spawn
 *     neighbours;
 *   - the domain box planes get ids -1..-6 (x<=1, x>=-1, y<=1, y>=-1, z<=1,
 *     z>=-1); max-pool comparison rows get id N+i for head i;
 *   - cycles run counter-clockwise seen from +grad F and start at the edge
 *     with the smallest id; faces are sorted by code words (unsigned,
 *     word 0 first), then argmax.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TAU (1.0 / 1099511627776.0) /* 2^-40 */

/* ORC_MUTATE (0 = the oracle) plants one known mistake, so that a test can
 * show that the pins catch it; the mutants are only ever built by that test. */
#ifndef ORC_MUTATE
#define ORC_MUTATE 0
#endif
#define SQUARE_HALF 2.0             /* the box section lies in a disc of radius sqrt(3) */

typedef struct {
    int32_t n_layers;        /* L + 2: input, L hidden layers, head layer */
    const int32_t *width;    /* width[l], l = 0..n_layers-1, width[0] == 3 */
    int32_t n_blocks;
    const int32_t *blk_dst;  /* block b adds W_b @ act[blk_src[b]] to pre[blk_dst[b]] */
    const int32_t *blk_src;
    const int64_t *blk_off;  /* offset of block b's row-major W in weights */
    const double *weights;
    const int64_t *bias_off; /* offset of layer l's bias in biases (l >= 1) */
    const double *biases;
} orc_net;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

static int n_hidden(const orc_net *net) {
    int n = 0;
    for (int l = 1; l < net->n_layers - 1; l++) n += net->width[l];
    return n;
}

static int n_heads(const orc_net *net) { return net->width[net->n_layers - 1]; }

/* first unit of layer l in the global (layer-major) unit order; layer
 * n_layers-1 (the heads) starts right after the last hidden unit */
static int layer_offset(const orc_net *net, int l) {
    int o = 0;
    for (int j = 1; j < l; j++) o += net->width[j];
    return o;
}

int orc_code_words(const orc_net *net) {
    int n = n_hidden(net);
    int w = (n + 63) / 64;
    return w < 1 ? 1 : w;
}

static int get_bit(const uint64_t *code, int g) { return (int)((code[g >> 6] >> (g & 63)) & 1u); }

/* ------------------------------------------------------------------ */
/* forward pass and activation code (Sec. 2.2)                          */
/* ------------------------------------------------------------------ */

/* pre: N + M values (hidden units in layer-major order, then heads).
 * Returns F = max over heads; *argmax gets the lowest index attaining it. */
double orc_forward(const orc_net *net, const double *x, double *pre, int32_t *argmax) {
    int L2 = net->n_layers;
    int total = 0;
    for (int l = 0; l < L2; l++) total += net->width[l];
    double *act = (double *)malloc(sizeof(double) * total);
    int *aoff = (int *)malloc(sizeof(int) * L2);
    int o = 0;
    for (int l = 0; l < L2; l++) { aoff[l] = o; o += net->width[l]; }
    for (int i = 0; i < 3; i++) act[i] = x[i];
    for (int l = 1; l < L2; l++) {
        double *a = act + aoff[l];
        const double *b = net->biases + net->bias_off[l];
        for (int k = 0; k < net->width[l]; k++) a[k] = b[k];
        for (int bk = 0; bk < net->n_blocks; bk++) {
            if (net->blk_dst[bk] != l) continue;
            int s = net->blk_src[bk];
            const double *W = net->weights + net->blk_off[bk];
            const double *in = act + aoff[s];
            for (int k = 0; k < net->width[l]; k++) {
                double acc = 0.0;
                for (int m = 0; m < net->width[s]; m++) acc += W[(int64_t)k * net->width[s] + m] * in[m];
                a[k] += acc;
            }
        }
        /* a now holds the pre-activation of layer l */
        int go = layer_offset(net, l);
        for (int k = 0; k < net->width[l]; k++) pre[go + k] = a[k];
        if (l < L2 - 1)
            for (int k = 0; k < net->width[l]; k++) a[k] = a[k] > 0.0 ? a[k] : 0.0;
    }
    int N = n_hidden(net), M = n_heads(net);
    int best = 0;
    for (int i = 1; i < M; i++)
        if (pre[N + i] > pre[N + best]) best = i;
    double F = pre[N + best];
    if (argmax) *argmax = best;
    free(act);
    free(aoff);
    return F;
}

/* Activation code s(x): bit g set iff the pre-activation of unit g is > 0. */
double orc_code(const orc_net *net, const double *x, uint64_t *code, int32_t *argmax) {
    int N = n_hidden(net), M = n_heads(net);
    double *pre = (double *)malloc(sizeof(double) * (N + M));
    double F = orc_forward(net, x, pre, argmax);
    int W = orc_code_words(net);
    memset(code, 0, sizeof(uint64_t) * W);
    for (int g = 0; g < N; g++)
        if (ORC_MUTATE == 7 ? pre[g] >= 0.0 : pre[g] > 0.0) code[g >> 6] |= (uint64_t)1 << (g & 63);
    free(pre);
    return F;
}

/* ------------------------------------------------------------------ */
/* affine chain (Lemma 1, Corollary 1, Sec. 5.1, Sec. 5.2)              */
/* ------------------------------------------------------------------ */

/* rows: (N + M) x 4, row g = coefficients (a, b, c, d) with
 * pre_g(x) = a x + b y + c z + d for every x in the cell of `code`. */
void orc_chain(const orc_net *net, const uint64_t *code, double *rows) {
    int L2 = net->n_layers;
    /* Z for the input layer: x = [I | 0] [x; 1] */
    double Z0[3][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}};
    for (int l = 1; l < L2; l++) {
        int go = layer_offset(net, l);
        const double *b = net->biases + net->bias_off[l];
        for (int k = 0; k < net->width[l]; k++) {
            double *z = rows + 4 * (int64_t)(go + k);
            z[0] = z[1] = z[2] = 0.0;
            z[3] = ORC_MUTATE == 1 ? 0.0 : b[k];
        }
        for (int bk = 0; bk < net->n_blocks; bk++) {
            if (net->blk_dst[bk] != l) continue;
            int s = net->blk_src[bk];
            if (ORC_MUTATE == 4 && s != l - 1) continue;
            const double *W = net->weights + net->blk_off[bk];
            int so = layer_offset(net, s);
            for (int k = 0; k < net->width[l]; k++) {
                double *z = rows + 4 * (int64_t)(go + k);
                for (int m = 0; m < net->width[s]; m++) {
                    double w = W[(int64_t)k * net->width[s] + m];
                    if (ORC_MUTATE == 9 && net->width[s] == net->width[l])
                        w = W[(int64_t)m * net->width[s] + k];
                    const double *src;
                    if (s == 0) {
                        src = Z0[m];                       /* input: never rectified */
                    } else {
                        if (ORC_MUTATE != 3 && !get_bit(code, so + m))
                            continue; /* diag(s_j) zeroes inactive units */
                        src = rows + 4 * (int64_t)(so + m);
                    }
                    for (int q = 0; q < 4; q++) z[q] += w * src[q];
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* constraint rows of a cell                                            */
/* ------------------------------------------------------------------ */

/* Oriented constraint row for id (feasible side: row . [x;1] <= 0). */
static void constraint_row(int id, int N, const uint64_t *code, int argmax, const double *rows,
                           double *c) {
    if (id < 0) {
        int a = (-id - 1) / 2, lower = (-id - 1) % 2;
        c[0] = c[1] = c[2] = 0.0;
        c[a] = lower ? -1.0 : 1.0;
        c[3] = -1.0;
    } else if (id < N) {
        double sgn = get_bit(code, id) ? -1.0 : 1.0; /* (1 - 2 s_k) */
        if (ORC_MUTATE == 2) sgn = -sgn;
        for (int q = 0; q < 4; q++) c[q] = sgn * rows[4 * (int64_t)id + q];
    } else {
        const double *hi = rows + 4 * (int64_t)id;
        const double *hj = rows + 4 * (int64_t)(N + argmax);
        for (int q = 0; q < 4; q++) c[q] = ORC_MUTATE == 5 ? hj[q] - hi[q] : hi[q] - hj[q];
    }
}

/* ------------------------------------------------------------------ */
/* halfplane clipping in the zero plane                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    double a, b; /* coordinates in the plane frame */
    int e;       /* id of the edge that starts at this vertex */
} pvert;

/* Clip polygon P (m vertices, CCW) by the halfplane cu*a + cv*b + cw <= 0
 * with id `id`.  Writes the result to Q and returns its size (0 = empty). */
static int clip_polygon(const pvert *P, int m, double cu, double cv, double cw, int id, pvert *Q) {
    double d[256];
    int cls[256]; /* +1 out, 0 on, -1 in */
    int n_out = 0, n_in = 0;
    double nrm = hypot(cu, cv);
    for (int i = 0; i < m; i++) {
        d[i] = cu * P[i].a + cv * P[i].b + cw;
        double tol = TAU * (nrm * (1.0 + hypot(P[i].a, P[i].b)) + fabs(cw));
        cls[i] = d[i] > tol ? 1 : (d[i] < -tol ? -1 : 0);
        if (ORC_MUTATE == 10 && cls[i] == 0) cls[i] = 1;
        n_out += cls[i] == 1;
        n_in += cls[i] == -1;
    }
    if (n_out == 0) {
        memcpy(Q, P, sizeof(pvert) * m);
        return m;
    }
    if (n_in == 0) return 0; /* nothing strictly inside: zero area */
    int q = 0;
    for (int i = 0; i < m; i++) {
        int j = (i + 1) % m;
        if (cls[i] != 1) {
            Q[q] = P[i];
            if (cls[j] == 1 && cls[i] == 0) Q[q].e = id; /* leaves along the new line */
            q++;
        }
        if ((cls[i] == -1 && cls[j] == 1) || (cls[i] == 1 && cls[j] == -1)) {
            double t = d[i] / (d[i] - d[j]);
            Q[q].a = P[i].a + t * (P[j].a - P[i].a);
            Q[q].b = P[i].b + t * (P[j].b - P[i].b);
            Q[q].e = cls[i] == -1 ? id : P[i].e;
            q++;
        }
        if (q > 250) return -1;
    }
    return q;
}

/* 3x3 solve by Gaussian elimination with partial pivoting: A x = r. */
static int solve3(double A[3][3], double r[3], double x[3]) {
    for (int c = 0; c < 3; c++) {
        int p = c;
        for (int i = c + 1; i < 3; i++)
            if (fabs(A[i][c]) > fabs(A[p][c])) p = i;
        if (A[p][c] == 0.0) return -1;
        if (p != c) {
            for (int k = 0; k < 3; k++) { double t = A[c][k]; A[c][k] = A[p][k]; A[p][k] = t; }
            double t = r[c]; r[c] = r[p]; r[p] = t;
        }
        for (int i = c + 1; i < 3; i++) {
            double f = A[i][c] / A[c][c];
            for (int k = c; k < 3; k++) A[i][k] -= f * A[c][k];
            r[i] -= f * r[c];
        }
    }
    for (int i = 2; i >= 0; i--) {
        double s = r[i];
        for (int k = i + 1; k < 3; k++) s -= A[i][k] * x[k];
        x[i] = s / A[i][i];
    }
    return 0;
}

/* Face flags */
#define ORC_FACE_EMPTY 1     /* no positive-area face in the domain */
#define ORC_FACE_DEGEN 2     /* repeated line id or leftover frame edge */
#define ORC_FACE_SINGULAR 4  /* a vertex system was singular */
#define ORC_FACE_TOOBIG 8

/* Face of the cell (code, argmax).  ids/verts need room for max_m entries.
 * Returns the vertex count m (0 if empty) and sets *flags, *area. */
int orc_face_from_rows(const orc_net *net, const uint64_t *code, int32_t argmax, const double *rows,
                       int max_m, int32_t *ids, double *verts, double *area, int32_t *flags) {
    int N = n_hidden(net), M = n_heads(net);
    const double *aF = rows + 4 * (int64_t)(N + argmax);
    *flags = 0;
    *area = 0.0;
    double nx = aF[0], ny = aF[1], nz = aF[2];
    double nn = nx * nx + ny * ny + nz * nz;
    if (nn == 0.0) { *flags = ORC_FACE_EMPTY; return 0; }
    double p0[3] = {-aF[3] * nx / nn, -aF[3] * ny / nn, -aF[3] * nz / nn};
    double nl = sqrt(nn), n[3] = {nx / nl, ny / nl, nz / nl};
    /* u = normalize(n x e_a) for the axis with the smallest |n_a|; v = n x u */
    int ax = 0;
    if (fabs(n[1]) < fabs(n[ax])) ax = 1;
    if (fabs(n[2]) < fabs(n[ax])) ax = 2;
    double e[3] = {0, 0, 0};
    e[ax] = 1.0;
    double u[3] = {n[1] * e[2] - n[2] * e[1], n[2] * e[0] - n[0] * e[2], n[0] * e[1] - n[1] * e[0]};
    double ul = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int i = 0; i < 3; i++) u[i] /= ul;
    double v[3] = {n[1] * u[2] - n[2] * u[1], n[2] * u[0] - n[0] * u[2], n[0] * u[1] - n[1] * u[0]};

    pvert bufA[256], bufB[256];
    pvert *P = bufA, *Q = bufB;
    int m = 4;
    P[0] = (pvert){-SQUARE_HALF, -SQUARE_HALF, -7};
    P[1] = (pvert){SQUARE_HALF, -SQUARE_HALF, -8};
    P[2] = (pvert){SQUARE_HALF, SQUARE_HALF, -9};
    P[3] = (pvert){-SQUARE_HALF, SQUARE_HALF, -10};

    int n_lines = 6 + N + M;
    for (int t = 0; t < n_lines && m > 0; t++) {
        int id;
        if (t < 6) id = -1 - t;
        else if (t < 6 + N) id = t - 6;
        else {
            int i = t - 6 - N;
            if (i == argmax) continue;
            id = N + i;
        }
        double c[4];
        constraint_row(id, N, code, argmax, rows, c);
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double cv = c[0] * v[0] + c[1] * v[1] + c[2] * v[2];
        double cw = c[0] * p0[0] + c[1] * p0[1] + c[2] * p0[2] + c[3];
        int q = clip_polygon(P, m, cu, cv, cw, id, Q);
        if (q < 0) { *flags = ORC_FACE_TOOBIG; return 0; }
        pvert *tmp = P; P = Q; Q = tmp;
        m = q;
    }
    if (m < 3) { *flags = ORC_FACE_EMPTY; return 0; }
    for (int i = 0; i < m; i++) {
        if (P[i].e <= -7) { /* a frame edge survived the box planes: unusable face */
            *flags |= ORC_FACE_DEGEN | ORC_FACE_EMPTY;
            return 0;
        }
        for (int j = i + 1; j < m; j++)
            if (P[i].e == P[j].e) *flags |= ORC_FACE_DEGEN;
    }
    /* twice the area, from the first vertex so that rounding scales with the
     * polygon's own size (the absolute shoelace loses tiny faces) */
    double A2 = 0.0;
    for (int i = 1; i + 1 < m; i++) {
        double ax = P[i].a - P[0].a, ay = P[i].b - P[0].b;
        double bx = P[i + 1].a - P[0].a, by = P[i + 1].b - P[0].b;
        A2 += ax * by - bx * ay;
    }
    if (ORC_MUTATE == 15) { /* the absolute shoelace about the frame origin */
        A2 = 0.0;
        for (int i = 0; i < m; i++) A2 += P[i].a * P[(i + 1) % m].b - P[(i + 1) % m].a * P[i].b;
    }
    *area = 0.5 * A2;
    if (!(A2 > 0.0)) { *flags |= ORC_FACE_EMPTY; return 0; }
    if (m > max_m) { *flags |= ORC_FACE_TOOBIG; return 0; }
    /* rotate so that the smallest edge id comes first */
    int r = 0;
    for (int i = 1; i < m; i++)
        if (P[i].e < P[r].e) r = i;
    for (int i = 0; i < m; i++) Q[i] = P[(i + r) % m];
    /* vertex i starts edge i and ends edge i-1: solve [c_{i-1}; c_i; aF] x = -[...] */
    for (int i = 0; i < m; i++) {
        int ea = Q[(i + m - 1) % m].e, eb = Q[i].e;
        if (ORC_MUTATE == 6) ea = Q[(i + 1) % m].e;
        double ca[4], cb[4];
        constraint_row(ea, N, code, argmax, rows, ca);
        constraint_row(eb, N, code, argmax, rows, cb);
        double A[3][3] = {{ca[0], ca[1], ca[2]}, {cb[0], cb[1], cb[2]}, {aF[0], aF[1], aF[2]}};
        double rr[3] = {-ca[3], -cb[3], -aF[3]};
        double x[3];
        if (solve3(A, rr, x) != 0) {
            *flags |= ORC_FACE_SINGULAR;
            x[0] = x[1] = x[2] = NAN;
        }
        ids[i] = eb;
        verts[3 * i + 0] = x[0];
        verts[3 * i + 1] = x[1];
        verts[3 * i + 2] = x[2];
    }
    return m;
}

int orc_face(const orc_net *net, const uint64_t *code, int32_t argmax, int max_m, int32_t *ids,
             double *verts, double *area, int32_t *flags) {
    int N = n_hidden(net), M = n_heads(net);
    double *rows = (double *)malloc(sizeof(double) * 4 * (N + M));
    orc_chain(net, code, rows);
    int m = orc_face_from_rows(net, code, argmax, rows, max_m, ids, verts, area, flags);
    free(rows);
    return m;
}

/* ------------------------------------------------------------------ */
/* pivoting enumeration of a face (Sec. 4.2.1, Alg. 2)                  */
/* ------------------------------------------------------------------ */

/* Constraint value and its on-plane tolerance at x (the TAU reading). */
static double row_value(const double *c, const double *x, double *tol) {
    double d = c[0] * x[0] + c[1] * x[1] + c[2] * x[2] + c[3];
    double xn = fmax(fabs(x[0]), fmax(fabs(x[1]), fabs(x[2])));
    *tol = TAU * ((fabs(c[0]) + fabs(c[1]) + fabs(c[2])) * (1.0 + xn) + fabs(c[3]));
    return d;
}

/* Candidate vertex of planes a and b on the zero plane aF. */
static int pair_vertex(const double *ca, const double *cb, const double *aF, double *x) {
    double A[3][3] = {{ca[0], ca[1], ca[2]}, {cb[0], cb[1], cb[2]}, {aF[0], aF[1], aF[2]}};
    double r[3] = {-ca[3], -cb[3], -aF[3]};
    return solve3(A, r, x);
}

/* The boundary condition of the cell, Eqn (AnalyticCellSystem), with the box
 * and comparison rows: every oriented row is <= its tolerance at x. */
static int point_valid(const double *C, int nl, const double *x) {
    for (int k = 0; k < nl; k++) {
        double tol, d = row_value(C + 4 * k, x, &tol);
        if (d > tol) return 0;
    }
    return 1;
}

static int same_point(const double *x, const double *y) {
    double s = 1.0 + fmax(fabs(x[0]), fmax(fabs(x[1]), fabs(x[2])));
    return fabs(x[0] - y[0]) <= 1e-12 * s && fabs(x[1] - y[1]) <= 1e-12 * s && fabs(x[2] - y[2]) <= 1e-12 * s;
}

/* Plane b carries a valid vertex other than v (with some plane other than
 * itself): the segment of the face on b has positive length. */
static int carries_edge(const double *C, int nl, int b, const double *aF, const double *v) {
    for (int k = 0; k < nl; k++) {
        if (k == b) continue;
        double x[3];
        if (pair_vertex(C + 4 * b, C + 4 * k, aF, x) != 0) continue;
        if (!same_point(x, v) && point_valid(C, nl, x)) return 1;
    }
    return 0;
}

typedef struct {
    double dist;
    int k;
} orc_order;

static int cmp_order(const void *pa, const void *pb) {
    const orc_order *a = (const orc_order *)pa, *b = (const orc_order *)pb;
    if (a->dist < b->dist) return -1;
    if (a->dist > b->dist) return 1;
    return a->k - b->k;
}

/* Face of the cell (code, argmax) by pivoting from a true boundary plane
 * start_id through the point xs on the face's edge on that plane.
 *
 * The planes are ordered by their distance from xs.  Phase 1 takes the
 * first plane t'' in that order whose vertex with the start plane satisfies
 * the cell's boundary condition; phase 2 repeats from the newest plane,
 * scanning the order again each time, until the accepted plane is the start
 * plane.  Readings where the paper is silent:
 *   - the plane list holds the hidden units, the comparison rows of other
 *     heads and the six box planes (the face is clipped to the box);
 *   - a candidate equal to the current vertex (up to 1e-12 relative) is not
 *     a new vertex, so a vertex where several planes meet is visited once;
 *   - a plane is accepted only if it also carries a valid vertex other than
 *     the candidate, i.e. the face has an edge of positive length on it
 *     (otherwise a plane that only touches the face at the candidate could
 *     be taken and the walk would stall);
 *   - the walk may go either way round; the cycle is then oriented
 *     counter-clockwise seen from +grad F and rotated to start at the
 *     smallest id, and vertices are re-solved from consecutive ids, as in
 *     the clipping routine.
 * Returns m (0 on failure, flags set as for orc_face). */
int orc_face_pivot(const orc_net *net, const uint64_t *code, int32_t argmax, int32_t start_id,
                   const double *xs, int max_m, int32_t *ids, double *verts, int32_t *flags) {
    int N = n_hidden(net), M = n_heads(net);
    double *rows = (double *)malloc(sizeof(double) * 4 * (N + M));
    orc_chain(net, code, rows);
    const double *aF = rows + 4 * (int64_t)(N + argmax);
    *flags = 0;
    int nl_max = 6 + N + M;
    double *C = (double *)malloc(sizeof(double) * 4 * nl_max);
    int *cid = (int *)malloc(sizeof(int) * nl_max);
    orc_order *ord = (orc_order *)malloc(sizeof(orc_order) * nl_max);
    int32_t *walk = (int32_t *)malloc(sizeof(int32_t) * (max_m + 1));
    double *wv = (double *)malloc(sizeof(double) * 3 * (max_m + 1));
    int nl = 0, star = -1, m = 0;
    for (int t = 0; t < nl_max; t++) {
        int id;
        if (t < 6) id = -1 - t;
        else if (t < 6 + N) id = t - 6;
        else {
            int i = t - 6 - N;
            if (i == argmax) continue;
            id = N + i;
        }
        constraint_row(id, N, code, argmax, rows, C + 4 * nl);
        cid[nl] = id;
        if (id == start_id) star = nl;
        double nrm = sqrt(C[4 * nl] * C[4 * nl] + C[4 * nl + 1] * C[4 * nl + 1] + C[4 * nl + 2] * C[4 * nl + 2]);
        double d = C[4 * nl] * xs[0] + C[4 * nl + 1] * xs[1] + C[4 * nl + 2] * xs[2] + C[4 * nl + 3];
        ord[nl].dist = nrm > 0.0 ? fabs(d) / nrm : INFINITY;
        ord[nl].k = nl;
        nl++;
    }
    if (star < 0) { *flags = ORC_FACE_EMPTY; goto done; }
    qsort(ord, nl, sizeof(orc_order), cmp_order);

    int t = star, tp = -1;
    double cur[3] = {0.0, 0.0, 0.0};
    int have_cur = 0;
    for (;;) {
        int accepted = -1;
        double v[3];
        for (int q = 0; q < nl; q++) {
            int k = ord[q].k;
            if (k == t || k == tp) continue;
            if (pair_vertex(C + 4 * t, C + 4 * k, aF, v) != 0) continue;
            if (!point_valid(C, nl, v)) continue;
            if (have_cur && same_point(v, cur)) continue;
            if (ORC_MUTATE != 13 && !carries_edge(C, nl, k, aF, v)) continue;
            accepted = k;
            break;
        }
        if (accepted < 0 || m >= max_m) { *flags = accepted < 0 ? ORC_FACE_EMPTY : ORC_FACE_TOOBIG; m = 0; goto done; }
        /* the vertex joins the edge on t and the edge on the accepted plane */
        walk[m] = accepted;
        wv[3 * m] = v[0]; wv[3 * m + 1] = v[1]; wv[3 * m + 2] = v[2];
        m++;
        cur[0] = v[0]; cur[1] = v[1]; cur[2] = v[2];
        have_cur = 1;
        if (accepted == star) break;
        tp = t;
        t = accepted;
    }
    /* walk order: vertex i (i < m-1) starts the edge on walk[i]; the last
     * vertex lies on the start plane and starts the edge back to vertex 0 */
    {
        double nx = 0.0, ny = 0.0, nz = 0.0;
        for (int i = 1; i + 1 < m; i++) {
            double ax = wv[3 * i] - wv[0], ay = wv[3 * i + 1] - wv[1], az = wv[3 * i + 2] - wv[2];
            double bx = wv[3 * i + 3] - wv[0], by = wv[3 * i + 4] - wv[1], bz = wv[3 * i + 5] - wv[2];
            nx += ay * bz - az * by;
            ny += az * bx - ax * bz;
            nz += ax * by - ay * bx;
        }
        int32_t *e = (int32_t *)malloc(sizeof(int32_t) * (m + 1));
        for (int i = 0; i < m; i++) e[i] = cid[walk[i]];   /* edge starting at walk vertex i */
        /* walk[m-1] is the start plane: vertex m-1 starts the edge on it */
        int ccw = nx * aF[0] + ny * aF[1] + nz * aF[2] > 0.0;
        if (ORC_MUTATE == 14) ccw = 1;
        int32_t *cyc = (int32_t *)malloc(sizeof(int32_t) * (m + 1));
        if (ccw) {
            for (int i = 0; i < m; i++) cyc[i] = e[i];
        } else {
            /* reversed: vertex i (from the end) starts the edge that ended there */
            for (int i = 0; i < m; i++) cyc[i] = e[(2 * m - 2 - i) % m];
        }
        free(e);
        if (m < 3) { *flags = ORC_FACE_EMPTY; free(cyc); m = 0; goto done; }
        for (int i = 0; i < m; i++)
            for (int j = i + 1; j < m; j++)
                if (cyc[i] == cyc[j]) *flags |= ORC_FACE_DEGEN;
        int r = 0;
        for (int i = 1; i < m; i++)
            if (cyc[i] < cyc[r]) r = i;
        for (int i = 0; i < m; i++) {
            int ea = cyc[(i + r + m - 1) % m], eb = cyc[(i + r) % m];
            double ca[4], cb[4], x[3];
            constraint_row(ea, N, code, argmax, rows, ca);
            constraint_row(eb, N, code, argmax, rows, cb);
            double A[3][3] = {{ca[0], ca[1], ca[2]}, {cb[0], cb[1], cb[2]}, {aF[0], aF[1], aF[2]}};
            double rr[3] = {-ca[3], -cb[3], -aF[3]};
            if (solve3(A, rr, x) != 0) {
                *flags |= ORC_FACE_SINGULAR;
                x[0] = x[1] = x[2] = NAN;
            }
            ids[i] = eb;
            verts[3 * i] = x[0];
            verts[3 * i + 1] = x[1];
            verts[3 * i + 2] = x[2];
        }
        free(cyc);
    }
done:
    free(rows);
    free(C);
    free(cid);
    free(ord);
    free(walk);
    free(wv);
    return m;
}

/* ------------------------------------------------------------------ */
/* dichotomy seeding along a ray (Sec. 4.3.2)                           */
/* ------------------------------------------------------------------ */

/* Finds a zero crossing of F on o + t d, t in [0, 1].  Returns 0 on success
 * (x, code, argmax set), 1 if F does not change sign, 2 if the bracket never
 * shrank into one cell within max_iter halvings. */
int orc_seed_ray(const orc_net *net, const double *o, const double *d, int max_iter, double *x,
                 uint64_t *code, int32_t *argmax) {
    int W = orc_code_words(net);
    uint64_t *clo = (uint64_t *)malloc(8 * W), *chi = (uint64_t *)malloc(8 * W);
    int32_t alo, ahi;
    double tlo = 0.0, thi = 1.0, p[3];
    for (int i = 0; i < 3; i++) p[i] = o[i];
    double flo = orc_code(net, p, clo, &alo);
    for (int i = 0; i < 3; i++) p[i] = o[i] + d[i];
    double fhi = orc_code(net, p, chi, &ahi);
    int st = 0;
    if ((flo > 0.0) == (fhi > 0.0)) { st = 1; goto done; }
    for (int it = 0;; it++) {
        if (alo == ahi && memcmp(clo, chi, 8 * W) == 0) break;
        if (it >= max_iter) { st = 2; goto done; }
        double tm = 0.5 * (tlo + thi);
        for (int i = 0; i < 3; i++) p[i] = o[i] + tm * d[i];
        uint64_t *cm = (uint64_t *)malloc(8 * W);
        int32_t am;
        double fm = orc_code(net, p, cm, &am);
        if ((fm > 0.0) == (flo > 0.0)) {
            tlo = tm; flo = fm; alo = am; memcpy(clo, cm, 8 * W);
        } else {
            thi = tm; fhi = fm; ahi = am; memcpy(chi, cm, 8 * W);
        }
        free(cm);
    }
    {
        double ts = tlo - flo * (thi - tlo) / (fhi - flo);
        for (int i = 0; i < 3; i++) x[i] = o[i] + ts * d[i];
        orc_code(net, x, code, argmax);
    }
done:
    free(clo);
    free(chi);
    return st;
}

/* ------------------------------------------------------------------ */
/* sphere-tracing seeding (Sec. 4.3.1, Eqn (SphereTracing))             */
/* ------------------------------------------------------------------ */

/* From x0, repeats x <- x - F(x) g / |g|^2, where g is the gradient of F in
 * the cell of x (the xyz part of the selected head's row of the cell's affine
 * chain); for an exact SDF |g| = 1 and this is the paper's update with step
 * size 1.  It stops when a step lands in the cell it started from: that point
 * lies on the cell's zero plane, so it is a surface point of that cell.
 * Returns 0 on success (x, code, argmax and *iters set), 1 if max_iter steps
 * do not settle, 2 if the gradient vanishes, 3 if the settled point lies
 * outside [-1, 1]^3.  A start point with F exactly 0 is returned as it is. */
int orc_seed_st(const orc_net *net, const double *x0, int max_iter, double *x, uint64_t *code,
                int32_t *argmax, int32_t *iters) {
    int W = orc_code_words(net), N = n_hidden(net), M = n_heads(net);
    uint64_t *cc = (uint64_t *)malloc(8 * W), *cn = (uint64_t *)malloc(8 * W);
    double *rows = (double *)malloc(sizeof(double) * 4 * (N + M));
    double p[3] = {x0[0], x0[1], x0[2]}, q[3];
    int32_t ac, an;
    int st = 1, it = 0;
    double F = orc_code(net, p, cc, &ac);
    if (F == 0.0) {
        st = 0;
        goto settled;
    }
    for (it = 0; it < max_iter; it++) {
        orc_chain(net, cc, rows);
        const double *g = rows + 4 * (N + (ORC_MUTATE == 12 ? 0 : ac));
        double gg = ORC_MUTATE == 11 ? 1.0 : g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        if (!(gg > 0.0)) { st = 2; goto done; }
        for (int i = 0; i < 3; i++) q[i] = p[i] - F * g[i] / gg;
        double Fq = orc_code(net, q, cn, &an);
        for (int i = 0; i < 3; i++) p[i] = q[i];
        if (an == ac && memcmp(cn, cc, 8 * W) == 0) {
            it++;
            st = 0;
            goto settled;
        }
        memcpy(cc, cn, 8 * W);
        ac = an;
        F = Fq;
    }
    goto done;
settled:
    for (int i = 0; i < 3; i++)
        if (fabs(p[i]) > 1.0) st = 3;
    for (int i = 0; i < 3; i++) x[i] = p[i];
    memcpy(code, cc, 8 * W);
    *argmax = ac;
    *iters = it;
done:
    free(cc);
    free(cn);
    free(rows);
    return st;
}

/* ------------------------------------------------------------------ */
/* marching (Algorithm 1)                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int W, N, M;
    int64_t n_cells, cap_cells;
    uint64_t *codes;     /* [cap][W] */
    int32_t *argmax;     /* [cap] */
    int32_t *m;          /* [cap] vertex count (0 = no face) */
    int32_t *fflags;     /* [cap] */
    int64_t *voff;       /* [cap] offset into ids/verts/nbr */
    int64_t n_v, cap_v;
    int32_t *ids;
    double *verts;
    int64_t *nbr;        /* neighbour cell index, -1 = domain edge */
    /* hash set of cell indices keyed by (code, argmax) */
    int64_t hcap;
    int64_t *htab;
    /* stats */
    int64_t n_seeds_in, n_seed_dup, n_seed_empty, n_degenerate;
} orc_result;

static uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static uint64_t key_hash(const uint64_t *code, int W, int32_t argmax) {
    uint64_t h = mix64((uint64_t)(uint32_t)argmax);
    for (int i = 0; i < W; i++) h = mix64(h ^ code[i]);
    return h;
}

static int key_eq(const orc_result *R, int64_t c, const uint64_t *code, int32_t argmax) {
    return R->argmax[c] == argmax && memcmp(R->codes + (int64_t)c * R->W, code, 8 * R->W) == 0;
}

static void hash_insert_index(orc_result *R, int64_t c) {
    uint64_t h = key_hash(R->codes + c * R->W, R->W, R->argmax[c]);
    int64_t i = (int64_t)(h & (uint64_t)(R->hcap - 1));
    while (R->htab[i] >= 0) i = (i + 1) & (R->hcap - 1);
    R->htab[i] = c;
}

static void grow_cells(orc_result *R) {
    if (R->n_cells < R->cap_cells) return;
    int64_t nc = R->cap_cells * 2;
    R->codes = (uint64_t *)realloc(R->codes, sizeof(uint64_t) * nc * R->W);
    R->argmax = (int32_t *)realloc(R->argmax, sizeof(int32_t) * nc);
    R->m = (int32_t *)realloc(R->m, sizeof(int32_t) * nc);
    R->fflags = (int32_t *)realloc(R->fflags, sizeof(int32_t) * nc);
    R->voff = (int64_t *)realloc(R->voff, sizeof(int64_t) * nc);
    R->cap_cells = nc;
}

/* Returns the index of (code, argmax), inserting it if unseen (*fresh = 1). */
static int64_t find_or_add(orc_result *R, const uint64_t *code, int32_t argmax, int *fresh) {
    uint64_t h = key_hash(code, R->W, argmax);
    int64_t i = (int64_t)(h & (uint64_t)(R->hcap - 1));
    while (R->htab[i] >= 0) {
        if (key_eq(R, R->htab[i], code, argmax)) { *fresh = 0; return R->htab[i]; }
        i = (i + 1) & (R->hcap - 1);
    }
    grow_cells(R);
    int64_t c = R->n_cells++;
    memcpy(R->codes + c * R->W, code, 8 * R->W);
    R->argmax[c] = argmax;
    R->m[c] = 0;
    R->fflags[c] = 0;
    R->voff[c] = -1;
    R->htab[i] = c;
    *fresh = 1;
    if (2 * R->n_cells > R->hcap) { /* keep the load factor <= 1/2 */
        free(R->htab);
        R->hcap *= 2;
        R->htab = (int64_t *)malloc(sizeof(int64_t) * R->hcap);
        for (int64_t k = 0; k < R->hcap; k++) R->htab[k] = -1;
        for (int64_t k = 0; k < R->n_cells; k++) hash_insert_index(R, k);
    }
    return c;
}

#define ORC_MAX_M 128

/* March from the given seed cells.  max_cells bounds the work (0 = none);
 * returns NULL on allocation failure. */
orc_result *orc_march(const orc_net *net, const uint64_t *seed_codes, const int32_t *seed_argmax,
                      int64_t n_seeds, int64_t max_cells) {
    orc_result *R = (orc_result *)calloc(1, sizeof(orc_result));
    R->W = orc_code_words(net);
    R->N = n_hidden(net);
    R->M = n_heads(net);
    R->cap_cells = 1024;
    R->codes = (uint64_t *)malloc(sizeof(uint64_t) * R->cap_cells * R->W);
    R->argmax = (int32_t *)malloc(sizeof(int32_t) * R->cap_cells);
    R->m = (int32_t *)malloc(sizeof(int32_t) * R->cap_cells);
    R->fflags = (int32_t *)malloc(sizeof(int32_t) * R->cap_cells);
    R->voff = (int64_t *)malloc(sizeof(int64_t) * R->cap_cells);
    R->cap_v = 4096;
    R->ids = (int32_t *)malloc(sizeof(int32_t) * R->cap_v);
    R->verts = (double *)malloc(sizeof(double) * 3 * R->cap_v);
    R->nbr = (int64_t *)malloc(sizeof(int64_t) * R->cap_v);
    R->hcap = 4096;
    R->htab = (int64_t *)malloc(sizeof(int64_t) * R->hcap);
    for (int64_t k = 0; k < R->hcap; k++) R->htab[k] = -1;
    R->n_seeds_in = n_seeds;

    for (int64_t s = 0; s < n_seeds; s++) {
        int fresh;
        find_or_add(R, seed_codes + s * R->W, seed_argmax[s], &fresh);
        if (!fresh) R->n_seed_dup++;
    }
    int64_t n_seed_cells = R->n_cells;

    double *rows = (double *)malloc(sizeof(double) * 4 * (R->N + R->M));
    int32_t ids[ORC_MAX_M];
    double verts[3 * ORC_MAX_M];
    uint64_t *ncode = (uint64_t *)malloc(8 * R->W);
    /* the active set is the tail of the cell list: FIFO order */
    for (int64_t c = 0; c < R->n_cells; c++) {
        if (max_cells > 0 && c >= max_cells) break;
        const uint64_t *code = R->codes + c * R->W;
        int32_t am = R->argmax[c];
        orc_chain(net, code, rows);
        double area;
        int32_t fl;
        int m = orc_face_from_rows(net, code, am, rows, ORC_MAX_M, ids, verts, &area, &fl);
        R->fflags[c] = fl;
        if (m == 0) {
            if (c < n_seed_cells) R->n_seed_empty++;
            else R->n_degenerate++;
            continue;
        }
        if (fl) R->n_degenerate++;
        while (R->n_v + m > R->cap_v) {
            R->cap_v *= 2;
            R->ids = (int32_t *)realloc(R->ids, sizeof(int32_t) * R->cap_v);
            R->verts = (double *)realloc(R->verts, sizeof(double) * 3 * R->cap_v);
            R->nbr = (int64_t *)realloc(R->nbr, sizeof(int64_t) * R->cap_v);
        }
        int64_t off = R->n_v;
        R->voff[c] = off;
        R->m[c] = m;
        R->n_v += m;
        for (int i = 0; i < m; i++) {
            R->ids[off + i] = ids[i];
            memcpy(R->verts + 3 * (off + i), verts + 3 * i, sizeof(double) * 3);
            int id = ids[i];
            if (id < 0) { R->nbr[off + i] = -1; continue; }
            /* re-read the code: find_or_add may have moved the arrays */
            memcpy(ncode, R->codes + c * R->W, 8 * R->W);
            int32_t nam = R->argmax[c];
            if (ORC_MUTATE == 8 && id < R->N) id ^= 1;
            if (id < R->N) ncode[id >> 6] ^= (uint64_t)1 << (id & 63);
            else nam = id - R->N;
            int fresh;
            R->nbr[off + i] = find_or_add(R, ncode, nam, &fresh);
        }
    }
    free(rows);
    free(ncode);
    return R;
}

/* The same march, with the faces of each batch of active cells computed in
 * parallel.  Algorithm 1 pops the active cells one at a time; the face of a
 * cell depends only on its code, and every cell of the batch [lo, hi) is
 * already in the list when the batch starts, so solving the batch first and
 * then appending faces and neighbours in cell order (as the one-at-a-time
 * loop does) gives the same cell ids, faces and adjacency.  Built without
 * OpenMP the pragmas are ignored and it runs on one thread.  batch <= 0 means
 * 16384 cells. */
orc_result *orc_march_batched(const orc_net *net, const uint64_t *seed_codes, const int32_t *seed_argmax,
                              int64_t n_seeds, int64_t max_cells, int64_t batch) {
    if (batch <= 0) batch = 16384;
    orc_result *R = (orc_result *)calloc(1, sizeof(orc_result));
    R->W = orc_code_words(net);
    R->N = n_hidden(net);
    R->M = n_heads(net);
    R->cap_cells = 1024;
    R->codes = (uint64_t *)malloc(sizeof(uint64_t) * R->cap_cells * R->W);
    R->argmax = (int32_t *)malloc(sizeof(int32_t) * R->cap_cells);
    R->m = (int32_t *)malloc(sizeof(int32_t) * R->cap_cells);
    R->fflags = (int32_t *)malloc(sizeof(int32_t) * R->cap_cells);
    R->voff = (int64_t *)malloc(sizeof(int64_t) * R->cap_cells);
    R->cap_v = 4096;
    R->ids = (int32_t *)malloc(sizeof(int32_t) * R->cap_v);
    R->verts = (double *)malloc(sizeof(double) * 3 * R->cap_v);
    R->nbr = (int64_t *)malloc(sizeof(int64_t) * R->cap_v);
    R->hcap = 4096;
    R->htab = (int64_t *)malloc(sizeof(int64_t) * R->hcap);
    for (int64_t k = 0; k < R->hcap; k++) R->htab[k] = -1;
    R->n_seeds_in = n_seeds;
    for (int64_t s = 0; s < n_seeds; s++) {
        int fresh;
        find_or_add(R, seed_codes + s * R->W, seed_argmax[s], &fresh);
        if (!fresh) R->n_seed_dup++;
    }
    int64_t n_seed_cells = R->n_cells;
    int32_t *bm = (int32_t *)malloc(sizeof(int32_t) * batch);
    int32_t *bfl = (int32_t *)malloc(sizeof(int32_t) * batch);
    int32_t *bids = (int32_t *)malloc(sizeof(int32_t) * batch * ORC_MAX_M);
    double *bverts = (double *)malloc(sizeof(double) * 3 * batch * ORC_MAX_M);
    uint64_t *ncode = (uint64_t *)malloc(8 * R->W);
    int64_t lo = 0;
    while (lo < R->n_cells) {
        int64_t hi = R->n_cells;
        if (hi - lo > batch) hi = lo + batch;
        if (max_cells > 0 && hi > max_cells) hi = max_cells;
        if (lo >= hi) break;
        /* faces of the batch: read-only access to R->codes (nothing is
         * inserted until the batch is solved) */
#pragma omp parallel
        {
            double *rows = (double *)malloc(sizeof(double) * 4 * (R->N + R->M));
#pragma omp for schedule(dynamic, 16)
            for (int64_t c = lo; c < hi; c++) {
                double area;
                int64_t b = c - lo;
                orc_chain(net, R->codes + c * R->W, rows);
                bm[b] = orc_face_from_rows(net, R->codes + c * R->W, R->argmax[c], rows, ORC_MAX_M,
                                           bids + b * ORC_MAX_M, bverts + 3 * b * ORC_MAX_M, &area, &bfl[b]);
            }
            free(rows);
        }
        /* append faces and neighbours in cell order */
        for (int64_t c = lo; c < hi; c++) {
            int64_t b = c - lo;
            int m = bm[b];
            R->fflags[c] = bfl[b];
            if (m == 0) {
                if (c < n_seed_cells) R->n_seed_empty++;
                else R->n_degenerate++;
                continue;
            }
            if (bfl[b]) R->n_degenerate++;
            while (R->n_v + m > R->cap_v) {
                R->cap_v *= 2;
                R->ids = (int32_t *)realloc(R->ids, sizeof(int32_t) * R->cap_v);
                R->verts = (double *)realloc(R->verts, sizeof(double) * 3 * R->cap_v);
                R->nbr = (int64_t *)realloc(R->nbr, sizeof(int64_t) * R->cap_v);
            }
            int64_t off = R->n_v;
            R->voff[c] = off;
            R->m[c] = m;
            R->n_v += m;
            for (int i = 0; i < m; i++) {
                int id = bids[b * ORC_MAX_M + i];
                R->ids[off + i] = id;
                memcpy(R->verts + 3 * (off + i), bverts + 3 * (b * ORC_MAX_M + i), sizeof(double) * 3);
                if (id < 0) { R->nbr[off + i] = -1; continue; }
                memcpy(ncode, R->codes + c * R->W, 8 * R->W);
                int32_t nam = R->argmax[c];
                if (id < R->N) ncode[id >> 6] ^= (uint64_t)1 << (id & 63);
                else nam = id - R->N;
                int fresh;
                R->nbr[off + i] = find_or_add(R, ncode, nam, &fresh);
            }
        }
        lo = hi;
    }
    free(bm); free(bfl); free(bids); free(bverts); free(ncode);
    return R;
}

/* Faces of n given cells (orc_face for each), in parallel when built with
 * OpenMP.  ids [n][max_m], verts [n][max_m][3], m [n], flags [n]. */
void orc_faces_batched(const orc_net *net, const uint64_t *codes, const int32_t *argmax, int64_t n, int max_m,
                       int32_t *m, int32_t *ids, double *verts, int32_t *flags) {
    int W = orc_code_words(net), NM = n_hidden(net) + n_heads(net);
#pragma omp parallel
    {
        double *rows = (double *)malloc(sizeof(double) * 4 * NM);
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < n; i++) {
            double area;
            orc_chain(net, codes + i * W, rows);
            m[i] = orc_face_from_rows(net, codes + i * W, argmax ? argmax[i] : 0, rows, max_m,
                                      ids + i * max_m, verts + 3 * i * max_m, &area, &flags[i]);
        }
        free(rows);
    }
}

/* Threads the batched routines use (1 when built without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_result_free(orc_result *R) {
    if (!R) return;
    free(R->codes); free(R->argmax); free(R->m); free(R->fflags); free(R->voff);
    free(R->ids); free(R->verts); free(R->nbr); free(R->htab);
    free(R);
}

/* counts: [faces, total face vertices, cells discovered, seeds_in, seed_dup,
 *          seed_empty, degenerate] */
void orc_result_counts(const orc_result *R, int64_t *out) {
    int64_t F = 0;
    for (int64_t c = 0; c < R->n_cells; c++) F += R->m[c] > 0;
    out[0] = F;
    out[1] = R->n_v;
    out[2] = R->n_cells;
    out[3] = R->n_seeds_in;
    out[4] = R->n_seed_dup;
    out[5] = R->n_seed_empty;
    out[6] = R->n_degenerate;
}

static const orc_result *g_sort_R;
static int cmp_cells(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    const uint64_t *ca = g_sort_R->codes + a * g_sort_R->W, *cb = g_sort_R->codes + b * g_sort_R->W;
    for (int i = 0; i < g_sort_R->W; i++)
        if (ca[i] != cb[i]) return ca[i] < cb[i] ? -1 : 1;
    int32_t x = g_sort_R->argmax[a], y = g_sort_R->argmax[b];
    return x < y ? -1 : (x > y);
}

/* Faces in canonical order.  offsets: F+1; ids, nbr: n_v; verts: 3 n_v;
 * codes: F x W; argmax: F.  nbr holds face indices (-1 = domain edge,
 * -2 = the neighbour cell has no face). */
void orc_result_fetch(const orc_result *R, int64_t *offsets, int32_t *ids, double *verts,
                      int64_t *nbr, uint64_t *codes, int32_t *argmax) {
    int64_t F = 0;
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (R->n_cells + 1));
    for (int64_t c = 0; c < R->n_cells; c++)
        if (R->m[c] > 0) order[F++] = c;
    g_sort_R = R;
    qsort(order, F, sizeof(int64_t), cmp_cells);
    int64_t *face_of = (int64_t *)malloc(sizeof(int64_t) * (R->n_cells + 1));
    for (int64_t c = 0; c < R->n_cells; c++) face_of[c] = -2;
    for (int64_t f = 0; f < F; f++) face_of[order[f]] = f;
    int64_t o = 0;
    for (int64_t f = 0; f < F; f++) {
        int64_t c = order[f];
        offsets[f] = o;
        memcpy(codes + f * R->W, R->codes + c * R->W, 8 * R->W);
        argmax[f] = R->argmax[c];
        for (int i = 0; i < R->m[c]; i++) {
            int64_t s = R->voff[c] + i;
            ids[o] = R->ids[s];
            memcpy(verts + 3 * o, R->verts + 3 * s, sizeof(double) * 3);
            nbr[o] = R->nbr[s] < 0 ? -1 : face_of[R->nbr[s]];
            o++;
        }
    }
    offsets[F] = o;
    free(order);
    free(face_of);
}
