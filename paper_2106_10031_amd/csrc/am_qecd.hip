// am_qecd.hip -- quadric edge-collapse simplification (Sec. 4.4) of a welded
// triangle mesh, in parallel rounds.
//
// Each vertex carries the quadric of the planes of its triangles (area
// weighted; Garland and Heckbert's error metric, which the paper adopts).
// An edge (a, b) costs v^T (Q_a + Q_b) v at the point v that minimises it
// (or the best of a, b and their midpoint when that system is singular).
// A round:
//   1. vertex -> triangle adjacency of the live triangles (count, scan, fill);
//   2. every collapsible edge (link condition, no flipped triangle) posts its
//      cost key (cost bits, edge id) to both endpoints with an atomic minimum;
//   3. an edge that is the minimum at both endpoints (listed once, by its
//      first end) claims every vertex of the triangles around a and b
//      (atomic minimum of its key);
//   4. an edge that holds all its claims owns that neighbourhood: it checks
//      again that it is collapsible, takes a ticket from the round's budget,
//      collapses b into a at v, and locks the neighbourhood;
//   5. steps 3-4 repeat (kClaimPasses in all) among the candidates whose
//      neighbourhoods hold no locked vertex: a vertex that is not locked has
//      the same triangles, position and quadric as at the start of the round,
//      so its adjacency and edge keys are still exact.
// Neighbourhoods of committed collapses are disjoint, so their updates do not
// race.  Vertices flagged as boundary never move.  Rounds repeat until the
// live triangle count reaches the target, nothing collapses, or max_rounds.
// Whenever fewer than half the rows in use hold live triangles, the live ones
// are compacted (in order) so that later rounds scan fewer rows.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "am_internal.h"

namespace am {

namespace {

unsigned qblocks(long long n) {
    long long b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return (unsigned)b;
}

// symmetric 4x4 quadric, 10 entries: q00 q01 q02 q03 q11 q12 q13 q22 q23 q33
__device__ __forceinline__ double quad_eval(const double q[10], const double v[3]) {
    const double x = v[0], y = v[1], z = v[2];
    return q[0] * x * x + 2 * q[1] * x * y + 2 * q[2] * x * z + 2 * q[3] * x + q[4] * y * y + 2 * q[5] * y * z +
           2 * q[6] * y + q[7] * z * z + 2 * q[8] * z + q[9];
}

__global__ void k_q_init(const double *vin, long long V, double *pos, double *Q, int *rep) {
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V;
         v += (long long)gridDim.x * blockDim.x) {
        pos[v * 3] = vin[v * 3];
        pos[v * 3 + 1] = vin[v * 3 + 1];
        pos[v * 3 + 2] = vin[v * 3 + 2];
        for (int k = 0; k < 10; ++k) Q[v * 10 + k] = 0.0;
        rep[v] = (int)v;
    }
}

__device__ void tri_normal(const double *pos, int a, int b, int c, double n[3]) {
    const double ux = pos[b * 3] - pos[a * 3], uy = pos[b * 3 + 1] - pos[a * 3 + 1], uz = pos[b * 3 + 2] - pos[a * 3 + 2];
    const double wx = pos[c * 3] - pos[a * 3], wy = pos[c * 3 + 1] - pos[a * 3 + 1], wz = pos[c * 3 + 2] - pos[a * 3 + 2];
    n[0] = uy * wz - uz * wy;
    n[1] = uz * wx - ux * wz;
    n[2] = ux * wy - uy * wx;
}

__global__ void k_q_accumulate(const int *tri, const unsigned char *tlive, long long T, const double *pos,
                               double *Q) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < T;
         t += (long long)gridDim.x * blockDim.x) {
        if (!tlive[t]) continue;
        const int a = tri[t * 3], b = tri[t * 3 + 1], c = tri[t * 3 + 2];
        double n[3];
        tri_normal(pos, a, b, c, n);
        const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(len > 0.0)) continue;
        const double w = 0.5 * len;   // triangle area
        const double p[4] = {n[0] / len, n[1] / len, n[2] / len,
                             -(n[0] * pos[a * 3] + n[1] * pos[a * 3 + 1] + n[2] * pos[a * 3 + 2]) / len};
        const double k[10] = {p[0] * p[0], p[0] * p[1], p[0] * p[2], p[0] * p[3], p[1] * p[1],
                              p[1] * p[2], p[1] * p[3], p[2] * p[2], p[2] * p[3], p[3] * p[3]};
        const int vs[3] = {a, b, c};
        for (int j = 0; j < 3; ++j)
            for (int e = 0; e < 10; ++e) atomicAdd(&Q[(long long)vs[j] * 10 + e], w * k[e]);
    }
}

// Placement and cost of collapsing edge (a, b).
__device__ double edge_cost(const double *pos, const double *Q, int a, int b, double out[3]) {
    double q[10];
    for (int e = 0; e < 10; ++e) q[e] = Q[(long long)a * 10 + e] + Q[(long long)b * 10 + e];
    const double pa[3] = {pos[a * 3], pos[a * 3 + 1], pos[a * 3 + 2]};
    const double pb[3] = {pos[b * 3], pos[b * 3 + 1], pos[b * 3 + 2]};
    // minimiser of the quadric: [q00 q01 q02; q01 q11 q12; q02 q12 q22] v = -[q03 q13 q23]
    const double A00 = q[0], A01 = q[1], A02 = q[2], A11 = q[4], A12 = q[5], A22 = q[7];
    const double r0 = -q[3], r1 = -q[6], r2 = -q[8];
    const double c00 = A11 * A22 - A12 * A12, c01 = A02 * A12 - A01 * A22, c02 = A01 * A12 - A02 * A11;
    const double det = A00 * c00 + A01 * c01 + A02 * c02;
    const double scale = fabs(A00) + fabs(A11) + fabs(A22);
    double best = 1e300;
    if (fabs(det) > 1e-10 * scale * scale * scale && scale > 0.0) {
        const double c11 = A00 * A22 - A02 * A02, c12 = A01 * A02 - A00 * A12, c22 = A00 * A11 - A01 * A01;
        const double v[3] = {(c00 * r0 + c01 * r1 + c02 * r2) / det, (c01 * r0 + c11 * r1 + c12 * r2) / det,
                             (c02 * r0 + c12 * r1 + c22 * r2) / det};
        // keep the optimum only near the edge (a far optimum means a near-flat quadric)
        const double ex = pb[0] - pa[0], ey = pb[1] - pa[1], ez = pb[2] - pa[2];
        const double el = sqrt(ex * ex + ey * ey + ez * ez);
        const double mx = 0.5 * (pa[0] + pb[0]), my = 0.5 * (pa[1] + pb[1]), mz = 0.5 * (pa[2] + pb[2]);
        const double dm = sqrt((v[0] - mx) * (v[0] - mx) + (v[1] - my) * (v[1] - my) + (v[2] - mz) * (v[2] - mz));
        if (dm <= 2.0 * el) {
            best = fmax(quad_eval(q, v), 0.0);
            out[0] = v[0];
            out[1] = v[1];
            out[2] = v[2];
        }
    }
    const double cand[3][3] = {{pa[0], pa[1], pa[2]}, {pb[0], pb[1], pb[2]},
                               {0.5 * (pa[0] + pb[0]), 0.5 * (pa[1] + pb[1]), 0.5 * (pa[2] + pb[2])}};
    for (int i = 0; i < 3; ++i) {
        const double c = fmax(quad_eval(q, cand[i]), 0.0);
        if (c < best) {
            best = c;
            out[0] = cand[i][0];
            out[1] = cand[i][1];
            out[2] = cand[i][2];
        }
    }
    return best;
}

__device__ __forceinline__ unsigned long long edge_key(double cost, long long e) {
    const float c = (float)fmin(cost, 3.0e38);
    return ((unsigned long long)__float_as_uint(c) << 32) | (unsigned long long)(unsigned)e;
}

__global__ void k_adj_count(const int *tri, const unsigned char *tlive, long long T, int *cnt) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < T;
         t += (long long)gridDim.x * blockDim.x) {
        if (!tlive[t]) continue;
        for (int k = 0; k < 3; ++k) atomicAdd(&cnt[tri[t * 3 + k]], 1);
    }
}

__global__ void k_adj_fill(const int *tri, const unsigned char *tlive, long long T, const int *off, int *cur,
                           int *adj) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < T;
         t += (long long)gridDim.x * blockDim.x) {
        if (!tlive[t]) continue;
        for (int k = 0; k < 3; ++k) {
            const int v = tri[t * 3 + k];
            adj[off[v] + atomicAdd(&cur[v], 1)] = (int)t;
        }
    }
}

__global__ void k_fill_u64(unsigned long long *p, long long n, unsigned long long v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_uchar(unsigned char *p, long long n, unsigned char v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_int(int *p, long long n, int v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Link condition (a and b share exactly two neighbours and two triangles)
// and no surviving triangle around a or b turning by more than about 78
// degrees or collapsing, when a and b move to v.
__device__ bool edge_valid(const int *tri, const int *adj_off, const int *adj, const double *pos, int a, int b,
                       const double v[3]) {
    // link condition: a and b have exactly two common neighbours, and
    // exactly two triangles contain both (the edge is manifold)
    int common = 0, shared = 0;
    for (int i = adj_off[a]; i < adj_off[a + 1]; ++i) {
        const int ta = adj[i];
        const int x0 = tri[ta * 3], x1 = tri[ta * 3 + 1], x2 = tri[ta * 3 + 2];
        if (x0 == b || x1 == b || x2 == b) ++shared;
    }
    for (int i = adj_off[a]; i < adj_off[a + 1]; ++i) {
        const int ta = adj[i];
        for (int ca = 0; ca < 3; ++ca) {
            const int w = tri[ta * 3 + ca];
            if (w == a || w == b) continue;
            // count w once: only at its first occurrence around a
            bool first = true;
            for (int i2 = adj_off[a]; i2 < i && first; ++i2) {
                const int tb = adj[i2];
                if (tri[tb * 3] == w || tri[tb * 3 + 1] == w || tri[tb * 3 + 2] == w) first = false;
            }
            for (int c2 = 0; c2 < ca && first; ++c2)
                if (tri[ta * 3 + c2] == w) first = false;
            if (!first) continue;
            bool in_b = false;
            for (int j = adj_off[b]; j < adj_off[b + 1] && !in_b; ++j) {
                const int tb = adj[j];
                in_b = tri[tb * 3] == w || tri[tb * 3 + 1] == w || tri[tb * 3 + 2] == w;
            }
            common += in_b ? 1 : 0;
        }
    }
    if (shared != 2 || common != 2) return false;
    // no surviving triangle around a or b may flip or collapse to nothing
    bool ok = true;
    for (int side = 0; side < 2 && ok; ++side) {
        const int s = side ? b : a;
        for (int i = adj_off[s]; i < adj_off[s + 1] && ok; ++i) {
            const int tt = adj[i];
            int c[3] = {tri[tt * 3], tri[tt * 3 + 1], tri[tt * 3 + 2]};
            if ((c[0] == a || c[1] == a || c[2] == a) && (c[0] == b || c[1] == b || c[2] == b)) continue;
            double n0[3];
            tri_normal(pos, c[0], c[1], c[2], n0);
            double p[3][3];
            for (int j = 0; j < 3; ++j)
                for (int d = 0; d < 3; ++d) p[j][d] = (c[j] == a || c[j] == b) ? v[d] : pos[c[j] * 3 + d];
            const double u0 = p[1][0] - p[0][0], u1 = p[1][1] - p[0][1], u2 = p[1][2] - p[0][2];
            const double w0 = p[2][0] - p[0][0], w1 = p[2][1] - p[0][1], w2 = p[2][2] - p[0][2];
            const double n1[3] = {u1 * w2 - u2 * w1, u2 * w0 - u0 * w2, u0 * w1 - u1 * w0};
            const double l0 = sqrt(n0[0] * n0[0] + n0[1] * n0[1] + n0[2] * n0[2]);
            const double l1 = sqrt(n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2]);
            const double dp = n0[0] * n1[0] + n0[1] * n1[1] + n0[2] * n1[2];
            if (!(l1 > 1e-12 * l0) || !(dp > 0.2 * l0 * l1)) ok = false;
        }
    }
    return ok;
}

__global__ void k_edge_min(const int *tri, const unsigned char *tlive, long long T, const double *pos,
                           const double *Q, const unsigned char *boundary, const int *adj_off, const int *adj,
                           unsigned long long *vmin) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < T * 3;
         e += (long long)gridDim.x * blockDim.x) {
        const long long t = e / 3;
        const int k = (int)(e - t * 3);
        if (!tlive[t]) continue;
        const int a = tri[t * 3 + k], b = tri[t * 3 + (k + 1) % 3];
        if (a >= b) continue;   // each edge once per triangle pair orientation
        if (boundary && (boundary[a] || boundary[b])) continue;
        double v[3];
        const unsigned long long key = edge_key(edge_cost(pos, Q, a, b, v), e);
        // minima only fall and keys are unique: a key above both current minima
        // can never be the minimum at either end, so it needs no validity check
        if (key > vmin[a] && key > vmin[b]) continue;
        // only collapsible edges compete, so an invalid cheapest edge cannot block a vertex
        if (!edge_valid(tri, adj_off, adj, pos, a, b, v)) continue;
        atomicMin(&vmin[a], key);
        atomicMin(&vmin[b], key);
    }
}

// Calls f(w) for every vertex of every triangle around vertex v.
template <class Fn>
__device__ void for_ring(const int *tri, const int *adj_off, const int *adj, int v, Fn f) {
    for (int i = adj_off[v]; i < adj_off[v + 1]; ++i) {
        const int t = adj[i];
        f(tri[t * 3]);
        f(tri[t * 3 + 1]);
        f(tri[t * 3 + 2]);
    }
}

constexpr int kClaimPasses = 3;

// Candidates of the round: the edge e named by vertex a's minimum, when a is
// the edge's first end and the edge is the minimum at its other end too.
// Each vertex adds at most one edge, so the list holds at most V entries.
__global__ void k_cand_list(const unsigned long long *vmin, long long V, const int *tri, long long T, int *cand,
                            unsigned long long *n_cand) {
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V;
         v += (long long)gridDim.x * blockDim.x) {
        const unsigned long long key = vmin[v];
        if (key == ~0ull) continue;
        const long long e = (long long)(unsigned)key;
        if (e >= 3 * T) continue;
        const long long t = e / 3;
        const int k = (int)(e - t * 3);
        const int a = tri[t * 3 + k], b = tri[t * 3 + (k + 1) % 3];
        if (a != v || vmin[b] != key) continue;
        cand[atomicAdd(n_cand, 1ull)] = (int)e;
    }
}

__global__ void k_edge_claim(const int *tri, const unsigned char *tlive, long long T, const double *pos,
                             const double *Q, const unsigned char *boundary, const unsigned long long *vmin,
                             const int *adj_off, const int *adj, const unsigned char *lock, const int *cand,
                             const unsigned long long *n_cand, unsigned long long *claim) {
    const long long nc = (long long)*n_cand;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nc;
         i += (long long)gridDim.x * blockDim.x) {
        const long long e = cand[i];
        if (e >= 3 * T) continue;
        const long long t = e / 3;
        const int k = (int)(e - t * 3);
        if (!tlive[t]) continue;
        const int a = tri[t * 3 + k], b = tri[t * 3 + (k + 1) % 3];
        if (a >= b) continue;
        if (boundary && (boundary[a] || boundary[b])) continue;
        // a candidate's key (edge id in the low word) is the minimum at both ends
        const unsigned long long va = vmin[a];
        if ((unsigned)va != (unsigned)e || vmin[b] != va) continue;
        double v[3];
        const unsigned long long key = edge_key(edge_cost(pos, Q, a, b, v), e);
        if (va != key) continue;
        bool free = true;
        auto unlocked = [&](int w) { free = free && !lock[w]; };
        for_ring(tri, adj_off, adj, a, unlocked);
        for_ring(tri, adj_off, adj, b, unlocked);
        if (!free) continue;
        auto mark = [&](int w) { atomicMin(&claim[w], key); };
        for_ring(tri, adj_off, adj, a, mark);
        for_ring(tri, adj_off, adj, b, mark);
    }
}

__global__ void k_edge_collapse(int *tri, unsigned char *tlive, long long T, double *pos, double *Q,
                                const unsigned char *boundary, const unsigned long long *vmin, const int *adj_off,
                                const int *adj, const unsigned long long *claim, int *rep,
                                unsigned char *lock, const int *cand, const unsigned long long *n_cand,
                                unsigned long long *tickets, unsigned long long budget,
                                unsigned long long *removed) {
    const long long nc = (long long)*n_cand;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nc;
         i += (long long)gridDim.x * blockDim.x) {
        const long long e = cand[i];
        if (e >= 3 * T) continue;
        const long long t = e / 3;
        const int k = (int)(e - t * 3);
        if (!tlive[t]) continue;
        const int a = tri[t * 3 + k], b = tri[t * 3 + (k + 1) % 3];
        if (a >= b) continue;
        if (boundary && (boundary[a] || boundary[b])) continue;
        // a candidate's key (edge id in the low word) is the minimum at both ends
        const unsigned long long va = vmin[a];
        if ((unsigned)va != (unsigned)e || vmin[b] != va) continue;
        double v[3];
        const unsigned long long key = edge_key(edge_cost(pos, Q, a, b, v), e);
        if (va != key) continue;
        bool own = true;
        auto check = [&](int w) { own = own && claim[w] == key && !lock[w]; };
        for_ring(tri, adj_off, adj, a, check);
        for_ring(tri, adj_off, adj, b, check);
        if (!own) continue;
        if (!edge_valid(tri, adj_off, adj, pos, a, b, v)) continue;
        if (atomicAdd(tickets, 1ull) >= budget) continue;
        // lock the neighbourhood for the round's later passes
        auto take = [&](int w) { lock[w] = 1; };
        for_ring(tri, adj_off, adj, a, take);
        for_ring(tri, adj_off, adj, b, take);
        // collapse b into a at v (the neighbourhood is this edge's alone)
        pos[a * 3] = v[0];
        pos[a * 3 + 1] = v[1];
        pos[a * 3 + 2] = v[2];
        for (int q = 0; q < 10; ++q) Q[(long long)a * 10 + q] += Q[(long long)b * 10 + q];
        rep[b] = a;
        for (int i = adj_off[b]; i < adj_off[b + 1]; ++i) {
            const int tt = adj[i];
            int *c = tri + tt * 3;
            const bool has_a = c[0] == a || c[1] == a || c[2] == a;
            if (has_a) {
                tlive[tt] = 0;
                atomicAdd(removed, 1ull);
            } else {
                for (int j = 0; j < 3; ++j)
                    if (c[j] == b) c[j] = a;
            }
        }
    }
}

// Compaction: vertex flags for live triangles, then renumbering.
__global__ void k_vert_used(const int *tri, const unsigned char *tlive, long long T, int *used) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < T;
         t += (long long)gridDim.x * blockDim.x) {
        if (!tlive[t]) continue;
        for (int k = 0; k < 3; ++k) used[tri[t * 3 + k]] = 1;
    }
}

__global__ void k_tri_flags(const unsigned char *tlive, long long T, int *f) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < T;
         t += (long long)gridDim.x * blockDim.x)
        f[t] = tlive[t] ? 1 : 0;
}

__global__ void k_compact(const int *tri, const unsigned char *tlive, long long T, const int *tidx,
                          const int *used, const int *vidx, long long V, const double *pos, long long *tri_out,
                          double *v_out) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < T;
         t += (long long)gridDim.x * blockDim.x) {
        if (!tlive[t]) continue;
        const long long o = tidx[t];
        for (int k = 0; k < 3; ++k) tri_out[o * 3 + k] = vidx[tri[t * 3 + k]];
    }
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V;
         v += (long long)gridDim.x * blockDim.x) {
        if (!used[v]) continue;
        const long long o = vidx[v];
        v_out[o * 3] = pos[v * 3];
        v_out[o * 3 + 1] = pos[v * 3 + 1];
        v_out[o * 3 + 2] = pos[v * 3 + 2];
    }
}

// Stable compaction of the live triangles: triangle t goes to row tidx[t].
__global__ void k_tri_compact(const int *tri, const unsigned char *tlive, long long T, const int *tidx, int *tri2) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < T;
         t += (long long)gridDim.x * blockDim.x) {
        if (!tlive[t]) continue;
        const long long o = tidx[t];
        tri2[o * 3] = tri[t * 3];
        tri2[o * 3 + 1] = tri[t * 3 + 1];
        tri2[o * 3 + 2] = tri[t * 3 + 2];
    }
}

__global__ void k_tri_load(const long long *tri_in, long long T, long long V, int *tri, unsigned char *tlive,
                           unsigned long long *bad) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < T;
         t += (long long)gridDim.x * blockDim.x) {
        bool ok = true;
        for (int k = 0; k < 3; ++k) {
            const long long v = tri_in[t * 3 + k];
            ok = ok && v >= 0 && v < V;
            tri[t * 3 + k] = ok ? (int)v : 0;
        }
        ok = ok && tri[t * 3] != tri[t * 3 + 1] && tri[t * 3 + 1] != tri[t * 3 + 2] && tri[t * 3] != tri[t * 3 + 2];
        tlive[t] = ok ? 1 : 0;
        if (!ok) atomicAdd(bad, 1ull);
    }
}

}  // namespace

// Device scratch the simplification needs for V vertices and T triangles.
size_t qecd_scratch_bytes(long long V, long long T) {
    size_t scan = 0, s2 = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (int *)nullptr, (int *)nullptr, (int)(V + 1));
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, s2, (int *)nullptr, (int *)nullptr, (int)(T > V ? T : V));
    if (s2 > scan) scan = s2;
    const size_t v = (size_t)V + 1, t = (size_t)T;
    // 21 carved arrays, each padded to 256 bytes; 165 B per vertex, 52 per triangle
    return 256 * 32 + v * 165 + t * 52 + scan;
}

struct QecdScratch {
    double *pos, *Q;
    int *rep, *tri, *tri2, *cand, *cnt, *off, *cur, *adj, *tflag, *tidx, *used, *vidx;
    unsigned char *tlive, *lock;
    unsigned long long *vmin, *claim, *ctr;   // ctr: [0] tickets, [1] removed, [2] bad input, [3] candidates
    void *scan;
    size_t scan_bytes;
};

static QecdScratch carve(void *base, long long V, long long T, size_t scan_bytes) {
    char *p = (char *)base;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += (bytes + 255) & ~(size_t)255;
        return (void *)q;
    };
    QecdScratch s;
    s.ctr = (unsigned long long *)take(8 * 8);
    s.pos = (double *)take(sizeof(double) * 3 * V);
    s.Q = (double *)take(sizeof(double) * 10 * V);
    s.rep = (int *)take(sizeof(int) * V);
    s.cand = (int *)take(sizeof(int) * V);
    s.vmin = (unsigned long long *)take(8 * V);
    s.claim = (unsigned long long *)take(8 * V);
    s.cnt = (int *)take(sizeof(int) * (V + 1));
    s.off = (int *)take(sizeof(int) * (V + 1));
    s.cur = (int *)take(sizeof(int) * V);
    s.used = (int *)take(sizeof(int) * V);
    s.vidx = (int *)take(sizeof(int) * V);
    s.tri = (int *)take(sizeof(int) * 3 * T);
    s.tri2 = (int *)take(sizeof(int) * 3 * T);
    s.tlive = (unsigned char *)take(T);
    s.lock = (unsigned char *)take(V);
    s.adj = (int *)take(sizeof(int) * 3 * T);
    s.tflag = (int *)take(sizeof(int) * T);
    s.tidx = (int *)take(sizeof(int) * T);
    s.scan = take(scan_bytes);
    s.scan_bytes = scan_bytes;
    return s;
}

// Simplifies (vin [V][3], tri_in [T][3]) towards target_tris triangles.  out:
// v_out [<= V][3], tri_out [<= T][3]; *V_out, *T_out, *rounds, *bad (input
// triangles out of range or degenerate, dropped).  Synchronises (the host
// reads the live count after each round).
hipError_t run_qecd(const double *vin, long long V, const long long *tri_in, long long T,
                    const unsigned char *boundary, long long target_tris, int max_rounds, void *scratch,
                    double *v_out, long long *tri_out, long long *V_out, long long *T_out, int *rounds_out,
                    long long *bad_out, hipStream_t st) {
    size_t scan = 0, s2 = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (int *)nullptr, (int *)nullptr, (int)(V + 1));
    if (e != hipSuccess) return e;
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, s2, (int *)nullptr, (int *)nullptr, (int)(T > V ? T : V));
    if (e != hipSuccess) return e;
    if (s2 > scan) scan = s2;
    QecdScratch s = carve(scratch, V, T, scan);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, s.ctr, 8, 0ull);
    hipLaunchKernelGGL(k_q_init, dim3(qblocks(V)), dim3(256), 0, st, vin, V, s.pos, s.Q, s.rep);
    hipLaunchKernelGGL(k_tri_load, dim3(qblocks(T)), dim3(256), 0, st, tri_in, T, V, s.tri, s.tlive, s.ctr + 2);
    hipLaunchKernelGGL(k_q_accumulate, dim3(qblocks(T)), dim3(256), 0, st, s.tri, s.tlive, T, s.pos, s.Q);
    unsigned long long h[3] = {0, 0, 0};
    e = hipMemcpyAsync(h, s.ctr, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    long long live = T - (long long)h[2];
    *bad_out = (long long)h[2];
    int rounds = 0;
    long long Tc = T;   // rows of tri / tlive in use
    while (live > target_tris && rounds < max_rounds) {
        if (live < Tc / 2) {
            // drop dead triangles (stable), so that later rounds scan fewer rows
            hipLaunchKernelGGL(k_tri_flags, dim3(qblocks(Tc)), dim3(256), 0, st, s.tlive, Tc, s.tflag);
            size_t cb = s.scan_bytes;
            e = hipcub::DeviceScan::ExclusiveSum(s.scan, cb, s.tflag, s.tidx, (int)Tc, st);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_tri_compact, dim3(qblocks(Tc)), dim3(256), 0, st, s.tri, s.tlive, Tc, s.tidx,
                               s.tri2);
            int last[2] = {0, 0};
            e = hipMemcpyAsync(&last[0], s.tidx + Tc - 1, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) return e;
            e = hipMemcpyAsync(&last[1], s.tflag + Tc - 1, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) return e;
            e = hipStreamSynchronize(st);
            if (e != hipSuccess) return e;
            const long long n = (long long)last[0] + last[1];
            if (n > 0) {
                e = hipMemcpyAsync(s.tri, s.tri2, sizeof(int) * 3 * (size_t)n, hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(k_fill_uchar, dim3(qblocks(n)), dim3(256), 0, st, s.tlive, n, (unsigned char)1);
            Tc = n;
            live = n;
        }
        // adjacency of the live triangles
        hipLaunchKernelGGL(k_fill_int, dim3(qblocks(V + 1)), dim3(256), 0, st, s.cnt, V + 1, 0);
        hipLaunchKernelGGL(k_fill_int, dim3(qblocks(V)), dim3(256), 0, st, s.cur, V, 0);
        hipLaunchKernelGGL(k_adj_count, dim3(qblocks(Tc)), dim3(256), 0, st, s.tri, s.tlive, Tc, s.cnt);
        size_t tb = s.scan_bytes;
        e = hipcub::DeviceScan::ExclusiveSum(s.scan, tb, s.cnt, s.off, (int)(V + 1), st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_adj_fill, dim3(qblocks(Tc)), dim3(256), 0, st, s.tri, s.tlive, Tc, s.off, s.cur, s.adj);
        // costs, local minima, claims, collapses
        hipLaunchKernelGGL(k_fill_u64, dim3(qblocks(V)), dim3(256), 0, st, s.vmin, V, ~0ull);
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, s.ctr, 2, 0ull);
        hipLaunchKernelGGL(k_fill_uchar, dim3(qblocks(V)), dim3(256), 0, st, s.lock, V, (unsigned char)0);
        hipLaunchKernelGGL(k_edge_min, dim3(qblocks(3 * Tc)), dim3(256), 0, st, s.tri, s.tlive, Tc, s.pos, s.Q,
                           boundary, s.off, s.adj, s.vmin);
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, s.ctr + 3, 1, 0ull);
        hipLaunchKernelGGL(k_cand_list, dim3(qblocks(V)), dim3(256), 0, st, s.vmin, V, s.tri, Tc, s.cand,
                           s.ctr + 3);
        const unsigned long long budget = (unsigned long long)((live - target_tris + 1) / 2);
        for (int pass = 0; pass < kClaimPasses; ++pass) {
            hipLaunchKernelGGL(k_fill_u64, dim3(qblocks(V)), dim3(256), 0, st, s.claim, V, ~0ull);
            hipLaunchKernelGGL(k_edge_claim, dim3(qblocks(V)), dim3(256), 0, st, s.tri, s.tlive, Tc, s.pos, s.Q,
                               boundary, s.vmin, s.off, s.adj, s.lock, s.cand, s.ctr + 3, s.claim);
            hipLaunchKernelGGL(k_edge_collapse, dim3(qblocks(V)), dim3(256), 0, st, s.tri, s.tlive, Tc, s.pos,
                               s.Q, boundary, s.vmin, s.off, s.adj, s.claim, s.rep, s.lock, s.cand, s.ctr + 3,
                               s.ctr, budget, s.ctr + 1);
        }
        e = hipMemcpyAsync(h, s.ctr, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        ++rounds;
        if (h[1] == 0) break;   // nothing collapsed: stuck
        live -= (long long)h[1];
    }
    // compaction
    hipLaunchKernelGGL(k_fill_int, dim3(qblocks(V)), dim3(256), 0, st, s.used, V, 0);
    hipLaunchKernelGGL(k_vert_used, dim3(qblocks(Tc)), dim3(256), 0, st, s.tri, s.tlive, Tc, s.used);
    size_t tb = s.scan_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(s.scan, tb, s.used, s.vidx, (int)V, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tri_flags, dim3(qblocks(Tc)), dim3(256), 0, st, s.tlive, Tc, s.tflag);
    tb = s.scan_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(s.scan, tb, s.tflag, s.tidx, (int)Tc, st);
    if (e != hipSuccess) return e;
    long long VT = V > Tc ? V : Tc;
    hipLaunchKernelGGL(k_compact, dim3(qblocks(VT)), dim3(256), 0, st, s.tri, s.tlive, Tc, s.tidx, s.used, s.vidx, V,
                       s.pos, tri_out, v_out);
    int tail[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(&tail[0], s.vidx + V - 1, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&tail[1], s.used + V - 1, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    if (Tc > 0) {
        e = hipMemcpyAsync(&tail[2], s.tidx + Tc - 1, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(&tail[3], s.tflag + Tc - 1, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    *V_out = (long long)tail[0] + tail[1];
    *T_out = (long long)tail[2] + tail[3];
    *rounds_out = rounds;
    return hipGetLastError();
}

}  // namespace am
