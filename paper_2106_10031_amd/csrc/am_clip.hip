// am_clip.hip -- analytic face of each cell by halfplane clipping (gfx950).
//
// The face of a cell (Eqn (AnalyticFace)) is the part of the zero plane
// a_F . [x;1] = 0 where every oriented constraint (1 - 2 s_k) a_k . [x;1] <= 0
// holds (Eqn (AnalyticCellSystem)), plus the max-pool sub-cell rows
// (a_F(i) - a_F(j)) . [x;1] <= 0 of Eqn (AnalyticCellSystemMaxPooling), inside
// the domain box.  Instead of the paper's pair enumeration (Algorithm 1) or
// pivoting (Sec. 4.2.1), one wave clips a polygon in a 2-D frame of the plane:
//   * lane i holds vertex i (frame coordinates, id of the edge it starts);
//   * constraints are tested 64 at a time, one per lane, against every
//     vertex (broadcast with readlane); only the lines that cut are applied;
//   * a cut is one Sutherland-Hodgman pass: each lane emits 0-2 vertices,
//     positions come from two ballots and a popcount (wave compaction), the
//     new polygon goes through the wave's LDS scratch.
// Vertices are then recomputed in FP64 from their two edge ids and the plane
// (Eqn (VertexEquationSystem)), and each edge on a hidden unit or head
// comparison becomes a neighbour candidate (state flip, Sec. 3.1).
#include "am_internal.h"

namespace am {

struct PolyScratch {
    double a[kMaxPoly];
    double b[kMaxPoly];
    double r[kMaxPoly];
    int e[kMaxPoly];
};

struct Poly {
    double a, b;   // this lane's vertex in the plane frame
    double r;      // 1 + |(a, b)|, the vertex scale of the on-line tolerance
    int e;         // id of the edge starting at this vertex
    int m;         // vertex count (uniform)
};

enum : int { kFlagEmpty = 1, kFlagDegen = 2, kFlagSingular = 4, kFlagTooBig = 8 };

// One Sutherland-Hodgman pass with the halfplane cu a + cv b + cw <= 0 (id).
// Returns false when the polygon has no interior left.
__device__ bool sh_clip(Poly &P, double cu, double cv, double cw, int id, PolyScratch &s, int &flags) {
    const int lane = lane_id();
    const bool act = lane < P.m;
    const double nrm = sqrt(cu * cu + cv * cv);
    const double d = cu * P.a + cv * P.b + cw;
    const double tol = kTau * (nrm * P.r + fabs(cw));
    const int cls = !act ? 0 : (d > tol ? 1 : (d < -tol ? -1 : 0));
    const uint64_t outm = ballot(act && cls == 1);
    if (!outm) return true;
    const uint64_t inm = ballot(act && cls == -1);
    if (!inm) {
        P.m = 0;
        return false;
    }
    const int j = (lane + 1 >= P.m) ? 0 : lane + 1;
    const double ja = shfl(P.a, j), jb = shfl(P.b, j), jd = shfl(d, j);
    const int jc = shfl(cls, j);
    const bool c1 = act && cls != 1;
    const bool c2 = act && ((cls == -1 && jc == 1) || (cls == 1 && jc == -1));
    const uint64_t b1 = ballot(c1), b2 = ballot(c2);
    const uint64_t lt = lanemask_lt();
    const int pos = __popcll(b1 & lt) + __popcll(b2 & lt);
    const int nm = __popcll(b1) + __popcll(b2);
    if (nm > kMaxPoly) {
        flags |= kFlagTooBig;
        P.m = 0;
        return false;
    }
    if (c1) {
        s.a[pos] = P.a;
        s.b[pos] = P.b;
        s.r[pos] = P.r;
        s.e[pos] = (cls == 0 && jc == 1) ? id : P.e;
    }
    if (c2) {
        const double t = d / (d - jd);
        const double xa = P.a + t * (ja - P.a);
        const double xb = P.b + t * (jb - P.b);
        const int p2 = pos + (c1 ? 1 : 0);
        s.a[p2] = xa;
        s.b[p2] = xb;
        s.r[p2] = 1.0 + sqrt(xa * xa + xb * xb);
        s.e[p2] = (cls == -1) ? id : P.e;
    }
    wave_lds_sync();
    P.m = nm;
    if (lane < nm) {
        P.a = s.a[lane];
        P.b = s.b[lane];
        P.r = s.r[lane];
        P.e = s.e[lane];
    }
    wave_lds_sync();
    return true;
}

// Oriented constraint row of id (feasible side <= 0).
__device__ __forceinline__ void constraint_row(const DevNet &net, int id, const uint64_t *code, int am,
                                               const double *crow, double c[4]) {
    if (id < 0) {
        const int t = -id - 1;
        const int ax = t >> 1;
        c[0] = c[1] = c[2] = 0.0;
        c[ax] = (t & 1) ? -1.0 : 1.0;
        c[3] = -1.0;
    } else if (id < net.N) {
        const double *z = crow + (long long)net.row_of_unit[id] * 4;
        const double sg = code_bit(code, id) ? -1.0 : 1.0;
        c[0] = sg * z[0];
        c[1] = sg * z[1];
        c[2] = sg * z[2];
        c[3] = sg * z[3];
    } else {
        const double *zi = crow + (long long)net.row_of_unit[id] * 4;
        const double *zj = crow + (long long)net.row_of_unit[net.N + am] * 4;
        c[0] = zi[0] - zj[0];
        c[1] = zi[1] - zj[1];
        c[2] = zi[2] - zj[2];
        c[3] = zi[3] - zj[3];
    }
}

// Solves A x = r (3x3) by elimination with row pivoting; false if singular.
__device__ bool solve3(double A[3][3], double r[3], double x[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int i = c + 1; i < 3; ++i)
            if (fabs(A[i][c]) > fabs(A[p][c])) p = i;
        if (A[p][c] == 0.0) return false;
        if (p != c) {
            for (int k = 0; k < 3; ++k) {
                const double t = A[c][k];
                A[c][k] = A[p][k];
                A[p][k] = t;
            }
            const double t = r[c];
            r[c] = r[p];
            r[p] = t;
        }
        const double inv = 1.0 / A[c][c];
        for (int i = c + 1; i < 3; ++i) {
            const double f = A[i][c] * inv;
            for (int k = c; k < 3; ++k) A[i][k] -= f * A[c][k];
            r[i] -= f * r[c];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = r[i];
        for (int k = i + 1; k < 3; ++k) s -= A[i][k] * x[k];
        x[i] = s / A[i][i];
    }
    return true;
}

// One wave per cell, four cells per workgroup.  rows holds the padded chain of
// cells lo..hi-1.  When cand.parent != NULL, every edge on a hidden unit or a
// head comparison is appended to the candidate list.
__global__ __launch_bounds__(256) void k_clip_f64(DevNet net, const uint64_t *__restrict__ codes,
                                                  const int *__restrict__ argmax,
                                                  const uint64_t *__restrict__ cell_hash, long long lo,
                                                  long long hi, long long n_seed_cells,
                                                  const double *__restrict__ rows, ClipOut out,
                                                  Candidates cand, unsigned long long cand_cap,
                                                  Counters *ctr) {
    __shared__ PolyScratch scratch[4];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const long long cell = lo + 4LL * blockIdx.x + wave;
    if (cell >= hi) return;
    PolyScratch &S = scratch[wave];
    const uint64_t *code = codes + cell * net.W;
    const int am_in = argmax ? argmax[cell] : 0;
    const bool am_ok = am_in >= 0 && am_in < net.M;   // a bad argmax gives an empty face
    const int am = am_ok ? am_in : 0;
    const double *crow = rows + (cell - lo) * (long long)net.R * 4;
    const long long oi = cell - out.out_base;
    int flags = 0;

    // ---- plane frame: n = a_F[0:3], foot point p0, orthonormal u, v with u x v = n/|n|
    const double *aF = crow + (long long)net.row_of_unit[net.N + am] * 4;
    const double fx = aF[0], fy = aF[1], fz = aF[2], fw = aF[3];
    const double nn = fx * fx + fy * fy + fz * fz;
    Poly P;
    P.m = 0;
    double p0[3], u[3], v[3];
    if (nn > 0.0 && am_ok) {
        p0[0] = -fw * fx / nn;
        p0[1] = -fw * fy / nn;
        p0[2] = -fw * fz / nn;
        const double inl = 1.0 / sqrt(nn);
        const double n0 = fx * inl, n1 = fy * inl, n2 = fz * inl;
        int ax = 0;
        if (fabs(n1) < fabs(n0)) ax = 1;
        if (fabs(n2) < fabs(ax == 0 ? n0 : n1)) ax = 2;
        // u = normalize(n x e_ax)
        double ux = ax == 0 ? 0.0 : (ax == 1 ? -n2 : n1);
        double uy = ax == 0 ? n2 : (ax == 1 ? 0.0 : -n0);
        double uz = ax == 0 ? -n1 : (ax == 1 ? n0 : 0.0);
        const double iu = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
        u[0] = ux * iu;
        u[1] = uy * iu;
        u[2] = uz * iu;
        v[0] = n1 * u[2] - n2 * u[1];
        v[1] = n2 * u[0] - n0 * u[2];
        v[2] = n0 * u[1] - n1 * u[0];
        // starting square, counter-clockwise, edges -7..-10
        const double sa[4] = {-kSquareHalf, kSquareHalf, kSquareHalf, -kSquareHalf};
        const double sb[4] = {-kSquareHalf, -kSquareHalf, kSquareHalf, kSquareHalf};
        const int li = lane < 4 ? lane : 0;
        P.a = sa[li];
        P.b = sb[li];
        P.r = 1.0 + sqrt(P.a * P.a + P.b * P.b);
        P.e = -7 - li;
        P.m = 4;
        // the six box planes, ids -1..-6
        for (int t = 0; t < 6 && P.m > 0; ++t) {
            const int axb = t >> 1;
            const double sg = (t & 1) ? -1.0 : 1.0;
            sh_clip(P, sg * u[axb], sg * v[axb], sg * p0[axb] - 1.0, -1 - t, S, flags);
        }
        // hidden units, 64 lines per pass
        for (int base = 0; base < net.N && P.m > 0; base += kWave) {
            const int g = base + lane;
            const bool valid = g < net.N;
            double cu = 0.0, cv = 0.0, cw = 0.0, nrm = 0.0;
            bool cuts = false;
            if (valid) {
                const double *z = crow + (long long)net.row_of_unit[g] * 4;
                const double sg = code_bit(code, g) ? -1.0 : 1.0;
                const double c0 = sg * z[0], c1 = sg * z[1], c2 = sg * z[2], c3 = sg * z[3];
                cu = c0 * u[0] + c1 * u[1] + c2 * u[2];
                cv = c0 * v[0] + c1 * v[1] + c2 * v[2];
                cw = c0 * p0[0] + c1 * p0[1] + c2 * p0[2] + c3;
                nrm = sqrt(cu * cu + cv * cv);
            }
            for (int i = 0; i < P.m; ++i) {
                const double ai = bcast(P.a, i), bi = bcast(P.b, i), ri = bcast(P.r, i);
                cuts |= (cu * ai + cv * bi + cw) > kTau * (nrm * ri + fabs(cw));
            }
            uint64_t mask = ballot(valid && cuts);
            while (mask) {
                const int t = __builtin_ctzll(mask);
                mask &= mask - 1;
                if (!sh_clip(P, bcast(cu, t), bcast(cv, t), bcast(cw, t), base + t, S, flags)) break;
            }
        }
        // max-pool comparisons with every other head
        if (net.M > 1 && P.m > 0) {
            const int hd = lane;
            const bool valid = hd < net.M && hd != am;
            double cu = 0.0, cv = 0.0, cw = 0.0;
            if (valid) {
                const double *zi = crow + (long long)net.row_of_unit[net.N + hd] * 4;
                const double c0 = zi[0] - fx, c1 = zi[1] - fy, c2 = zi[2] - fz, c3 = zi[3] - fw;
                cu = c0 * u[0] + c1 * u[1] + c2 * u[2];
                cv = c0 * v[0] + c1 * v[1] + c2 * v[2];
                cw = c0 * p0[0] + c1 * p0[1] + c2 * p0[2] + c3;
            }
            uint64_t mask = ballot(valid);
            while (mask && P.m > 0) {
                const int t = __builtin_ctzll(mask);
                mask &= mask - 1;
                if (!sh_clip(P, bcast(cu, t), bcast(cv, t), bcast(cw, t), net.N + t, S, flags)) break;
            }
        }
    }

    // ---- validity: >= 3 vertices, positive area, distinct ids, no frame edge
    int m = P.m;
    const bool act = lane < m;
    if (m >= 3) {
        const int j = (lane + 1 >= m) ? 0 : lane + 1;
        const double ja = shfl(P.a, j), jb = shfl(P.b, j);
        const double area2 = wave_sum(act ? (P.a * jb - ja * P.b) : 0.0);
        bool dup = false;
        for (int k = 0; k < m; ++k) {
            const int ek = bcast(P.e, k);
            dup |= act && k != lane && ek == P.e;
        }
        if (ballot(dup)) flags |= kFlagDegen;
        // a starting-square edge cannot survive the box planes; if one did, the
        // face is unusable (and its id names no constraint row)
        if (ballot(act && P.e <= -7)) {
            flags |= kFlagDegen;
            m = 0;
        }
        if (!(area2 > 0.0)) m = 0;
    } else {
        m = 0;
    }
    if (m == 0) flags |= kFlagEmpty;

    if (m > out.stride) {
        flags |= kFlagTooBig;
        m = 0;
    }

    int e_out = 0;
    if (m > 0) {
        // rotate so that the smallest edge id comes first
        const int minid = wave_min(lane < m ? P.e : 0x7fffffff);
        const int r0 = __builtin_ctzll(ballot(lane < m && P.e == minid));
        int src = lane + r0;
        if (src >= m) src -= m;
        if (lane >= m) src = lane;
        const int e = shfl(P.e, src);
        const int eprev = shfl(e, lane == 0 ? m - 1 : lane - 1);
        e_out = e;
        if (lane < m) {
            // vertex i = [c_{e(i-1)}; c_{e(i)}; a_F] x = -[...]
            double ca[4], cb[4];
            constraint_row(net, eprev, code, am, crow, ca);
            constraint_row(net, e, code, am, crow, cb);
            double A[3][3] = {{ca[0], ca[1], ca[2]}, {cb[0], cb[1], cb[2]}, {fx, fy, fz}};
            double rr[3] = {-ca[3], -cb[3], -fw};
            double x[3];
            if (!solve3(A, rr, x)) {
                flags |= kFlagSingular;
                x[0] = x[1] = x[2] = __builtin_nan("");
            }
            const long long o = oi * out.stride + lane;
            out.ids[o] = e;
            out.verts[o * 3 + 0] = x[0];
            out.verts[o * 3 + 1] = x[1];
            out.verts[o * 3 + 2] = x[2];
            if (out.nbr) out.nbr[o] = -1;
        }
        for (int o = 32; o > 0; o >>= 1) flags |= __shfl_xor(flags, o, kWave);
    }
    if (lane == 0) {
        out.m[oi] = m;
        if (out.flags) out.flags[oi] = flags;
    }

    if (ctr && lane == 0) {
        if (m == 0) {
            if (cell >= n_seed_cells) atomicAdd(&ctr->degenerate, 1ull);
        } else {
            atomicAdd(&ctr->face_verts, (unsigned long long)m);
            if (flags & kFlagDegen) atomicAdd(&ctr->degenerate, 1ull);
        }
        if (flags & kFlagTooBig) atomicAdd(&ctr->too_big, 1ull);
    }

    // ---- neighbour candidates: flip the unit (or the argmax) behind each edge
    if (cand.parent && m > 0) {
        const bool want = lane < m && e_out >= 0;
        if (ctr) {
            const uint64_t dm = ballot(lane < m && e_out < 0);
            if (lane == 0 && dm) atomicAdd(&ctr->domain_edges, (unsigned long long)__popcll(dm));
        }
        unsigned long long basev;
        const unsigned long long idx = wave_reserve(&ctr->n_cand, want, &basev);
        if (want) {
            if (idx < cand_cap) {
                const uint64_t h = cell_hash[cell];
                uint64_t hn;
                if (e_out < net.N) hn = h ^ net.zobrist[e_out];
                else hn = h ^ net.zobrist[net.N + am] ^ net.zobrist[e_out];
                cand.parent[idx] = (int)cell;
                cand.slot[idx] = lane;
                cand.unit[idx] = e_out;
                cand.hash[idx] = hn;
            } else {
                atomicAdd(&ctr->overflow_cand, 1ull);
            }
        }
    }
}

void launch_clip(const DevNet &net, const uint64_t *codes, const int *argmax, const uint64_t *cell_hash,
                 long long lo, long long hi, long long n_seed_cells, const double *rows, const ClipOut &out,
                 const Candidates &cand, unsigned long long cand_cap, Counters *ctr, hipStream_t st) {
    if (hi <= lo) return;
    const long long blocks = (hi - lo + 3) / 4;
    hipLaunchKernelGGL(k_clip_f64, dim3((unsigned)blocks), dim3(256), 0, st, net, codes, argmax, cell_hash,
                       lo, hi, n_seed_cells, rows, out, cand, cand_cap, ctr);
}

}  // namespace am
