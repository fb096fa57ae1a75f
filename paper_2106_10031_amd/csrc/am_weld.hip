// am_weld.hip -- the mesh Z = {V, {P}} (Sec. 3) with shared vertices.
//
// A march emits every face with its own copy of its vertices (corner c of
// face f = entry offsets[f] + c of the CSR arrays).  Two corners are the same
// mesh vertex when an edge links them: across edge i of face f (to face g,
// where the same plane is edge j) the start of edge i is the end of edge j
// and the end of edge i is the start of edge j.  Welding joins those corner
// pairs with a lock-free union-find (parent pointers linked by CAS, smaller
// root wins), so every class of corners around a vertex collapses to its
// smallest corner index, whatever the number of faces meeting there.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "am_internal.h"

namespace am {

namespace {

__device__ __forceinline__ long long find_root(long long *parent, long long x) {
    long long p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (p != x) {
        const long long gp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (gp != p) atomicCAS((unsigned long long *)&parent[x], (unsigned long long)p, (unsigned long long)gp);
        x = p;
        p = gp;
    }
    return x;
}

__device__ void unite(long long *parent, long long a, long long b) {
    // bounded: every failed CAS means another thread lowered a root, and roots
    // only decrease, so the loop ends after at most (corner count) rounds
    for (;;) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a < b) {
            const long long t = a;
            a = b;
            b = t;
        }
        // hang the larger root under the smaller
        if (atomicCAS((unsigned long long *)&parent[a], (unsigned long long)a, (unsigned long long)b) ==
            (unsigned long long)a)
            return;
    }
}

__global__ void k_weld_init(long long *parent, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) parent[i] = i;
}

// One thread per face: links each edge's corners with its twin's in the
// neighbouring face (only from the face with the smaller index, so each edge
// is linked once).  twin id: a hidden-unit edge keeps its id; comparison
// edge N + i of a face whose argmax is a is edge N + a of the neighbour.
__global__ void k_weld_link(long long F, long long n, const long long *__restrict__ off,
                            const int *__restrict__ ids, const long long *__restrict__ nbr,
                            const int *__restrict__ argmax, int N, long long *parent,
                            unsigned long long *unpaired) {
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const long long a0 = off[f], m = off[f + 1] - a0;
    if (a0 < 0 || m < 0 || a0 + m > n) {   // malformed CSR: counted, not followed
        atomicAdd(unpaired, 1ull);
        return;
    }
    for (long long i = 0; i < m; ++i) {
        const long long g = nbr[a0 + i];
        if (g < 0 || g >= F || g <= f) continue;
        const int e = ids[a0 + i];
        const int twin = (e >= N && argmax) ? N + argmax[f] : e;
        const long long b0 = off[g], mg = off[g + 1] - b0;
        long long j = -1;
        if (b0 >= 0 && mg > 0 && b0 + mg <= n)
            for (long long k = 0; k < mg; ++k)
                if (ids[b0 + k] == twin && nbr[b0 + k] == f) {
                    j = k;
                    break;
                }
        if (j < 0) {
            atomicAdd(unpaired, 1ull);
            continue;
        }
        unite(parent, a0 + i, b0 + (j + 1 == mg ? 0 : j + 1));
        unite(parent, a0 + (i + 1 == m ? 0 : i + 1), b0 + j);
    }
}

// Full compression; is_root[c] = 1 for class representatives.
__global__ void k_weld_flatten(long long *parent, long long n, int *is_root) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long r = find_root(parent, i);
    parent[i] = r;
    is_root[i] = r == i ? 1 : 0;
}

// corner -> vertex id; vertex coordinates from the representative corner.
__global__ void k_weld_emit(const long long *__restrict__ parent, const int *__restrict__ vid_of_root, long long n,
                            const double *__restrict__ verts, long long *corner_vertex, double *vxyz,
                            long long vxyz_rows) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long r = parent[i];
    const int v = vid_of_root[r];
    if (corner_vertex) corner_vertex[i] = v;
    if (vxyz && r == i && v < vxyz_rows) {
        vxyz[(long long)v * 3] = verts[i * 3];
        vxyz[(long long)v * 3 + 1] = verts[i * 3 + 1];
        vxyz[(long long)v * 3 + 2] = verts[i * 3 + 2];
    }
}

// Fan triangles: face f with corners c0..c(m-1) gives (c0, ck, ck+1),
// k = 1..m-2, at triangle index off[f] - 2 f + k - 1 (rows past tri_rows,
// which only faces with fewer than 2 corners could cause, are not written).
__global__ void k_triangles(long long F, long long n, const long long *__restrict__ off,
                            const long long *__restrict__ corner_vertex, long long *tri, long long tri_rows) {
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const long long a0 = off[f], m = off[f + 1] - off[f];
    if (a0 < 0 || m < 0 || a0 + m > n) return;
    const long long t0 = a0 - 2 * f;
    for (long long k = 1; k + 1 < m; ++k) {
        const long long r = t0 + k - 1;
        if (r < 0 || r >= tri_rows) continue;
        long long *t = tri + r * 3;
        t[0] = corner_vertex[a0];
        t[1] = corner_vertex[a0 + k];
        t[2] = corner_vertex[a0 + k + 1];
    }
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// Scratch: parent [n] i64, is_root [n] i32, vid [n] i32, scan tmp.
hipError_t weld_tmp_bytes(long long n, size_t *bytes) {
    size_t b = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, b, (int *)nullptr, (int *)nullptr, (int)n);
    *bytes = b;
    return e;
}

hipError_t launch_weld(long long F, long long n, const long long *off, const int *ids, const long long *nbr,
                       const int *argmax, const double *verts, int N, long long vxyz_rows, long long *parent,
                       int *is_root, int *vid,
                       void *tmp, size_t tmp_bytes, unsigned long long *unpaired, long long *corner_vertex,
                       double *vxyz, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_weld_init, dim3(blocks_for(n)), dim3(256), 0, st, parent, n);
    if (F > 0)
        hipLaunchKernelGGL(k_weld_link, dim3(blocks_for(F)), dim3(256), 0, st, F, n, off, ids, nbr, argmax, N,
                           parent, unpaired);
    hipLaunchKernelGGL(k_weld_flatten, dim3(blocks_for(n)), dim3(256), 0, st, parent, n, is_root);
    size_t tb = tmp_bytes;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(tmp, tb, is_root, vid, (int)n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_weld_emit, dim3(blocks_for(n)), dim3(256), 0, st, parent, vid, n, verts, corner_vertex,
                       vxyz, vxyz_rows);
    return hipSuccess;
}

void launch_triangles(long long F, long long n, const long long *off, const long long *corner_vertex, long long *tri,
                      long long tri_rows, hipStream_t st) {
    if (F <= 0) return;
    hipLaunchKernelGGL(k_triangles, dim3(blocks_for(F)), dim3(256), 0, st, F, n, off, corner_vertex, tri,
                       tri_rows);
}

}  // namespace am
