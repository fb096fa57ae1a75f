"""Python access to the FP64 CPU oracle (``am_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
SRC = os.path.join(HERE, "am_oracle.c")


def build(force: bool = True, out: str = LIB_PATH, mutate: int = 0) -> str:
    """Compile the oracle with gcc (generic x86-64, -O2, no GPU code).

    ``mutate`` > 0 builds a deliberately broken variant (see ORC_MUTATE in the
    C source); only the mutation test asks for one, into a temporary path.
    """
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]
        if mutate:
            cmd.append(f"-DORC_MUTATE={int(mutate)}")
        subprocess.check_call(cmd + [SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


OMP_LIB_PATH = os.path.join(HERE, "liborc_omp.so")


def build_omp(force: bool = True, out: str = OMP_LIB_PATH) -> str:
    """The same source built with OpenMP (-O3) for the batched routines.

    Contraction and reassociation stay off (no -march, -ffp-contract=off), so
    every face is computed with the same IEEE operations as in the -O2 build
    and the two give identical meshes (checked by a test); only the batch
    driver runs on several threads.
    """
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall",
               "-Wno-unused-function"]
        subprocess.check_call(cmd + [SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


class _Net(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("width", C.POINTER(C.c_int32)),
                ("n_blocks", C.c_int32), ("blk_dst", C.POINTER(C.c_int32)),
                ("blk_src", C.POINTER(C.c_int32)), ("blk_off", C.POINTER(C.c_int64)),
                ("weights", C.POINTER(C.c_double)), ("bias_off", C.POINTER(C.c_int64)),
                ("biases", C.POINTER(C.c_double))]


_libs = {}


def lib(path: str = LIB_PATH):
    L = _libs.get(path)
    if L is None:
        if not os.path.exists(path):
            if path == LIB_PATH:
                build()
            elif path == OMP_LIB_PATH:
                build_omp()
            else:
                raise FileNotFoundError(path)
        L = C.CDLL(path)
        P = C.POINTER
        L.orc_code_words.argtypes = [P(_Net)]
        L.orc_code_words.restype = C.c_int
        L.orc_forward.argtypes = [P(_Net), P(C.c_double), P(C.c_double), P(C.c_int32)]
        L.orc_forward.restype = C.c_double
        L.orc_code.argtypes = [P(_Net), P(C.c_double), P(C.c_uint64), P(C.c_int32)]
        L.orc_code.restype = C.c_double
        L.orc_chain.argtypes = [P(_Net), P(C.c_uint64), P(C.c_double)]
        L.orc_chain.restype = None
        L.orc_face.argtypes = [P(_Net), P(C.c_uint64), C.c_int32, C.c_int, P(C.c_int32),
                               P(C.c_double), P(C.c_double), P(C.c_int32)]
        L.orc_face.restype = C.c_int
        L.orc_face_pivot.argtypes = [P(_Net), P(C.c_uint64), C.c_int32, C.c_int32, P(C.c_double), C.c_int,
                                     P(C.c_int32), P(C.c_double), P(C.c_int32)]
        L.orc_face_pivot.restype = C.c_int
        L.orc_seed_ray.argtypes = [P(_Net), P(C.c_double), P(C.c_double), C.c_int,
                                   P(C.c_double), P(C.c_uint64), P(C.c_int32)]
        L.orc_seed_ray.restype = C.c_int
        L.orc_seed_st.argtypes = [P(_Net), P(C.c_double), C.c_int, P(C.c_double), P(C.c_uint64),
                                  P(C.c_int32), P(C.c_int32)]
        L.orc_seed_st.restype = C.c_int
        L.orc_march.argtypes = [P(_Net), P(C.c_uint64), P(C.c_int32), C.c_int64, C.c_int64]
        L.orc_march.restype = C.c_void_p
        L.orc_march_batched.argtypes = [P(_Net), P(C.c_uint64), P(C.c_int32), C.c_int64, C.c_int64, C.c_int64]
        L.orc_march_batched.restype = C.c_void_p
        L.orc_faces_batched.argtypes = [P(_Net), P(C.c_uint64), P(C.c_int32), C.c_int64, C.c_int,
                                        P(C.c_int32), P(C.c_int32), P(C.c_double), P(C.c_int32)]
        L.orc_faces_batched.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = C.c_int
        L.orc_result_free.argtypes = [C.c_void_p]
        L.orc_result_counts.argtypes = [C.c_void_p, P(C.c_int64)]
        L.orc_result_fetch.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32), P(C.c_double),
                                       P(C.c_int64), P(C.c_uint64), P(C.c_int32)]
        _libs[path] = L
    return L


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


class OracleNet:
    """A :class:`am_workloads.nets.Net` marshalled for the C oracle."""

    def __init__(self, net, lib_path: str = LIB_PATH):
        self.net = net
        self._L = lib(lib_path)
        self.width = np.asarray(net.widths, np.int32)
        self.dst = np.asarray([d for d, _, _ in net.blocks], np.int32)
        self.src = np.asarray([s for _, s, _ in net.blocks], np.int32)
        offs, o = [], 0
        for _, _, W in net.blocks:
            offs.append(o)
            o += W.size
        self.blk_off = np.asarray(offs, np.int64)
        self.weights = np.concatenate([W.ravel() for _, _, W in net.blocks]).astype(np.float64)
        boffs, o = [0], 0
        for b in net.bias:
            boffs.append(o)
            o += b.size
        self.bias_off = np.asarray(boffs, np.int64)
        self.biases = np.concatenate(net.bias).astype(np.float64)
        self.s = _Net(len(self.width), _ptr(self.width, C.c_int32), len(self.dst),
                      _ptr(self.dst, C.c_int32), _ptr(self.src, C.c_int32),
                      _ptr(self.blk_off, C.c_int64), _ptr(self.weights, C.c_double),
                      _ptr(self.bias_off, C.c_int64), _ptr(self.biases, C.c_double))
        self.N = net.n_hidden
        self.M = net.n_heads
        self.W = self._L.orc_code_words(C.byref(self.s))

    # -- per-point / per-cell primitives ----------------------------------
    def forward(self, x):
        x = np.ascontiguousarray(x, np.float64)
        pre = np.zeros(self.N + self.M)
        am = C.c_int32()
        F = self._L.orc_forward(C.byref(self.s), _ptr(x, C.c_double), _ptr(pre, C.c_double), C.byref(am))
        return F, pre, am.value

    def code(self, x):
        x = np.ascontiguousarray(x, np.float64)
        code = np.zeros(self.W, np.uint64)
        am = C.c_int32()
        F = self._L.orc_code(C.byref(self.s), _ptr(x, C.c_double), _ptr(code, C.c_uint64), C.byref(am))
        return code, am.value, F

    def chain(self, code):
        code = np.ascontiguousarray(code, np.uint64)
        rows = np.zeros((self.N + self.M, 4))
        self._L.orc_chain(C.byref(self.s), _ptr(code, C.c_uint64), _ptr(rows, C.c_double))
        return rows

    def face(self, code, argmax=0, max_m=128):
        code = np.ascontiguousarray(code, np.uint64)
        ids = np.zeros(max_m, np.int32)
        verts = np.zeros((max_m, 3))
        area = C.c_double()
        flags = C.c_int32()
        m = self._L.orc_face(C.byref(self.s), _ptr(code, C.c_uint64), int(argmax), max_m,
                           _ptr(ids, C.c_int32), _ptr(verts, C.c_double), C.byref(area),
                           C.byref(flags))
        return ids[:m].copy(), verts[:m].copy(), area.value, flags.value

    def face_pivot(self, code, argmax, start_id, xs, max_m=128):
        """Face by pivoting enumeration (Alg. 2) from plane start_id through
        the point xs on the face's edge there: (ids, verts, flags)."""
        code = np.ascontiguousarray(code, np.uint64)
        xs = np.ascontiguousarray(xs, np.float64)
        ids = np.zeros(max_m, np.int32)
        verts = np.zeros((max_m, 3))
        flags = C.c_int32()
        m = self._L.orc_face_pivot(C.byref(self.s), _ptr(code, C.c_uint64), int(argmax), int(start_id),
                                   _ptr(xs, C.c_double), max_m, _ptr(ids, C.c_int32), _ptr(verts, C.c_double),
                                   C.byref(flags))
        return ids[:m].copy(), verts[:m].copy(), flags.value

    def seed_ray(self, o, d, max_iter=200):
        o = np.ascontiguousarray(o, np.float64)
        d = np.ascontiguousarray(d, np.float64)
        x = np.zeros(3)
        code = np.zeros(self.W, np.uint64)
        am = C.c_int32()
        st = self._L.orc_seed_ray(C.byref(self.s), _ptr(o, C.c_double), _ptr(d, C.c_double),
                                int(max_iter), _ptr(x, C.c_double), _ptr(code, C.c_uint64),
                                C.byref(am))
        return st, x, code, am.value

    def seed_st(self, x0, max_iter=64):
        """Sphere-tracing seed from x0: (status, x, code, argmax, iterations)."""
        x0 = np.ascontiguousarray(x0, np.float64)
        x = np.zeros(3)
        code = np.zeros(self.W, np.uint64)
        am = C.c_int32()
        it = C.c_int32()
        st = self._L.orc_seed_st(C.byref(self.s), _ptr(x0, C.c_double), int(max_iter), _ptr(x, C.c_double),
                                 _ptr(code, C.c_uint64), C.byref(am), C.byref(it))
        return st, x, code, am.value, it.value

    def seed_rays(self, origins, dirs, max_iter=200):
        """Seeds for a batch of rays; returns (codes[S,W], argmax[S], points[S,3], status[R])."""
        codes, ams, pts, sts = [], [], [], []
        for o, d in zip(origins, dirs):
            st, x, code, am = self.seed_ray(o, d, max_iter)
            sts.append(st)
            if st == 0:
                codes.append(code)
                ams.append(am)
                pts.append(x)
        W = self.W
        return (np.asarray(codes, np.uint64).reshape(-1, W), np.asarray(ams, np.int32),
                np.asarray(pts, np.float64).reshape(-1, 3), np.asarray(sts, np.int32))

    def threads(self):
        """Threads of the batched routines in the loaded build."""
        return int(self._L.orc_threads())

    def faces_batched(self, codes, argmax=None, max_m=128):
        """orc_face of every given cell (parallel in the OpenMP build):
        (m [n], ids [n, max_m], verts [n, max_m, 3], flags [n])."""
        codes = np.ascontiguousarray(np.asarray(codes, np.uint64).reshape(-1, self.W))
        n = codes.shape[0]
        am = None if argmax is None else np.ascontiguousarray(argmax, np.int32)
        m = np.zeros(n, np.int32)
        ids = np.zeros((n, max_m), np.int32)
        verts = np.zeros((n, max_m, 3))
        flags = np.zeros(n, np.int32)
        self._L.orc_faces_batched(C.byref(self.s), _ptr(codes, C.c_uint64),
                                  None if am is None else _ptr(am, C.c_int32), n, int(max_m),
                                  _ptr(m, C.c_int32), _ptr(ids, C.c_int32), _ptr(verts, C.c_double),
                                  _ptr(flags, C.c_int32))
        return m, ids, verts, flags

    def march(self, seed_codes, seed_argmax=None, max_cells=0, batch=None):
        """Algorithm 1 from the seed cells (FIFO).  batch: None = one cell at
        a time (orc_march); an int = orc_march_batched with that batch size
        (the same mesh; parallel in the OpenMP build)."""
        seed_codes = np.ascontiguousarray(np.asarray(seed_codes, np.uint64).reshape(-1, self.W))
        S = seed_codes.shape[0]
        if seed_argmax is None:
            seed_argmax = np.zeros(S, np.int32)
        seed_argmax = np.ascontiguousarray(seed_argmax, np.int32)
        L = self._L
        if batch is None:
            R = L.orc_march(C.byref(self.s), _ptr(seed_codes, C.c_uint64), _ptr(seed_argmax, C.c_int32),
                            S, int(max_cells))
        else:
            R = L.orc_march_batched(C.byref(self.s), _ptr(seed_codes, C.c_uint64), _ptr(seed_argmax, C.c_int32),
                                    S, int(max_cells), int(batch))
        if not R:
            raise MemoryError("oracle march failed")
        try:
            cnt = np.zeros(7, np.int64)
            L.orc_result_counts(R, _ptr(cnt, C.c_int64))
            F, nv = int(cnt[0]), int(cnt[1])
            offsets = np.zeros(F + 1, np.int64)
            ids = np.zeros(nv, np.int32)
            verts = np.zeros((nv, 3))
            nbr = np.zeros(nv, np.int64)
            codes = np.zeros((F, self.W), np.uint64)
            am = np.zeros(F, np.int32)
            L.orc_result_fetch(R, _ptr(offsets, C.c_int64), _ptr(ids, C.c_int32),
                               _ptr(verts, C.c_double), _ptr(nbr, C.c_int64),
                               _ptr(codes, C.c_uint64), _ptr(am, C.c_int32))
        finally:
            L.orc_result_free(R)
        stats = dict(faces=F, face_verts=nv, cells=int(cnt[2]), seeds_in=int(cnt[3]),
                     seed_dup=int(cnt[4]), seed_empty=int(cnt[5]), degenerate=int(cnt[6]))
        return Mesh(codes, am, offsets, ids, verts, nbr, stats)


@dataclasses.dataclass
class Mesh:
    """Polygon mesh in canonical face order (faces sorted by code, then argmax)."""
    codes: np.ndarray     # [F, W] uint64
    argmax: np.ndarray    # [F] int32
    offsets: np.ndarray   # [F+1] int64
    ids: np.ndarray       # [V] int32 edge (constraint) id of edge i of each face
    verts: np.ndarray     # [V, 3] float64, vertex i starts edge i
    nbr: np.ndarray       # [V] int64 face across edge i (-1 domain, -2 missing)
    stats: dict

    @property
    def n_faces(self):
        return len(self.offsets) - 1

    def face(self, f):
        a, b = self.offsets[f], self.offsets[f + 1]
        return self.ids[a:b], self.verts[a:b], self.nbr[a:b]


# ------------------------------------------------------------- welded mesh

def weld(mesh, n_hidden: int, _mutate: int = 0):
    """Shared vertices of a march's mesh: the output Z = {V, {P}} of Sec. 3.

    Corner i of face f is entry offsets[f] + i; it starts edge i, so edge i
    runs from corner i to corner i+1 (cyclic).  Across edge i (to face
    g = nbr[i], where the same edge is edge j of g: same constraint, or for a
    max-pool comparison edge N + k of f the row N + argmax[f] of g) the two
    faces traverse the edge in opposite directions, so corner i of f is
    corner j+1 of g and corner i+1 of f is corner j of g.  The vertices are
    the classes of the equivalence these identifications generate (union-find
    over the corners).  Vertex ids follow each class's smallest corner; a
    vertex's position is that corner's.

    Returns (corner_vertex [corners] int64, vxyz [V][3] float64, unpaired).
    ``_mutate`` plants a mistake for the checks of the checks
    (1: corner i of f joined to corner j of g instead of j+1).
    """
    off = np.asarray(mesh.offsets, np.int64)
    ids = np.asarray(mesh.ids)
    nbr = np.asarray(mesh.nbr, np.int64)
    am = np.asarray(mesh.argmax)
    n = int(off[-1])
    parent = list(range(n))

    def find(a):
        root = a
        while parent[root] != root:
            root = parent[root]
        while parent[a] != root:
            parent[a], a = root, parent[a]
        return root

    def union(a, b):
        a, b = find(a), find(b)
        if a != b:
            parent[max(a, b)] = min(a, b)

    unpaired = 0
    for f in range(len(off) - 1):
        a0, m = int(off[f]), int(off[f + 1] - off[f])
        for i in range(m):
            g = int(nbr[a0 + i])
            if g < 0:
                continue
            e = int(ids[a0 + i])
            twin = e if e < n_hidden else n_hidden + int(am[f])
            b0, mg = int(off[g]), int(off[g + 1] - off[g])
            js = [k for k in range(mg) if ids[b0 + k] == twin and nbr[b0 + k] == f]
            if len(js) != 1:
                unpaired += 1
                continue
            j = js[0]
            if _mutate == 1:
                union(a0 + i, b0 + j)
                union(a0 + (i + 1) % m, b0 + (j + 1) % mg)
            else:
                union(a0 + i, b0 + (j + 1) % mg)
                union(a0 + (i + 1) % m, b0 + j)
    roots = np.array([find(a) for a in range(n)], np.int64)
    is_root = roots == np.arange(n)
    vid = np.cumsum(is_root) - 1
    corner_vertex = vid[roots]
    vxyz = np.asarray(mesh.verts, np.float64).reshape(-1, 3)[is_root]
    return corner_vertex.astype(np.int64), vxyz, unpaired


def fan_triangles(offsets, corner_vertex):
    """Triangles (c0, ck, ck+1), k = 1..m-2, of each convex polygon in order."""
    off = np.asarray(offsets, np.int64)
    cv = np.asarray(corner_vertex, np.int64)
    out = []
    for f in range(len(off) - 1):
        a0, m = int(off[f]), int(off[f + 1] - off[f])
        for k in range(1, m - 1):
            out.append((cv[a0], cv[a0 + k], cv[a0 + k + 1]))
    return np.array(out, np.int64).reshape(-1, 3)


# ----------------------------------------------- quadric edge collapse

def qecd(verts, tris, target_tris: int, _mutate: int = 0):
    """Sequential quadric edge-collapse decimation (Sec. 4.4; Garland and
    Heckbert's metric, which the paper adopts), the reference for the GPU's
    parallel rounds.  Vertex quadrics are area-weighted sums of their
    triangles' plane quadrics; an edge collapses to the minimiser of the
    summed quadric when that 3x3 system is well conditioned and the point
    lies within two edge lengths of the midpoint, else to the best of its two
    ends and midpoint.  The cheapest edge whose ends share exactly two
    neighbours and two triangles, and whose collapse turns no surviving
    triangle by more than the angle with cosine 0.2, collapses first (a lazy
    heap).  Returns (verts [V'][3], tris [T'][3]) with unused vertices
    dropped.  Plain numpy and Python loops: small meshes only.
    ``_mutate`` plants a mistake for the checks of the checks (1: every edge
    collapses to its midpoint).
    """
    import heapq

    P = np.array(verts, np.float64).copy()
    T = [list(map(int, t)) for t in tris]
    nV = len(P)
    Q = np.zeros((nV, 4, 4))
    for a, b, c in T:
        n = np.cross(P[b] - P[a], P[c] - P[a])
        ln = np.linalg.norm(n)
        if ln == 0.0:
            continue
        p = np.append(n / ln, -np.dot(n / ln, P[a]))
        K = np.outer(p, p) * 0.5 * ln
        for v in (a, b, c):
            Q[v] += K
    live = [True] * len(T)
    adj = [set() for _ in range(nV)]
    for t, (a, b, c) in enumerate(T):
        for v in (a, b, c):
            adj[v].add(t)

    def placement(a, b):
        q = Q[a] + Q[b]
        if _mutate == 1:
            v = 0.5 * (P[a] + P[b])
            h = np.append(v, 1.0)
            return max(h @ q @ h, 0.0), v
        A, r = q[:3, :3], -q[:3, 3]
        best, vb = None, None
        det = np.linalg.det(A)
        scale = abs(A[0, 0]) + abs(A[1, 1]) + abs(A[2, 2])
        if scale > 0.0 and abs(det) > 1e-10 * scale ** 3:
            v = np.linalg.solve(A, r)
            if np.linalg.norm(v - 0.5 * (P[a] + P[b])) <= 2.0 * np.linalg.norm(P[b] - P[a]):
                h = np.append(v, 1.0)
                best, vb = max(h @ q @ h, 0.0), v
        for v in (P[a], P[b], 0.5 * (P[a] + P[b])):
            h = np.append(v, 1.0)
            c = max(h @ q @ h, 0.0)
            if best is None or c < best:
                best, vb = c, v.copy()
        return best, vb

    def valid(a, b, v):
        shared = [t for t in adj[a] if b in T[t]]
        na = {w for t in adj[a] for w in T[t]} - {a, b}
        nb = {w for t in adj[b] for w in T[t]} - {a, b}
        if len(shared) != 2 or len(na & nb) != 2:
            return False
        for s in (a, b):
            for t in adj[s]:
                c = T[t]
                if a in c and b in c:
                    continue
                n0 = np.cross(P[c[1]] - P[c[0]], P[c[2]] - P[c[0]])
                q = [v if x in (a, b) else P[x] for x in c]
                n1 = np.cross(q[1] - q[0], q[2] - q[0])
                l0, l1 = np.linalg.norm(n0), np.linalg.norm(n1)
                if not (l1 > 1e-12 * l0) or not (np.dot(n0, n1) > 0.2 * l0 * l1):
                    return False
        return True

    heap = []
    stamp = [0] * nV

    def push_edges(v):
        for t in adj[v]:
            for w in T[t]:
                if w != v:
                    a, b = min(v, w), max(v, w)
                    c, _ = placement(a, b)
                    heapq.heappush(heap, (c, a, b, stamp[a], stamp[b]))

    for v in range(nV):
        push_edges(v)
    n_live = sum(live)
    while n_live > target_tris and heap:
        c, a, b, sa, sb = heapq.heappop(heap)
        if sa != stamp[a] or sb != stamp[b] or not adj[a] or not adj[b]:
            continue
        if not any(b in T[t] for t in adj[a]):
            continue
        c, v = placement(a, b)
        if not valid(a, b, v):
            continue
        P[a] = v
        Q[a] = Q[a] + Q[b]
        for t in list(adj[b]):
            if a in T[t]:
                live[t] = False
                n_live -= 1
                for w in T[t]:
                    adj[w].discard(t)
            else:
                T[t] = [a if x == b else x for x in T[t]]
                adj[a].add(t)
        adj[b] = set()
        stamp[a] += 1
        stamp[b] += 1
        push_edges(a)
    kept = [T[t] for t in range(len(T)) if live[t]]
    used = sorted({v for t in kept for v in t})
    remap = {v: i for i, v in enumerate(used)}
    return P[used], np.array([[remap[v] for v in t] for t in kept], np.int64).reshape(-1, 3)
