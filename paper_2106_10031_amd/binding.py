"""Thin Python binding of the C ABI in include/am.h (argument marshalling only).

Every step of analytic marching runs in the HIP kernels of libam.so; this
module only passes pointers.  PyTorch supplies device memory and the stream.
The library must have been built (``paper_2106_10031_amd/build.py``); there is
no fallback: if it is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libam.so")

AM_OK, AM_E_INVALID, AM_E_OOM, AM_E_CAPACITY, AM_E_SEED, AM_E_DEGENERATE, AM_E_HIP, AM_E_STATE, AM_E_STALL = range(9)
STATUS_NAMES = {0: "AM_OK", 1: "AM_E_INVALID", 2: "AM_E_OOM", 3: "AM_E_CAPACITY", 4: "AM_E_SEED",
                5: "AM_E_DEGENERATE", 6: "AM_E_HIP", 7: "AM_E_STATE", 8: "AM_E_STALL"}

# every symbol include/am.h declares
EXPORTS = ["am_create", "am_destroy", "am_last_error", "am_load_net", "am_load_batch", "am_net_dims", "am_codes",
           "am_chain", "am_faces", "am_seed_rays", "am_seed_cells", "am_march", "am_get_counts", "am_fetch",
           "am_prop_param_count", "am_prop_set", "am_prop_collect", "am_prop_collected", "am_prop_grad",
           "am_prop_adam", "am_prop_score", "am_tune_chain", "am_set_chain_groups", "am_get_chain_groups",
           "am_seed_points_st", "am_weld", "am_triangles", "am_fetch_sorted",
           "am_seed_points", "am_simplify", "am_faces_noalloc", "am_wait", "am_busy"]


# chain tile variants (am_march_opts.chain_groups, am_tune_chain)
CHAIN_VARIANTS = 8


class AmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


AM_F64, AM_F32 = 0, 1          # am_net_desc.dtype
AM_DEVICE, AM_HOST = 0, 1      # am_fetch's `where`


class NetDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("width", C.POINTER(C.c_int32)), ("n_blocks", C.c_int32),
                ("blk_dst", C.POINTER(C.c_int32)), ("blk_src", C.POINTER(C.c_int32)),
                ("blk_w", C.POINTER(C.c_void_p)), ("bias", C.POINTER(C.c_void_p)),
                ("n_heads", C.c_int32), ("dtype", C.c_int32)]


class MarchOpts(C.Structure):
    _fields_ = [("max_cells", C.c_int64), ("max_steps", C.c_int32), ("strict", C.c_int32),
                ("time_kernels", C.c_int32), ("kernel_path", C.c_int32), ("precision", C.c_int32),
                ("propose", C.c_int32), ("chain_groups", C.c_int32), ("graph_steps", C.c_int32),
                ("face_routine", C.c_int32), ("async_", C.c_int32),
                ("margin", C.c_double),
                ("vertex_tol", C.c_double), ("wait_limit", C.c_int32)]


class MarchStats(C.Structure):
    _fields_ = [("faces", C.c_int64), ("face_verts", C.c_int64), ("triangles", C.c_int64),
                ("cells", C.c_int64), ("steps", C.c_int64), ("max_frontier", C.c_int64),
                ("seeds_in", C.c_int64), ("seed_cells", C.c_int64), ("seed_empty", C.c_int64),
                ("degenerate", C.c_int64), ("domain_edges", C.c_int64), ("required_cells", C.c_int64),
                ("march_ms", C.c_double), ("chain_ms", C.c_double), ("clip_ms", C.c_double),
                ("hash_ms", C.c_double), ("chain_launches", C.c_int64), ("clip_launches", C.c_int64),
                ("hash_launches", C.c_int64), ("fused", C.c_int32), ("pad", C.c_int32),
                ("escalated", C.c_int64), ("prop_cells", C.c_int64), ("prop_accepted", C.c_int64),
                ("prop_cuts", C.c_int64), ("graph_launches", C.c_int64), ("pivot_cells", C.c_int64),
                ("pivot_fallback", C.c_int64), ("split_row_eps", C.c_double), ("split_margin", C.c_double),
                ("calib_vertices", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("user", C.c_void_p)]


def _torch_alloc(user, nbytes, device, stream):
    """am_allocator.alloc backed by PyTorch's caching allocator."""
    import torch
    try:
        return int(torch.cuda.caching_allocator_alloc(int(nbytes), int(device), _STREAMS.get(stream or 0)))
    except Exception:   # out of memory: the library reports AM_E_OOM
        return None


def _torch_release(user, ptr, device, stream):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


_TORCH_ALLOC = Allocator(ALLOC_FN(_torch_alloc), RELEASE_FN(_torch_release), None)
_STREAMS = {}          # hipStream_t -> the torch stream it belongs to
_LIVE = None           # contexts still open (closed at exit, while torch is alive)

_lib = None


def lib(path: str = LIB_PATH):
    """Loads libam.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python paper_2106_10031_amd/build.py")
    L = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.am_create.argtypes = [C.POINTER(vp), C.c_int, vp, C.POINTER(Allocator)]
    L.am_destroy.argtypes = [vp]
    L.am_destroy.restype = None
    L.am_last_error.argtypes = [vp]
    L.am_last_error.restype = C.c_char_p
    L.am_load_net.argtypes = [vp, C.POINTER(NetDesc)]
    L.am_load_batch.argtypes = [vp, C.POINTER(NetDesc), i32, vp]
    L.am_net_dims.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.am_codes.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.am_chain.argtypes = [vp, vp, vp, i64, i32, vp]
    L.am_faces.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, vp, vp]
    L.am_faces_noalloc.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, vp, vp]
    L.am_seed_rays.argtypes = [vp, vp, vp, vp, i64, C.c_double, i32, vp]
    L.am_seed_cells.argtypes = [vp, vp, vp, vp, i64]
    L.am_march.argtypes = [vp, C.POINTER(MarchOpts), C.POINTER(MarchStats)]
    L.am_wait.argtypes = [vp, C.POINTER(MarchStats)]
    L.am_busy.argtypes = [vp, C.POINTER(i32)]
    L.am_get_counts.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.am_fetch.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.am_fetch_sorted.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.am_seed_points.argtypes = [vp, vp, vp, i64]
    L.am_simplify.argtypes = [vp, i64, vp, i64, vp, vp, i64, i32, vp, vp, C.POINTER(i64), C.POINTER(i64),
                              C.POINTER(i32), C.POINTER(i64)]
    L.am_prop_param_count.argtypes = []
    L.am_prop_set.argtypes = [vp, vp, i64, i32, C.c_float]
    L.am_prop_collect.argtypes = [vp, vp, vp, i64, C.c_float]
    L.am_prop_collected.argtypes = [vp, C.POINTER(i64)]
    L.am_prop_grad.argtypes = [vp, vp, vp, i64, vp, vp, C.POINTER(C.c_double)]
    L.am_prop_adam.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float]
    L.am_prop_score.argtypes = [vp, vp, i64, vp]
    L.am_tune_chain.argtypes = [vp, i32, vp]
    L.am_seed_points_st.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp]
    L.am_set_chain_groups.argtypes = [vp, vp]
    L.am_get_chain_groups.argtypes = [vp, vp]
    L.am_weld.argtypes = [vp, i64, vp, vp, vp, vp, vp, i64, vp, vp, i64, C.POINTER(i64), C.POINTER(i64)]
    L.am_triangles.argtypes = [vp, i64, vp, vp, vp, i64]
    for name in EXPORTS:
        if name == "am_prop_param_count":
            L.am_prop_param_count.restype = C.c_int64
        elif name not in ("am_destroy", "am_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _p(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """One am_ctx bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream=None, allocator: str = "torch"):
        """allocator: "torch" (device memory from PyTorch's caching allocator,
        the default) or None (the library's own hipMalloc)."""
        global _LIVE
        import atexit
        import weakref
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.L = lib()
        h = C.c_void_p()
        if allocator not in ("torch", None):
            raise ValueError("allocator must be 'torch' or None")
        if allocator == "torch":
            _STREAMS[stream.cuda_stream or 0] = stream
        alloc = C.byref(_TORCH_ALLOC) if allocator == "torch" else None
        st = self.L.am_create(C.byref(h), int(device), C.c_void_p(stream.cuda_stream), alloc)
        if st != AM_OK:
            raise AmError(st, "am_create failed")
        self.h = h
        self.N = self.M = self.W = self.S = None
        if _LIVE is None:
            _LIVE = weakref.WeakSet()
            atexit.register(lambda: [c.close() for c in list(_LIVE)])
        _LIVE.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.L.am_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != AM_OK:
            raise AmError(st, self.L.am_last_error(self.h).decode())

    # ------------------------------------------------------------------ net
    def load_net(self, net, shape_bias=None, dtype=AM_F64):
        """Loads a network given as (widths, blocks [(dst, src, W)], bias [per layer >= 1]).

        With ``shape_bias`` ([S, sum of widths of layers >= 1]), loads S shapes
        that share the weights and use row s as their biases (am_load_batch).
        dtype AM_F32 hands the library FP32 arrays (each value rounded to
        FP32 first; exact for nets stored in FP32).
        """
        widths = np.asarray(net.widths, np.int32)
        dst = np.asarray([d for d, _, _ in net.blocks], np.int32)
        src = np.asarray([s for _, s, _ in net.blocks], np.int32)
        npt = np.float32 if dtype == AM_F32 else np.float64
        ws = [np.ascontiguousarray(W, npt) for _, _, W in net.blocks]
        bs = [np.zeros(3, npt)] + [np.ascontiguousarray(b, npt) for b in net.bias]
        wp = (C.c_void_p * len(ws))(*[w.ctypes.data for w in ws])
        bp = (C.c_void_p * len(bs))(*[b.ctypes.data for b in bs])
        desc = NetDesc(len(widths), widths.ctypes.data_as(C.POINTER(C.c_int32)), len(ws),
                       dst.ctypes.data_as(C.POINTER(C.c_int32)), src.ctypes.data_as(C.POINTER(C.c_int32)),
                       wp, bp, int(widths[-1]), int(dtype))
        if shape_bias is None:
            self._check(self.L.am_load_net(self.h, C.byref(desc)))
        else:
            sb = np.ascontiguousarray(shape_bias, np.float64)
            self._check(self.L.am_load_batch(self.h, C.byref(desc), int(sb.shape[0]), C.c_void_p(sb.ctypes.data)))
        n, m, w, sh = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.L.am_net_dims(self.h, C.byref(n), C.byref(m), C.byref(w), C.byref(sh)))
        self.N, self.M, self.W, self.S = n.value, m.value, w.value, sh.value
        return self

    # ------------------------------------------------------------ per point
    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.device)

    def _shape(self, shape_id):
        return None if shape_id is None else self._dev(shape_id, self.torch.int32)

    def codes(self, pts, shape_id=None):
        t = self.torch
        pts = self._dev(pts, t.float64).reshape(-1, 3)
        n = pts.shape[0]
        sh = self._shape(shape_id)
        codes = t.empty((n, self.W), dtype=t.int64, device=self.device)
        am = t.empty(n, dtype=t.int32, device=self.device)
        F = t.empty(n, dtype=t.float64, device=self.device)
        self._check(self.L.am_codes(self.h, _p(pts), _p(sh), n, _p(codes), _p(am), _p(F)))
        return codes, am, F

    def chain(self, codes, shape_id=None, precision=0):
        t = self.torch
        codes = self._dev(codes, t.int64).reshape(-1, self.W)
        n = codes.shape[0]
        sh = self._shape(shape_id)
        rows = t.empty((n, self.N + self.M, 4), dtype=t.float64, device=self.device)
        self._keep = (codes, sh)
        self._check(self.L.am_chain(self.h, _p(codes), _p(sh), n, int(precision), _p(rows)))
        return rows

    def faces(self, codes, argmax=None, max_m=32, shape_id=None):
        t = self.torch
        codes = self._dev(codes, t.int64).reshape(-1, self.W)
        n = codes.shape[0]
        am = None if argmax is None else self._dev(argmax, t.int32)
        sh = self._shape(shape_id)
        m = t.empty(n, dtype=t.int32, device=self.device)
        ids = t.empty((n, max_m), dtype=t.int32, device=self.device)
        verts = t.empty((n, max_m, 3), dtype=t.float64, device=self.device)
        flags = t.empty(n, dtype=t.int32, device=self.device)
        self._check(self.L.am_faces(self.h, _p(codes), _p(am), _p(sh), n, int(max_m), _p(m), _p(ids), _p(verts),
                                    _p(flags)))
        return m, ids, verts, flags

    def faces_into(self, codes, argmax, shape_id, m, ids, verts, flags, noalloc=True):
        """am_faces_noalloc (or am_faces) into caller-allocated outputs:
        codes [n][W] i64, argmax [n] i32 or None, shape_id [n] i32 or None,
        m [n] i32, ids [n][max_m] i32, verts [n][max_m][3] f64, flags [n] i32
        or None (all device tensors, contiguous)."""
        n = codes.shape[0]
        fn = self.L.am_faces_noalloc if noalloc else self.L.am_faces
        self._check(fn(self.h, _p(codes), _p(argmax), _p(shape_id), n, int(ids.shape[1]), _p(m), _p(ids),
                       _p(verts), _p(flags)))

    # --------------------------------------------------------------- march
    def seed_rays(self, orig, dirs, max_iter=200, shape_id=None, t_max=1.0):
        t = self.torch
        o = self._dev(orig, t.float64).reshape(-1, 3)
        d = self._dev(dirs, t.float64).reshape(-1, 3)
        sh = self._shape(shape_id)
        status = t.empty(o.shape[0], dtype=t.int32, device=self.device)
        self._seed_keep = (o, d, sh)        # the kernel reads them on the stream
        self._check(self.L.am_seed_rays(self.h, _p(o), _p(d), _p(sh), o.shape[0], float(t_max), int(max_iter),
                                        _p(status)))
        return status

    def seed_cells(self, codes, argmax=None, shape_id=None):
        t = self.torch
        codes = self._dev(codes, t.int64).reshape(-1, self.W)
        am = None if argmax is None else self._dev(argmax, t.int32)
        sh = self._shape(shape_id)
        self._seed_keep = (codes, am, sh)   # the copy is enqueued on the stream
        self._check(self.L.am_seed_cells(self.h, _p(codes), _p(am), _p(sh), codes.shape[0]))

    def seed_points(self, pts, shape_id=None):
        """Seeds from the cells of points (forward pass on the device)."""
        t = self.torch
        P = self._dev(pts, t.float64).reshape(-1, 3)
        sh = self._shape(shape_id)
        self._seed_keep = (P, sh)           # the kernel reads them on the stream
        self._check(self.L.am_seed_points(self.h, _p(P), _p(sh), P.shape[0]))

    def seed_points_st(self, pts, max_iter=64, shape_id=None):
        """Sphere-tracing seeds from start points; returns (status, iters, x) device tensors."""
        t = self.torch
        P = self._dev(pts, t.float64).reshape(-1, 3)
        sh = self._shape(shape_id)
        n = P.shape[0]
        status = t.empty(n, dtype=t.int32, device=self.device)
        iters = t.empty(n, dtype=t.int32, device=self.device)
        x = t.empty((n, 3), dtype=t.float64, device=self.device)
        self._seed_keep = (P, sh)           # the kernel reads them on the stream
        self._check(self.L.am_seed_points_st(self.h, _p(P), _p(sh), n, int(max_iter), _p(status), _p(iters), _p(x)))
        return status, iters, x

    def march(self, max_cells=0, max_steps=0, strict=False, time_kernels=False, kernel_path=0, precision=0,
              margin=0.0, vertex_tol=0.0, propose=0, chain_groups=0, graph_steps=0, face_routine=0,
              wait=True, wait_limit=0):
        """am_march; with wait=False it returns None at once (asynchronous
        march) and wait() gives its stats."""
        opts = MarchOpts(int(max_cells), int(max_steps), int(bool(strict)), int(bool(time_kernels)),
                         int(kernel_path), int(precision), int(propose), int(chain_groups), int(graph_steps),
                         int(face_routine), 0 if wait else 1)
        opts.margin = float(margin)
        opts.vertex_tol = float(vertex_tol)
        opts.wait_limit = int(wait_limit)
        stats = MarchStats()
        st = self.L.am_march(self.h, C.byref(opts), C.byref(stats))
        if st != AM_OK:
            err = AmError(st, self.L.am_last_error(self.h).decode())
            err.stats = stats.as_dict()
            raise err
        return stats.as_dict() if wait else None

    def wait(self):
        """am_wait: the stats of the asynchronous march (raises on its error)."""
        stats = MarchStats()
        st = self.L.am_wait(self.h, C.byref(stats))
        if st != AM_OK:
            err = AmError(st, self.L.am_last_error(self.h).decode())
            err.stats = stats.as_dict()
            raise err
        return stats.as_dict()

    def busy(self):
        b = C.c_int32()
        self._check(self.L.am_busy(self.h, C.byref(b)))
        return bool(b.value)

    # ------------------------------------------------------------ chain tiles
    def tune_chain(self, reps=5):
        """Times the chain tiles on the last march's cells and keeps the
        fastest per launch size; returns (variants[4], ms[4][CHAIN_VARIANTS])
        (-1 for a variant that cannot run on the loaded net)."""
        import numpy as np
        ms = np.zeros(4 * CHAIN_VARIANTS, dtype=np.float32)
        self._check(self.L.am_tune_chain(self.h, int(reps), ms.ctypes.data_as(C.c_void_p)))
        return self.chain_groups(), ms.reshape(4, CHAIN_VARIANTS)

    def chain_groups(self):
        import numpy as np
        g = np.zeros(4, dtype=np.int32)
        self._check(self.L.am_get_chain_groups(self.h, g.ctypes.data_as(C.c_void_p)))
        return [int(x) for x in g]

    def set_chain_groups(self, groups):
        import numpy as np
        g = np.ascontiguousarray(np.asarray(groups, dtype=np.int32))
        assert g.shape == (4,)
        self._check(self.L.am_set_chain_groups(self.h, g.ctypes.data_as(C.c_void_p)))

    # ------------------------------------------------------------ learned form
    def prop_param_count(self):
        return int(self.L.am_prop_param_count())

    def prop_set(self, params, k=16, rho=6.0):
        """Loads the proposal scorer (host FP32 parameters, flat)."""
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        self._check(self.L.am_prop_set(self.h, p.ctypes.data_as(C.c_void_p), p.size, int(k), float(rho)))

    def prop_collect(self, samples, labels, rho=6.0):
        """Later marches append training rows to the device tensors samples
        [cap][32] float32 and labels [cap] uint8 (None: stop collecting)."""
        if samples is None:
            self._check(self.L.am_prop_collect(self.h, None, None, 0, float(rho)))
            return
        assert samples.dtype == self.torch.float32 and samples.shape[1] == 32 and labels.dtype == self.torch.uint8
        assert samples.is_contiguous() and labels.is_contiguous() and labels.shape[0] == samples.shape[0]
        self._check(self.L.am_prop_collect(self.h, _p(samples), _p(labels), samples.shape[0], float(rho)))

    def prop_collected(self):
        n = C.c_int64()
        self._check(self.L.am_prop_collected(self.h, C.byref(n)))
        return n.value

    def prop_grad(self, X, y, params, grad):
        """Mean BCE loss (returned) and its gradient into `grad` (device tensors)."""
        loss = C.c_double()
        n = X.shape[0]
        assert X.dtype == self.torch.float32 and X.shape[1] == 32 and X.is_contiguous()
        assert y.dtype == self.torch.uint8 and y.shape[0] == n and params.is_contiguous() and grad.is_contiguous()
        self._check(self.L.am_prop_grad(self.h, _p(X), _p(y), n, _p(params), _p(grad), C.byref(loss)))
        return loss.value

    def prop_adam(self, params, grad, m, v, step, lr):
        self._check(self.L.am_prop_adam(self.h, _p(params), _p(grad), _p(m), _p(v), int(step), float(lr)))

    def prop_score(self, X):
        """Logits of the rows of X (device float32 [n][32]) by the loaded scorer."""
        assert X.dtype == self.torch.float32 and X.shape[1] == 32 and X.is_contiguous()
        z = self.torch.empty(X.shape[0], dtype=self.torch.float32, device=self.device)
        self._check(self.L.am_prop_score(self.h, _p(X), X.shape[0], _p(z)))
        return z

    def counts(self):
        """(faces, corners, triangles, cells) of the last march."""
        f, v, tr, c = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.L.am_get_counts(self.h, C.byref(f), C.byref(v), C.byref(tr), C.byref(c)))
        return f.value, v.value, tr.value, c.value

    def fetch(self, sorted=False, where=AM_DEVICE):
        """The mesh (faces in discovery order, or with sorted=True in
        canonical order: shape, code words, argmax) as device tensors, or with
        where=AM_HOST as numpy arrays filled by the library's host copy."""
        t = self.torch
        F, V, _, _ = self.counts()
        if where == AM_HOST:
            out = dict(offsets=np.empty(F + 1, np.int64), ids=np.empty(V, np.int32), verts=np.empty((V, 3)),
                       nbr=np.empty(V, np.int64), codes=np.empty((F, self.W), np.int64), argmax=np.empty(F, np.int32),
                       shape=np.empty(F, np.int32))
            ptr = {k: C.c_void_p(v.ctypes.data) for k, v in out.items()}
        else:
            dev = self.device
            out = dict(offsets=t.empty(F + 1, dtype=t.int64, device=dev), ids=t.empty(V, dtype=t.int32, device=dev),
                       verts=t.empty((V, 3), dtype=t.float64, device=dev), nbr=t.empty(V, dtype=t.int64, device=dev),
                       codes=t.empty((F, self.W), dtype=t.int64, device=dev),
                       argmax=t.empty(F, dtype=t.int32, device=dev), shape=t.empty(F, dtype=t.int32, device=dev))
            ptr = {k: _p(v) for k, v in out.items()}
        fn = self.L.am_fetch_sorted if sorted else self.L.am_fetch
        self._check(fn(self.h, int(where), ptr["offsets"], ptr["ids"], ptr["verts"], ptr["nbr"], ptr["codes"],
                       ptr["argmax"], ptr["shape"]))
        return out


    def weld(self, mesh, positions=True):
        """Shared vertices of a fetched mesh (the dict fetch() returns).

        Returns (corner_vertex [corners] int64, vxyz [V][3] float64 or None,
        n_unpaired), all on the device but n_unpaired.
        """
        t = self.torch
        F = mesh["offsets"].shape[0] - 1
        n = mesh["ids"].shape[0]
        cv = t.empty(n, dtype=t.int64, device=self.device)
        vx = t.empty((max(n, 1), 3), dtype=t.float64, device=self.device) if positions else None
        nv, unp = C.c_int64(), C.c_int64()
        am = mesh.get("argmax")
        self._check(self.L.am_weld(self.h, F, _p(mesh["offsets"]), _p(mesh["ids"]), _p(mesh["nbr"]), _p(am),
                                   _p(mesh["verts"]), n, _p(cv), _p(vx), vx.shape[0] if positions else 0,
                                   C.byref(nv), C.byref(unp)))
        return cv, (vx[:nv.value] if positions else None), unp.value

    def triangles(self, offsets, corner_vertex):
        """Fan triangles [corners - 2 faces][3] int64 (device) of welded polygons."""
        t = self.torch
        F = offsets.shape[0] - 1
        T = max(corner_vertex.shape[0] - 2 * F, 0)
        tri = t.empty((max(T, 1), 3), dtype=t.int64, device=self.device)
        self._check(self.L.am_triangles(self.h, F, _p(offsets), _p(corner_vertex), _p(tri), T))
        return tri[:T]


    def simplify(self, vxyz, tri, target_tris, max_rounds=0, boundary=None):
        """Quadric edge-collapse simplification of a welded triangle mesh
        (device tensors); returns (vertices, triangles, rounds, dropped)."""
        t = self.torch
        V, T = vxyz.shape[0], tri.shape[0]
        assert vxyz.dtype == t.float64 and tri.dtype == t.int64 and vxyz.is_contiguous() and tri.is_contiguous()
        v_out = t.empty((V, 3), dtype=t.float64, device=self.device)
        t_out = t.empty((T, 3), dtype=t.int64, device=self.device)
        nv, nt, r, bad = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int64()
        self._check(self.L.am_simplify(self.h, V, _p(vxyz), T, _p(tri), _p(boundary), int(target_tris),
                                       int(max_rounds), _p(v_out), _p(t_out), C.byref(nv), C.byref(nt), C.byref(r),
                                       C.byref(bad)))
        return v_out[:nv.value], t_out[:nt.value], r.value, bad.value


def mesh_to_host(out):
    """Device mesh dict -> numpy arrays (codes as uint64)."""
    h = {k: v.cpu().numpy() for k, v in out.items()}
    h["codes"] = h["codes"].view(np.uint64)
    return h
