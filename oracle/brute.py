"""Brute-force analytic faces for tiny nets: a pin for the marching oracle.

TEST INFRASTRUCTURE ONLY.  Independent of ``am_oracle.c`` (shares no code with
it): numpy, every activation code enumerated, each face found by the paper's
naive enumeration (Algorithm 1, the pair loop): solve the 3x3 system of Eqn
(VertexEquationSystem) for every pair of constraint planes, keep the solutions
that satisfy the cell system of Eqn (AnalyticCellSystem) (plus the max-pool
sub-cell rows of Eqn (AnalyticCellSystemMaxPooling) and the domain box), and
order the valid vertices around their centroid.

A code whose face has positive area is an analytic cell; the result is the set
of all analytic faces in the domain box, each with its CCW cycle of constraint
ids (seen from +grad F), starting at the smallest id, and its vertices.

Conventions shared with the oracle as a *specification* (not code): box plane
ids -1..-6 = x<=1, x>=-1, y<=1, y>=-1, z<=1, z>=-1; max-pool comparison rows
have id N+i; tolerance rule |c.[x;1]| <= TAU (|c_xyz| (1 + |x|) + |c_w|),
TAU = 2^-40.
"""
from __future__ import annotations

import itertools

import numpy as np

TAU = 2.0 ** -40


def forward_pre(net, X):
    """Pre-activations of every hidden unit and head at points X[P,3]."""
    X = np.atleast_2d(np.asarray(X, np.float64))
    acts = {0: X}
    pres = []
    L2 = len(net.widths)
    for l in range(1, L2):
        a = np.tile(net.bias[l - 1], (X.shape[0], 1))
        for d, s, W in net.blocks:
            if d == l:
                a = a + acts[s] @ W.T
        pres.append(a)
        acts[l] = np.maximum(a, 0.0) if l < L2 - 1 else a
    return np.concatenate(pres, axis=1)


def chains(net, bits):
    """Affine rows for many codes at once: bits[C, N] (0/1) -> rows[C, N+M, 4].

    Row g of code c gives the pre-activation of unit g as an affine function of
    x inside the region of code c (Lemma 1 / Corollary 1 of the paper).
    """
    Cn = bits.shape[0]
    L2 = len(net.widths)
    offs = np.cumsum([0] + net.widths[1:])       # global offset of layer l is offs[l-1]
    Z = {0: np.broadcast_to(np.hstack([np.eye(3), np.zeros((3, 1))]), (Cn, 3, 4))}
    out = []
    for l in range(1, L2):
        z = np.zeros((Cn, net.widths[l], 4))
        z[:, :, 3] = net.bias[l - 1]
        for d, s, W in net.blocks:
            if d != l:
                continue
            src = Z[s]
            if s > 0:
                o = offs[s - 1]
                src = src * bits[:, o:o + net.widths[s], None]
            z = z + np.einsum("km,cmq->ckq", W, src)
        Z[l] = z
        out.append(z)
    return np.concatenate(out, axis=1)


def _box_rows():
    rows, ids = [], []
    for a in range(3):
        for lower in (0, 1):
            c = np.zeros(4)
            c[a] = -1.0 if lower else 1.0
            c[3] = -1.0
            rows.append(c)
            ids.append(-1 - (2 * a + lower))
    return np.array(rows), np.array(ids)


def _tol(c, x):
    return TAU * (np.linalg.norm(c[..., :3], axis=-1) * (1.0 + np.linalg.norm(x, axis=-1)) + np.abs(c[..., 3]))


def face_by_pairs(rows_all, bits, argmax, N, M):
    """Face of one cell by naive pair enumeration.

    Returns (ids cycle, vertices) or None if the face has no positive area.
    """
    box_rows, box_ids = _box_rows()
    aF = rows_all[N + argmax]
    if not np.any(aF[:3]):
        return None
    sgn = 1.0 - 2.0 * bits[:N]
    cons = [box_rows, sgn[:, None] * rows_all[:N]]
    ids = [box_ids, np.arange(N)]
    others = [i for i in range(M) if i != argmax]
    if others:
        cons.append(rows_all[N + np.array(others)] - aF[None])
        ids.append(N + np.array(others))
    cons = np.concatenate(cons)
    ids = np.concatenate(ids)
    K = len(ids)
    pairs = np.array(list(itertools.combinations(range(K), 2)))
    A = np.stack([cons[pairs[:, 0], :3], cons[pairs[:, 1], :3],
                  np.broadcast_to(aF[:3], (len(pairs), 3))], axis=1)
    r = -np.stack([cons[pairs[:, 0], 3], cons[pairs[:, 1], 3],
                   np.broadcast_to(aF[3], (len(pairs),))], axis=1)
    det = np.linalg.det(A)
    scale = np.prod(np.linalg.norm(A, axis=2), axis=1)
    ok = np.abs(det) > 1e-13 * scale
    if not ok.any():
        return None
    X = np.linalg.solve(A[ok], r[ok][..., None])[..., 0]
    vals = X @ cons[:, :3].T + cons[None, :, 3]                      # [P, K]
    tol = TAU * (np.linalg.norm(cons[None, :, :3], axis=-1) * (1.0 + np.linalg.norm(X, axis=-1))[:, None]
                 + np.abs(cons[None, :, 3]))
    valid = np.all(vals <= tol, axis=1)
    X = X[valid]
    vals = vals[valid]
    tol = tol[valid]
    if len(X) < 3:
        return None
    # merge coincident solutions (several pairs meet at one point)
    pts, on = [], []
    for x, v, t in zip(X, vals, tol):
        for j, p in enumerate(pts):
            if np.max(np.abs(p - x)) <= 1e-9 * (1.0 + np.max(np.abs(x))):
                on[j] |= np.abs(v) <= t
                break
        else:
            pts.append(x)
            on.append(np.abs(v) <= t)
    if len(pts) < 3:
        return None
    pts = np.array(pts)
    on = np.array(on)                                                # [V, K]
    n = aF[:3] / np.linalg.norm(aF[:3])
    cen = pts.mean(axis=0)
    ref = pts[0] - cen
    ref2 = np.cross(n, ref)
    ang = np.arctan2((pts - cen) @ ref2, (pts - cen) @ ref)
    order = np.argsort(ang)                                          # CCW about +n
    pts, on = pts[order], on[order]
    m = len(pts)
    area2 = sum(np.dot(np.cross(pts[i] - cen, pts[(i + 1) % m] - cen), n) for i in range(m))
    if not area2 > 0:
        return None
    cyc = []
    for i in range(m):
        shared = np.nonzero(on[i] & on[(i + 1) % m])[0]
        if len(shared) != 1:
            raise RuntimeError(f"edge {i} lies on {len(shared)} constraints (degenerate net)")
        cyc.append(int(ids[shared[0]]))
    cyc = np.array(cyc)
    r0 = int(np.argmin(cyc))
    return np.roll(cyc, -r0), np.roll(pts, -r0, axis=0)


def all_faces(net):
    """Every analytic face of a net with at most ~16 hidden units.

    Returns a dict {(code bits as a tuple, argmax): (ids, verts)}.  A cheap
    vectorised pass first keeps the codes with at least three valid pair
    solutions; those get the full per-face construction above.
    """
    N, M = net.n_hidden, net.n_heads
    if N > 20:
        raise ValueError("brute force is for tiny nets")
    box_rows, _ = _box_rows()
    faces = {}
    n_codes = 1 << N
    chunk = 2048
    for c0 in range(0, n_codes, chunk):
        cs = np.arange(c0, min(n_codes, c0 + chunk))
        bits = ((cs[:, None] >> np.arange(N)[None, :]) & 1).astype(np.float64)
        R = chains(net, bits)
        for am in range(M):
            aF = R[:, N + am]                                          # [C, 4]
            cons = [np.broadcast_to(box_rows, (len(cs), 6, 4)),
                    (1.0 - 2.0 * bits)[:, :, None] * R[:, :N]]
            others = [i for i in range(M) if i != am]
            if others:
                cons.append(R[:, N + np.array(others)] - aF[:, None])
            cons = np.concatenate(cons, axis=1)                        # [C, K, 4]
            K = cons.shape[1]
            pairs = np.array(list(itertools.combinations(range(K), 2)))
            A = np.stack([cons[:, pairs[:, 0], :3], cons[:, pairs[:, 1], :3],
                          np.broadcast_to(aF[:, None, :3], (len(cs), len(pairs), 3))], axis=2)
            r = -np.stack([cons[:, pairs[:, 0], 3], cons[:, pairs[:, 1], 3],
                           np.broadcast_to(aF[:, None, 3], (len(cs), len(pairs)))], axis=2)
            # Cramer's rule, vectorised (only a filter: faces are rebuilt below)
            c0_, c1_, c2_ = A[..., 0], A[..., 1], A[..., 2]
            det = np.einsum("...i,...i->...", c0_, np.cross(c1_, c2_))
            scale = np.prod(np.linalg.norm(A, axis=3), axis=2)
            ok = np.abs(det) > 1e-13 * np.maximum(scale, 1e-300)
            dsafe = np.where(ok, det, 1.0)
            X = np.stack([np.einsum("...i,...i->...", r, np.cross(c1_, c2_)),
                          np.einsum("...i,...i->...", c0_, np.cross(r, c2_)),
                          np.einsum("...i,...i->...", c0_, np.cross(c1_, r))], axis=-1) / dsafe[..., None]
            vals = np.einsum("cpj,ckj->cpk", X, cons[:, :, :3]) + cons[:, None, :, 3]
            tol = TAU * (np.linalg.norm(cons[:, None, :, :3], axis=-1)
                         * (1.0 + np.linalg.norm(X, axis=-1))[:, :, None] + np.abs(cons[:, None, :, 3]))
            valid = np.all(vals <= tol, axis=2) & ok
            cand = np.nonzero(valid.sum(axis=1) >= 3)[0]
            for i in cand:
                f = face_by_pairs(R[i], bits[i], am, N, M)
                if f is not None:
                    faces[(tuple(int(b) for b in bits[i]), am)] = f
    return faces


def bits_to_words(bits, n_words):
    w = np.zeros(n_words, np.uint64)
    for g, b in enumerate(bits):
        if b:
            w[g >> 6] |= np.uint64(1) << np.uint64(g & 63)
    return w


def words_to_bits(words, N):
    words = np.asarray(words, np.uint64)
    return tuple(int((int(words[g >> 6]) >> (g & 63)) & 1) for g in range(N))
