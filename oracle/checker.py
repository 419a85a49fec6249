"""TEST INFRASTRUCTURE ONLY -- brute-force topology used to pin the oracle.

Nothing here is shared with the oracle's C++ or with the GPU library: the mesh
is rebuilt from its simplices (the Kuhn/Freudenthal subdivision of each grid
cube into d! simplices along the main diagonal), links are read off the
simplicial complex, and merge trees are computed by the textbook union-find
sweep (Carr, Snoeyink and Axen 2003), which the paper cites as the reference
construction of join, split and contour trees (Sec. 3.1).

Everything is pure Python on tiny fields (a few hundred vertices).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


# ----------------------------------------------------------------------------
# simplicial complex of the grid


class Complex:
    """Kuhn triangulation of an nx x ny x nz vertex grid (unused dims = 1)."""

    def __init__(self, shape_xyz):
        dims = [d for d in shape_xyz]
        self.ndim = len(dims)
        self.dims = dims + [1] * (3 - len(dims))
        nx, ny, nz = self.dims
        self.n = nx * ny * nz
        d = self.ndim
        simplices = set()
        # every grid cell [c, c+1]^d is cut into d! simplices, one per
        # permutation of the axes: corner, +e_p1, +e_p1+e_p2, ...
        cells = itertools.product(*[range(max(self.dims[k] - 1, 0)) for k in range(d)])
        for c in cells:
            for perm in itertools.permutations(range(d)):
                p = list(c)
                verts = [self._index(p)]
                for ax in perm:
                    p[ax] += 1
                    verts.append(self._index(p))
                simplices.add(tuple(sorted(verts)))
        if self.n == 1:
            simplices.add((0,))
        # all faces
        faces = set()
        for s in simplices:
            for k in range(1, len(s) + 1):
                for sub in itertools.combinations(s, k):
                    faces.add(sub)
        for v in range(self.n):
            faces.add((v,))
        self.faces = faces
        self.nbrs = [set() for _ in range(self.n)]
        for s in faces:
            if len(s) == 2:
                a, b = s
                self.nbrs[a].add(b)
                self.nbrs[b].add(a)
        # link of v: faces tau with v not in tau and tau + v a face
        self.link = [[] for _ in range(self.n)]
        for s in faces:
            for v in s:
                tau = tuple(u for u in s if u != v)
                if tau:
                    self.link[v].append(tau)

    def _index(self, p):
        p = list(p) + [0] * (3 - len(p))
        return p[0] + self.dims[0] * (p[1] + self.dims[1] * p[2])

    def coords(self, i):
        nx, ny, _ = self.dims
        return (i % nx, (i // nx) % ny, i // (nx * ny))


def sos_less(h, i, j):
    return h[i] < h[j] or (h[i] == h[j] and i < j)


def _components(verts, edges):
    parent = {v: v for v in verts}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    return len({find(v) for v in verts})


def local(cx: Complex, h, v):
    """Lower/upper link sub-complexes of v, their component counts, Euler char."""
    lower = [t for t in cx.link[v] if all(sos_less(h, u, v) for u in t)]
    upper = [t for t in cx.link[v] if all(sos_less(h, v, u) for u in t)]
    lv = {t[0] for t in lower if len(t) == 1}
    uv = {t[0] for t in upper if len(t) == 1}
    lc = _components(lv, [t for t in lower if len(t) == 2])
    uc = _components(uv, [t for t in upper if len(t) == 2])
    chi = sum((-1) ** (len(t) - 1) for t in lower)
    return lv, uv, lc, uc, chi


REGULAR, MINIMUM, MAXIMUM, SADDLE = 0, 1, 2, 3


def classify(cx: Complex, h):
    """Per vertex: type, lc, uc, chi(lower link), asc, desc."""
    h = np.asarray(h).ravel()
    out = []
    for v in range(cx.n):
        lv, uv, lc, uc, chi = local(cx, h, v)
        if not lv:
            t = MINIMUM
        elif not uv:
            t = MAXIMUM
        elif lc == 1 and uc == 1:
            t = REGULAR
        else:
            t = SADDLE
        closed = list(cx.nbrs[v]) + [v]
        asc = closed[0]
        desc = closed[0]
        for u in closed:
            if sos_less(h, asc, u):
                asc = u
            if sos_less(h, u, desc):
                desc = u
        out.append({"type": t, "lc": lc, "uc": uc, "chi": chi, "asc": asc,
                    "desc": desc, "lower": lv, "upper": uv})
    return out


def euler_sum(cx: Complex, h):
    """Sum over vertices of 1 - chi(lower link); equals chi(domain) = 1."""
    h = np.asarray(h).ravel()
    return sum(1 - local(cx, h, v)[4] for v in range(cx.n))


# ----------------------------------------------------------------------------
# extremum graph


def extremum_graph(cx: Complex, h, info=None):
    """Critical points with types, and saddle -> extremum edges.

    An edge joins saddle s to minimum m when the steepest-descent path from a
    lower neighbour of s ends at m, and to maximum M when the steepest-ascent
    path from an upper neighbour ends at M (Sec. 3.1-3.2).
    """
    h = np.asarray(h).ravel()
    info = info or classify(cx, h)

    def term(v, key):
        while info[v][key] != v:
            v = info[v][key]
        return v

    cps = {v: info[v]["type"] for v in range(cx.n) if info[v]["type"] != REGULAR}
    edges = set()
    for s, t in cps.items():
        if t != SADDLE:
            continue
        for k in info[s]["lower"]:
            edges.add((s, "min", term(k, "desc")))
        for k in info[s]["upper"]:
            edges.add((s, "max", term(k, "asc")))
    return cps, edges


def saddle_sequence(cx: Complex, f, h):
    """Saddles of f (by the brute-force link analysis of f), listed in
    ascending SoS order of h.  The saddle ordering constraint (Sec. 4.2, C2)
    holds on h exactly when this equals the list in f's order."""
    f = np.asarray(f).ravel()
    h = np.asarray(h).ravel()
    info = classify(cx, f)
    sad = [v for v in range(cx.n) if info[v]["type"] == SADDLE]
    return sorted(sad, key=lambda v: (h[v], v))


def event_selections(cx: Complex, f, h):
    """Per saddle of f, the extremum EGP pairs it with in h (Sec. 4.2, C3).

    For a join saddle s of f (lower link of s in f has two or more pieces):
    the highest minimum in h among the minima that steepest-descent paths of
    h reach from the lower neighbours of s in h.  For a split saddle of f:
    the lowest maximum among those steepest-ascent paths of h reach from its
    upper neighbours in h.  Paths, links and pointers are the checker's own
    (simplicial complex, closed-neighbourhood SoS pointers).  Returns a dict
    {(s, "join"|"split"): extremum}.
    """
    f = np.asarray(f).ravel()
    h = np.asarray(h).ravel()
    fi = classify(cx, f)
    hi = classify(cx, h)

    def term(v, key):
        while hi[v][key] != v:
            v = hi[v][key]
        return v

    out = {}
    for s in range(cx.n):
        if fi[s]["type"] != SADDLE:
            continue
        if fi[s]["lc"] >= 2 and hi[s]["lower"]:
            reach = {term(k, "desc") for k in hi[s]["lower"]}
            out[(s, "join")] = max(reach, key=lambda m: (h[m], m))
        if fi[s]["uc"] >= 2 and hi[s]["upper"]:
            reach = {term(k, "asc") for k in hi[s]["upper"]}
            out[(s, "split")] = min(reach, key=lambda m: (h[m], m))
    return out


# ----------------------------------------------------------------------------
# merge trees and contour tree (union-find sweeps)


def _sweep(cx: Complex, h, ascending=True):
    """Augmented merge tree: for each vertex, the vertices it connects down to.

    Sweeping in SoS order, vertex v is joined to the current "tip" (last added
    vertex) of every distinct earlier component among its neighbours.
    Returns dict v -> sorted list of earlier vertices (tree arcs), and the
    persistence pairs (born-at extremum, died-at vertex) by the elder rule.
    """
    order = sorted(range(cx.n), key=lambda i: (h[i], i), reverse=not ascending)
    # SoS with index ties: sorting by (value, index) is exactly SoS order.
    pos = {v: k for k, v in enumerate(order)}
    parent = list(range(cx.n))
    tip = list(range(cx.n))
    birth = list(range(cx.n))  # extremum that created the component (root-indexed)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    down = {}
    pairs = []
    for v in order:
        roots = sorted({find(u) for u in cx.nbrs[v] if pos[u] < pos[v]},
                       key=lambda r: pos[birth[r]])
        down[v] = sorted(tip[r] for r in roots)
        # elder rule: the component born earliest survives
        for r in roots[1:]:
            pairs.append((birth[r], v))
        if roots:
            keep = roots[0]
            for r in roots[1:]:
                parent[r] = keep
            parent[v] = keep
            tip[keep] = v
        else:
            tip[v] = v
            birth[v] = v
    return down, pairs


def join_tree(cx, h):
    h = np.asarray(h).ravel()
    return _sweep(cx, h, ascending=True)


def split_tree(cx, h):
    h = np.asarray(h).ravel()
    return _sweep(cx, h, ascending=False)


def _contract(adj):
    """Remove degree-2 vertices whose arcs go one up and one down."""
    adj = {v: set(a) for v, a in adj.items()}
    changed = True
    while changed:
        changed = False
        for v in list(adj):
            if len(adj[v]) == 2:
                a, b = tuple(adj[v])
                adj[a].discard(v)
                adj[b].discard(v)
                adj[a].add(b)
                adj[b].add(a)
                del adj[v]
                changed = True
    return {frozenset((a, b)) for a in adj for b in adj[a]}, set(adj)


def tree_arcs(down):
    """Unaugmented tree: arcs between nodes after contracting degree-2 vertices."""
    adj = {v: set() for v in down}
    for v, ds in down.items():
        for u in ds:
            adj[v].add(u)
            adj[u].add(v)
    return _contract(adj)


def contour_tree(cx, h):
    """Contour tree from the augmented join and split trees (Carr et al.)."""
    h = np.asarray(h).ravel()
    jdown, _ = join_tree(cx, h)
    sdown, _ = split_tree(cx, h)
    # join tree: arcs from v down to earlier (lower) vertices; split tree:
    # arcs from v to earlier (higher) vertices.
    J_up = {v: set() for v in range(cx.n)}
    J_dn = {v: set(jdown[v]) for v in range(cx.n)}
    for v, ds in jdown.items():
        for u in ds:
            J_up[u].add(v)
    S_dn = {v: set() for v in range(cx.n)}
    S_up = {v: set(sdown[v]) for v in range(cx.n)}
    for v, us in sdown.items():
        for u in us:
            S_dn[u].add(v)
    alive = set(range(cx.n))
    ct = set()
    queue = [v for v in alive if len(J_dn[v]) + len(S_up[v]) == 1]
    while len(alive) > 1:
        progressed = False
        for v in list(queue):
            if v not in alive or len(J_dn[v]) + len(S_up[v]) != 1:
                continue
            if len(J_dn[v]) == 0:  # lower leaf: arc to its join-tree parent
                (w,) = J_up[v]
                ct.add(frozenset((v, w)))
            else:  # upper leaf: arc to its split-tree child
                (w,) = S_dn[v]
                ct.add(frozenset((v, w)))
            for T_up, T_dn in ((J_up, J_dn), (S_dn, S_up)):
                # remove v from the tree, splicing its neighbours together
                ups, dns = T_up[v], T_dn[v]
                for a in ups:
                    T_dn[a].discard(v)
                for b in dns:
                    T_up[b].discard(v)
                for a in ups:
                    for b in dns:
                        T_dn[a].add(b)
                        T_up[b].add(a)
                T_up[v] = set()
                T_dn[v] = set()
            alive.discard(v)
            progressed = True
        queue = [v for v in alive if len(J_dn[v]) + len(S_up[v]) == 1]
        if not progressed and len(alive) > 1:
            raise RuntimeError("contour tree combine stalled")
    adj = {v: set() for v in range(cx.n)}
    for e in ct:
        a, b = tuple(e)
        adj[a].add(b)
        adj[b].add(a)
    return _contract(adj)


def eg_pairs(cx, h, info=None):
    """Minimum--join-saddle pairs extracted from the extremum graph alone.

    Join saddles are visited in ascending order; each merges the minimum
    components it is connected to in the extremum graph, and every component
    except the one with the lowest minimum is paired with the saddle (the
    pairing rule of Extremum Graph Pairing, Sec. 3.2).  By the merge-tree
    equivalence of ExTreeM this must equal the elder-rule pairs of the full
    sublevel-set sweep.
    """
    h = np.asarray(h).ravel()
    info = info or classify(cx, h)
    cps, edges = extremum_graph(cx, h, info)
    conn = {}
    for s, kind, m in edges:
        if kind == "min":
            conn.setdefault(s, set()).add(m)
    parent = {m: m for m, t in cps.items() if t == MINIMUM}

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a

    pairs = []
    for s in sorted(conn, key=lambda v: (h[v], v)):
        roots = sorted({find(m) for m in conn[s]}, key=lambda r: (h[r], r))
        for r in roots[1:]:
            pairs.append((r, s))
            parent[r] = roots[0]
    return sorted(pairs)


def topology_signature(cx, h):
    """Everything the corrected field must share with the original."""
    h = np.asarray(h).ravel()
    info = classify(cx, h)
    cps, eg = extremum_graph(cx, h, info)
    jd, jp = join_tree(cx, h)
    sd, sp = split_tree(cx, h)
    return {
        "critical": cps,
        "eg": eg,
        "join_arcs": tree_arcs(jd)[0],
        "split_arcs": tree_arcs(sd)[0],
        "join_pairs": sorted(jp),
        "split_pairs": sorted(sp),
        "contour_arcs": contour_tree(cx, h)[0],
    }


# ----------------------------------------------------------------------------
# vulnerability graph and iteration bound (Sec. 4.4)


def _frac(x):
    return Fraction(float(x))


def lower_bounds_exact(f, xi_T):
    """L_u = smallest value of f's dtype >= f_u - xi_T, by exact rationals."""
    f = np.asarray(f)
    out = np.empty_like(f)
    for idx, v in np.ndenumerate(f):
        target = _frac(v) - _frac(xi_T)
        c = f.dtype.type(float(target))  # round to nearest in the dtype
        if _frac(c) < target:
            c = np.nextafter(c, f.dtype.type(np.inf))
        elif _frac(c) > target:
            p = np.nextafter(c, f.dtype.type(-np.inf))
            if _frac(p) >= target:
                c = p
        out[idx] = c
    return out


def vulnerability(cx, f, g_hat, xi_T, extra_pairs=()):
    """Weak/strong/reduced vulnerability graphs and D_max of the reduced one.

    Candidate pairs are the vertex pairs that a check can compare: any two
    members of a closed neighbourhood N[i], plus consecutive critical points
    of f in sorted order.  Edge u -> v when f ranks u above v (SoS) and
    |f_u - f_v| <= 2 xi_T (G_V); kept in G_S unless g_hat_v < L_u; seeds are
    G_S edges already inverted in g_hat.  D_max counts vertices on the
    longest path of G_S that starts at a seed endpoint.
    """
    f = np.asarray(f).ravel()
    g = np.asarray(g_hat).ravel()
    L = lower_bounds_exact(f, xi_T)
    info = classify(cx, f)
    critical_order = sorted((v for v in range(cx.n) if info[v]["type"] != REGULAR),
                            key=lambda v: (f[v], v))
    pairs = set()
    for i in range(cx.n):
        closed = sorted(cx.nbrs[i] | {i})
        for a, b in itertools.combinations(closed, 2):
            pairs.add((a, b))
    for a, b in zip(critical_order[:-1], critical_order[1:]):
        pairs.add((min(a, b), max(a, b)))
    for a, b in extra_pairs:
        pairs.add((min(a, b), max(a, b)))
    two_xi = 2 * _frac(xi_T)
    GV, GS, seeds = set(), set(), set()
    for a, b in pairs:
        u, v = (a, b) if sos_less(f, b, a) else (b, a)  # u above v in f
        if abs(_frac(f[u]) - _frac(f[v])) <= two_xi:
            GV.add((u, v))
            if not (g[v] < L[u]):
                GS.add((u, v))
                if sos_less(g, u, v):
                    seeds.add((u, v))
    succ = {}
    for u, v in GS:
        succ.setdefault(u, []).append(v)
    start = {u for u, v in seeds} | {v for u, v in seeds}
    reach = set(start)
    stack = list(start)
    while stack:
        u = stack.pop()
        for v in succ.get(u, ()):
            if v not in reach:
                reach.add(v)
                stack.append(v)
    # longest path (vertex count) within the reachable part of the DAG G_S,
    # starting at seed endpoints; edges go strictly down in SoS(f).
    order = sorted(reach, key=lambda i: (f[i], i), reverse=True)
    dep = {v: (1 if v in start else 0) for v in reach}
    for u in order:
        if dep[u] == 0:
            continue
        for v in succ.get(u, ()):
            if v in reach and dep[u] + 1 > dep[v]:
                dep[v] = dep[u] + 1
    dmax = max(dep.values(), default=0)
    verts = lambda E: {x for e in E for x in e}
    return {"GV": GV, "GS": GS, "seeds": seeds, "GR_vertices": reach,
            "V_GV": verts(GV), "V_GS": verts(GS), "D_max": dmax}
