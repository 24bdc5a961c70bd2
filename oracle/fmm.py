"""ORACLE -- test infrastructure only.

The cubed sphere fast multipole method (CSFMM) of Chen & Krasny written out
step by step in NumPy, in the order of the paper, for checking the GPU
library's tree, interaction lists, passes and results.  It shares no code with
the GPU library.  Every array is float64.

Steps and the passages they follow:
  * faces, local angles, quadtree ....... §3 (tree building)
  * Chebyshev points, barycentric L_k ... §4, eq. (barycentric), 2-D tensor form
  * proxy points in a cell .............. §4 (reference square mapped to the cell)
  * PP, PC, CP, CC ...................... §5, eqs. (PP), (PC), (CP), (CC)
  * upward pass ......................... §6, eqs. (upwardpass1), (upwardpass2)
  * dual tree traversal ................. §8, Algorithm 2 and the MAC below it
  * accumulated proxy potentials ........ §8, eq. (CP_CC_accumulated)
  * downward pass ....................... §8.1, eqs. (downward_1), (downward_2)
  * cubed sphere treecode (CSTC) ......... §7, Algorithm 1 (the comparison method)

Readings taken where the paper is silent or ambiguous:
  * Cells are equiangular: a level-l cell of a face is a square of side
    (pi/2)/2^l in the local angles (xi, eta) in [-pi/4, pi/4]^2.  A point with
    scaled angle t = (xi + pi/4)/(pi/2) lies in the level-l cell with index
    floor(2^l t) (clamped to 0..2^l-1): half-open intervals, the upper cell
    takes points on a split line.
  * The face of a point is the axis of its largest |coordinate|, ties broken
    x before y before z.  Each face carries a fixed right-handed frame
    (normal n, tangents e_a, e_b with e_a x e_b = n); xi = atan(x.e_a / x.n),
    eta = atan(x.e_b / x.n).
  * A cluster with more than N0 particles is split into its four quadrants
    (also when some are empty) unless it is at the deepest level MAX_LEVEL;
    a leaf is a cluster without children ("small" = leaf).  Without
    shrinking every cluster is its exact cubed-sphere cell.
  * Shrinking (§3, last remark on nonuniform particles; optional): the tree
    keeps the same quadrants and the same points per cluster, but the box of a
    non-empty cluster -- what its centre, radius, proxy points and local
    coordinates refer to -- is the smallest (xi, eta) rectangle holding its
    points, each half width at least SHRINK_FLOOR times the cell's half width
    (so that a cluster of one point, or of points on one grid line, keeps an
    interval to interpolate on).  The interpolation identity of §6 then holds
    with each child's own box, so the parent-child operators of eqs.
    (upwardpass2) and (downward_2) are computed per cluster.
  * Cluster centre = image of the (xi, eta) midpoint; radius = largest chord
    distance from the centre to the four corners; R = chord distance between
    centres.  Well separated means (r_t + r_s)^2 < MAC^2 R^2 (strict).
  * The reference square is mapped to a cell affinely in (xi, eta).
  * Barycentric L_k(u) at u equal to a node s_k is the Kronecker delta.
  * Traversal, one exclusive outcome per pair (T, S) with both non-empty:
      separated and not both leaves -> PC if T is a leaf, else CP if S is a
        leaf, else CC;
      not separated and not both leaves -> recurse into the children of the
        larger cluster, "larger" meaning the coarser level (tie: the target),
        and the other one if the larger is a leaf;
      both leaves -> PP.
  * The singular self term: a source is skipped for a target exactly when
    their coordinates are equal bit for bit (the i=j rule for one point set).
  * 1 - x.y is evaluated as |x-y|^2/2 (equal on the unit sphere).
  * CSTC: target x and source cluster C are well separated when
    r_C^2 < MAC^2 R^2 (strict), R = chord distance from x to the centre of C.
    A separated cluster with more than N0 points takes PC, a separated one
    with at most N0 points takes PP; a cluster that is not separated is
    opened into its children, and a leaf that is not separated takes PP
    (it has no children to open).  Empty clusters are skipped.
"""

import math

import numpy as np

MAX_LEVEL = 20
PI_4 = math.pi / 4.0
PI_2 = math.pi / 2.0
SHRINK_FLOOR = 2.0 ** -20

# (normal, e_a, e_b) for faces +x, +y, -x, -y, +z, -z, with e_a x e_b = normal
FACE_FRAMES = np.array([
    [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
    [[0, 1, 0], [-1, 0, 0], [0, 0, 1]],
    [[-1, 0, 0], [0, -1, 0], [0, 0, 1]],
    [[0, -1, 0], [1, 0, 0], [0, 0, 1]],
    [[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
    [[0, 0, -1], [0, 1, 0], [1, 0, 0]],
], dtype=np.float64)

KERNEL_POISSON = 1
KERNEL_BIOT_SAVART = 2
KERNEL_INV_DIST = 3
KERNEL_BIHARMONIC = 4
KERNEL_SAL = 5

# eq. (G_SAL_approx): Load Love number fit k'_n ~ a1/n, h'_n ~ b0 + b1/n (§2.4)
SAL_A1, SAL_B0, SAL_B1 = -2.7, -6.21196, 6.1
# seawater over mean Earth density; the paper names the ratio, not its value
SAL_RHO_RATIO = 1025.0 / 5514.0


# ---------------------------------------------------------------- kernels

def kernel_matrix(kernel, X, Y):
    """K(x_i, y_j) for all pairs; exact coincidences give 0 (self term).

    Poisson (eq. G_L): -(1/4pi) ln(1 - x.y).  Biot-Savart (eq. K_BS):
    -(1/4pi) (x cross y)/(1 - x.y), shape [M,N,3].  Inverse distance: 1/|x-y|.
    Biharmonic (eq. G_B): (1/4pi) dilog((1 + x.y)/2), with SciPy's Spence
    function spence(z) = dilog(1 - z) taken at z = 1 - (1 + x.y)/2 = |x-y|^2/4.
    SAL (eq. G_SAL_approx): (3 rw/(4 pi re)) ((1 - b0)/g - (a1 - b1)
    ln(g/2 + g^2/4)), g = |x-y|.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    D = X[:, None, :] - Y[None, :, :]
    d = 0.5 * np.einsum("ijk,ijk->ij", D, D)  # 1 - x.y on the sphere
    same = np.all(X[:, None, :] == Y[None, :, :], axis=-1)
    dd = np.where(same, 1.0, d)
    if kernel == KERNEL_POISSON:
        K = -np.log(dd) / (4.0 * np.pi)
        K[same] = 0.0
    elif kernel == KERNEL_INV_DIST:
        K = 1.0 / np.sqrt(2.0 * dd)
        K[same] = 0.0
    elif kernel == KERNEL_BIHARMONIC:
        from scipy.special import spence
        K = spence(np.minimum(0.5 * d, 1.0)) / (4.0 * np.pi)
        K[same] = 0.0
    elif kernel == KERNEL_SAL:
        g = np.sqrt(2.0 * dd)
        K = (3.0 * SAL_RHO_RATIO / (4.0 * np.pi)) * (
            (1.0 - SAL_B0) / g - (SAL_A1 - SAL_B1) * np.log(0.5 * g + 0.25 * g * g))
        K[same] = 0.0
    elif kernel == KERNEL_BIOT_SAVART:
        C = np.cross(X[:, None, :], Y[None, :, :])
        K = -C / (4.0 * np.pi * dd[:, :, None])
        K[same] = 0.0
    else:
        raise ValueError("unknown kernel %r" % (kernel,))
    return K


def apply_kernel(kernel, X, Y, w):
    """sum_j K(x_i, y_j) w_j (vector valued for Biot-Savart)."""
    K = kernel_matrix(kernel, X, Y)
    if K.ndim == 3:
        return np.einsum("ijk,j->ik", K, w)
    return K @ w


# ----------------------------------------------- §4 barycentric Lagrange

def chebyshev_points(n):
    """s_k = cos(k pi / n), k = 0..n (§4)."""
    return np.cos(np.arange(n + 1) * np.pi / n)


def barycentric_weights(n):
    """(-1)^k, halved at k = 0 and k = n (eq. barycentric)."""
    b = np.array([(-1.0) ** k for k in range(n + 1)])
    b[0] *= 0.5
    b[n] *= 0.5
    return b


def lagrange(n, u):
    """L_k(u) for every u (rows) and k = 0..n (columns), eq. (barycentric)."""
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    s = chebyshev_points(n)
    beta = barycentric_weights(n)
    diff = u[:, None] - s[None, :]
    hit = diff == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        t = beta[None, :] / diff
        L = t / np.sum(t, axis=1, keepdims=True)
    rows = np.any(hit, axis=1)
    L[rows] = hit[rows].astype(np.float64)
    return L


# ------------------------------------------------------ §3 faces and tree

def face_and_angles(P):
    """Face index and local angles (xi, eta) of every point."""
    P = np.asarray(P, dtype=np.float64)
    A = np.abs(P)
    axis = np.where((A[:, 0] >= A[:, 1]) & (A[:, 0] >= A[:, 2]), 0,
                    np.where(A[:, 1] >= A[:, 2], 1, 2))
    sign_pos = P[np.arange(P.shape[0]), axis] > 0
    face = np.select([axis == 0, axis == 1, axis == 2],
                     [np.where(sign_pos, 0, 2), np.where(sign_pos, 1, 3),
                      np.where(sign_pos, 4, 5)])
    F = FACE_FRAMES[face]
    c = np.einsum("ij,ij->i", P, F[:, 0])
    a = np.einsum("ij,ij->i", P, F[:, 1])
    b = np.einsum("ij,ij->i", P, F[:, 2])
    xi = np.arctan(a / c)
    eta = np.arctan(b / c)
    return face.astype(np.int64), xi, eta


def cell_index(angle, level):
    """Index of the level-`level` cell holding a local angle (half-open)."""
    t = (angle + PI_4) / PI_2
    k = np.floor(t * float(2 ** level))
    return np.clip(k, 0, 2 ** level - 1).astype(np.int64)


def angles_to_sphere(face, xi, eta):
    """Image on the unit sphere of local angles on a face (gnomonic map)."""
    F = FACE_FRAMES[np.asarray(face)]
    v = F[:, 0] + np.tan(xi)[:, None] * F[:, 1] + np.tan(eta)[:, None] * F[:, 2]
    return v / np.sqrt(np.einsum("ij,ij->i", v, v))[:, None]


class Cell:
    """A cluster: one cubed-sphere cell (face, level, i, j) and its points."""

    __slots__ = ("face", "level", "i", "j", "idx", "children", "parent", "id",
                 "xi_mid", "eta_mid", "half", "half_xi", "half_eta", "center", "radius",
                 "proxies")

    def __init__(self, face, level, i, j, idx, parent):
        self.face, self.level, self.i, self.j = face, level, i, j
        self.idx = idx
        self.children = None
        self.parent = parent
        self.id = -1
        d = PI_2 / 2 ** level
        self.xi_mid = -PI_4 + (i + 0.5) * d
        self.eta_mid = -PI_4 + (j + 0.5) * d
        self.half = 0.5 * d          # the cell's half width
        self.half_xi = self.half     # the box's half widths (the cell unless shrunk)
        self.half_eta = self.half

    def shrink(self, xi, eta):
        """Make the box the smallest rectangle holding the angles (xi, eta)
        of the cluster's points (half widths floored, see the module notes)."""
        lo, hi = float(np.min(xi)), float(np.max(xi))
        self.xi_mid, self.half_xi = 0.5 * (lo + hi), max(0.5 * (hi - lo), SHRINK_FLOOR * self.half)
        lo, hi = float(np.min(eta)), float(np.max(eta))
        self.eta_mid, self.half_eta = 0.5 * (lo + hi), max(0.5 * (hi - lo), SHRINK_FLOOR * self.half)

    @property
    def key(self):
        return (self.level, self.face, self.i, self.j)

    @property
    def is_leaf(self):
        return self.children is None

    @property
    def count(self):
        return len(self.idx)

    def local(self, xi, eta):
        """Local coordinates in [-1,1]^2 of angles inside this cluster's box."""
        return (xi - self.xi_mid) / self.half_xi, (eta - self.eta_mid) / self.half_eta


class Tree:
    """Forest of six quadtrees over the cubed sphere (§3)."""

    def __init__(self, points, N0, n, shrink=False):
        self.points = np.asarray(points, dtype=np.float64)
        self.shrink = bool(shrink)
        self.N0 = int(N0)
        self.n = int(n)
        self.face, self.xi, self.eta = face_and_angles(self.points)
        self.levels = []
        roots = [Cell(f, 0, 0, 0, np.nonzero(self.face == f)[0], None) for f in range(6)]
        frontier = roots
        while frontier:
            self.levels.append(frontier)
            nxt = []
            for C in frontier:
                if C.count > self.N0 and C.level < MAX_LEVEL:
                    l = C.level + 1
                    ii = cell_index(self.xi[C.idx], l)
                    jj = cell_index(self.eta[C.idx], l)
                    C.children = []
                    for q in range(4):
                        ci, cj = 2 * C.i + (q >> 1), 2 * C.j + (q & 1)
                        sel = C.idx[(ii == ci) & (jj == cj)]
                        ch = Cell(C.face, l, ci, cj, sel, C)
                        C.children.append(ch)
                        nxt.append(ch)
            frontier = nxt
        self.cells = [C for lev in self.levels for C in lev]
        for k, C in enumerate(self.cells):
            C.id = k
            if self.shrink and C.count > 0:
                C.shrink(self.xi[C.idx], self.eta[C.idx])
            self._geometry(C)

    def _geometry(self, C):
        """Centre, radius (chord to the farthest corner) and proxy points of
        the cluster's box."""
        f = np.array([C.face])
        C.center = angles_to_sphere(f, np.array([C.xi_mid]), np.array([C.eta_mid]))[0]
        cx = C.xi_mid + C.half_xi * np.array([-1.0, -1.0, 1.0, 1.0])
        cy = C.eta_mid + C.half_eta * np.array([-1.0, 1.0, -1.0, 1.0])
        corners = angles_to_sphere(np.full(4, C.face), cx, cy)
        C.radius = float(np.max(np.sqrt(np.sum((corners - C.center) ** 2, axis=1))))
        sx, sy = self.proxy_angles(C)
        px = np.repeat(sx, self.n + 1)
        py = np.tile(sy, self.n + 1)
        C.proxies = angles_to_sphere(np.full(px.shape[0], C.face), px, py)

    def proxy_angles(self, C):
        s = chebyshev_points(self.n)
        return C.xi_mid + C.half_xi * s, C.eta_mid + C.half_eta * s

    @property
    def leaves(self):
        return [C for C in self.cells if C.is_leaf]


# ------------------------------------------------------------ §6 upward

def upward_pass(tree, w):
    """Proxy weights wbar(C), shape [(n+1),(n+1)] (k1, k2), for every cell.

    Leaves by eq. (PC): wbar_k = sum_j L_k1(u_j) L_k2(v_j) w_j.  Parents by
    eq. (upwardpass2): wbar_k(P) = sum_c sum_m L_k^P(s_m^c) wbar_m(c).
    """
    n = tree.n
    wbar = {}
    for lev in reversed(tree.levels):
        for C in lev:
            if C.is_leaf:
                u, v = C.local(tree.xi[C.idx], tree.eta[C.idx])
                L1 = lagrange(n, u)
                L2 = lagrange(n, v)
                wbar[C.id] = np.einsum("jk,jl,j->kl", L1, L2, w[C.idx])
            else:
                acc = np.zeros((n + 1, n + 1))
                for ch in C.children:
                    sx, sy = tree.proxy_angles(ch)
                    u, v = C.local(sx, sy)
                    A = lagrange(n, u)  # A[m1, k1] = L^P_k1(s^c_m1)
                    B = lagrange(n, v)
                    acc += np.einsum("mk,ql,mq->kl", A, B, wbar[ch.id])
                wbar[C.id] = acc
    return wbar


# -------------------------------------------------- §8 dual traversal

def well_separated(T, S, theta):
    s = T.radius + S.radius
    d = T.center - S.center
    R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
    return s * s < (theta * theta) * R2


def dual_traversal(ttree, stree, theta):
    """Lists of (target cell, source cell) pairs: PP, PC, CP, CC (Alg. 2)."""
    lists = {"PP": [], "PC": [], "CP": [], "CC": []}
    stack = [(T, S) for T in reversed(ttree.levels[0]) for S in reversed(stree.levels[0])]
    # depth-first, root pairs in (target face, source face) order
    while stack:
        T, S = stack.pop()
        if T.count == 0 or S.count == 0:
            continue
        both_leaves = T.is_leaf and S.is_leaf
        if not both_leaves and well_separated(T, S, theta):
            if T.is_leaf:
                lists["PC"].append((T, S))
            elif S.is_leaf:
                lists["CP"].append((T, S))
            else:
                lists["CC"].append((T, S))
        elif not both_leaves:
            split_target = (not T.is_leaf) and (S.is_leaf or T.level <= S.level)
            if split_target:
                for ch in reversed(T.children):
                    stack.append((ch, S))
            else:
                for ch in reversed(S.children):
                    stack.append((T, ch))
        else:
            lists["PP"].append((T, S))
    return lists


# ------------------------------------------------------- driver (Alg. 2)

class FMM:
    """One CSFMM evaluation: phi_i = sum_j K(x_i, y_j) w_j, approximated."""

    def __init__(self, targets, sources, kernel, n, theta, N0, shrink=False):
        self.kernel = int(kernel)
        self.n = int(n)
        self.theta = float(theta)
        self.N0 = int(N0)
        self.same = sources is None
        self.ttree = Tree(targets, N0, n, shrink)
        self.stree = self.ttree if self.same else Tree(sources, N0, n, shrink)
        self.lists = dual_traversal(self.ttree, self.stree, self.theta)

    @property
    def vdim(self):
        return 3 if self.kernel == KERNEL_BIOT_SAVART else 1

    def evaluate(self, w, sample=None, stages=False):
        """phi at every target, or only at the target indices in `sample`.

        With a sample, target-side work is done only for the cells that hold
        sampled targets; the sampled values are the same numbers the full
        evaluation gives.  With stages=True also returns a dict with the proxy
        weights {cell id: [n+1,n+1]}, the proxy potentials after the downward
        pass {cell id: [n+1,n+1,vdim]} and the PP+PC part of phi.
        """
        tt, st = self.ttree, self.stree
        w = np.asarray(w, dtype=np.float64)
        nt = tt.points.shape[0]
        vd = self.vdim
        n1 = self.n + 1
        want = np.ones(nt, dtype=bool) if sample is None else np.zeros(nt, dtype=bool)
        if sample is not None:
            want[np.asarray(sample)] = True
        live = set()
        for C in tt.cells:
            if np.any(want[C.idx]):
                live.add(C.id)

        # Algorithm 2, upward pass on the source tree
        wbar = upward_pass(st, w)

        # Algorithm 2, interactions by list type, grouped by target cluster
        phi = np.zeros((nt, vd))
        psi = {}
        by_t = {}
        for kind in ("PP", "PC", "CP", "CC"):
            for T, S in self.lists[kind]:
                if T.id in live:
                    by_t.setdefault((kind, T.id), []).append(S)
        for (kind, tid), Ss in by_t.items():
            T = tt.cells[tid]
            if kind in ("PP", "PC"):
                X = tt.points[T.idx[want[T.idx]]]
                rows = T.idx[want[T.idx]]
                if kind == "PP":
                    Y = np.concatenate([st.points[S.idx] for S in Ss])
                    wy = np.concatenate([w[S.idx] for S in Ss])
                else:
                    Y = np.concatenate([S.proxies for S in Ss])
                    wy = np.concatenate([wbar[S.id].reshape(-1) for S in Ss])
                phi[rows] += apply_kernel(self.kernel, X, Y, wy).reshape(len(rows), vd)
            else:
                if kind == "CP":
                    Y = np.concatenate([st.points[S.idx] for S in Ss])
                    wy = np.concatenate([w[S.idx] for S in Ss])
                else:
                    Y = np.concatenate([S.proxies for S in Ss])
                    wy = np.concatenate([wbar[S.id].reshape(-1) for S in Ss])
                # eq. (CP_CC_accumulated)
                val = apply_kernel(self.kernel, T.proxies, Y, wy).reshape(n1, n1, vd)
                psi[tid] = psi.get(tid, 0.0) + val

        near = phi.copy()

        # Algorithm 2, downward pass: eq. (downward_2) through all levels, then
        # eq. (downward_1) at the leaves
        for lev in tt.levels:
            for C in lev:
                if C.id not in live or C.id not in psi:
                    continue
                if C.is_leaf:
                    rows = C.idx[want[C.idx]]
                    u, v = C.local(tt.xi[rows], tt.eta[rows])
                    L1 = lagrange(self.n, u)
                    L2 = lagrange(self.n, v)
                    phi[rows] += np.einsum("ik,il,klv->iv", L1, L2, psi[C.id])
                else:
                    for ch in C.children:
                        if ch.id not in live:
                            continue
                        tx, ty = tt.proxy_angles(ch)
                        u, v = C.local(tx, ty)
                        A = lagrange(self.n, u)  # A[n1, m1] = L^P_m1(t^c_n1)
                        B = lagrange(self.n, v)
                        add = np.einsum("am,bq,mqv->abv", A, B, psi[C.id])
                        psi[ch.id] = psi.get(ch.id, 0.0) + add
        out = phi if sample is None else phi[np.asarray(sample)]
        out = out[:, 0] if vd == 1 else out
        if stages:
            return out, {"wbar": wbar, "psi": psi, "near": near}
        return out


def fmm(targets, sources, weights, kernel, n, theta, N0, sample=None, shrink=False):
    """Convenience wrapper: build the trees and lists, then evaluate."""
    F = FMM(targets, sources, kernel, n, theta, N0, shrink)
    return F.evaluate(weights, sample=sample)


# ------------------------------------------------------ CSTC (Alg. 1)

def point_separated(x, S, theta):
    """r/R < MAC for a target point x and a source cluster S (Algorithm 1)."""
    d = x - S.center
    R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
    return S.radius * S.radius < (theta * theta) * R2


def treecode(targets, sources, weights, kernel, n, theta, N0, sample=None):
    """Cubed sphere treecode (Algorithm 1): the source tree and its upward
    pass, then for every target particle a traversal from the six source
    roots: PC for separated clusters with more than N0
    points, PP for separated small clusters and for leaves that are not
    separated, children otherwise.  `kernel` is a kernel id or a function
    (X, Y) -> matrix of kernel values (for tests).  Returns phi at every
    target (or at the indices in `sample`).
    """
    X = np.asarray(targets, dtype=np.float64)
    src = X if sources is None else np.asarray(sources, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    st = Tree(src, N0, n)
    wbar = upward_pass(st, w)
    if callable(kernel):
        kmat, vd = kernel, 1
    else:
        kmat = lambda A, B: kernel_matrix(int(kernel), A, B)  # noqa: E731
        vd = 3 if int(kernel) == KERNEL_BIOT_SAVART else 1
    rows = np.arange(X.shape[0]) if sample is None else np.asarray(sample)
    out = np.zeros((rows.shape[0], vd))
    for r, i in enumerate(rows):
        x = X[i]
        acc = np.zeros(vd)
        stack = list(reversed(st.levels[0]))
        while stack:
            S = stack.pop()
            if S.count == 0:
                continue
            sep = point_separated(x, S, theta)
            if sep and S.count > st.N0:
                K = kmat(x[None, :], S.proxies)
                acc += np.tensordot(K[0], wbar[S.id].reshape(-1), axes=([0], [0])).reshape(vd)
            elif sep or S.is_leaf:
                K = kmat(x[None, :], st.points[S.idx])
                acc += np.tensordot(K[0], w[S.idx], axes=([0], [0])).reshape(vd)
            else:
                for ch in reversed(S.children):
                    stack.append(ch)
        out[r] = acc
    return out[:, 0] if vd == 1 else out

