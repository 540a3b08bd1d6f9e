"""Structured laminate meshes of 20-node serendipity hexahedra (oracle; test infrastructure).

The paper meshes laminates on a tensor-product grid with a fixed number of element layers
through each ply and interface (section 2.2, "6 elements in each of the 12 fibrous and the
11 interface layers") and builds curved wrinkled parts by mapping a flat mesh (section 3,
Eq. eq-wrinkle and the curved mapping that follows it).  The 20-node element carries
nodes at its 8 vertices and 12 edge midpoints (section 2.1).

Readings where the paper is silent:

* nodes live on a doubled index lattice (i2, j2, k2); a lattice point is a node when at
  most one of its indices is odd (vertices: none odd; edge midpoints: exactly one);
* the canonical node number is the rank of (k2, j2, i2) in lexicographic order with i2
  fastest, counting nodes only; element e = (ez*ny + ey)*nx + ex;
* element-local node order: 8 vertices with (di, dj, dk) in lexicographic order, i fastest;
  then 4 x-directed edges at (dj, dk) = (0,0),(1,0),(0,1),(1,1); then 4 y-directed edges at
  (di, dk); then 4 z-directed edges at (di, dj);
* each node's coordinates are the geometry map evaluated at its lattice parameter
  (curved isoparametric edges);
* wrinkle: zeta_hat = zeta + w(s - s_c), w(s) = A exp(-(s/L_w)^2) cos(2 pi s/L_w), the
  same shift for every layer and across the whole width;
* L-section: limb 1 (clamped) for s < s_a, a 90 degree arc of mid-surface radius
  R_ref = R + T/2 around the centre (limb, 0), limb 2 for s > s_b; s = 0 at mid-arc,
  s_b = -s_a = pi R_ref / 4; each of the three segments carries a uniform element size.
"""
from __future__ import annotations

import math

import numpy as np

# reference coordinates of the 20 element nodes, in the element-local order above
def reference_nodes():
    pts = []
    for dk in (0, 1):
        for dj in (0, 1):
            for di in (0, 1):
                pts.append((2 * di - 1, 2 * dj - 1, 2 * dk - 1))
    for dk in (0, 1):          # x-directed edges
        for dj in (0, 1):
            pts.append((0, 2 * dj - 1, 2 * dk - 1))
    for dk in (0, 1):          # y-directed edges
        for di in (0, 1):
            pts.append((2 * di - 1, 0, 2 * dk - 1))
    for dj in (0, 1):          # z-directed edges
        for di in (0, 1):
            pts.append((2 * di - 1, 2 * dj - 1, 0))
    return np.array(pts, dtype=np.float64)


def total_thickness(cfg):
    return float(sum(L["t"] for L in cfg["layers"]))


def graded(n, bias, fine):
    """Boundaries (fractions of the segment, n + 1 values) of n elements graded with the
    paper's bias ratio (largest over smallest element, section 2.2): element sizes grow
    geometrically, q^e, symmetric about the segment's middle, with e = min(k, n - 1 - k) for
    elements refined towards both ends (fine="ends") and m - e for elements refined towards
    the middle (fine="middle"), m = (n - 1) // 2 and q = bias^(1/m).  bias <= 1: uniform."""
    m = (n - 1) // 2
    k = np.arange(n)
    e = np.minimum(k, n - 1 - k)
    if bias <= 1.0 or m == 0:
        h = np.ones(n)
    else:
        q = bias ** (1.0 / m)
        h = q ** (e if fine == "ends" else m - e)
    b = np.concatenate([[0.0], np.cumsum(h)])
    return b / b[-1]


def _bias(cfg, axis):
    return float(cfg.get("bias", {}).get(axis, 1.0))


def zeta_boundaries(cfg):
    """Element-layer boundaries through the thickness and the material layer of each; each
    layer's elements are graded towards its two faces (bias "z", section 2.2)."""
    zb, lay = [0.0], []
    z0 = 0.0
    for li, L in enumerate(cfg["layers"]):
        g = graded(L["nel"], _bias(cfg, "z"), "ends")
        for k in range(L["nel"]):
            zb.append(z0 + L["t"] * g[k + 1])
            lay.append(li)
        z0 += L["t"]
    return np.array(zb), np.array(lay, dtype=np.int64)


def l_boundaries(cfg):
    """Element boundaries across the width: with resin edge strips (section 2.2, 3) each
    strip carries ny_strip uniform elements and the laminate between them is graded towards
    its two edges (bias "l"); without strips the whole width is graded towards the free
    edges."""
    ny, W = cfg["ny"], cfg["width"]
    st = cfg.get("edge_strip")
    if not st:
        return W * graded(ny, _bias(cfg, "l"), "ends")
    e, ns = st["width"], st["ny"]
    mid = e + (W - 2 * e) * graded(ny - 2 * ns, _bias(cfg, "l"), "ends")
    left = e * np.arange(ns) / ns
    right = W - e + e * np.arange(1, ns + 1) / ns
    return np.concatenate([left, mid, right])


def s_boundaries(cfg):
    """Element boundaries along s (the arc-length / length coordinate).  A flat part is
    graded towards its middle and the arc of an L-section towards mid-arc (where the
    defects sit), with bias "s" (section 3.1: refinement towards the defect); limbs are
    uniform."""
    nx = cfg["nx"]
    bs = _bias(cfg, "s")
    if cfg["geometry"] == "flat":
        return cfg["length"] * graded(nx, bs, "middle")
    R, T, limb = cfg["radius"], total_thickness(cfg), cfg["limb"]
    rref = R + 0.5 * T
    sb = 0.25 * math.pi * rref
    sa = -sb
    nl = cfg["nx_limb"]
    na = nx - 2 * nl
    ga = graded(na, bs, "middle")
    out = []
    for i in range(nx + 1):
        if i <= nl:
            out.append(sa - limb + limb * i / nl)
        elif i <= nl + na:
            out.append(sa + (sb - sa) * ga[i - nl])
        else:
            out.append(sb + limb * (i - nl - na) / nl)
    return np.array(out)


def lattice_params(bounds):
    """Parameter values on the doubled lattice: boundaries at even, midpoints at odd."""
    n = len(bounds) - 1
    p = np.empty(2 * n + 1)
    p[0::2] = bounds
    p[1::2] = 0.5 * (bounds[:-1] + bounds[1:])
    return p


def wrinkle(cfg, s):
    """Out-of-plane wrinkle offset w(s - s_c) (zero when the config has no wrinkle)."""
    if "wrinkle" not in cfg:
        return np.zeros_like(s)
    A, Lw = cfg["wrinkle"]
    sc = 0.5 * cfg["length"] if cfg["geometry"] == "flat" else 0.0
    u = s - sc
    return A * np.exp(-(u / Lw) ** 2) * np.cos(2.0 * math.pi * u / Lw)


def sech2(x):
    """sech^2 x = 1 / cosh^2 x (written to stay analytic for complex steps)."""
    return 1.0 / np.cosh(x) ** 2


def defect(cfg, s, l, zeta):
    """The paper's localised wrinkle defect, Eq. eq-f (section 3), as a shift of zeta.

    f = d sech^2(pi (s_p - s_p,def) / (pi b1)) sech^2(pi (r - r_def) / (R b2))
          sech^2(pi (l - l_def) / (W b3)),
    b2 = b2_in for r < r_def (towards the inner radius) and b2_out otherwise.  Readings:
    the paper's s runs over [0, pi] along the 90 degree arc (angle = s / 2), so
    s_p - s_p,def = 2 (s - s_def) / R_ref in this mesh's arc length s (R_ref = R + T/2, s = 0
    at mid-arc); r = R + zeta is the unperturbed radius; R in the second factor is the
    inner radius as printed.  Zero when the descriptor has no "defect".
    """
    D = cfg.get("defect")
    if not D:
        return np.zeros(np.broadcast(s, l, zeta).shape)
    T = total_thickness(cfg)
    R = cfg["radius"]
    rref = R + 0.5 * T
    sp = 2.0 * (s - D["s_def"]) / rref
    r = R + zeta
    rdef = R + D["zeta_def"]
    b2 = np.where(np.real(r - rdef) < 0, D["b2_in"], D["b2_out"])
    return (D["d"] * sech2(sp / D["b1"]) * sech2(np.pi * (r - rdef) / (R * b2)) *
            sech2(np.pi * (l - D["l_def"]) / (cfg["width"] * D["b3"])))


def geometry_map(cfg, s, l, zeta):
    """Physical coordinates of parameter points (s, l, zeta) (section 3 mapping)."""
    zh = zeta + wrinkle(cfg, s)
    if cfg.get("defect"):
        if cfg["geometry"] != "lsection":
            raise ValueError("the sech^2 defect is defined on the curved L-section")
        zh = zh + defect(cfg, s, l, zeta)
    if cfg["geometry"] == "flat":
        return np.stack([s, l, zh], axis=-1)
    R, T, limb = cfg["radius"], total_thickness(cfg), cfg["limb"]
    rref = R + 0.5 * T
    sb = 0.25 * math.pi * rref
    sa = -sb
    rho = R + zh
    x = np.empty(s.shape, dtype=np.result_type(s, zh))
    z = np.empty(s.shape, dtype=np.result_type(s, zh))
    m1 = s < sa
    m3 = s > sb
    m2 = ~(m1 | m3)
    x[m1] = limb + (s[m1] - sa)
    z[m1] = rho[m1]
    th = (s[m2] - sa) / rref
    x[m2] = limb + rho[m2] * np.sin(th)
    z[m2] = rho[m2] * np.cos(th)
    x[m3] = limb + rho[m3]
    z[m3] = -(s[m3] - sb)
    return np.stack([x, l, z], axis=-1)


class Mesh:
    """Node coordinates, connectivity and per-element material layer of a laminate."""

    def __init__(self, cfg):
        self.cfg = cfg
        nx, ny = cfg["nx"], cfg["ny"]
        zb, elay = zeta_boundaries(cfg)
        nz = len(zb) - 1
        self.nx, self.ny, self.nz = nx, ny, nz
        sp = lattice_params(s_boundaries(cfg))
        lp = lattice_params(l_boundaries(cfg))
        zp = lattice_params(zb)
        # enumerate the lattice in (k2, j2, i2) lexicographic order and keep the nodes; a
        # laminate periodic across the width (section 3: periodic boundary conditions at the
        # free edge) identifies the lattice plane j2 = 2 ny with j2 = 0
        self.periodic = bool(cfg.get("periodic"))
        if self.periodic and cfg.get("edge_strip"):
            raise ValueError("a periodic laminate has no free edges for resin strips")
        nj = 2 * ny if self.periodic else 2 * ny + 1
        K2, J2, I2 = np.meshgrid(np.arange(2 * nz + 1), np.arange(nj),
                                 np.arange(2 * nx + 1), indexing="ij")
        odd = (K2 % 2) + (J2 % 2) + (I2 % 2)
        isnode = odd <= 1
        self.node_of = -np.ones((2 * nz + 1, 2 * ny + 1, 2 * nx + 1), dtype=np.int64)
        self.node_of[:, :nj][isnode] = np.arange(int(isnode.sum()))
        if self.periodic:
            self.node_of[:, 2 * ny] = self.node_of[:, 0]
        self.n_nodes = int(isnode.sum())
        self.lat = np.stack([I2[isnode], J2[isnode], K2[isnode]], axis=1)   # (i2, j2, k2)
        self.param = np.stack([sp[self.lat[:, 0]], lp[self.lat[:, 1]], zp[self.lat[:, 2]]],
                              axis=1)
        self.xyz = geometry_map(cfg, self.param[:, 0], self.param[:, 1], self.param[:, 2])
        # connectivity
        ref = reference_nodes().astype(np.int64)          # entries in {-1, 0, 1}
        ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
        self.n_elems = ex.size
        conn = np.empty((self.n_elems, 20), dtype=np.int64)
        for a in range(20):
            i2 = 2 * ex + 1 + ref[a, 0]
            j2 = 2 * ey + 1 + ref[a, 1]
            k2 = 2 * ez + 1 + ref[a, 2]
            conn[:, a] = self.node_of[k2, j2, i2]
        assert (conn >= 0).all()
        self.conn = conn
        # element nodes that stand for the wrapped plane j2 = 2 ny take the period W along l
        self.wrap = np.zeros((self.n_elems, 20), dtype=bool)
        if self.periodic:
            self.wrap = (ey[:, None] == ny - 1) & (ref[None, :, 1] == 1)
        self.period = np.array([0.0, cfg["width"], 0.0])
        self.eidx = np.stack([ex, ey, ez], axis=1)
        self.elayer = elay[ez]
        # material overrides: resin edge strips (elements across the strip width), then the
        # stiff end column of the loaded limb (section 2.2); their materials follow the
        # layers' in the material table (material.layer_material)
        nlay = len(cfg["layers"])
        if cfg.get("edge_strip"):
            ns = cfg["edge_strip"]["ny"]
            self.elayer = np.where((ey < ns) | (ey >= ny - ns), nlay, self.elayer)
        if cfg.get("stiff_end"):
            self.elayer = np.where(ex == nx - 1, nlay + (1 if cfg.get("edge_strip") else 0),
                                   self.elayer)
        self.n_dofs = 3 * self.n_nodes

    def elem_coords(self, elems=None):
        """Node coordinates (E, 20, 3) of elements, the wrapped nodes of a periodic laminate
        shifted by the period."""
        c = self.conn if elems is None else self.conn[elems]
        w = self.wrap if elems is None else self.wrap[elems]
        X = self.xyz[c]
        if self.periodic:
            X = X + w[..., None] * self.period
        return X

    # --- boundary description (clamp at s = s_min, load on the s = s_max face) ---
    def clamped_nodes(self):
        return np.nonzero(self.lat[:, 0] == 0)[0]

    def free_mask(self):
        m = np.ones(self.n_dofs, dtype=bool)
        cn = self.clamped_nodes()
        for c in range(3):
            m[3 * cn + c] = False
        return m

    def load_elements(self):
        """Elements whose local xi = +1 face lies on the s = s_max end."""
        return np.nonzero(self.eidx[:, 0] == self.nx - 1)[0]

    def arc_elements(self):
        """Elements whose s-centroid lies on the arc (all elements for a flat part)."""
        if self.cfg["geometry"] == "flat":
            return np.arange(self.n_elems)
        nl = self.cfg["nx_limb"]
        return np.nonzero((self.eidx[:, 0] >= nl) & (self.eidx[:, 0] < self.nx - nl))[0]
