"""Seeded synthetic workload descriptors shared by the oracle tests, the GPU tests and the bench.

This module holds *data only*: layer tables, mesh sizes, load cases, solver options and the
seeded draws of the wrinkle-sample sweep.  It contains none of the method's arithmetic
(no mesh coordinates, no stiffness, no loads): each implementation turns a descriptor into
numbers on its own.

Material constants are the values of the paper's Table 1 (section 2.2), converted from GPa
to MPa (1 GPa = 1000 MPa); lengths are in mm, moments in N*mm/mm.

Descriptor format
-----------------
``layers``: list of dicts ``{"mat": "ply"|"resin", "t": thickness_mm, "nel": element
layers, "angle": ply angle in degrees}`` listed from the inner radius (zeta = 0) outwards.
``geometry``: ``"flat"`` (s along x, l along y, zeta along z) or ``"lsection"`` (two
straight limbs joined by a 90 degree arc, the laminate normal pointing away from the
centre of curvature).
``load``: ``{"kind": "traction", "t0": (tx, ty, tz)}`` uniform traction (MPa) on the
s = s_max end face, or ``{"kind": "moment", "M": m}`` end moment per unit width.
The s = s_min end face is clamped in all three components.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Table 1 (section 2.2): orthotropic fibrous layer and isotropic interface layer, MPa.
PLY = dict(E1=162e3, E2=10e3, E3=10e3, G12=5.2e3, G13=5.2e3, G23=3.5e3,
           nu12=0.35, nu13=0.35, nu23=0.5)
RESIN = dict(E=10e3, nu=0.35)
# Resin edge material of Table 1 (used only by edge-treated models).
RESIN_EDGE = dict(E=8.5e3, nu=0.35)

# Moment applied in the corner-unfolding verification model, N*mm/mm (section 2.2).
PAPER_MOMENT = 96.8


def ply_layers(angles, ply_t, ply_nel, resin_t, resin_nel):
    """Alternate plies with resin interfaces (no resin outside the outermost plies)."""
    out = []
    for i, a in enumerate(angles):
        out.append({"mat": "ply", "t": ply_t, "nel": ply_nel, "angle": float(a)})
        if i + 1 < len(angles):
            out.append({"mat": "resin", "t": resin_t, "nel": resin_nel, "angle": 0.0})
    return out


CFG1_ANGLES = [0, 45, 90, -45, 0, 45, 45, 0, -45, 90, 45, 0]


def cfg0():
    """Flat 10x10x1.2 mm, [0,R,90,R,0,R,90,R], 8x8x12 elements, 2x2 subdomains, nev=6."""
    layers = []
    for a in (0, 90, 0, 90):
        layers.append({"mat": "ply", "t": 0.25, "nel": 2, "angle": float(a)})
        layers.append({"mat": "resin", "t": 0.05, "nel": 1, "angle": 0.0})
    return dict(name="cfg0_flat_8x8x12", geometry="flat", length=10.0, width=10.0,
                nx=8, ny=8, layers=layers,
                load={"kind": "traction", "t0": (1.0, 0.0, 0.0)},
                solver=dict(px=2, py=2, overlap=1, nev=6, tau=None, nev_max=32, rtol=1e-8))


def cfg1(nx=64, ny=64, ply_nel=4, px=8, py=8):
    """Flat 50x50 mm, 12 plies [0/45/90/-45/0/45]s with resin, 64x64x59, 8x8 subdomains."""
    layers = ply_layers(CFG1_ANGLES, 0.25, ply_nel, 0.05, 1)
    return dict(name=f"cfg1_flat_{nx}x{ny}x{sum(l['nel'] for l in layers)}",
                geometry="flat", length=50.0, width=50.0, nx=nx, ny=ny, layers=layers,
                load={"kind": "traction", "t0": (1.0, 0.0, 0.0)},
                solver=dict(px=px, py=py, overlap=2, nev=0, tau=0.1, nev_max=32, rtol=1e-8))


def _limb_elems(nx, limb, radius, layers):
    """Elements per straight limb: the arc and limbs share nx in proportion to length."""
    thick = sum(l["t"] for l in layers)
    s_total = 2 * limb + 0.5 * math.pi * (radius + 0.5 * thick)
    return int(round(nx * limb / s_total))


def cfg2(nx=240, ny=18, ply_nel=4, px=32, py=2, amp=0.3, wlen=4.0, limb=40.0):
    """Wrinkled L-section: R=5, 90 degree arc, 40 mm limbs, W=10, cfg1 layup, end moment."""
    layers = ply_layers(CFG1_ANGLES, 0.25, ply_nel, 0.05, 1)
    return dict(name=f"cfg2_lsection_{nx}x{ny}x{sum(l['nel'] for l in layers)}",
                geometry="lsection", radius=5.0, limb=limb, width=10.0,
                nx=nx, ny=ny, nx_limb=_limb_elems(nx, limb, 5.0, layers),
                layers=layers, wrinkle=(float(amp), float(wlen)),
                load={"kind": "moment", "M": PAPER_MOMENT},
                solver=dict(px=px, py=py, overlap=2, nev=0, tau=0.1, nev_max=32, rtol=1e-8))


def cfg3(nx=240, ny=4, px=16, py=1):
    """Adjoint workload: cfg2 geometry with 2 elements per ply, 240x4x35 (490,377 DOFs).

    16 x 1 subdomains: across 4 elements of width, two subdomains grown by an overlap of 2
    would each cover the full width and coincide."""
    return cfg2(nx=nx, ny=ny, ply_nel=2, px=px, py=py)


def cfg4_samples(n=32, seed=170704228):
    """Seeded wrinkle-sample sweep: amplitude, wavelength, ply count and DOF target.

    Draw order is fixed: amplitude, wavelength, ply count, DOF target, each a vector of n.
    """
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.0, 0.5, n)
    wlen = rng.uniform(2.0, 8.0, n)
    nplies = rng.integers(6, 13, n)
    target = rng.uniform(5e4, 4e5, n)
    out = []
    for i in range(n):
        angles = [(0, 45, 90, -45)[k % 4] for k in range(int(nplies[i]))]
        out.append(dict(amp=float(amp[i]), wlen=float(wlen[i]), angles=angles,
                        target=float(target[i])))
    return out


def cfg4(i, samples=None, nx_override=None):
    """One sample of the sweep as a laminate descriptor (limbs 10 mm, R=5, W=10)."""
    smp = (samples or cfg4_samples())[i]
    layers = ply_layers(smp["angles"], 0.25, 2, 0.05, 1)
    nz = sum(l["nel"] for l in layers)
    thick = sum(l["t"] for l in layers)
    limb, radius = 10.0, 5.0
    # Element counts are mesh-resolution choices (>= 10 elements per wrinkle length).
    s_total = 2 * limb + 0.5 * math.pi * (radius + 0.5 * thick)
    nx = nx_override or int(4 * math.ceil(math.ceil(10 * s_total / smp["wlen"]) / 4))
    ny = int(min(16, max(2, round(smp["target"] / (12 * nx * nz)))))
    n_dofs_guess = 12 * nx * ny * nz
    nsub = max(2, int(round(n_dofs_guess / 4e4)))
    # wide samples are split across the width as well (keeps the subdomain bandwidth small)
    py = 2 if ny > 8 else 1
    px = max(1, int(round(nsub / py)))
    return dict(name=f"cfg4_sample{i}", geometry="lsection", radius=radius, limb=limb,
                width=10.0, nx=nx, ny=ny, nx_limb=_limb_elems(nx, limb, radius, layers),
                layers=layers, wrinkle=(smp["amp"], smp["wlen"]),
                load={"kind": "moment", "M": PAPER_MOMENT},
                solver=dict(px=px, py=py, overlap=2, nev=0, tau=0.1, nev_max=32, rtol=1e-8))


def small_flat(nx=4, ny=3, layers=None, length=4.0, width=3.0):
    """A tiny flat laminate used by unit tests."""
    if layers is None:
        layers = [{"mat": "ply", "t": 0.25, "nel": 2, "angle": 30.0},
                  {"mat": "resin", "t": 0.05, "nel": 1, "angle": 0.0},
                  {"mat": "ply", "t": 0.25, "nel": 1, "angle": -60.0}]
    return dict(name=f"flat_{nx}x{ny}", geometry="flat", length=length, width=width,
                nx=nx, ny=ny, layers=copy.deepcopy(layers),
                load={"kind": "traction", "t0": (1.0, 0.0, 0.0)},
                solver=dict(px=2, py=1, overlap=1, nev=6, tau=None, nev_max=32, rtol=1e-8))


def small_lsection(nx=12, ny=2, amp=0.3, wlen=4.0, limb=3.0, layers=None):
    """A tiny wrinkled L-section used by unit tests."""
    if layers is None:
        layers = ply_layers([0, 45, -45], 0.25, 1, 0.05, 1)
    return dict(name=f"lsec_{nx}x{ny}", geometry="lsection", radius=5.0, limb=limb,
                width=2.0, nx=nx, ny=ny, nx_limb=_limb_elems(nx, limb, 5.0, layers),
                layers=layers, wrinkle=(float(amp), float(wlen)),
                load={"kind": "moment", "M": PAPER_MOMENT},
                solver=dict(px=3, py=1, overlap=1, nev=6, tau=None, nev_max=32, rtol=1e-8))


def seeded_vector(n, seed):
    """A seeded standard-normal vector of length n (test input shared by the oracle runs
    that write stored results and the GPU tests that read them)."""
    return np.random.default_rng(seed).standard_normal(n)


def sample_indices(n, k, seed=170704228):
    """k distinct seeded positions in [0, n), ascending (the entries of large vectors that
    stored results keep)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(k, n), replace=False))


# Extents of the sech^2 defect of section 3 (b2: towards the inner radius, outwards).
DEFECT_B = dict(b1=0.2, b2_in=0.5, b2_out=0.25, b3=0.5)


def defect_lsection(nx=24, ny=4, d=0.3, angles=(0, 45, 90, -45), ply_nel=1, limb=3.0,
                    width=4.0, zeta_def=None, px=4, py=1, nev=6):
    """A small curved L-section with the paper's sech^2 wrinkle defect (section 3, Eq. eq-f)
    at mid-arc and mid-width, centred through the thickness unless zeta_def is given, under
    the end moment; resin interfaces between the plies."""
    layers = ply_layers(list(angles), 0.25, ply_nel, 0.05, 1)
    T = sum(l["t"] for l in layers)
    D = dict(DEFECT_B, d=float(d), s_def=0.0, l_def=0.5 * width,
             zeta_def=0.5 * T if zeta_def is None else float(zeta_def))
    return dict(name=f"defect_lsec_{nx}x{ny}", geometry="lsection", radius=5.0, limb=limb,
                width=width, nx=nx, ny=ny, nx_limb=_limb_elems(nx, limb, 5.0, layers),
                layers=layers, defect=D, load={"kind": "moment", "M": PAPER_MOMENT},
                solver=dict(px=px, py=py, overlap=1, nev=nev, tau=None, nev_max=32,
                            rtol=1e-8))


# The "very stiff" end layer that carries the moment (section 2.2); the paper gives no
# value: ten times the ply's fibre modulus, isotropic.
STIFF_END = dict(E=10 * PLY["E1"], nu=0.3)


def graded_lsection(nx=20, ny=8, ny_strip=2, strip=0.5, bias=None, stiff=True, d=0.25,
                    angles=(0, 90, 0), ply_nel=2, limb=3.0, width=4.0, px=4, py=2, nev=6):
    """A small edge-treated, graded L-section (section 2.2 / 3.1 features): resin edge strips
    of `strip` mm with ny_strip elements each, the laminate graded towards its edges, every
    layer towards its faces and the arc towards mid-arc, a stiff end column on the loaded
    limb, and the sech^2 defect at mid-arc."""
    cfg = defect_lsection(nx=nx, ny=ny, d=d, angles=angles, ply_nel=ply_nel, limb=limb,
                          width=width, px=px, py=py, nev=nev)
    cfg["name"] = f"graded_lsec_{nx}x{ny}"
    cfg["bias"] = dict(s=2.0, l=20.0, z=4.0) if bias is None else dict(bias)
    if strip:
        cfg["edge_strip"] = dict(width=float(strip), ny=int(ny_strip), **RESIN_EDGE)
    if stiff:
        cfg["stiff_end"] = dict(STIFF_END)
    return cfg


def verification_model(px=8, py=8, overlap=1):
    """The corner-unfolding verification model of section 2.2: R = 6.6 mm, 3 mm limbs,
    W = 15 mm, the 12-ply layup [+-45/90/0/-+45/-+45/0/90/+-45] of 0.23 mm plies and 0.02 mm
    resin interfaces (T = 2.98 mm), 6 elements in every layer, 56 elements along s and l
    (432,768 elements, 5,362,047 DOFs); 2 mm resin edge strips, the mesh graded with bias
    400 across the width (towards the laminate's edges) and 10 through every layer, a stiff
    end layer carrying the 96.8 N mm/mm moment.  The strips carry 4 of the 56 elements
    each (the paper does not say how many)."""
    angles = [45, -45, 90, 0, -45, 45, -45, 45, 0, 90, 45, -45]
    layers = ply_layers(angles, 0.23, 6, 0.02, 6)
    return dict(name="verification_56x56x138", geometry="lsection", radius=6.6, limb=3.0,
                width=15.0, nx=56, ny=56, nx_limb=_limb_elems(56, 3.0, 6.6, layers),
                layers=layers, bias=dict(s=1.0, l=400.0, z=10.0),
                edge_strip=dict(width=2.0, ny=4, **RESIN_EDGE), stiff_end=dict(STIFF_END),
                load={"kind": "moment", "M": PAPER_MOMENT},
                solver=dict(px=px, py=py, overlap=overlap, nev=0, tau=0.1, nev_max=32,
                            rtol=1e-8))
