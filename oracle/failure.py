"""Through-thickness stresses and the quadratic delamination-onset criterion (oracle; test
infrastructure).

Section 3.3: the strength of the curved laminate is assessed with the criterion of Camanho
et al. (Eq. eq-Camanho),

    F = sqrt( (sigma_r^+ / s33)^2 + (tau_rs / s13)^2 + (tau_rl / s13)^2 ),

with negative sigma_r counted as zero, s33 = 61 MPa and s13 = 97 MPa, evaluated only in the
resin-rich interface layers; failure initiates at F = 1.  Since the problem is linear, F
scales with the load, and the moment at which failure initiates is M / max F.  The paper's
Table table-per lists, for each model, max F, the interface where it occurs (counted from
the outer radius) and the six stresses there in the (s, l, r) directions.

Readings where the paper is silent:

* stresses are recovered at the 3x3x3 Gauss points of each element, sigma = C_g B u_e in
  global axes, and expressed in the local frame (s, l, r) = (e1, e2, e3) of the
  isoparametric Jacobian (the frame the material is rotated into);
* "resin-rich interface zones" are the isotropic layers between plies;
* the steepest slope of the defect (the paper differentiates Eq. eq-f in its own s) is taken
  as a physical angle: d f / d(arc length at the defect's radius r_def), with
  ds_paper / d(arc length) = 2 / r_def.
"""
from __future__ import annotations

import math

import numpy as np

from .element import gauss_point_data, local_frame, material_at_points, strain_matrix
from .fem import element_data, element_dofs

S33 = 61.0       # MPa, through-thickness tensile allowable (section 3.3)
S13 = 97.0       # MPa, interlaminar shear allowable


def local_stresses(mesh, u_full, elems):
    """Stresses (E, 27, 6) at the Gauss points of `elems` in the local frame, ordered
    [sigma_s, sigma_l, sigma_r, tau_lr, tau_sr, tau_sl] (Voigt order of (e1, e2, e3))."""
    X, C, ang = element_data(mesh)
    X, C, ang = X[elems], C[elems], ang[elems]
    gp = gauss_point_data(X)
    Cq = material_at_points(gp["J"], C, ang)
    B = strain_matrix(gp["G"])
    ue = u_full[element_dofs(mesh)[elems]]
    sig = np.einsum("eqIJ,eqJb,eb->eqI", Cq, B, ue)
    S = np.empty(sig.shape[:2] + (3, 3))
    S[..., 0, 0], S[..., 1, 1], S[..., 2, 2] = sig[..., 0], sig[..., 1], sig[..., 2]
    S[..., 1, 2] = S[..., 2, 1] = sig[..., 3]
    S[..., 0, 2] = S[..., 2, 0] = sig[..., 4]
    S[..., 0, 1] = S[..., 1, 0] = sig[..., 5]
    Q = local_frame(gp["J"])                          # rows e1, e2, e3
    L = np.einsum("eqai,eqij,eqbj->eqab", Q, S, Q)
    return np.stack([L[..., 0, 0], L[..., 1, 1], L[..., 2, 2], L[..., 1, 2], L[..., 0, 2],
                     L[..., 0, 1]], axis=-1)


def camanho(loc, s33=S33, s13=S13):
    """F of Eq. eq-Camanho from local stresses [..., 6] (see local_stresses)."""
    sr = np.maximum(loc[..., 2], 0.0)
    return np.sqrt((sr / s33) ** 2 + (loc[..., 4] / s13) ** 2 + (loc[..., 3] / s13) ** 2)


def interface_layers(cfg):
    """Material layers where the criterion applies: the isotropic (resin) layers."""
    return np.array([k for k, L in enumerate(cfg["layers"]) if L["mat"] == "resin"])


def failure(mesh, u_full, layers=None):
    """max F over the Gauss points of the interface layers' elements, where it occurs, the
    local stresses there, and the per-element maximum of F (0 outside those layers)."""
    layers = interface_layers(mesh.cfg) if layers is None else np.asarray(layers)
    elems = np.nonzero(np.isin(mesh.elayer, layers))[0]
    loc = local_stresses(mesh, u_full, elems)
    F = camanho(loc)
    per = np.zeros(mesh.n_elems)
    per[elems] = F.max(axis=1)
    k = int(np.argmax(F.ravel()))
    e, q = divmod(k, F.shape[1])
    layer = int(mesh.elayer[elems[e]])
    resin = list(interface_layers(mesh.cfg))
    return dict(F_max=float(F.ravel()[k]), elem=int(elems[e]), gauss=int(q),
                stresses=loc[e, q], F_elem=per, layer=layer,
                interface_from_outer=len(resin) - resin.index(layer) if layer in resin else -1)


def failure_moment(M, F_max):
    """The moment at which failure initiates: F is homogeneous of degree one in the load."""
    return M / F_max


def steepest_slope_deg(d, b1, r_def):
    """Steepest slope of the sech^2 defect along the arc at its own radius, in degrees.

    In the paper's s: df/ds = -(2 / b1) tanh(x) f, x = (s - s_def) / b1, whose largest
    magnitude is (2 / b1) d max sech^2 x tanh x = 4 d / (3 sqrt(3) b1) (at tanh x = 1/sqrt 3);
    per unit arc length at radius r_def that is multiplied by 2 / r_def.
    """
    return math.degrees(math.atan(8.0 * d / (3.0 * math.sqrt(3.0) * b1 * r_def)))


def amplitude_for_slope(theta_deg, b1, r_def):
    """Defect amplitude d whose steepest slope (steepest_slope_deg) is theta_deg."""
    return math.tan(math.radians(theta_deg)) * 3.0 * math.sqrt(3.0) * b1 * r_def / 8.0
