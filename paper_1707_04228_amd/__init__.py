"""Python binding of libgx (ctypes): AS-GenEO preconditioned CG for laminates on MI355X.

Argument marshalling only: every step of the solve runs in the library's HIP kernels.
Device arrays are torch tensors on the context's device; descriptors are plain dicts (the
laminate descriptors of the ``workloads`` module) turned into the C structs of gx.h.

The library must be built (``python -m paper_1707_04228_amd.build``); importing this module
on a machine without the built library raises immediately — there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch is imported before libgx is loaded so that the process holds a single HIP runtime:
# libgx's libamdhip64.so.7 dependency then resolves to the one torch already mapped.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libgx.so is not built ({LIB_PATH}); run python -m "
                      "paper_1707_04228_amd.build")
lib = C.CDLL(LIB_PATH)

GX_OK, GX_EINVAL, GX_ENOMEM, GX_EHIP, GX_ENOTSPD, GX_ENOCONV, GX_EBREAKDOWN, GX_ESTATE = range(8)
STATUS = {0: "GX_OK", 1: "GX_EINVAL", 2: "GX_ENOMEM", 3: "GX_EHIP", 4: "GX_ENOTSPD",
          5: "GX_ENOCONV", 6: "GX_EBREAKDOWN", 7: "GX_ESTATE"}
GX_GEOM_FLAT, GX_GEOM_LSECTION = 0, 1
GX_FP64, GX_MIXED = 0, 1

i32p, i64p, f64p, vp = (C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                        C.c_void_p)


class Laminate(C.Structure):
    _fields_ = [("geometry", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nx_limb", C.c_int32), ("n_layers", C.c_int32),
                ("layer_t", f64p), ("layer_nel", i32p),
                ("length", C.c_double), ("width", C.c_double), ("radius", C.c_double),
                ("limb", C.c_double), ("wrinkle_amp", C.c_double),
                ("wrinkle_len", C.c_double), ("defect_amp", C.c_double),
                ("defect_s", C.c_double), ("defect_l", C.c_double),
                ("defect_zeta", C.c_double), ("defect_b1", C.c_double),
                ("defect_b2_in", C.c_double), ("defect_b2_out", C.c_double),
                ("defect_b3", C.c_double), ("bias_s", C.c_double), ("bias_l", C.c_double),
                ("bias_z", C.c_double), ("strip_width", C.c_double),
                ("strip_ny", C.c_int32), ("strip_mat", C.c_int32),
                ("end_column", C.c_int32), ("end_mat", C.c_int32),
                ("periodic_l", C.c_int32)]


class PlyStack(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("eng", f64p), ("angle_deg", f64p)]


class Mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_elems", C.c_int64), ("xyz", vp), ("conn", vp),
                ("elem_layer", vp), ("elem_wrap", vp), ("period", C.c_double * 3)]


class Traction(C.Structure):
    _fields_ = [("t0", C.c_double * 3), ("k", C.c_double), ("c", C.c_double * 3),
                ("d", C.c_double * 3)]


class Loads(C.Structure):
    _fields_ = [("n_clamped", C.c_int64), ("clamped", vp), ("n_faces", C.c_int64),
                ("face_elem", vp), ("face_id", vp), ("traction", Traction)]


class FailureResult(C.Structure):
    _fields_ = [("F_max", C.c_double), ("elem", C.c_int64), ("gauss", C.c_int32),
                ("layer", C.c_int32), ("stress", C.c_double * 6)]


class GeneoOpts(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("elem_part", vp), ("overlap", C.c_int32),
                ("tau", C.c_double), ("nev", C.c_int32), ("nev_max", C.c_int32),
                ("precision", C.c_int32), ("coarse", C.c_int32), ("nev_per_sub", i32p),
                ("eig_tol", C.c_double), ("eig_maxit", C.c_int32)]


def _sig(name, args, res=C.c_int32):
    f = getattr(lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("gx_create", [C.POINTER(vp), C.c_int32, vp])
_sig("gx_destroy", [vp], None)
_sig("gx_last_error", [vp], C.c_char_p)
_sig("gx_version", [], C.c_char_p)
_sig("gx_laminate_counts", [C.POINTER(Laminate), i64p, i64p, i64p, i64p])
_sig("gx_laminate_mesh", [vp, C.POINTER(Laminate), vp, vp, vp, vp, vp, vp])
_sig("gx_laminate_partition", [vp, C.POINTER(Laminate), C.c_int32, C.c_int32, vp])
_sig("gx_laminate_wrap", [vp, C.POINTER(Laminate), vp])
_sig("gx_laminate_traction", [C.POINTER(Laminate), C.c_int32, f64p, C.POINTER(Traction)])
_sig("gx_assemble", [vp, C.POINTER(Mesh), C.POINTER(PlyStack), C.POINTER(Loads), vp])
_sig("gx_matrix_info", [vp, i64p, i64p])
_sig("gx_matrix_copy", [vp, vp, vp, vp])
_sig("gx_spmv", [vp, vp, vp])
_sig("gx_matrix_load", [vp, C.c_int64, C.c_int64, vp, vp, vp])
_sig("gx_phase_times", [vp, f64p])
for _name, _args in [("gx_geneo_setup", [vp, C.POINTER(GeneoOpts), i32p, i64p]),
                     ("gx_subdomain_info", [vp, i64p, i64p, i64p]),
                     ("gx_geneo_eigenvalues", [vp, C.c_int32, f64p]),
                     ("gx_precond_apply", [vp, vp, vp]),
                     ("gx_pcg_solve", [vp, vp, vp, C.c_double, C.c_int32, i32p, f64p, f64p]),
                     ("gx_kernel_time", [vp, C.c_int32, C.c_int32, f64p, f64p]),
                     ("gx_stats", [vp, i64p]),
                     ("gx_band_stats", [vp, f64p]),
                     ("gx_failure", [vp, vp, i32p, C.c_double, C.c_double, vp, vp,
                                     C.POINTER(FailureResult)]),
                     ("gx_tune", [vp, C.c_int32, C.c_int64]),
                     ("gx_band_factor_solve", [vp, C.c_int32, i64p, i64p, vp, C.c_int32,
                                               C.c_int32, C.c_int32, vp]),
                     ("gx_objective", [vp, C.POINTER(Laminate), C.c_int32, vp, f64p]),
                     ("gx_objective_noalloc", [vp, C.POINTER(Laminate), C.c_int32, vp, f64p]),
                     ("gx_pcg_solve_batch", [C.c_int32, C.POINTER(vp), C.POINTER(vp),
                                             C.POINTER(vp), C.c_double, C.c_int32, i32p, f64p,
                                             i32p]),
                     ("gx_geneo_setup_batch", [C.c_int32, C.POINTER(vp),
                                               C.POINTER(C.POINTER(GeneoOpts)), C.c_int32,
                                               C.POINTER(i32p), i64p, i32p]),
                     ("gx_adjoint", [vp, C.POINTER(Laminate), C.c_int32, vp, C.c_double,
                                     C.c_int32, f64p, f64p, i32p])]:
    if hasattr(lib, _name):
        _sig(_name, _args)

EXPORTS = ["gx_create", "gx_destroy", "gx_last_error", "gx_version", "gx_laminate_counts",
           "gx_laminate_mesh", "gx_laminate_partition", "gx_laminate_traction",
           "gx_laminate_wrap",
           "gx_assemble", "gx_matrix_info", "gx_matrix_copy", "gx_matrix_load", "gx_spmv",
           "gx_geneo_setup",
           "gx_subdomain_info", "gx_geneo_eigenvalues", "gx_precond_apply", "gx_pcg_solve",
           "gx_phase_times", "gx_kernel_time", "gx_stats", "gx_band_stats", "gx_tune",
           "gx_band_factor_solve", "gx_failure",
           "gx_objective", "gx_objective_noalloc", "gx_adjoint", "gx_pcg_solve_batch",
           "gx_geneo_setup_batch"]


class GxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def laminate_struct(cfg):
    """gx_laminate for a workload descriptor; returns (struct, keep-alive arrays)."""
    t = np.array([L["t"] for L in cfg["layers"]], dtype=np.float64)
    nel = np.array([L["nel"] for L in cfg["layers"]], dtype=np.int32)
    s = Laminate()
    s.geometry = GX_GEOM_FLAT if cfg["geometry"] == "flat" else GX_GEOM_LSECTION
    s.nx, s.ny = cfg["nx"], cfg["ny"]
    s.nx_limb = cfg.get("nx_limb", 0)
    s.n_layers = len(t)
    s.layer_t = t.ctypes.data_as(f64p)
    s.layer_nel = nel.ctypes.data_as(i32p)
    s.length = cfg.get("length", 0.0)
    s.width = cfg["width"]
    s.radius = cfg.get("radius", 0.0)
    s.limb = cfg.get("limb", 0.0)
    A, Lw = cfg.get("wrinkle", (0.0, 0.0))
    s.wrinkle_amp, s.wrinkle_len = A, Lw
    D = cfg.get("defect")
    if D:
        s.defect_amp, s.defect_s, s.defect_l, s.defect_zeta = (D["d"], D["s_def"], D["l_def"],
                                                                D["zeta_def"])
        s.defect_b1, s.defect_b2_in, s.defect_b2_out, s.defect_b3 = (D["b1"], D["b2_in"],
                                                                     D["b2_out"], D["b3"])
    bias = cfg.get("bias", {})
    s.bias_s, s.bias_l, s.bias_z = (float(bias.get(k, 1.0)) for k in ("s", "l", "z"))
    n_lay = len(cfg["layers"])
    if cfg.get("edge_strip"):
        s.strip_width, s.strip_ny = cfg["edge_strip"]["width"], cfg["edge_strip"]["ny"]
        s.strip_mat = n_lay                       # extra materials follow the layers
    if cfg.get("stiff_end"):
        s.end_column = 1
        s.end_mat = n_lay + (1 if cfg.get("edge_strip") else 0)
    s.periodic_l = 1 if cfg.get("periodic") else 0
    return s, (t, nel)


def plystack_arrays(cfg):
    """Engineering constants and angles per layer (isotropic layers as E, nu with G12 = 0)."""
    from workloads import PLY, RESIN
    eng, ang = [], []
    for L in cfg["layers"]:
        if L["mat"] == "ply":
            p = dict(PLY)
            if "E1" in L:
                p["E1"] = L["E1"]
            eng.append([p["E1"], p["E2"], p["E3"], p["G12"], p["G13"], p["G23"],
                        p["nu12"], p["nu13"], p["nu23"]])
        else:
            eng.append([L.get("E", RESIN["E"]), 0, 0, 0, 0, 0, RESIN["nu"], 0, 0])
        ang.append(L["angle"])
    for key in ("edge_strip", "stiff_end"):       # extra materials, after the layers
        if cfg.get(key):
            eng.append([cfg[key]["E"], 0, 0, 0, 0, 0, cfg[key]["nu"], 0, 0])
            ang.append(0.0)
    return np.array(eng, dtype=np.float64), np.array(ang, dtype=np.float64)


def _on_stream(fn):
    """Run a Solver method with the solver's stream current (torch work and allocations)."""
    import functools

    @functools.wraps(fn)
    def wrapped(self, *a, **k):
        if self.stream is None:
            return fn(self, *a, **k)
        with self.torch.cuda.stream(self.stream):
            return fn(self, *a, **k)
    return wrapped


class Solver:
    """One gx context on a torch CUDA (HIP) device, holding mesh, K, P and work vectors."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        torch.cuda.init()
        # the library and the binding's own tensor work share one torch stream (the given
        # one, else the current one unless that is the default stream, in which case the
        # library runs on a stream of its own and every entry point synchronises it)
        cur = torch.cuda.current_stream(self.device)
        if stream is None and cur.cuda_stream != 0:
            stream = cur
        self.stream = stream
        h = vp()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else None
        self._check_plain(lib.gx_create(C.byref(h), device, st), "gx_create")
        self.h = h
        self.nev = None

    def close(self):
        if getattr(self, "h", None) and lib is not None:
            lib.gx_destroy(self.h)
            self.h = None

    __del__ = close

    def _check_plain(self, code, what):
        if code != GX_OK:
            raise GxError(code, what)

    def _check(self, code):
        if code != GX_OK:
            raise GxError(code, lib.gx_last_error(self.h).decode())
        return code

    # ---- mesh --------------------------------------------------------------------
    @_on_stream
    def laminate(self, cfg):
        """Build the laminate mesh and boundary lists of a workload descriptor."""
        torch = self.torch
        lam, keep = laminate_struct(cfg)
        nn, ne, nc, nf = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        self._check_plain(lib.gx_laminate_counts(C.byref(lam), C.byref(nn), C.byref(ne),
                                                 C.byref(nc), C.byref(nf)),
                          "gx_laminate_counts")
        d = self.device
        m = dict(n_nodes=nn.value, n_elems=ne.value,
                 xyz=torch.empty(3 * nn.value, dtype=torch.float64, device=d),
                 conn=torch.empty(20 * ne.value, dtype=torch.int32, device=d),
                 elem_layer=torch.empty(ne.value, dtype=torch.int32, device=d),
                 clamped=torch.empty(nc.value, dtype=torch.int32, device=d),
                 face_elem=torch.empty(nf.value, dtype=torch.int32, device=d),
                 face_id=torch.empty(nf.value, dtype=torch.int32, device=d))
        self._check(lib.gx_laminate_mesh(self.h, C.byref(lam), _ptr(m["xyz"]),
                                         _ptr(m["conn"]), _ptr(m["elem_layer"]),
                                         _ptr(m["clamped"]), _ptr(m["face_elem"]),
                                         _ptr(m["face_id"])))
        load = cfg["load"]
        tr = Traction()
        if load["kind"] == "traction":
            v = np.array(load["t0"], dtype=np.float64)
            kind = 0
        else:
            v = np.array([load["M"], 0, 0], dtype=np.float64)
            kind = 1
        self._check_plain(lib.gx_laminate_traction(C.byref(lam), kind,
                                                   v.ctypes.data_as(f64p), C.byref(tr)),
                          "gx_laminate_traction")
        m["traction"] = tr
        m["cfg"] = cfg
        m["wrap"] = None
        if cfg.get("periodic"):
            m["wrap"] = torch.empty(ne.value, dtype=torch.int32, device=d)
            self._check(lib.gx_laminate_wrap(self.h, C.byref(lam), _ptr(m["wrap"])))
            m["period"] = (0.0, float(cfg["width"]), 0.0)
        self.mesh = m
        return m

    @_on_stream
    def partition(self, cfg, px, py):
        lam, keep = laminate_struct(cfg)
        part = self.torch.empty(self.mesh["n_elems"], dtype=self.torch.int32,
                                device=self.device)
        self._check(lib.gx_laminate_partition(self.h, C.byref(lam), px, py, _ptr(part)))
        return part

    # ---- assembly ------------------------------------------------------------------
    @_on_stream
    def assemble(self, cfg=None, mesh=None):
        m = mesh or self.mesh
        cfg = cfg or m["cfg"]
        eng, ang = plystack_arrays(cfg)
        ps = PlyStack(len(ang), eng.ctypes.data_as(f64p), ang.ctypes.data_as(f64p))
        ms = Mesh(m["n_nodes"], m["n_elems"], _ptr(m["xyz"]), _ptr(m["conn"]),
                  _ptr(m["elem_layer"]), _ptr(m.get("wrap")),
                  (C.c_double * 3)(*m.get("period", (0.0, 0.0, 0.0))))
        ld = Loads(m["clamped"].numel(), _ptr(m["clamped"]), m["face_elem"].numel(),
                   _ptr(m["face_elem"]), _ptr(m["face_id"]), m["traction"])
        f = self.torch.empty(3 * m["n_nodes"], dtype=self.torch.float64, device=self.device)
        self._check(lib.gx_assemble(self.h, C.byref(ms), C.byref(ps), C.byref(ld), _ptr(f)))
        self.f = f
        self.n_dofs = 3 * m["n_nodes"]
        return f

    @_on_stream
    def matrix(self):
        """K as (row_ptr, col, val) torch tensors on the device."""
        torch = self.torch
        nr, nb = C.c_int64(), C.c_int64()
        self._check(lib.gx_matrix_info(self.h, C.byref(nr), C.byref(nb)))
        rp = torch.empty(nr.value + 1, dtype=torch.int32, device=self.device)
        col = torch.empty(nb.value, dtype=torch.int32, device=self.device)
        val = torch.empty(9 * nb.value, dtype=torch.float64, device=self.device)
        self._check(lib.gx_matrix_copy(self.h, _ptr(rp), _ptr(col), _ptr(val)))
        return rp, col, val

    @_on_stream
    def load_matrix(self, row_ptr, col, val):
        """Install a 3x3-block CSR matrix (torch tensors: int32 row_ptr, int32 col, float64
        val with 9 entries per block, row-major) as K for spmv."""
        n_rows = row_ptr.numel() - 1
        self._check(lib.gx_matrix_load(self.h, n_rows, col.numel(), _ptr(row_ptr), _ptr(col),
                                       _ptr(val)))
        self.n_dofs = 3 * n_rows

    @_on_stream
    def spmv(self, x, y=None):
        y = self.torch.empty_like(x) if y is None else y
        self._check(lib.gx_spmv(self.h, _ptr(x), _ptr(y)))
        return y

    # ---- preconditioner and solve ----------------------------------------------------
    @_on_stream
    def geneo_setup(self, part, n_sub, overlap=1, tau=0.1, nev=0, nev_max=32,
                    precision=GX_FP64, coarse=True, nev_per_sub=None, eig_tol=0.0,
                    eig_maxit=0):
        nps = None
        keep = None
        if nev_per_sub is not None:
            keep = np.ascontiguousarray(nev_per_sub, dtype=np.int32)
            nps = keep.ctypes.data_as(i32p)
        o = GeneoOpts(n_sub, _ptr(part), overlap, tau, nev, nev_max, precision,
                      1 if coarse else 0, nps, eig_tol, eig_maxit)
        nev_out = np.zeros(n_sub, dtype=np.int32)
        n0 = C.c_int64()
        self._check(lib.gx_geneo_setup(self.h, C.byref(o), nev_out.ctypes.data_as(i32p),
                                       C.byref(n0)))
        self.nev = nev_out
        self.n0 = n0.value
        self.n_sub = n_sub
        return nev_out, n0.value

    def subdomain_info(self):
        n = self.n_sub
        a, b, c = (np.zeros(n, dtype=np.int64) for _ in range(3))
        self._check(lib.gx_subdomain_info(self.h, a.ctypes.data_as(i64p),
                                          b.ctypes.data_as(i64p), c.ctypes.data_as(i64p)))
        return a, b, c

    def eigenvalues(self, j):
        lam = np.zeros(max(1, int(self.nev[j])), dtype=np.float64)
        self._check(lib.gx_geneo_eigenvalues(self.h, j, lam.ctypes.data_as(f64p)))
        return lam[: int(self.nev[j])]

    @_on_stream
    def precond(self, r, z=None):
        z = self.torch.empty_like(r) if z is None else z
        self._check(lib.gx_precond_apply(self.h, _ptr(r), _ptr(z)))
        return z

    @_on_stream
    def pcg(self, b, x=None, rtol=1e-8, maxit=1000, history=False, allow_noconv=False):
        x = self.torch.zeros_like(b) if x is None else x
        it = C.c_int32()
        rr = C.c_double()
        hist = np.zeros(maxit + 1) if history else None
        code = lib.gx_pcg_solve(self.h, _ptr(b), _ptr(x), rtol, maxit, C.byref(it),
                                C.byref(rr), hist.ctypes.data_as(f64p) if history else None)
        if not (code == GX_OK or (allow_noconv and code == GX_ENOCONV)):
            self._check(code)
        out = dict(x=x, iters=it.value, relres=rr.value, status=code)
        if history:
            out["hist"] = hist[: it.value + 1]
        return out

    @_on_stream
    def kernel_time(self, which, reps=5):
        """(average ms, algorithmic bytes per launch) of library kernel `which`."""
        ms, b = C.c_double(), C.c_double()
        self._check(lib.gx_kernel_time(self.h, which, reps, C.byref(ms), C.byref(b)))
        return ms.value, b.value

    # ---- sensitivities ------------------------------------------------------------
    @_on_stream
    def objective(self, u, cfg=None, region=1):
        """J = sum over the region of sigma_33^2 (region 1: the L-section arc; 0: all)."""
        lam, keep = laminate_struct(cfg or self.mesh["cfg"])
        J = C.c_double()
        self._check(lib.gx_objective(self.h, C.byref(lam), region, _ptr(u), C.byref(J)))
        return J.value

    @_on_stream
    def failure(self, u, layers=None, s33=61.0, s13=97.0, per_gauss=False):
        """Delamination onset (gx_failure): max F of Eq. eq-Camanho over the selected layers
        (default: the resin interface layers, not edge strips or the stiff end), where it
        occurs, the local stresses there, the per-element maxima (device tensor) and, with
        per_gauss, F at every Gauss point."""
        torch = self.torch
        n_e = self.mesh["n_elems"]
        Fe = torch.empty(n_e, dtype=torch.float64, device=self.device)
        Fq = torch.empty(27 * n_e, dtype=torch.float64, device=self.device) if per_gauss else None
        cfg = self.mesh["cfg"]
        if layers is None:
            layers = [k for k, L in enumerate(cfg["layers"]) if L["mat"] == "resin"]
        keep = np.zeros(len(plystack_arrays(cfg)[1]), dtype=np.int32)
        keep[np.asarray(layers, dtype=np.int64)] = 1
        mask = keep.ctypes.data_as(i32p)
        r = FailureResult()
        self._check(lib.gx_failure(self.h, _ptr(u), mask, s33, s13, _ptr(Fq), _ptr(Fe),
                                   C.byref(r)))
        out = dict(F_max=r.F_max, elem=int(r.elem), gauss=int(r.gauss), layer=int(r.layer),
                   stresses=np.array(list(r.stress)), F_elem=Fe)
        if per_gauss:
            out["F_gauss"] = Fq
        return out

    @_on_stream
    def objective_noalloc(self, u, cfg=None, region=1):
        """gx_objective_noalloc: J with the library's static scratch, no device allocation."""
        lam, keep = laminate_struct(cfg or self.mesh["cfg"])
        J = C.c_double()
        self._check(lib.gx_objective_noalloc(self.h, C.byref(lam), region, _ptr(u),
                                             C.byref(J)))
        return J.value

    @_on_stream
    def adjoint(self, u, cfg=None, region=1, rtol=1e-12, maxit=2000, allow_noconv=False):
        """(J, dJ/dp, adjoint iterations); dJ/dp = [dA, dL_w, dE11 of every layer]."""
        cfg = cfg or self.mesh["cfg"]
        lam, keep = laminate_struct(cfg)
        out = np.zeros(2 + len(plystack_arrays(cfg)[1]))
        J, it = C.c_double(), C.c_int32()
        code = lib.gx_adjoint(self.h, C.byref(lam), region, _ptr(u), rtol, maxit, C.byref(J),
                              out.ctypes.data_as(f64p), C.byref(it))
        if not (code == GX_OK or (allow_noconv and code == GX_ENOCONV)):
            self._check(code)
        return J.value, out, it.value

    def tune(self, param, value):
        self._check(lib.gx_tune(self.h, param, value))

    @_on_stream
    def autotune(self, candidates=(1, 2, 3, 4), reps=3):
        """Pick the work-groups per subdomain of the preconditioner's band solves by timing
        them (gx_kernel_time 1) for each candidate; returns {candidate: ms} and keeps the
        fastest."""
        times = {}
        for g in candidates:
            self.tune(0, g)
            times[g] = self.kernel_time(1, reps=reps)[0]
        best = min(times, key=times.get)
        self.tune(0, best)
        return times

    @_on_stream
    def band_factor_solve(self, n, bw, band, x, precision=GX_FP64, groups=0):
        """Factor the band matrices (row-major band storage, device FP64 tensor `band`) and
        solve in place for x (device FP64, n[j] x nrhs per matrix, concatenated)."""
        n = np.ascontiguousarray(n, dtype=np.int64)
        bw = np.ascontiguousarray(bw, dtype=np.int64)
        nrhs = x.numel() // int(n.sum())
        self._check(lib.gx_band_factor_solve(self.h, len(n), n.ctypes.data_as(i64p),
                                             bw.ctypes.data_as(i64p), _ptr(band), precision,
                                             nrhs, groups, _ptr(x)))
        return x

    def stats(self):
        out = np.zeros(5, dtype=np.int64)
        self._check(lib.gx_stats(self.h, out.ctypes.data_as(i64p)))
        return dict(eig_iters=int(out[0]), pcg_iters=int(out[1]),
                    interior_band_entries=int(out[2]), neumann_band_entries=int(out[3]),
                    fp64_fallbacks=int(out[4]))

    def band_stats(self):
        """Subdomain and eigensolver factor sizes: band and envelope entries, flops, and the
        envelope (algorithmic) and stored bytes of one PCG subdomain solve."""
        out = np.zeros(8)
        self._check(lib.gx_band_stats(self.h, out.ctypes.data_as(f64p)))
        keys = ["interior_band_entries", "interior_envelope_entries", "interior_factor_flops",
                "neumann_band_entries", "neumann_envelope_entries", "neumann_factor_flops",
                "solve_envelope_bytes", "solve_stored_bytes"]
        return dict(zip(keys, out.tolist()))

    def phase_times(self):
        t = np.zeros(8)
        lib.gx_phase_times(self.h, t.ctypes.data_as(f64p))
        return dict(zip(["assemble", "decomposition", "local_factors", "eigensolves",
                         "coarse", "pcg", "pcg_precond", "pcg_spmv"], t.tolist()))


# ---- differentiable solve --------------------------------------------------------------
def with_parameters(cfg, params):
    """Copy of a laminate descriptor with p = [A, L_w, E11 of every layer] applied (E of an
    isotropic layer)."""
    import copy
    c = copy.deepcopy(cfg)
    p = [float(v) for v in params]
    c["wrinkle"] = (p[0], p[1])
    for k, L in enumerate(c["layers"]):
        L["E1" if L["mat"] == "ply" else "E"] = p[2 + k]
    return c


def parameters_of(cfg):
    """p = [A, L_w, E11 of every layer] of a descriptor (defaults from the material table)."""
    from workloads import PLY, RESIN
    A, Lw = cfg.get("wrinkle", (0.0, 1.0))
    p = [A, Lw]
    for L in cfg["layers"]:
        p.append(L.get("E1", PLY["E1"]) if L["mat"] == "ply" else L.get("E", RESIN["E"]))
    return np.array(p, dtype=np.float64)


def _laminate_objective_fn():
    import torch

    class LaminateObjective(torch.autograd.Function):
        """J(p) = sum over the region of sigma_33^2 for the laminate with parameters p
        (wrinkle amplitude, wavelength, layer moduli): forward = mesh, assembly, GenEO
        set-up and PCG solve on the device; backward = the adjoint solve with the same
        preconditioner (gx_adjoint).  p is a CPU float64 tensor; J a CPU scalar."""

        @staticmethod
        def forward(ctx, p, cfg, region=1, rtol=1e-12, device=0):
            c = with_parameters(cfg, p.detach().cpu().numpy())
            s = Solver(device=device)
            s.laminate(c)
            f = s.assemble()
            sv = c["solver"]
            part = s.partition(c, sv["px"], sv["py"])
            s.geneo_setup(part, sv["px"] * sv["py"], overlap=sv["overlap"],
                          tau=sv["tau"] or 0.1, nev=sv["nev"] or 0, nev_max=sv["nev_max"])
            # an unconverged primal or adjoint solve raises GxError (GX_ENOCONV)
            u = s.pcg(f, rtol=rtol, maxit=5000)["x"]
            J, g, _ = s.adjoint(u, c, region=region, rtol=rtol, maxit=5000)
            s.close()
            ctx.save_for_backward(torch.tensor(g, dtype=torch.float64))
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            (g,) = ctx.saved_tensors
            return gJ * g, None, None, None, None

    return LaminateObjective


def laminate_objective(p, cfg, region=1, rtol=1e-12, device=0):
    """Differentiable J(p); see LaminateObjective."""
    global _LAMINATE_OBJECTIVE
    if _LAMINATE_OBJECTIVE is None:
        _LAMINATE_OBJECTIVE = _laminate_objective_fn()
    return _LAMINATE_OBJECTIVE.apply(p, cfg, region, rtol, device)


_LAMINATE_OBJECTIVE = None


# ---- batches of laminates -------------------------------------------------------------
class Batch:
    """Many laminates solved together: one Solver per laminate, each on its own torch
    stream (default priority) so that their kernels overlap, and one lockstep batched PCG
    (gx_pcg_solve_batch) with a per-laminate convergence test."""

    def __init__(self, cfgs, precision=GX_FP64, device=0):
        import torch
        self.torch = torch
        self.cfgs = list(cfgs)
        self.solvers, self.f = [], []
        for cfg in self.cfgs:
            s = Solver(device=device, stream=torch.cuda.Stream(device=device))
            s.laminate(cfg)
            self.f.append(s.assemble())
            self.solvers.append(s)
        self.precision = precision

    def setup(self, progress=None, concurrent=4):
        """Decomposition, GenEO coarse spaces and factors of every laminate, up to
        `concurrent` set-ups at a time (gx_geneo_setup_batch); progress(n - 1, n) is called
        when all are done.  Returns [(nev per subdomain, n0)] per laminate.  More than four
        at a time pays off only with more hardware queues than HIP's default of 4
        (GPU_MAX_HW_QUEUES in the environment before the HIP runtime starts)."""
        n = len(self.solvers)
        parts, opts = [], []
        for cfg, s in zip(self.cfgs, self.solvers):
            sv = cfg["solver"]
            with self.torch.cuda.stream(s.stream):
                part = s.partition(cfg, sv["px"], sv["py"])
            parts.append(part)
            opts.append(GeneoOpts(sv["px"] * sv["py"], _ptr(part), sv["overlap"],
                                  sv["tau"] or 0.1, sv["nev"] or 0, sv["nev_max"],
                                  self.precision, 1, None, 0.0, 0))
        nevs = [np.zeros(o.n_sub, dtype=np.int32) for o in opts]
        n0 = np.zeros(n, dtype=np.int64)
        st = np.zeros(n, dtype=np.int32)
        H = (vp * n)(*[s.h for s in self.solvers])
        O = (C.POINTER(GeneoOpts) * n)(*[C.pointer(o) for o in opts])
        NV = (i32p * n)(*[a.ctypes.data_as(i32p) for a in nevs])
        code = lib.gx_geneo_setup_batch(n, H, O, int(concurrent), NV, n0.ctypes.data_as(i64p),
                                        st.ctypes.data_as(i32p))
        if code == GX_EINVAL and not st.any():
            raise GxError(code, "gx_geneo_setup_batch: bad arguments")
        for k, s in enumerate(self.solvers):
            if st[k] != GX_OK:
                raise GxError(int(st[k]), f"laminate {k}: " + lib.gx_last_error(s.h).decode())
            s.nev, s.n0, s.n_sub = nevs[k], int(n0[k]), opts[k].n_sub
        if progress:
            progress(n - 1, n)
        return [(nevs[k], int(n0[k])) for k in range(n)]

    def solve(self, rtol=1e-8, maxit=2000):
        """x_i for every laminate; (list of x, iterations, relative residuals, statuses)."""
        n = len(self.solvers)
        xs = []
        for s, f in zip(self.solvers, self.f):
            with self.torch.cuda.stream(s.stream):
                xs.append(self.torch.zeros_like(f))
        H = (vp * n)(*[s.h for s in self.solvers])
        Bp = (vp * n)(*[f.data_ptr() for f in self.f])
        Xp = (vp * n)(*[x.data_ptr() for x in xs])
        it = np.zeros(n, dtype=np.int32)
        rr = np.zeros(n)
        st = np.zeros(n, dtype=np.int32)
        lib.gx_pcg_solve_batch(n, H, Bp, Xp, rtol, maxit, it.ctypes.data_as(i32p),
                               rr.ctypes.data_as(f64p), st.ctypes.data_as(i32p))
        return xs, it, rr, st

    def close(self):
        for s in self.solvers:
            s.close()
