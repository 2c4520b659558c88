"""Python binding of liblbddc.so (include/lbddc.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module only
converts numpy arrays and torch tensors to pointers and sizes and maps status
codes to exceptions.  It refuses to run without the compiled library.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbddc.so")

OK, E_ARG, E_NOMEM, E_HIP, E_STATE, E_DEGENERATE_MAP, E_PARAM_RANGE, E_ROM, E_NOT_CONVERGED, E_BREAKDOWN, \
    E_NUMERIC, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_NOMEM", -3: "E_HIP", -4: "E_STATE", -5: "E_DEGENERATE_MAP",
                -6: "E_PARAM_RANGE", -7: "E_ROM", -8: "E_NOT_CONVERGED", -9: "E_BREAKDOWN", -10: "E_NUMERIC",
                -11: "E_UNSUPPORTED"}
FP64, MIXED, FP32_CONTRACTION = 0, 1, 2
X_K, X_THETA, X_ITIL, X_S, X_D, X_PSI, X_SC, X_LOAD, X_FINE, X_RU, X_RC, X_CONS = range(12)
Q_NCELL, Q_NDOF_FREE, Q_N_SKELETON, Q_N_INTERIOR, Q_N_COARSE, Q_N_I_ROM, Q_NU_CELL, Q_NC_CELL, Q_NRHS, \
    Q_NR_MAX, Q_DEVICE_BYTES, Q_COARSE_SOLVE_BYTES, Q_COARSE_LEVELS, Q_COARSE_FWD_BYTES, \
    Q_COARSE_SWEEP_LAUNCHES, Q_NPAIR = range(16)
TIME_OP, TIME_PRE, TIME_COARSE, TIME_ALL, TIME_SAMPLE = 1, 2, 4, 7, 8
SIDE_LEFT, SIDE_RIGHT, SIDE_BOTTOM, SIDE_TOP = 1, 2, 4, 8
SIDES = {"left": SIDE_LEFT, "right": SIDE_RIGHT, "bottom": SIDE_BOTTOM, "top": SIDE_TOP}
CON_CORNERS, CON_EDGE_AVG, CON_EDGE_MOMENT = 1, 2, 4
PHASES = ["assembly_kernel", "assemble", "schur_kernel", "setup", "coarse_factor", "solve", "op_kernel",
          "pre_kernel", "coarse_solve", "recovery", "gradient", "adjoint_kernel", "coarse_fwd_sweep",
          "coarse_bwd_sweep", "geometry"]

FUNCTIONS = ["lbddc_create", "lbddc_destroy", "lbddc_last_error", "lbddc_version", "lbddc_load_rom",
             "lbddc_set_problem", "lbddc_set_geometry_device", "lbddc_assemble", "lbddc_setup", "lbddc_solve",
             "lbddc_solve_sequential",
             "lbddc_get_displacement", "lbddc_get_displacement_device", "lbddc_compliance_gradient",
             "lbddc_compliance_gradient_device", "lbddc_query", "lbddc_export_cells", "lbddc_phase_times",
             "lbddc_set_timing", "lbddc_assemble_fp32_noalloc", "lbddc_coarse_solve", "lbddc_implicit_tensors",
             "lbddc_implicit_rule_host"]


class LbddcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class RomDesc(C.Structure):
    _fields_ = [("family", C.c_int32), ("p", C.c_int32), ("q", C.c_int32), ("n_k", C.c_int32),
                ("n_r", C.c_int32), ("r", C.c_int32), ("lo", C.c_double), ("hi", C.c_double),
                ("U", C.POINTER(C.c_double)), ("coeff", C.POINTER(C.c_double)), ("I_pi", C.POINTER(C.c_double)),
                ("dim", C.c_int32)]


class ProblemDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("p", C.c_int32), ("q", C.c_int32),
                ("map_order", C.c_int32), ("ctrl", C.POINTER(C.c_double)), ("family", C.POINTER(C.c_int32)),
                ("t", C.POINTER(C.c_double)), ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
                ("constraints", C.c_uint32), ("clamped_sides", C.c_uint32), ("loaded_side", C.c_int32),
                ("nrhs", C.c_int32), ("traction", C.POINTER(C.c_double)), ("mu", C.POINTER(C.c_double))]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_res", C.c_double), ("true_rel_res", C.c_double)]


_lib = None


def library():
    """Load liblbddc.so from the package directory (raises if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2604_09113_amd.build.build()")
    # torch brings its own copy of the HIP runtime; when both are in one process,
    # torch's has to start first (started after the library's, it finds no GPU),
    # so bring it up before the library is loaded
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    sig = {
        "lbddc_create": (C.c_int, [C.c_int, P, C.POINTER(P)]),
        "lbddc_destroy": (None, [P]),
        "lbddc_last_error": (C.c_char_p, [P]),
        "lbddc_version": (C.c_int, []),
        "lbddc_load_rom": (C.c_int, [P, C.POINTER(RomDesc)]),
        "lbddc_set_problem": (C.c_int, [P, C.POINTER(ProblemDesc)]),
        "lbddc_set_geometry_device": (C.c_int, [P, P, P, P]),
        "lbddc_assemble": (C.c_int, [P, C.c_int]),
        "lbddc_setup": (C.c_int, [P, C.c_int]),
        "lbddc_solve": (C.c_int, [P, C.c_double, C.c_int32, C.POINTER(SolveInfo)]),
        "lbddc_solve_sequential": (C.c_int, [P, C.c_double, C.c_int32, C.POINTER(SolveInfo)]),
        "lbddc_get_displacement": (C.c_int, [P, C.c_int32, dp]),
        "lbddc_get_displacement_device": (C.c_int, [P, C.c_int32, P]),
        "lbddc_compliance_gradient": (C.c_int, [P, dp, dp, dp, dp]),
        "lbddc_compliance_gradient_device": (C.c_int, [P, P, P, P, P]),
        "lbddc_query": (C.c_int, [P, C.c_int32, C.POINTER(C.c_int64)]),
        "lbddc_export_cells": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32, dp]),
        "lbddc_phase_times": (C.c_int, [P, dp, C.c_int32]),
        "lbddc_set_timing": (C.c_int, [P, C.c_int32]),
        "lbddc_assemble_fp32_noalloc": (C.c_int, [P, P]),
        "lbddc_coarse_solve": (C.c_int, [P, dp, dp]),
        "lbddc_implicit_tensors": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp, C.c_int32,
                                             C.POINTER(C.c_int64), C.c_int32, dp]),
        "lbddc_implicit_rule_host": (C.c_int, [C.c_int32, dp, C.c_int32, C.c_int32, dp, dp, dp,
                                               C.POINTER(C.c_int32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Solver:
    """One lbddc context on a HIP device.  `stream` is a hipStream_t handle
    (an int, e.g. torch.cuda.current_stream().cuda_stream) or None."""

    def __init__(self, device=0, stream=None):
        self.lib = library()
        self.ctx = C.c_void_p()
        st = self.lib.lbddc_create(device, C.c_void_p(stream) if stream else None, C.byref(self.ctx))
        if st != OK:
            raise LbddcError(st, "lbddc_create failed (no HIP device?)")
        # the stream the library enqueues on: the given one, or (None) a stream
        # the library creates and owns
        self.stream = stream if stream else None
        self._keep = []

    def close(self):
        if self.ctx:
            self.lib.lbddc_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise LbddcError(st, self.lib.lbddc_last_error(self.ctx).decode())
        return st

    def load_rom(self, family, p, q, n_k, n_r, r, lo, hi, U, coeff, I_pi, dim=1):
        """U [n_k^dim, n_i, n_r], coeff [n_k^dim, (r+1)^dim, n_r], I_pi [n_i]
        (float64); dim 1 (thickness t) or 4 (corner thresholds mu)."""
        U, coeff, I_pi = _f64(U), _f64(coeff), _f64(I_pi)
        d = RomDesc(family, p, q, n_k, n_r, r, lo, hi, _dptr(U), _dptr(coeff), _dptr(I_pi), dim)
        self._check(self.lib.lbddc_load_rom(self.ctx, C.byref(d)))

    def set_problem(self, nx, ny, p, q, m, ctrl, family, t, E, nu, rho, moments, traction,
                    clamped=("left",), loaded="right", constraints=None, mu=None):
        """`moments` selects the coarse set CORNERS | EDGE_AVG (| EDGE_MOMENT);
        `constraints` (a CON_* mask) overrides it.  `clamped` is a sequence of
        side names, `loaded` one side name; traction [nrhs, n_side, 2];
        mu [ncell, 4] the corner thresholds of cells of four-parameter
        families (None when there are none)."""
        ctrl, t, traction = _f64(ctrl), _f64(t), _f64(traction)
        mu = None if mu is None else _f64(mu)
        family = np.ascontiguousarray(family, dtype=np.int32)
        if constraints is None:
            constraints = CON_CORNERS | CON_EDGE_AVG | (CON_EDGE_MOMENT if moments else 0)
        cmask = 0
        for sd in clamped:
            cmask |= SIDES[sd]
        d = ProblemDesc(nx, ny, p, q, m, _dptr(ctrl), family.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(t),
                        E, nu, rho, int(constraints), cmask, SIDES[loaded], traction.shape[0], _dptr(traction),
                        None if mu is None else _dptr(mu))
        self._check(self.lib.lbddc_set_problem(self.ctx, C.byref(d)))
        self.nrhs = traction.shape[0]
        self.shape = (nx, ny, p, q, m)

    def set_geometry_device(self, ctrl_ptr, t_ptr, mu_ptr=None):
        self._check(self.lib.lbddc_set_geometry_device(self.ctx, C.c_void_p(ctrl_ptr), C.c_void_p(t_ptr),
                                                       C.c_void_p(mu_ptr)))

    def assemble(self, prec=FP64):
        self._check(self.lib.lbddc_assemble(self.ctx, prec))

    def assemble_fp32_noalloc(self, dptr):
        """FP32 contraction into the caller's device buffer (packed node-pair
        triangle, float32 [ncell][npair][4]); no device allocation."""
        self._check(self.lib.lbddc_assemble_fp32_noalloc(self.ctx, C.c_void_p(dptr)))

    def setup(self, prec=FP64):
        self._check(self.lib.lbddc_setup(self.ctx, prec))

    def solve(self, rtol=1e-8, max_iter=1000, raise_on_not_converged=True, sequential=False):
        """lbddc_solve (load cases in blocks), or lbddc_solve_sequential."""
        info = (SolveInfo * self.nrhs)()
        fn = self.lib.lbddc_solve_sequential if sequential else self.lib.lbddc_solve
        st = fn(self.ctx, rtol, max_iter, info)
        if st != OK and (st != E_NOT_CONVERGED or raise_on_not_converged):
            self._check(st)
        return [dict(iters=i.iters, rel_res=i.rel_res, true_rel_res=i.true_rel_res) for i in info]

    def query(self, what):
        v = C.c_int64()
        self._check(self.lib.lbddc_query(self.ctx, what, C.byref(v)))
        return v.value

    def displacement(self, rhs=0):
        nx, ny, p, _, _ = self.shape
        out = np.zeros(((p * ny + 1), (p * nx + 1), 2))
        self._check(self.lib.lbddc_get_displacement(self.ctx, rhs, _dptr(out)))
        return out

    def displacement_device(self, rhs, dptr):
        self._check(self.lib.lbddc_get_displacement_device(self.ctx, rhs, C.c_void_p(dptr)))

    def compliance_gradient(self, thresholds=False):
        """(J, dJ/dctrl, dJ/dt), and dJ/dmu [nrhs, ncell, 4] with `thresholds`."""
        nx, ny, p, q, m = self.shape
        J = np.zeros(self.nrhs)
        gX = np.zeros((self.nrhs, m * ny + 1, m * nx + 1, 2))
        gt = np.zeros((self.nrhs, nx * ny))
        gmu = np.zeros((self.nrhs, nx * ny, 4)) if thresholds else None
        self._check(self.lib.lbddc_compliance_gradient(self.ctx, _dptr(J), _dptr(gX), _dptr(gt),
                                                       None if gmu is None else _dptr(gmu)))
        return (J, gX, gt, gmu) if thresholds else (J, gX, gt)

    def compliance_gradient_device(self, J_ptr, gX_ptr, gt_ptr, gmu_ptr=None):
        self._check(self.lib.lbddc_compliance_gradient_device(self.ctx, C.c_void_p(J_ptr), C.c_void_p(gX_ptr),
                                                              C.c_void_p(gt_ptr), C.c_void_p(gmu_ptr)))

    def implicit_tensors(self, family, p, q, mu, entries=None):
        """Offline snapshots of a Table 1 family on the GPU: I(mu) for every row
        of mu [count, 4], whole ([count, n_i]) or at `entries` ([count, ne]):
        one list [ne] for all rows, or one per row [count, ne]."""
        mu = _f64(np.atleast_2d(mu))
        count = mu.shape[0]
        n_i = (p + 1) ** 4 * 4 * (q + 1) ** 2
        per_rule = 0
        if entries is None:
            out = np.zeros((count, n_i))
            ne, ep = 0, None
        else:
            ent = np.ascontiguousarray(entries, dtype=np.int64)
            per_rule = int(ent.ndim == 2)
            ne = ent.shape[-1]
            out = np.zeros((count, ne))
            ep = ent.ctypes.data_as(C.POINTER(C.c_int64))
        self._check(self.lib.lbddc_implicit_tensors(self.ctx, family, p, q, count, _dptr(mu), ne, ep, per_rule,
                                                    _dptr(out)))
        return out

    def export(self, which, first, count):
        nx, ny, p, q, m = self.shape
        nB, nU, nC, nL = (p + 1) ** 2, 8 * p, self.query(Q_NC_CELL), (q + 1) ** 2
        per = {X_K: (2 * nB, 2 * nB), X_THETA: (2, 2, 2, 2, nL), X_ITIL: (self.query(Q_NR_MAX),),
               X_S: (nU, nU), X_D: (nU,), X_PSI: (nU, nC), X_SC: (nC, nC), X_LOAD: (self.nrhs, nU),
               X_FINE: (nU, nU), X_RU: (nU,), X_RC: (nC,), X_CONS: (4, (nC - 8) // 4, p + 1, 2)}[which]
        out = np.zeros((count,) + per)
        self._check(self.lib.lbddc_export_cells(self.ctx, which, first, count, _dptr(out)))
        return out

    def coarse_solve(self, z):
        """g = S_C^-1 z with the library's factored coarse matrix (host vectors)."""
        z = _f64(z)
        g = np.zeros_like(z)
        self._check(self.lib.lbddc_coarse_solve(self.ctx, _dptr(z), _dptr(g)))
        return g

    def set_timing(self, mask):
        """PCG phases timed by solve (TIME_OP | TIME_PRE | TIME_COARSE, optionally | TIME_SAMPLE for one
        iteration in eight; TIME_ALL after creation)."""
        self._check(self.lib.lbddc_set_timing(self.ctx, int(mask)))

    def phase_times(self):
        out = np.zeros(len(PHASES))
        self._check(self.lib.lbddc_phase_times(self.ctx, _dptr(out), len(PHASES)))
        return dict(zip(PHASES, out.tolist()))


def implicit_rule_host(family, mu, n, cap=1 << 18):
    """The offline implicit-domain rule computed on the host (a test entry):
    points x, y and weights w of the trimmed cell {phi_0 < mu}."""
    lib = library()
    x, y, w = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    cnt = C.c_int32()
    st = lib.lbddc_implicit_rule_host(family, _dptr(_f64(mu)), n, cap, _dptr(x), _dptr(y), _dptr(w), C.byref(cnt))
    if st != OK:
        raise LbddcError(st, "implicit_rule_host failed")
    k = cnt.value
    return x[:k], y[:k], w[:k]
