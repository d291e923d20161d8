"""ctypes binding of libpimc.so: same names as the C ABI, argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

PIMC_OK = 0
PIMC_EINVAL = -1
PIMC_EUNSUPPORTED = -2
PIMC_ENOMEM = -3
PIMC_EDEVICE = -4
PIMC_WNONFINITE = 1
PIMC_WNOTCONVERGED = 2
PIMC_CHUNK_PATHS = 4096          # paths per canonical chunk (include/pimc.h)

FLAG_FP64 = 0
FLAG_FP32_POLY = 1
FLAG_HIERARCHY = 2

MAX_DEGREE = 8
MAX_P = 18
FLOW_NPARAM = 24832
FLOW_MAX_LAYERS = 16


class PimcLibraryMissing(RuntimeError):
    """libpimc.so is not built: there is no other implementation to fall back to."""


class PimcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pimc status {status}: {msg}")
        self.status = status


class Potential(C.Structure):
    _fields_ = [("degree", C.c_int), ("coef", C.c_double * (MAX_DEGREE + 1))]


class Task(C.Structure):
    _fields_ = [("system", C.c_uint32), ("m", C.c_double), ("a", C.c_double), ("b", C.c_double), ("T", C.c_double),
                ("N", C.c_uint32), ("p", C.c_int), ("n_samples", C.c_uint64), ("stream", C.c_uint32)]


class GeneralPotential(C.Structure):
    _fields_ = [("degree", C.c_int), ("coef", C.c_double * (MAX_DEGREE + 1)), ("n_sech2", C.c_int),
                ("sech2_A", C.c_double * 4), ("sech2_alpha", C.c_double * 4), ("n_gauss", C.c_int),
                ("gauss_B", C.c_double * 4), ("gauss_beta", C.c_double * 4)]


def general_potential(poly=(), sech2=(), gauss=()) -> GeneralPotential:
    """V = sum poly[j] q^j + sum A / cosh^2(alpha q) for (A, alpha) in sech2 + sum B exp(-beta q^2)."""
    V = GeneralPotential()
    poly = list(poly)
    if len(poly) > MAX_DEGREE + 1 or len(sech2) > 4 or len(gauss) > 4:
        raise ValueError("too many terms")
    V.degree = max(len(poly) - 1, 0)
    for j in range(MAX_DEGREE + 1):
        V.coef[j] = float(poly[j]) if j < len(poly) else 0.0
    V.n_sech2 = len(sech2)
    for i, (A, a) in enumerate(sech2):
        V.sech2_A[i], V.sech2_alpha[i] = float(A), float(a)
    V.n_gauss = len(gauss)
    for i, (B, b) in enumerate(gauss):
        V.gauss_B[i], V.gauss_beta[i] = float(B), float(b)
    return V


class Mpt(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("alpha", C.c_double)]


MAX_DIM = 4
POLY_MAX_TERMS = 70
POLY_MAX_DEGREE = 4
MAX_RADIAL_DEGREE = 2


class RadialPotential(C.Structure):
    _fields_ = [("dim", C.c_int), ("degree", C.c_int), ("coef", C.c_double * (MAX_RADIAL_DEGREE + 1))]


class PolyPotential(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_terms", C.c_int), ("coef", C.c_double * POLY_MAX_TERMS),
                ("exps", (C.c_int * MAX_DIM) * POLY_MAX_TERMS)]


def poly_potential(terms, dim):
    """pimc_poly_potential for V(q) = sum coef q_1^e1 q_2^e2 q_3^e3 from ``terms`` = [(coef, (e1, ..))]."""
    terms = list(terms)
    if len(terms) > POLY_MAX_TERMS:
        raise ValueError(f"at most {POLY_MAX_TERMS} terms")
    V = PolyPotential()
    V.dim = int(dim)
    V.n_terms = len(terms)
    for t, (c, e) in enumerate(terms):
        V.coef[t] = float(c)
        e = list(e) + [0] * (MAX_DIM - len(e))
        for k in range(MAX_DIM):
            V.exps[t][k] = int(e[k])
    return V


def radial_potential(coefs, dim):
    """pimc_radial_potential for V = sum_n coefs[n] (q.q)^n in `dim` coordinates."""
    coefs = list(coefs)
    if not coefs or len(coefs) > MAX_RADIAL_DEGREE + 1:
        raise ValueError(f"radial potential needs 1..{MAX_RADIAL_DEGREE + 1} coefficients")
    V = RadialPotential()
    V.dim = int(dim)
    V.degree = len(coefs) - 1
    for n in range(MAX_RADIAL_DEGREE + 1):
        V.coef[n] = float(coefs[n]) if n < len(coefs) else 0.0
    return V


def _vec(x, dim):
    x = [float(v) for v in x]
    if len(x) != dim:
        raise ValueError(f"endpoint needs {dim} coordinates")
    return (C.c_double * dim)(*x)


class FlowConfig(C.Structure):
    _fields_ = [("layers", C.c_int), ("batch", C.c_uint32), ("lr", C.c_double), ("beta", C.c_double),
                ("init_seed", C.c_uint64), ("init_scale", C.c_double)]


class SpectrumInfo(C.Structure):
    _fields_ = [("iterations", C.c_uint32), ("converged", C.c_int), ("max_residual", C.c_double),
                ("matrix_ms", C.c_double), ("solve_ms", C.c_double)]


class _LevelResult(C.Structure):
    _fields_ = [("amp", C.c_double), ("err", C.c_double), ("log_amp", C.c_double), ("relvar", C.c_double),
                ("ess", C.c_double), ("n", C.c_uint64), ("n_nonfinite", C.c_uint64)]


class BatchClass(C.Structure):
    _fields_ = [("p", C.c_int), ("n16", C.c_int), ("n_tasks", C.c_uint64), ("n_items", C.c_uint64),
                ("shape", C.c_int), ("n_shapes", C.c_int), ("subtree_levels", C.c_int), ("block", C.c_int),
                ("waves_per_eu", C.c_int), ("slice_batch", C.c_int), ("tuned_ms", C.c_double),
                ("default_ms", C.c_double)]


@dataclass
class LevelResult:
    amp: float
    err: float
    log_amp: float
    relvar: float
    ess: float
    n: int
    n_nonfinite: int


_lib = None


def lib_path() -> str:
    return os.path.join(_HERE, "libpimc.so")


def load_library():
    """Load the in-tree libpimc.so (raises PimcLibraryMissing when absent)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise PimcLibraryMissing(f"{path} is missing: build it with `python -m paper_1105_0542_amd.build`")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7). Importing torch first
    # makes the dynamic loader bind libpimc.so to that already-loaded runtime, so the library and
    # torch's streams and allocations live in one HIP runtime. Loading libpimc.so first and torch
    # afterwards would put two HSA runtimes in the process, and the second cannot open the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp = C.c_void_p
    P = C.POINTER
    lib.pimc_strerror.restype = C.c_char_p
    lib.pimc_strerror.argtypes = [C.c_int]
    lib.pimc_last_error.restype = C.c_char_p
    lib.pimc_last_error.argtypes = [vp]
    lib.pimc_check_problem.restype = C.c_int
    lib.pimc_check_problem.argtypes = [P(Potential), C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_uint32, C.c_int, C.c_uint64]
    lib.pimc_level_table.restype = C.c_int
    lib.pimc_level_table.argtypes = [P(Potential), C.c_double, C.c_double, C.c_int, C.c_uint32, P(C.c_double),
                                     C.c_size_t, P(C.c_size_t), P(C.c_int), P(C.c_int), P(C.c_int)]
    lib.pimc_create.restype = C.c_int
    lib.pimc_create.argtypes = [P(vp), C.c_int, vp]
    lib.pimc_destroy.restype = C.c_int
    lib.pimc_destroy.argtypes = [vp]
    lib.pimc_amplitude.restype = C.c_int
    lib.pimc_amplitude.argtypes = [vp, P(Potential), C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32,
                                   C.c_int, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, P(_LevelResult)]
    lib.pimc_amplitude_noalloc.restype = C.c_int
    lib.pimc_amplitude_noalloc.argtypes = [vp, P(Potential), C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_uint32, C.c_int, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                           P(_LevelResult)]
    lib.pimc_path_actions.restype = C.c_int
    lib.pimc_path_actions.argtypes = [vp, P(Potential), C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_uint32, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64,
                                      C.c_uint64, P(C.c_double)]
    lib.pimc_last_partials.restype = C.c_int
    lib.pimc_last_partials.argtypes = [vp, C.c_uint32, C.c_uint64, C.c_uint64, P(C.c_double), P(C.c_uint64),
                                       P(C.c_uint64), P(C.c_double)]
    lib.pimc_normals.restype = C.c_int
    lib.pimc_normals.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32, P(C.c_double)]
    lib.pimc_batch_create.restype = C.c_int
    lib.pimc_batch_create.argtypes = [vp, P(Potential), C.c_int, P(Task), C.c_size_t, C.c_uint64, C.c_uint32, P(vp)]
    lib.pimc_batch_run.restype = C.c_int
    lib.pimc_batch_run.argtypes = [vp, P(_LevelResult), P(C.c_double)]
    lib.pimc_batch_set_tuning.restype = C.c_int
    lib.pimc_batch_set_tuning.argtypes = [vp, C.c_int, C.c_uint32]
    lib.pimc_batch_autotune.restype = C.c_int
    lib.pimc_batch_autotune.argtypes = [vp, C.c_char_p, P(C.c_int), P(C.c_uint32)]
    lib.pimc_batch_destroy.restype = C.c_int
    lib.pimc_batch_destroy.argtypes = [vp]
    lib.pimc_batch_last_error.restype = C.c_char_p
    lib.pimc_batch_last_error.argtypes = [vp]
    lib.pimc_amplitude_batch.restype = C.c_int
    lib.pimc_amplitude_batch.argtypes = [vp, P(Potential), C.c_int, P(Task), C.c_size_t, C.c_uint64, C.c_uint32,
                                         vp, C.c_int]
    lib.pimc_batch_run_to.restype = C.c_int
    lib.pimc_batch_run_to.argtypes = [vp, vp, C.c_int, P(C.c_double)]
    lib.pimc_batch_n_classes.restype = C.c_int
    lib.pimc_batch_n_classes.argtypes = [vp]
    lib.pimc_batch_class_info.restype = C.c_int
    lib.pimc_batch_class_info.argtypes = [vp, C.c_int, P(BatchClass)]
    lib.pimc_batch_set_shape.restype = C.c_int
    lib.pimc_batch_set_shape.argtypes = [vp, C.c_int, C.c_int]
    lib.pimc_last_kernel_ms.restype = C.c_int
    lib.pimc_last_kernel_ms.argtypes = [vp, P(C.c_double)]
    lib.pimc_flow_create.restype = C.c_int
    lib.pimc_flow_create.argtypes = [vp, P(Potential), C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32,
                                     C.c_int, P(FlowConfig), P(vp)]
    lib.pimc_flow_destroy.restype = C.c_int
    lib.pimc_flow_destroy.argtypes = [vp]
    lib.pimc_flow_get_params.restype = C.c_int
    lib.pimc_flow_get_params.argtypes = [vp, P(C.c_float), C.c_size_t, P(C.c_size_t)]
    lib.pimc_flow_set_params.restype = C.c_int
    lib.pimc_flow_set_params.argtypes = [vp, P(C.c_float), C.c_size_t]
    lib.pimc_flow_save.restype = C.c_int
    lib.pimc_flow_save.argtypes = [vp, C.c_char_p]
    lib.pimc_flow_load.restype = C.c_int
    lib.pimc_flow_load.argtypes = [vp, C.c_char_p]
    lib.pimc_flow_grad.restype = C.c_int
    lib.pimc_flow_grad.argtypes = [vp, C.c_uint64, C.c_uint32, P(C.c_double), P(C.c_double), P(C.c_float)]
    lib.pimc_flow_train.restype = C.c_int
    lib.pimc_flow_train.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, P(C.c_double), P(C.c_double)]
    lib.pimc_flow_log_weights.restype = C.c_int
    lib.pimc_flow_log_weights.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, P(C.c_double),
                                          P(C.c_double), P(C.c_double)]
    lib.pimc_flow_amplitude.restype = C.c_int
    lib.pimc_flow_amplitude.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_uint32, P(_LevelResult), P(C.c_double)]
    lib.pimc_amplitude_mpt.restype = C.c_int
    lib.pimc_amplitude_mpt.argtypes = [vp, P(Mpt), C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32,
                                       C.c_int, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, P(_LevelResult)]
    lib.pimc_path_actions_mpt.restype = C.c_int
    lib.pimc_path_actions_mpt.argtypes = [vp, P(Mpt), C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint32,
                                          C.c_int, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64,
                                          P(C.c_double)]
    lib.pimc_level_table_mpt.restype = C.c_int
    lib.pimc_level_table_mpt.argtypes = [P(Mpt), C.c_double, C.c_double, C.c_int, C.c_uint32, P(C.c_double),
                                         C.c_size_t, P(C.c_size_t), P(C.c_int), P(C.c_int)]
    lib.pimc_amplitude_radial.restype = C.c_int
    lib.pimc_amplitude_radial.argtypes = [vp, P(RadialPotential), C.c_double, P(C.c_double), P(C.c_double),
                                          C.c_double, C.c_uint32, C.c_int, C.c_uint64, C.c_uint64, C.c_uint32,
                                          C.c_uint32, P(_LevelResult)]
    lib.pimc_path_actions_radial.restype = C.c_int
    lib.pimc_path_actions_radial.argtypes = [vp, P(RadialPotential), C.c_double, P(C.c_double), P(C.c_double),
                                             C.c_double, C.c_uint32, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32,
                                             C.c_uint64, C.c_uint64, P(C.c_double)]
    lib.pimc_amplitude_poly.restype = C.c_int
    lib.pimc_amplitude_poly.argtypes = [vp, P(PolyPotential), C.c_double, P(C.c_double), P(C.c_double),
                                        C.c_double, C.c_uint32, C.c_int, C.c_uint64, C.c_uint64, C.c_uint32,
                                        C.c_uint32, P(_LevelResult)]
    lib.pimc_path_actions_poly.restype = C.c_int
    lib.pimc_path_actions_poly.argtypes = [vp, P(PolyPotential), C.c_double, P(C.c_double), P(C.c_double),
                                           C.c_double, C.c_uint32, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32,
                                           C.c_uint64, C.c_uint64, P(C.c_double)]
    lib.pimc_level_table_poly.restype = C.c_int
    lib.pimc_level_table_poly.argtypes = [P(PolyPotential), C.c_double, C.c_double, C.c_int, C.c_uint32,
                                          vp, C.c_size_t, vp, C.c_size_t, P(C.c_size_t)]
    lib.pimc_level_table_radial.restype = C.c_int
    lib.pimc_level_table_radial.argtypes = [P(RadialPotential), C.c_double, C.c_double, C.c_int, C.c_uint32,
                                            P(C.c_double), C.c_size_t, P(C.c_size_t), P(C.c_int), C.c_size_t,
                                            P(C.c_int)]
    lib.pimc_amplitude_general.restype = C.c_int
    lib.pimc_amplitude_general.argtypes = [vp, P(GeneralPotential), C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_uint32, C.c_int, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                           P(_LevelResult)]
    lib.pimc_path_actions_general.restype = C.c_int
    lib.pimc_path_actions_general.argtypes = [vp, P(GeneralPotential), C.c_double, C.c_double, C.c_double,
                                              C.c_double, C.c_uint32, C.c_int, C.c_uint64, C.c_uint32, C.c_uint32,
                                              C.c_uint64, C.c_uint64, P(C.c_double)]
    lib.pimc_evolution_matrix.restype = C.c_int
    lib.pimc_evolution_matrix.argtypes = [vp, P(Potential), C.c_double, C.c_double, C.c_int, C.c_double, C.c_uint32,
                                          vp, C.c_uint64]
    lib.pimc_spectrum.restype = C.c_int
    lib.pimc_spectrum.argtypes = [vp, P(Potential), C.c_double, C.c_double, C.c_int, C.c_double, C.c_uint32,
                                  C.c_uint32, C.c_uint32, C.c_double, P(C.c_double), P(C.c_double), P(SpectrumInfo)]
    _lib = lib
    return lib


def potential_from_coefs(coefs: Sequence[float]) -> Potential:
    coefs = list(coefs)
    if len(coefs) > MAX_DEGREE + 1:
        raise ValueError(f"degree > {MAX_DEGREE}")
    V = Potential()
    V.degree = max(len(coefs) - 1, 0)
    for j in range(MAX_DEGREE + 1):
        V.coef[j] = float(coefs[j]) if j < len(coefs) else 0.0
    return V


def quartic(A: float, g: float) -> List[float]:
    """Coefficients of V = A q^2/2 + g q^4/24."""
    return [0.0, 0.0, A / 2.0, 0.0, g / 24.0]


def _err(lib, ctx, status) -> PimcError:
    msg = lib.pimc_last_error(ctx)
    return PimcError(status, (msg or b"").decode() or lib.pimc_strerror(status).decode())


def check_problem(coefs, m, a, b, T, N, p, n_samples) -> int:
    lib = load_library()
    V = potential_from_coefs(coefs)
    return lib.pimc_check_problem(C.byref(V), m, a, b, T, N, p, n_samples)


def level_table(coefs, m, T, p, level):
    """(coef array, degrees per k, even flag) of pimc_level_table (host-only call)."""
    lib = load_library()
    V = potential_from_coefs(coefs)
    need = C.c_size_t(0)
    nk = C.c_int(0)
    deg = (C.c_int * max(MAX_P, int(p)))()
    ev = C.c_int(0)
    lib.pimc_level_table(C.byref(V), m, T, p, level, None, 0, C.byref(need), C.byref(nk), deg, C.byref(ev))
    out = np.zeros(need.value, dtype=np.float64)
    st = lib.pimc_level_table(C.byref(V), m, T, p, level, out.ctypes.data_as(C.POINTER(C.c_double)), out.size,
                              C.byref(need), C.byref(nk), deg, C.byref(ev))
    if st != PIMC_OK:
        raise _err(lib, None, st)
    return out, [deg[k] for k in range(nk.value)], bool(ev.value)


def level_table_mpt(lam, alpha, m, T, p, level):
    """(coef array, degrees per k) of pimc_level_table_mpt (host-only call): tables in tanh^2."""
    lib = load_library()
    V = Mpt(float(lam), float(alpha))
    need = C.c_size_t(0)
    nk = C.c_int(0)
    deg = (C.c_int * max(MAX_P, int(p)))()
    lib.pimc_level_table_mpt(C.byref(V), m, T, p, level, None, 0, C.byref(need), C.byref(nk), deg)
    out = np.zeros(need.value, dtype=np.float64)
    st = lib.pimc_level_table_mpt(C.byref(V), m, T, p, level, out.ctypes.data_as(C.POINTER(C.c_double)), out.size,
                                  C.byref(need), C.byref(nk), deg)
    if st != PIMC_OK:
        raise _err(lib, None, st)
    return out, [deg[k] for k in range(nk.value)]


def level_table_radial(coefs, dim, m, T, p, level):
    """(coef array, [(k, j, len) per group]) of pimc_level_table_radial (host-only call)."""
    lib = load_library()
    V = radial_potential(coefs, dim)
    need = C.c_size_t(0)
    ng = C.c_int(0)
    lib.pimc_level_table_radial(C.byref(V), m, T, p, level, None, 0, C.byref(need), None, 0, C.byref(ng))
    out = np.zeros(need.value, dtype=np.float64)
    shape = (C.c_int * (3 * ng.value))()
    st = lib.pimc_level_table_radial(C.byref(V), m, T, p, level, out.ctypes.data_as(C.POINTER(C.c_double)),
                                     out.size, C.byref(need), shape, 3 * ng.value, C.byref(ng))
    if st != PIMC_OK:
        raise _err(lib, None, st)
    return out, [(shape[3 * g], shape[3 * g + 1], shape[3 * g + 2]) for g in range(ng.value)]


def level_table_poly(terms, dim, m, T, p, level):
    """(coef array, exps array [terms, 2 dim]) of pimc_level_table_poly (host-only call)."""
    lib = load_library()
    V = poly_potential(terms, dim)
    need = C.c_size_t(0)
    lib.pimc_level_table_poly(C.byref(V), m, T, p, level, None, 0, None, 0, C.byref(need))
    n = need.value
    out = np.zeros(n, dtype=np.float64)
    exps = np.zeros((n, 2 * dim), dtype=np.int32)
    st = lib.pimc_level_table_poly(C.byref(V), m, T, p, level, out.ctypes.data_as(C.POINTER(C.c_double)), n,
                                   exps.ctypes.data_as(C.POINTER(C.c_int)), exps.size, C.byref(need))
    if st != PIMC_OK:
        raise _err(lib, None, st)
    return out, exps


def _torch_stream_handle() -> Optional[int]:
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream) or None
    except Exception:
        return None
    return None


class Context:
    """pimc_create/pimc_destroy. ``stream``: a hipStream_t handle (int); default = torch's current
    stream if torch sees a GPU, else a stream owned by the context."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, use_torch_stream: bool = True):
        self.lib = load_library()
        if stream is None and use_torch_stream:
            stream = _torch_stream_handle()
        h = C.c_void_p()
        st = self.lib.pimc_create(C.byref(h), device, C.c_void_p(stream) if stream else None)
        if st != PIMC_OK:
            raise _err(self.lib, None, st)
        self.h = h
        self._children = weakref.WeakSet()      # batches and proposals that use this context

    def close(self):
        """Destroy the context; batches and proposals created on it are destroyed first."""
        if getattr(self, "h", None):
            for child in list(getattr(self, "_children", ())):
                child.close()
            self.lib.pimc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st < 0:
            raise _err(self.lib, self.h, st)
        return st

    def amplitude(self, coefs, m, a, b, T, N, p, n_samples, seed, stream=0, flags=0):
        """pimc_amplitude -> (list of LevelResult for n = 0..s, status)."""
        V = potential_from_coefs(coefs)
        s = int(N).bit_length() - 1
        out = (_LevelResult * (s + 1))()
        st = self._check(self.lib.pimc_amplitude(self.h, C.byref(V), m, a, b, T, N, p, n_samples, seed, stream,
                                                 flags, out))
        res = [LevelResult(r.amp, r.err, r.log_amp, r.relvar, r.ess, int(r.n), int(r.n_nonfinite)) for r in out]
        return res, st

    def amplitude_noalloc(self, coefs, m, a, b, T, N, p, n_samples, seed, stream=0, flags=0):
        """pimc_amplitude_noalloc (no device allocation: the library's static workspace) -> (list of
        LevelResult for n = 0..s, status)."""
        V = potential_from_coefs(coefs)
        s = int(N).bit_length() - 1
        out = (_LevelResult * (s + 1))()
        st = self._check(self.lib.pimc_amplitude_noalloc(self.h, C.byref(V), m, a, b, T, N, p, n_samples, seed,
                                                         stream, flags, out))
        res = [LevelResult(r.amp, r.err, r.log_amp, r.relvar, r.ess, int(r.n), int(r.n_nonfinite)) for r in out]
        return res, st

    def amplitude_mpt(self, lam, alpha, m, a, b, T, N, p, n_samples, seed, stream=0, flags=0):
        """pimc_amplitude_mpt (V = -lam / cosh^2(alpha q)) -> (list of LevelResult, status)."""
        V = Mpt(float(lam), float(alpha))
        s = int(N).bit_length() - 1
        out = (_LevelResult * (s + 1))()
        st = self._check(self.lib.pimc_amplitude_mpt(self.h, C.byref(V), m, a, b, T, N, p, n_samples, seed, stream,
                                                     flags, out))
        res = [LevelResult(r.amp, r.err, r.log_amp, r.relvar, r.ess, int(r.n), int(r.n_nonfinite)) for r in out]
        return res, st

    def amplitude_general(self, m, a, b, T, N, p, n_samples, seed, stream=0, flags=0, poly=(), sech2=(), gauss=()):
        """pimc_amplitude_general (derivative-symbol mode) -> (list of LevelResult, status)."""
        V = general_potential(poly, sech2, gauss)
        s = int(N).bit_length() - 1
        out = (_LevelResult * (s + 1))()
        st = self._check(self.lib.pimc_amplitude_general(self.h, C.byref(V), m, a, b, T, N, p, n_samples, seed,
                                                         stream, flags, out))
        res = [LevelResult(r.amp, r.err, r.log_amp, r.relvar, r.ess, int(r.n), int(r.n_nonfinite)) for r in out]
        return res, st

    def path_actions_general(self, m, a, b, T, N, p, seed, stream, flags, first_path, k_paths, poly=(), sech2=(),
                             gauss=()):
        V = general_potential(poly, sech2, gauss)
        s = int(N).bit_length() - 1
        out = np.zeros((k_paths, s + 1), dtype=np.float64)
        self._check(self.lib.pimc_path_actions_general(self.h, C.byref(V), m, a, b, T, N, p, seed, stream, flags,
                                                       first_path, k_paths, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def amplitude_radial(self, coefs, dim, m, a, b, T, N, p, n_samples, seed, stream=0, flags=0):
        """pimc_amplitude_radial (V = sum_n coefs[n] (q.q)^n, q in R^dim) -> (list of LevelResult, status)."""
        V = radial_potential(coefs, dim)
        s = int(N).bit_length() - 1
        out = (_LevelResult * (s + 1))()
        st = self._check(self.lib.pimc_amplitude_radial(self.h, C.byref(V), m, _vec(a, dim), _vec(b, dim), T, N, p,
                                                        n_samples, seed, stream, flags, out))
        res = [LevelResult(r.amp, r.err, r.log_amp, r.relvar, r.ess, int(r.n), int(r.n_nonfinite)) for r in out]
        return res, st

    def path_actions_radial(self, coefs, dim, m, a, b, T, N, p, seed, stream, flags, first_path, k_paths):
        """pimc_path_actions_radial -> array [k_paths, s+1]."""
        V = radial_potential(coefs, dim)
        s = int(N).bit_length() - 1
        out = np.zeros((k_paths, s + 1), dtype=np.float64)
        self._check(self.lib.pimc_path_actions_radial(self.h, C.byref(V), m, _vec(a, dim), _vec(b, dim), T, N, p,
                                                      seed, stream, flags, first_path, k_paths,
                                                      out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def amplitude_poly(self, terms, dim, m, a, b, T, N, p, n_samples, seed, stream=0, flags=0):
        """pimc_amplitude_poly (V = sum coef prod_c q_c^e_c, q in R^dim) -> (list of LevelResult, status)."""
        V = poly_potential(terms, dim)
        s = int(N).bit_length() - 1
        out = (_LevelResult * (s + 1))()
        st = self._check(self.lib.pimc_amplitude_poly(self.h, C.byref(V), m, _vec(a, dim), _vec(b, dim), T, N, p,
                                                      n_samples, seed, stream, flags, out))
        res = [LevelResult(r.amp, r.err, r.log_amp, r.relvar, r.ess, int(r.n), int(r.n_nonfinite)) for r in out]
        return res, st

    def path_actions_poly(self, terms, dim, m, a, b, T, N, p, seed, stream, flags, first_path, k_paths):
        """pimc_path_actions_poly -> array [k_paths, s+1]."""
        V = poly_potential(terms, dim)
        s = int(N).bit_length() - 1
        out = np.zeros((k_paths, s + 1), dtype=np.float64)
        self._check(self.lib.pimc_path_actions_poly(self.h, C.byref(V), m, _vec(a, dim), _vec(b, dim), T, N, p,
                                                    seed, stream, flags, first_path, k_paths,
                                                    out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def path_actions_mpt(self, lam, alpha, m, a, b, T, N, p, seed, stream, flags, first_path, k_paths):
        V = Mpt(float(lam), float(alpha))
        s = int(N).bit_length() - 1
        out = np.zeros((k_paths, s + 1), dtype=np.float64)
        self._check(self.lib.pimc_path_actions_mpt(self.h, C.byref(V), m, a, b, T, N, p, seed, stream, flags,
                                                   first_path, k_paths, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def path_actions(self, coefs, m, a, b, T, N, p, seed, stream, flags, first_path, k_paths):
        """pimc_path_actions -> array [k_paths, s+1]."""
        V = potential_from_coefs(coefs)
        s = int(N).bit_length() - 1
        out = np.zeros((k_paths, s + 1), dtype=np.float64)
        self._check(self.lib.pimc_path_actions(self.h, C.byref(V), m, a, b, T, N, p, seed, stream, flags,
                                               first_path, k_paths, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def last_partials(self, level, first_chunk, n_chunks):
        """pimc_last_partials -> (array [n_chunks, 4], chunk_paths, total_chunks, shift)."""
        out = np.zeros((n_chunks, 4), dtype=np.float64)
        cp = C.c_uint64(0)
        tc = C.c_uint64(0)
        sh = C.c_double(0)
        self._check(self.lib.pimc_last_partials(self.h, level, first_chunk, n_chunks,
                                                out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(cp),
                                                C.byref(tc), C.byref(sh)))
        return out, cp.value, tc.value, sh.value

    def normals(self, seed, stream, first_path, k_paths, n_nodes):
        """pimc_normals -> array [k_paths, n_nodes] of z_h, h = 1..n_nodes."""
        out = np.zeros((k_paths, n_nodes), dtype=np.float64)
        self._check(self.lib.pimc_normals(self.h, seed, stream, first_path, k_paths, n_nodes,
                                          out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def evolution_matrix(self, coefs, m, t, p, L, n, device_ptr, ld):
        """pimc_evolution_matrix into caller-owned device memory (an address, e.g. a torch tensor's
        data_ptr(), of at least n*ld doubles)."""
        V = potential_from_coefs(coefs)
        self._check(self.lib.pimc_evolution_matrix(self.h, C.byref(V), m, t, p, L, n, C.c_void_p(device_ptr), ld))

    def spectrum(self, coefs, m, t, p, L, n, k, max_iter=None, tol=1e-10, want_psi=False):
        """pimc_spectrum -> (E [k], psi [k, n] or None, SpectrumInfo, status); max_iter defaults to
        min(n, 1024)."""
        V = potential_from_coefs(coefs)
        if max_iter is None:
            max_iter = min(int(n), 1024)
        E = np.zeros(k, dtype=np.float64)
        psi = np.zeros((k, n), dtype=np.float64) if want_psi else None
        info = SpectrumInfo()
        st = self._check(self.lib.pimc_spectrum(self.h, C.byref(V), m, t, p, L, n, k, max_iter, tol,
                                                E.ctypes.data_as(C.POINTER(C.c_double)),
                                                None if psi is None else psi.ctypes.data_as(C.POINTER(C.c_double)),
                                                C.byref(info)))
        return E, psi, info, st

    def last_kernel_ms(self) -> float:
        ms = C.c_double(0)
        self._check(self.lib.pimc_last_kernel_ms(self.h, C.byref(ms)))
        return ms.value


_RESULT_DTYPE = np.dtype([("amp", "f8"), ("err", "f8"), ("log_amp", "f8"), ("relvar", "f8"), ("ess", "f8"),
                          ("n", "u8"), ("n_nonfinite", "u8")])


def make_tasks(rows) -> "C.Array":
    """Task array from an iterable of (system, m, a, b, T, N, p, n_samples, stream)."""
    rows = list(rows)
    arr = (Task * len(rows))()
    for i, r in enumerate(rows):
        arr[i] = Task(*r)
    return arr


class Batch:
    """pimc_batch_create / run / set_tuning / autotune / destroy."""

    def __init__(self, ctx: Context, systems, tasks, seed: int, flags: int = 0):
        self.ctx = ctx
        self.lib = ctx.lib
        pots = (Potential * len(systems))(*[potential_from_coefs(c) for c in systems])
        self.tasks = tasks if isinstance(tasks, C.Array) else make_tasks(tasks)
        self.n_tasks = len(self.tasks)
        self.s_max = max(int(t.N).bit_length() - 1 for t in self.tasks)
        h = C.c_void_p()
        st = self.lib.pimc_batch_create(ctx.h, pots, len(systems), self.tasks, self.n_tasks, seed, flags, C.byref(h))
        if st != PIMC_OK:
            raise _err(self.lib, ctx.h, st)
        self.h = h
        ctx._children.add(self)
        self._out = (_LevelResult * (self.n_tasks * (self.s_max + 1)))()

    def _check(self, st):
        if st < 0:
            msg = self.lib.pimc_batch_last_error(self.h)
            raise PimcError(st, (msg or b"").decode())
        return st

    def run(self):
        """One graph replay -> (structured array [n_tasks, s_max+1], device ms, status)."""
        ms = C.c_double(0)
        st = self._check(self.lib.pimc_batch_run(self.h, self._out, C.byref(ms)))
        arr = np.frombuffer(self._out, dtype=_RESULT_DTYPE).reshape(self.n_tasks, self.s_max + 1).copy()
        return arr, ms.value, st

    def run_to_device(self, out):
        """One graph replay with the results written into the caller's device buffer `out` (a
        contiguous torch CUDA tensor of at least n_tasks * (s_max+1) * 56 bytes, e.g. float64 of
        shape [n_tasks, s_max+1, 7]: amp, err, log_amp, relvar, ess, then n and n_nonfinite as
        64-bit integers). Returns (device ms, status)."""
        need = self.n_tasks * (self.s_max + 1) * C.sizeof(_LevelResult)
        if not out.is_cuda or not out.is_contiguous() or out.numel() * out.element_size() < need:
            raise ValueError(f"need a contiguous device tensor of at least {need} bytes")
        ms = C.c_double(0)
        st = self._check(self.lib.pimc_batch_run_to(self.h, C.c_void_p(out.data_ptr()), 1, C.byref(ms)))
        return ms.value, st

    def set_tuning(self, grid_mult_x2: int, grab: int):
        self._check(self.lib.pimc_batch_set_tuning(self.h, grid_mult_x2, grab))

    def classes(self):
        """Kernel classes (p, N = 16 or not) with their launch shapes and autotuner timings."""
        out = []
        for k in range(self.lib.pimc_batch_n_classes(self.h)):
            ci = BatchClass()
            self._check(self.lib.pimc_batch_class_info(self.h, k, C.byref(ci)))
            out.append({f: getattr(ci, f) for f, _ in BatchClass._fields_})
        return out

    def set_shape(self, k: int, shape: int):
        self._check(self.lib.pimc_batch_set_shape(self.h, k, shape))

    def autotune(self, cache_path=None):
        g = C.c_int(0)
        gr = C.c_uint32(0)
        self._check(self.lib.pimc_batch_autotune(self.h, cache_path.encode() if cache_path else None, C.byref(g),
                                                 C.byref(gr)))
        return g.value, gr.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.pimc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


class Flow:
    """pimc_flow_create / get_params / set_params / grad / train / log_weights / amplitude / destroy.

    The proposal belongs to the context ``ctx`` (its device, stream and error text)."""

    def __init__(self, ctx: Context, coefs, m, a, b, T, N, p, layers=8, batch=4096, lr=1e-3, beta=0.0,
                 init_seed=0, init_scale=0.0):
        self.ctx = ctx
        self.lib = ctx.lib
        self.N = int(N)
        self.D = self.N - 1
        self.layers = int(layers)
        self.batch = int(batch)
        V = potential_from_coefs(coefs)
        cfg = FlowConfig(int(layers), int(batch), float(lr), float(beta), int(init_seed), float(init_scale))
        h = C.c_void_p()
        st = self.lib.pimc_flow_create(ctx.h, C.byref(V), m, a, b, T, N, p, C.byref(cfg), C.byref(h))
        if st != PIMC_OK:
            raise _err(self.lib, ctx.h, st)
        self.h = h
        ctx._children.add(self)

    def _check(self, st):
        if st < 0:
            raise _err(self.lib, self.ctx.h, st)
        return st

    def get_params(self) -> np.ndarray:
        """FP32 parameters, shape [layers, FLOW_NPARAM]."""
        out = np.zeros((self.layers, FLOW_NPARAM), dtype=np.float32)
        n = C.c_size_t(0)
        self._check(self.lib.pimc_flow_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), out.size,
                                                  C.byref(n)))
        return out

    def set_params(self, theta):
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).reshape(-1))
        self._check(self.lib.pimc_flow_set_params(self.h, th.ctypes.data_as(C.POINTER(C.c_float)), th.size))

    def save(self, path):
        self._check(self.lib.pimc_flow_save(self.h, os.fsencode(path)))

    def load(self, path):
        self._check(self.lib.pimc_flow_load(self.h, os.fsencode(path)))

    def grad(self, seed, stream):
        """(loss, ell [batch], grad [layers, FLOW_NPARAM] FP32) of one batch, no update."""
        loss = C.c_double(0)
        ell = np.zeros(self.batch, dtype=np.float64)
        g = np.zeros((self.layers, FLOW_NPARAM), dtype=np.float32)
        self._check(self.lib.pimc_flow_grad(self.h, seed, stream, C.byref(loss), _dptr(ell),
                                            g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, ell, g

    def train(self, seed, stream_base, steps):
        """(losses [steps], device ms)."""
        losses = np.zeros(int(steps), dtype=np.float64)
        ms = C.c_double(0)
        self._check(self.lib.pimc_flow_train(self.h, seed, stream_base, int(steps), _dptr(losses), C.byref(ms)))
        return losses, ms.value

    def log_weights(self, seed, stream, first_path, k_paths, want_z=False):
        """(ell [k], logdet [k], z [k, N-1] or None)."""
        ell = np.zeros(k_paths, dtype=np.float64)
        ld = np.zeros(k_paths, dtype=np.float64)
        z = np.zeros((k_paths, self.D), dtype=np.float64) if want_z else None
        self._check(self.lib.pimc_flow_log_weights(self.h, seed, stream, first_path, k_paths, _dptr(ell), _dptr(z),
                                                   _dptr(ld)))
        return ell, ld, z

    def amplitude(self, n_samples, seed, stream):
        """(LevelResult of level s, device ms, status)."""
        r = _LevelResult()
        ms = C.c_double(0)
        st = self._check(self.lib.pimc_flow_amplitude(self.h, n_samples, seed, stream, C.byref(r), C.byref(ms)))
        return LevelResult(r.amp, r.err, r.log_amp, r.relvar, r.ess, int(r.n), int(r.n_nonfinite)), ms.value, st

    def close(self):
        if getattr(self, "h", None):
            self.lib.pimc_flow_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
