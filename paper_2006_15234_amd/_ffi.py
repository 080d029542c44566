"""ctypes declarations of the C ABI in include/hpeps.h."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))

F64, C128, F32, BF16 = 0, 1, 2, 3
ABSORB_CARRY, ABSORB_RIGHT, ABSORB_NONE, ABSORB_LEFT, ABSORB_SQRT = 0, 1, 2, 3, 4
L2R, R2L = 0, 1

_STATUS = {0: "ok", 1: "invalid argument", 2: "shape mismatch", 3: "unsupported dtype",
           4: "allocation failed", 5: "HIP runtime error", 6: "non-finite values",
           7: "not converged", 8: "unsupported size"}


class HpepsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hpeps error {code} ({_STATUS.get(code, '?')}): {msg}")
        self.code = code


class EsvdOpts(C.Structure):
    _fields_ = [("rank", C.c_int64), ("oversample", C.c_int64), ("power_iters", C.c_int32),
                ("sketch_precision", C.c_int32), ("seed", C.c_uint64), ("stream_id", C.c_uint64),
                ("jacobi_max_sweeps", C.c_int32), ("orth", C.c_int32), ("method", C.c_int32), ("reserved", C.c_int32)]


class EsvdInfo(C.Structure):
    _fields_ = [("rank_kept", C.c_int64), ("sketch_width", C.c_int64),
                ("orth_extra_passes", C.c_int32), ("jacobi_sweeps", C.c_int32),
                ("numeric_errors", C.c_int32), ("not_converged", C.c_int32),
                ("orth_householder", C.c_int32), ("reserved", C.c_int32)]


class Peps(C.Structure):
    _fields_ = [("nrow", C.c_int32), ("ncol", C.c_int32), ("dtype", C.c_int32),
                ("reserved", C.c_int32), ("sites", C.POINTER(C.c_void_p)),
                ("shapes", C.POINTER(C.c_int64))]


class Tensor(C.Structure):
    _fields_ = [("data", C.c_void_p), ("ndim", C.c_int32), ("conj", C.c_int32),
                ("shape", C.c_int64 * 8), ("strides", C.c_int64 * 8)]


class Bmps(C.Structure):
    _fields_ = [("ncol", C.c_int32), ("dtype", C.c_int32), ("tensors", C.POINTER(C.c_void_p)),
                ("shapes", C.POINTER(C.c_int64)), ("capacity", C.POINTER(C.c_int64))]


def lib_path():
    return os.path.join(_HERE, "libhpeps.so")


_LIB = None

# name -> (restype, argtypes); mirrors include/hpeps.h
_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)
_SIGS = {
    "hpeps_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "hpeps_destroy": (C.c_int, [_P]),
    "hpeps_set_stream": (C.c_int, [_P, _P]),
    "hpeps_status_string": (C.c_char_p, [C.c_int]),
    "hpeps_last_error": (C.c_char_p, [_P]),
    "hpeps_set_workspace_limit": (C.c_int, [_P, C.c_int64]),
    "hpeps_workspace_peak": (C.c_int, [_P, _I64P, C.c_int32]),
    "hpeps_get_info": (C.c_int, [_P, C.POINTER(EsvdInfo)]),
    "hpeps_autotune_enable": (C.c_int, [_P, C.c_int32]),
    "hpeps_autotune_export": (C.c_int, [_P, C.c_char_p, C.c_int64, _I64P]),
    "hpeps_autotune_import": (C.c_int, [_P, C.c_char_p]),
    "hpeps_profile_start": (C.c_int, [_P, C.c_char_p]),
    "hpeps_profile_stop": (C.c_int, [_P]),
    "hpeps_profile_by_shape": (C.c_int, [_P, C.c_int32]),
    "hpeps_profile_read": (C.c_int, [_P, C.c_int32, C.c_void_p, C.POINTER(C.c_int32)]),
    "hpeps_sketch": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_uint64,
                               C.c_uint64, _P]),
    "hpeps_einsumsvd": (C.c_int, [_P, C.c_int, C.c_char_p, C.c_int32, C.POINTER(Tensor),
                                  C.POINTER(EsvdOpts), C.c_int, _P, _P, _P, _P]),
    "hpeps_einsumsvd_backward": (C.c_int, [_P, C.c_int, C.c_char_p, C.c_int32, C.POINTER(Tensor),
                                           C.POINTER(EsvdOpts), C.c_int, C.c_double, _P, _P, _P,
                                           C.POINTER(C.c_void_p)]),
    "hpeps_einsumsvd_batched": (C.c_int, [_P, C.c_int, C.c_int64, C.c_char_p, C.c_int32, C.POINTER(Tensor),
                                          C.POINTER(EsvdOpts), C.c_int, _P, _P, _P, _P]),
    "hpeps_einsumsvd_query": (C.c_int, [_P, C.c_char_p, C.c_int32, C.POINTER(Tensor),
                                        C.POINTER(EsvdOpts), _I64P, _I64P, _I64P]),
    "hpeps_einsumsvd_zipup": (C.c_int, [_P, C.c_int64, C.c_int, _I64P, _P, _P, _P, _P,
                                        C.POINTER(EsvdOpts), C.c_int, _P, _P, _P, _P]),
    "hpeps_einsumsvd_pair": (C.c_int, [_P, C.c_int64, C.c_int, _I64P, _P, _P, _P, _P,
                                       C.POINTER(EsvdOpts), C.c_int, _P, _P, _P]),
    "hpeps_einsumsvd_pair_backward": (C.c_int, [_P, C.c_int64, C.c_int, _I64P, _P, _P, _P, _P,
                                                C.POINTER(EsvdOpts), C.c_int, C.c_double, _P,
                                                _P, _P, _P, _P, _P, _P]),
    "hpeps_boundary_contract_row": (C.c_int, [_P, C.POINTER(Bmps), C.POINTER(Peps), C.POINTER(Peps),
                                              C.c_int32, C.c_int, C.POINTER(EsvdOpts),
                                              C.POINTER(Bmps), _DP]),
    "hpeps_peps_norm": (C.c_int, [_P, C.POINTER(Peps), C.POINTER(Peps), C.POINTER(EsvdOpts), _DP, _DP]),
    "hpeps_peps_amplitude": (C.c_int, [_P, C.POINTER(Peps), C.POINTER(C.c_int32), C.POINTER(EsvdOpts), _DP, _DP]),
    "hpeps_peps_amplitudes": (C.c_int, [_P, C.POINTER(Peps), C.c_int64, C.POINTER(C.c_int32), C.POINTER(EsvdOpts),
                                        _DP, _DP]),
    "hpeps_peps_energy": (C.c_int, [_P, C.POINTER(Peps), C.c_int32, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), _DP, _I64P, C.POINTER(EsvdOpts), _DP, _DP]),
    "hpeps_peps_energy_uncached": (C.c_int, [_P, C.POINTER(Peps), C.c_int32, C.POINTER(C.c_int32),
                                             C.POINTER(C.c_int32), _DP, _I64P, C.POINTER(EsvdOpts), _DP, _DP]),
    "hpeps_peps_trotter_expectation": (C.c_int, [_P, C.POINTER(Peps), C.c_int32, C.POINTER(C.c_int32), _DP,
                                                 C.c_double, C.POINTER(EsvdOpts), _DP, _DP]),
    "hpeps_peps_norm_backward": (C.c_int, [_P, C.POINTER(Peps), C.POINTER(EsvdOpts), C.c_double,
                                           C.POINTER(C.c_void_p), _DP]),
    "hpeps_peps_energy_backward": (C.c_int, [_P, C.POINTER(Peps), C.c_int32, C.POINTER(C.c_int32),
                                             C.POINTER(C.c_int32), _DP, _I64P, C.POINTER(EsvdOpts),
                                             C.c_double, C.POINTER(C.c_void_p), _DP]),
    "hpeps_apply_two_site_gate": (C.c_int, [_P, C.POINTER(Peps), _I64P, C.c_int32, C.c_int32,
                                            C.c_int32, _P, C.c_int64, _I64P, _P]),
    "hpeps_apply_two_site_gate_noalloc": (C.c_int, [_P, C.POINTER(Peps), _I64P, C.c_int32, C.c_int32,
                                            C.c_int32, _P, C.c_int64, _I64P, _P]),
    "hpeps_ite_plan_create": (C.c_int, [_P, C.POINTER(Peps), C.c_int32, _P, C.POINTER(C.c_int32),
                                        C.c_int64, C.POINTER(C.c_void_p)]),
    "hpeps_circuit_plan_create": (C.c_int, [_P, C.POINTER(Peps), C.c_int32, _DP, C.c_int32, _DP, C.c_int32,
                                            C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_void_p)]),
    "hpeps_ite_plan_layers": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "hpeps_apply_one_site_gate": (C.c_int, [_P, C.c_int, _I64P, _P, _P, _P]),
    "hpeps_ite_run": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "hpeps_ite_get_state": (C.c_int, [_P, _I64P, C.POINTER(C.c_void_p)]),
    "hpeps_ite_spectra": (C.c_int, [_P, _P]),
    "hpeps_ite_plan_destroy": (C.c_int, [_P]),
    # include/hpeps_testing.h
    "hpeps_test_gemm_variant": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32]),
    "hpeps_test_zip_order": (C.c_int, [_P, C.c_int32]),
    "hpeps_test_gemm_smallk": (C.c_int, [_P, C.c_int32]),
    "hpeps_test_gemm": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                  C.c_int32, _P, _P, _P]),
    "hpeps_test_orthogonalize": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, C.c_int64, _P, _P]),
    "hpeps_test_householder": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, C.c_int64, _P, _P, _P]),
    "hpeps_test_orthogonalize_eigh": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, C.c_int64, _P, _P, _P]),
    "hpeps_test_strip_chunk_bytes": (C.c_int, [_P, C.c_int64]),
    "hpeps_test_checkpoint_rows": (C.c_int, [_P, C.c_int32]),
    "hpeps_test_small_svd": (C.c_int, [_P, C.c_int, C.c_int64, C.c_int64, _P, _P, _P]),
    "hpeps_test_zip_apply": (C.c_int, [_P, C.c_int, C.c_int64, _I64P, _P, _P, _P, _P, C.c_int64,
                                       C.c_int32, _P, _P]),
}


def symbols():
    """Names of every entry point declared in include/hpeps.h."""
    return list(_SIGS)


def load_library(path=None):
    """Loads libhpeps.so (raises RuntimeError when it has not been built)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or lib_path()
    if not os.path.exists(p):
        raise RuntimeError(f"{p} not found: build it with `python -m paper_2006_15234_amd.build` "
                           "(there is no CPU fallback)")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _LIB = lib
    return lib


class Context:
    """Owns one hpeps_ctx on a device; calls run on torch's current stream."""

    def __init__(self, device=0):
        import torch
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        self._check(self.lib.hpeps_create(device, C.byref(h)), None)
        self.h = h
        self._torch = torch

    def _check(self, st, h=None):
        if st != 0:
            msg = self.lib.hpeps_last_error(h if h is not None else getattr(self, "h", None))
            raise HpepsError(st, (msg or b"").decode())

    def check(self, st):
        self._check(st, self.h)

    def sync_stream(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        self.check(self.lib.hpeps_set_stream(self.h, C.c_void_p(s)))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.hpeps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
