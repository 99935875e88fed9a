"""CPU oracle for the IBIP hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, single-threaded C (``ibip_oracle.c``) behind ctypes, with numpy
arrays in and out. The same source built with OpenMP (``build_openmp``; the
distance transform's lines and the x-planes of large spheres split over the
host's threads, nothing else changed) is the benchmark's data-parallel CPU
baseline, loaded in a child process through ``IBIP_ORACLE_LIB``. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does, and the
two share no code.

Each wrapper follows the paper (Gostick, Yang & Boek, arXiv 2101.03240):
  edt / edt_brute / edt_at   distance transform of the pore space, Section 2.1
  invade / invade(literal)   the invasion loop, Section 2.1, Figure 2(e)-(l)
  steps                      saturation and Washburn Pc per step, 2.2.1-2.2.2
  trap / trap_brute / rerank defender trapping and re-ranking, Section 2.2.3
  mio / mio_kept             morphological image opening drainage, 2.4.1
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibip_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libibip_oracle.so")
_lib = None

OK, EINVAL, ENOMEM, ENOSOLID, ECAPACITY = 0, -1, -2, -3, -5


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libibip_oracle.so``."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"],
                   check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path: str) -> str:
    """Compile the same source with AddressSanitizer and UndefinedBehaviour-
    Sanitizer into `path` (loaded through IBIP_ORACLE_LIB with libasan
    preloaded; used by the tests only)."""
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", path, _SRC, "-lm"],
                   check=True)
    return path


OPENMP_LIB = os.path.join(_HERE, "libibip_oracle_omp.so")


def build_openmp(path: str = OPENMP_LIB) -> str:
    """Compile the same source with OpenMP into `path`."""
    tmp = path + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-fopenmp", "-o", tmp, _SRC, "-lm"],
                   check=True)
    os.replace(tmp, path)
    return path


def threads() -> int:
    """Threads the loaded build uses (1 unless it is the OpenMP build)."""
    return int(_load().ibipref_threads())


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("IBIP_ORACLE_LIB") or _LIB_PATH
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.ibipref_threads.argtypes = []
    lib.ibipref_threads.restype = i32
    lib.ibipref_edt_brute.argtypes = [P, i32, i32, i32, P]
    lib.ibipref_edt_brute.restype = i32
    lib.ibipref_edt.argtypes = [P, i32, i32, i32, P]
    lib.ibipref_edt.restype = i32
    lib.ibipref_edt_at.argtypes = [P, i32, i32, i32, i32, i32, i32]
    lib.ibipref_edt_at.restype = i64
    for fn in (lib.ibipref_invade_literal, lib.ibipref_invade):
        fn.argtypes = [P, P, i32, i32, i32, i64, P, P, P, P, i64]
        fn.restype = i64
    for fn in (lib.ibipref_invade_literal_v, lib.ibipref_invade_v):
        fn.argtypes = [P, P, i32, i32, i32, i64, i32, P, P, P, P, i64]
        fn.restype = i64
    lib.ibipref_trap_c.argtypes = [P, P, i32, i32, i32, i32, P, P, P]
    lib.ibipref_trap_c.restype = i32
    lib.ibipref_trap_brute_c.argtypes = [P, P, i32, i32, i32, i32, P]
    lib.ibipref_trap_brute_c.restype = i32
    lib.ibipref_mio_v.argtypes = [P, P, i32, i32, i32, P, i32, i32, i32, P, P]
    lib.ibipref_mio_v.restype = i32
    lib.ibipref_mio_kept_v.argtypes = [P, P, P, i32, i32, i32, ctypes.c_uint32, i32, P]
    lib.ibipref_mio_kept_v.restype = i64
    lib.ibipref_steps.argtypes = [P, i64, i64, P, d, P, P, P]
    lib.ibipref_steps.restype = i32
    lib.ibipref_satmap.argtypes = [P, i64, i64, P, P]
    lib.ibipref_satmap.restype = i32
    lib.ibipref_remap_steps.argtypes = [P, P, i64, P, i64, i64, P]
    lib.ibipref_remap_steps.restype = i32
    lib.ibipref_trap.argtypes = [P, P, i32, i32, i32, P, P, P]
    lib.ibipref_trap.restype = i32
    lib.ibipref_trap_brute.argtypes = [P, P, i32, i32, i32, P]
    lib.ibipref_trap_brute.restype = i32
    lib.ibipref_rerank.argtypes = [P, P, i64, P, P]
    lib.ibipref_rerank.restype = i32
    lib.ibipref_mio.argtypes = [P, P, i32, i32, i32, P, i32, i32, P, P]
    lib.ibipref_mio.restype = i32
    lib.ibipref_mio_kept.argtypes = [P, P, P, i32, i32, i32, ctypes.c_uint32, P]
    lib.ibipref_mio_kept.restype = i64
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def _dims(a: np.ndarray):
    if a.ndim == 2:
        return (1,) + tuple(a.shape)
    if a.ndim != 3:
        raise ValueError("expected a 2D or 3D array")
    return tuple(a.shape)


def _check(code, what):
    if code < 0:
        raise OracleError(int(code), what)
    return code


def washburn_c0(sigma: float = 1.0, theta_rad: float = 0.0, voxel_size: float = 1.0) -> float:
    """Pc = c0 / r with c0 = 2 sigma cos(theta) / voxel_size (Section 2.2.2)."""
    return 2.0 * sigma * math.cos(theta_rad) / voxel_size


def edt(img) -> np.ndarray:
    img = _u8(img)
    X, Y, Z = _dims(img)
    out = np.empty(img.shape, dtype=np.uint32)
    _check(_load().ibipref_edt(_p(img), X, Y, Z, _p(out)), "edt")
    return out


def edt_brute(img) -> np.ndarray:
    img = _u8(img)
    X, Y, Z = _dims(img)
    out = np.empty(img.shape, dtype=np.uint32)
    _check(_load().ibipref_edt_brute(_p(img), X, Y, Z, _p(out)), "edt_brute")
    return out


def edt_at(img, x: int, y: int, z: int) -> int:
    img = _u8(img)
    X, Y, Z = _dims(img)
    return int(_load().ibipref_edt_at(_p(img), X, Y, Z, int(x), int(y), int(z)))


INTEGER_BALL = 1  # footnote 1's integer sphere rule (variant)
MASK_INLETS = 2   # solid inlet voxels contribute no neighbours to the seeds (variant)


def _flags(integer_ball: bool, mask_inlets: bool) -> int:
    return (INTEGER_BALL if integer_ball else 0) | (MASK_INLETS if mask_inlets else 0)


def invade(img, inlets, max_steps: int = 0, literal: bool = False, integer_ball: bool = False,
           mask_inlets: bool = False, paint: bool = True) -> dict:
    """Returns dict(seq int32, rad2 uint32, centre_step int32, M uint32[K], K).
    integer_ball / mask_inlets select the variant readings of the sphere rule
    and of the seeds. paint=False runs the selection alone (the candidate-set
    loop; seq and rad2 are None): sphere insertion never feeds back into which
    voxels are centres (Section 2.1), so centre_step and M are the same."""
    img = _u8(img)
    inl = _u8(inlets)
    if inl.shape != img.shape:
        raise ValueError("inlets shape")
    X, Y, Z = _dims(img)
    N = img.size
    if not paint and literal:
        raise ValueError("the literal loop always paints")
    seq = np.empty(img.shape, dtype=np.int32) if paint else None
    rad2 = np.empty(img.shape, dtype=np.uint32) if paint else None
    cs = np.empty(img.shape, dtype=np.int32)
    cap = int(N) + 1
    M = np.zeros(cap, dtype=np.uint32)
    fn = _load().ibipref_invade_literal_v if literal else _load().ibipref_invade_v
    K = _check(fn(_p(img), _p(inl), X, Y, Z, int(max_steps), _flags(integer_ball, mask_inlets),
                  _p(seq) if paint else None, _p(rad2) if paint else None, _p(cs), _p(M), cap), "invade")
    return {"seq": seq, "rad2": rad2, "centre_step": cs, "M": M[:K].copy(), "K": int(K)}


def steps(seq, M, c0: float = 2.0) -> dict:
    seq = np.ascontiguousarray(seq, dtype=np.int32)
    M = np.ascontiguousarray(M, dtype=np.uint32)
    K = M.shape[0]
    n_new = np.zeros(K, dtype=np.int64)
    sat = np.zeros(K, dtype=np.float64)
    pc = np.zeros(K, dtype=np.float64)
    _check(_load().ibipref_steps(_p(seq), seq.size, K, _p(M), float(c0), _p(n_new), _p(sat), _p(pc)),
           "steps")
    return {"n_new": n_new, "sat": sat, "pc": pc}


def satmap(seq, sat) -> np.ndarray:
    """Saturation map: sat[seq-1] on invaded voxels, 0 on uninvaded pore, -1
    on solid (Section 2.2.1, Figure 5 left)."""
    seq = np.ascontiguousarray(seq, dtype=np.int32)
    sat = np.ascontiguousarray(sat, dtype=np.float64)
    out = np.empty(seq.shape, dtype=np.float64)
    _check(_load().ibipref_satmap(_p(seq), seq.size, sat.shape[0], _p(sat), _p(out)), "satmap")
    return out


def remap_steps(seq, seq_after, M, K_after: int) -> np.ndarray:
    """Squared radius of each re-ranked step after trapping (Section 2.2.3)."""
    seq = np.ascontiguousarray(seq, dtype=np.int32)
    sa = np.ascontiguousarray(seq_after, dtype=np.int32)
    M = np.ascontiguousarray(M, dtype=np.uint32)
    out = np.empty(int(K_after), dtype=np.uint32)
    _check(_load().ibipref_remap_steps(_p(seq), _p(sa), seq.size, _p(M), M.shape[0], int(K_after), _p(out)),
           "remap_steps")
    return out


def compare_opening(satmap, mio_r2, T, sat_T, trapped=None) -> dict:
    """Equal-saturation comparison of IBIP and the opening (Section 3.1.1,
    Figures 8 and 9), level by level from the definition: at level i the IBIP
    configuration is {0 < satmap <= sat_T[i]} and the opening's is
    {mio_r2 >= T[i]}; ``disagree[i]`` = pixels in exactly one of them,
    ``mio_trapped[i]`` = pixels the opening holds that IBIP leaves trapped."""
    satmap = np.asarray(satmap, dtype=np.float64)
    r2 = np.asarray(mio_r2).astype(np.uint32)
    dis = np.zeros(len(T), dtype=np.int64)
    mt = np.zeros(len(T), dtype=np.int64)
    for i, (t, s) in enumerate(zip(T, sat_T)):
        a = (satmap > 0) & (satmap <= s)
        b = r2 >= np.uint32(t)
        dis[i] = int(np.count_nonzero(a ^ b))
        if trapped is not None:
            mt[i] = int(np.count_nonzero(b & (np.asarray(trapped) != 0)))
    return {"disagree": dis, "mio_trapped": mt}


def trap(seq, outlets, conn: int = 6) -> dict:
    """Trapping with 6- (faces) or 26-connectivity (faces, edges, corners)."""
    seq = np.ascontiguousarray(seq, dtype=np.int32)
    out = _u8(outlets)
    X, Y, Z = _dims(seq)
    trapped = np.empty(seq.shape, dtype=np.uint8)
    st = np.empty(seq.shape, dtype=np.int32)
    ka = ctypes.c_int64(0)
    _check(_load().ibipref_trap_c(_p(seq), _p(out), X, Y, Z, int(conn), _p(trapped), _p(st), ctypes.byref(ka)),
           "trap")
    return {"trapped": trapped, "seq_trapped": st, "K_after": int(ka.value)}


def trap_brute(seq, outlets, conn: int = 6) -> np.ndarray:
    seq = np.ascontiguousarray(seq, dtype=np.int32)
    out = _u8(outlets)
    X, Y, Z = _dims(seq)
    trapped = np.empty(seq.shape, dtype=np.uint8)
    _check(_load().ibipref_trap_brute_c(_p(seq), _p(out), X, Y, Z, int(conn), _p(trapped)), "trap_brute")
    return trapped


def rerank(seq, trapped) -> tuple[np.ndarray, int]:
    seq = np.ascontiguousarray(seq, dtype=np.int32)
    tr = _u8(trapped)
    st = np.empty(seq.shape, dtype=np.int32)
    ka = ctypes.c_int64(0)
    _check(_load().ibipref_rerank(_p(seq), _p(tr), seq.size, _p(st), ctypes.byref(ka)), "rerank")
    return st, int(ka.value)


def mio(img, inlets, thresholds, brute_erosion: bool = False, mask_inlets: bool = False) -> dict:
    img = _u8(img)
    inl = _u8(inlets)
    X, Y, Z = _dims(img)
    T = np.ascontiguousarray(thresholds, dtype=np.uint32)
    r2 = np.empty(img.shape, dtype=np.uint32)
    sat = np.zeros(T.shape[0], dtype=np.float64)
    _check(_load().ibipref_mio_v(_p(img), _p(inl), X, Y, Z, _p(T), int(T.shape[0]), int(brute_erosion),
                                 _flags(False, mask_inlets), _p(r2), _p(sat)), "mio")
    return {"mio_r2": r2, "mio_sat": sat}


def mio_kept(img, inlets, dt2, T: int, mask_inlets: bool = False) -> np.ndarray:
    img = _u8(img)
    inl = _u8(inlets)
    d = np.ascontiguousarray(dt2, dtype=np.uint32)
    X, Y, Z = _dims(img)
    kept = np.empty(img.shape, dtype=np.uint8)
    _check(_load().ibipref_mio_kept_v(_p(img), _p(inl), _p(d), X, Y, Z, int(T), _flags(False, mask_inlets),
                                      _p(kept)), "mio_kept")
    return kept.astype(bool)
