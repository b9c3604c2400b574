"""ctypes binding of libsfpath.so: the C ABI of include/sfpath.h, same names.

Argument marshalling only: every step of the path sum runs in the library's
HIP kernels.  Importing this module loads the library and raises if it has
not been built (``python -m paper_1807_10749_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfpath.so")

SF_OK, SF_ERR_INVALID, SF_ERR_OOM, SF_ERR_UNSUPPORTED, SF_ERR_NO_CUT, SF_ERR_DEVICE = 0, -1, -2, -3, -4, -5
SF_ACCUMULATE, SF_OUT_ON_DEVICE, SF_FP64_SWEEPS, SF_PLAIN, SF_BITS_ON_DEVICE, SF_TIMING = 1, 2, 4, 8, 16, 32
SF_SAMPLE_BASIC = 256

EXPORTS = ["create_circuit", "destroy_circuit", "set_cut", "choose_cut", "num_paths", "sample_paths",
           "run_paths", "workspace_size", "set_tuning", "get_tuning", "autotune", "get_run_stats",
           "describe_plan", "last_error", "server_create", "server_submit", "server_poll", "server_release",
           "server_drain", "server_stats", "server_destroy", "server_last_error", "rejection_m",
           "sample_bitstrings", "rejection_workspace_size", "rejection_accept", "frugal_sample",
           "fidelity_estimate", "xeb_fidelity", "verify_claim", "save_tuning_cache", "load_tuning_cache",
           "server_set_policy", "run_paths_noalloc", "read_bandwidth", "compile_segment_kernels"]
SF_PENDING = 1
SF_SERVE_OLDEST_FIRST, SF_SERVE_ROUND_ROBIN, SF_SERVE_LEAST_WORK = 0, 1, 2


class SFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sfpath error {code}: {msg}")
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [("reg_qubits", ctypes.c_uint32), ("leaf_batch", ctypes.c_uint32),
                ("max_slots", ctypes.c_uint32), ("waves_per_cu", ctypes.c_uint32),
                ("dense_qubits", ctypes.c_uint32), ("no_leaf_fold", ctypes.c_uint32),
                ("fold_levels", ctypes.c_uint32), ("chain_passes", ctypes.c_uint32),
                ("no_row_skip", ctypes.c_uint32), ("no_defer", ctypes.c_uint32),
                ("no_chain_merge", ctypes.c_uint32), ("jit", ctypes.c_uint32), ("no_tail_move", ctypes.c_uint32)]


class RunStats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_sweep", ctypes.c_double),
                ("ms_gather", ctypes.c_double), ("ms_other", ctypes.c_double),
                ("n_sweep_launches", ctypes.c_uint64), ("n_gather_launches", ctypes.c_uint64),
                ("sweep_bytes", ctypes.c_uint64), ("gather_bytes", ctypes.c_uint64),
                ("n_batches", ctypes.c_uint64), ("n_passes_a", ctypes.c_uint64),
                ("n_passes_b", ctypes.c_uint64), ("gather_row_bytes", ctypes.c_uint64),
                ("a_groups", ctypes.c_uint64), ("ms_plan", ctypes.c_double),
                ("n_paths_live", ctypes.c_uint64), ("n_chained_passes", ctypes.c_uint64),
                ("gather_ws_bytes", ctypes.c_uint64), ("row_mask_frac", ctypes.c_double * 2),
                ("n_jit_passes", ctypes.c_uint64), ("jit_compile_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: (list(getattr(self, name)) if name == "row_mask_frac" else getattr(self, name))
                for name, _ in self._fields_}


class Job(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int), ("cols", ctypes.c_int), ("gates", ctypes.c_void_p),
                ("n_gates", ctypes.c_size_t), ("block_a_mask", ctypes.c_uint64), ("bitstrings", ctypes.c_void_p),
                ("n_bits", ctypes.c_size_t), ("f", ctypes.c_double), ("path_seed", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


class JobInfo(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("n_paths", ctypes.c_uint64), ("k", ctypes.c_uint32), ("chunks", ctypes.c_uint32),
                ("status", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64), ("in_use_bytes", ctypes.c_uint64),
                ("chunks", ctypes.c_uint64), ("max_concurrent_chunks", ctypes.c_uint32),
                ("waiting", ctypes.c_uint32), ("active", ctypes.c_uint32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1807_10749_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t
    pu64 = ctypes.POINTER(ctypes.c_uint64)
    lib.create_circuit.argtypes = [ctypes.c_int, ctypes.c_int, vp, sz, ctypes.POINTER(vp)]
    lib.destroy_circuit.argtypes = [vp]
    lib.set_cut.argtypes = [vp, u64, ctypes.POINTER(u32)]
    lib.choose_cut.argtypes = [vp, pu64]
    lib.num_paths.argtypes = [u32, ctypes.c_double, pu64]
    lib.sample_paths.argtypes = [u32, ctypes.c_double, u64, vp, u64, pu64]
    lib.run_paths.argtypes = [vp, vp, u64, u64, vp, sz, vp, u32, vp, vp, sz]
    lib.run_paths_noalloc.argtypes = [vp, vp, u64, u64, vp, sz, vp, u32, vp]
    lib.workspace_size.argtypes = [vp, u64, sz, u32, ctypes.POINTER(sz)]
    lib.set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.save_tuning_cache.argtypes = [ctypes.c_char_p]
    lib.load_tuning_cache.argtypes = [ctypes.c_char_p, ctypes.POINTER(u32)]
    lib.get_run_stats.argtypes = [vp, ctypes.POINTER(RunStats)]
    lib.describe_plan.argtypes = [vp, ctypes.c_char_p, sz]
    lib.autotune.argtypes = [vp, vp, u64, u64, vp, sz, vp, u32, vp, vp, sz, u32, ctypes.POINTER(Tuning)]
    lib.server_create.argtypes = [sz, vp, u32, u64, ctypes.POINTER(vp)]
    lib.server_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]
    lib.server_poll.argtypes = [vp, u64, vp, ctypes.POINTER(JobInfo)]
    lib.server_release.argtypes = [vp, u64]
    lib.server_drain.argtypes = [vp]
    lib.server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.server_destroy.argtypes = [vp]
    lib.server_set_policy.argtypes = [vp, u32]
    lib.rejection_m.argtypes = [u32, ctypes.c_double, u32, ctypes.POINTER(ctypes.c_double)]
    lib.sample_bitstrings.argtypes = [u32, u64, u64, vp]
    lib.rejection_workspace_size.argtypes = [u64, ctypes.POINTER(sz)]
    lib.rejection_accept.argtypes = [vp, u64, u32, ctypes.c_double, u64, u32, vp, pu64,
                                     ctypes.POINTER(ctypes.c_double), vp, vp, sz]
    lib.frugal_sample.argtypes = [vp, vp, u64, u64, u64, ctypes.c_double, u64, u64, u32, vp, vp, sz, vp, pu64,
                                  ctypes.POINTER(ctypes.c_double)]
    pd = ctypes.POINTER(ctypes.c_double)
    lib.fidelity_estimate.argtypes = [vp, vp, u64, vp, pd, pd, pd]
    lib.xeb_fidelity.argtypes = [vp, u64, u32, vp, pd]
    lib.read_bandwidth.argtypes = [vp, sz, u32, u32, vp, pd]
    lib.compile_segment_kernels.argtypes = [vp, ctypes.c_int, u32, u32, u32, u32, u32, ctypes.POINTER(u32),
                                            ctypes.POINTER(u64)]
    lib.verify_claim.argtypes = [vp, vp, u64, u64, ctypes.c_double, u64, ctypes.c_double, u32, vp, vp, sz, pd,
                                 ctypes.POINTER(ctypes.c_int)]
    lib.server_last_error.restype = ctypes.c_char_p
    lib.last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("last_error", "server_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def last_error() -> str:
    return lib.last_error().decode()


def _check(rc: int):
    if rc != SF_OK:
        raise SFError(rc, last_error())


def _ptr(x) -> Optional[int]:
    """Address of a numpy array or torch tensor (None stays None)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


# ---------------------------------------------------------------- C ABI, same names

def create_circuit(rows: int, cols: int, gates: np.ndarray) -> int:
    g = np.ascontiguousarray(gates)
    if g.dtype.itemsize != 8:
        raise ValueError("gate records must be 8 bytes")
    out = ctypes.c_void_p()
    _check(lib.create_circuit(rows, cols, g.ctypes.data if g.size else None, g.size, ctypes.byref(out)))
    return out.value


def destroy_circuit(c: int):
    _check(lib.destroy_circuit(c))


def set_cut(c: int, block_a_mask: int) -> int:
    k = ctypes.c_uint32()
    _check(lib.set_cut(c, block_a_mask, ctypes.byref(k)))
    return k.value


def choose_cut(c: int) -> int:
    m = ctypes.c_uint64()
    _check(lib.choose_cut(c, ctypes.byref(m)))
    return m.value


def num_paths(k: int, f: float) -> int:
    n = ctypes.c_uint64()
    _check(lib.num_paths(k, f, ctypes.byref(n)))
    return n.value


def sample_paths(k: int, f: float, seed: int) -> np.ndarray:
    m = num_paths(k, f)
    out = np.empty(m, dtype=np.uint64)
    n = ctypes.c_uint64()
    _check(lib.sample_paths(k, f, seed, out.ctypes.data, m, ctypes.byref(n)))
    return out[: n.value]


def rejection_m(n_qubits: int, eps: float, flags: int = 0) -> float:
    m = ctypes.c_double()
    _check(lib.rejection_m(n_qubits, eps, flags, ctypes.byref(m)))
    return m.value


def sample_bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _check(lib.sample_bitstrings(n_qubits, count, seed, out.ctypes.data))
    return out


def rejection_workspace_size(n: int) -> int:
    b = ctypes.c_size_t()
    _check(lib.rejection_workspace_size(n, ctypes.byref(b)))
    return b.value


def rejection_accept(amps, n: int, n_qubits: int, m: float, seed: int, accepted, flags: int = 0, stream=None,
                     workspace=None, workspace_bytes: int = 0):
    """Raw call (device buffers as torch tensors or addresses); returns (n_accepted, err_est)."""
    na = ctypes.c_uint64()
    err = ctypes.c_double()
    _check(lib.rejection_accept(_ptr(amps), n, n_qubits, m, seed, flags, _ptr(accepted), ctypes.byref(na),
                                ctypes.byref(err), _stream_handle(stream), _ptr(workspace), workspace_bytes))
    return na.value, err.value


def frugal_sample(c: int, path_ids, path_begin: int, n_paths: int, n_candidates: int, m: float,
                  seed_candidates: int, seed_accept: int, flags: int = 0, stream=None, workspace=None,
                  workspace_bytes: int = 0):
    """Returns (accepted bitstrings as uint64 array, error estimate)."""
    ids = None
    if path_ids is not None:
        ids = np.ascontiguousarray(path_ids, dtype=np.uint64)
        n_paths = ids.size
    out = np.empty(max(n_candidates, 1), dtype=np.uint64)
    n = ctypes.c_uint64()
    err = ctypes.c_double()
    _check(lib.frugal_sample(c, _ptr(ids), path_begin, n_paths, n_candidates, m, seed_candidates, seed_accept, flags,
                             _stream_handle(stream), _ptr(workspace), workspace_bytes, out.ctypes.data,
                             ctypes.byref(n), ctypes.byref(err)))
    return out[: n.value], err.value


def fidelity_estimate(a, b, n: int, stream=None):
    """Device arrays; returns (f_e, sum |a|^2, sum |b|^2)."""
    f, na, nb = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib.fidelity_estimate(_ptr(a), _ptr(b), n, _stream_handle(stream), ctypes.byref(f), ctypes.byref(na),
                                 ctypes.byref(nb)))
    return f.value, na.value, nb.value


def xeb_fidelity(amps, n: int, n_qubits: int, stream=None) -> float:
    f = ctypes.c_double()
    _check(lib.xeb_fidelity(_ptr(amps), n, n_qubits, _stream_handle(stream), ctypes.byref(f)))
    return f.value


def read_bandwidth(buf, nbytes: int, reps: int, grid: int = 0, stream=None) -> float:
    """Milliseconds of one launch reading the first nbytes of device buffer buf reps times."""
    ms = ctypes.c_double()
    _check(lib.read_bandwidth(_ptr(buf), nbytes, reps, grid, _stream_handle(stream), ctypes.byref(ms)))
    return ms.value


def verify_claim(c: int, claimed, index_seed: int, f1: float, path_seed: int, delta: float, flags: int = 0,
                 stream=None, workspace=None, workspace_bytes: int = 0):
    """claimed: host complex128 array of the Claimant's amplitudes; returns (f_e, passed)."""
    a = np.ascontiguousarray(claimed, dtype=np.complex128)
    f, ok = ctypes.c_double(), ctypes.c_int()
    _check(lib.verify_claim(c, a.ctypes.data, a.size, index_seed, f1, path_seed, delta, flags, _stream_handle(stream),
                            _ptr(workspace), workspace_bytes, ctypes.byref(f), ctypes.byref(ok)))
    return f.value, bool(ok.value)


def run_paths(c: int, path_ids, path_begin: int, n_paths: int, bitstrings, n_bits: int, amps,
              flags: int = 0, stream=None, workspace=None, workspace_bytes: int = 0):
    """Raw call; bitstrings/amps/workspace are numpy arrays, torch tensors or addresses."""
    ids = None
    if path_ids is not None:
        ids = np.ascontiguousarray(path_ids, dtype=np.uint64)
        n_paths = ids.size
    _check(lib.run_paths(c, _ptr(ids), path_begin, n_paths, _ptr(bitstrings), n_bits, _ptr(amps), flags,
                         _stream_handle(stream), _ptr(workspace), workspace_bytes))


def run_paths_noalloc(c: int, path_ids, path_begin: int, n_paths: int, bitstrings, n_bits: int, amps,
                      flags: int = 0, stream=None):
    """Raw call of the entry point without device allocations (device bitstrings and amps)."""
    ids = None
    if path_ids is not None:
        ids = np.ascontiguousarray(path_ids, dtype=np.uint64)
        n_paths = ids.size
    _check(lib.run_paths_noalloc(c, _ptr(ids), path_begin, n_paths, _ptr(bitstrings), n_bits, _ptr(amps), flags,
                                 _stream_handle(stream)))


def workspace_size(c: int, n_paths: int, n_bits: int, flags: int = 0) -> int:
    b = ctypes.c_size_t()
    _check(lib.workspace_size(c, n_paths, n_bits, flags, ctypes.byref(b)))
    return b.value


def set_tuning(c: int, reg_qubits=0, leaf_batch=0, max_slots=0, waves_per_cu=0, dense_qubits=0, no_leaf_fold=0,
               fold_levels=0, chain_passes=0, no_row_skip=0, no_defer=0, no_chain_merge=0, jit=0, no_tail_move=0):
    t = Tuning(reg_qubits, leaf_batch, max_slots, waves_per_cu, dense_qubits, no_leaf_fold, fold_levels, chain_passes,
               no_row_skip, no_defer, no_chain_merge, jit, no_tail_move)
    _check(lib.set_tuning(c, ctypes.byref(t)))


def get_tuning(c: int) -> dict:
    t = Tuning()
    _check(lib.get_tuning(c, ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in Tuning._fields_}


def autotune(c: int, path_ids, path_begin: int, n_paths: int, bitstrings, n_bits: int, amps, flags: int = 0,
             stream=None, workspace=None, workspace_bytes: int = 0, n_measure: int = 6) -> dict:
    ids = None
    if path_ids is not None:
        ids = np.ascontiguousarray(path_ids, dtype=np.uint64)
        n_paths = ids.size
    t = Tuning()
    _check(lib.autotune(c, _ptr(ids), path_begin, n_paths, _ptr(bitstrings), n_bits, _ptr(amps), flags,
                        _stream_handle(stream), _ptr(workspace), workspace_bytes, n_measure, ctypes.byref(t)))
    return {name: getattr(t, name) for name, _ in Tuning._fields_}


def save_tuning_cache(path: str) -> None:
    _check(lib.save_tuning_cache(str(path).encode()))


def load_tuning_cache(path: str) -> int:
    n = ctypes.c_uint32(0)
    _check(lib.load_tuning_cache(str(path).encode(), ctypes.byref(n)))
    return n.value


def get_run_stats(c: int) -> dict:
    s = RunStats()
    _check(lib.get_run_stats(c, ctypes.byref(s)))
    return s.as_dict()


def compile_segment_kernels(c: int, half: int, first_level: int, last_level: int, slot_bits: int, reg_qubits: int,
                            fp64: bool = False) -> tuple:
    """(kernels, code-object bytes) of the compiled passes of one segment plan (host only)."""
    n = ctypes.c_uint32()
    nb = ctypes.c_uint64()
    _check(lib.compile_segment_kernels(c, half, first_level, last_level, slot_bits, reg_qubits, int(bool(fp64)),
                                       ctypes.byref(n), ctypes.byref(nb)))
    return n.value, nb.value


def describe_plan(c: int) -> str:
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib.describe_plan(c, buf, len(buf)))
    return buf.value.decode()


def server_last_error() -> str:
    return lib.server_last_error().decode()


def _scheck(rc: int):
    if rc not in (SF_OK, SF_PENDING):
        raise SFError(rc, server_last_error())
    return rc


def server_create(arena_bytes: int, arena=None, n_workers: int = 4, chunk_paths: int = 0) -> int:
    out = ctypes.c_void_p()
    _scheck(lib.server_create(arena_bytes, _ptr(arena), n_workers, chunk_paths, ctypes.byref(out)))
    return out.value


def server_submit(s: int, rows: int, cols: int, gates: np.ndarray, bitstrings: np.ndarray, f: float = 1.0,
                  path_seed: int = 0, block_a_mask: int = 0, flags: int = 0) -> int:
    g = np.ascontiguousarray(gates)
    b = np.ascontiguousarray(bitstrings, dtype=np.uint64)
    job = Job(rows, cols, g.ctypes.data, g.size, block_a_mask, b.ctypes.data if b.size else None, b.size, f,
              path_seed, flags)
    jid = ctypes.c_uint64()
    _scheck(lib.server_submit(s, ctypes.byref(job), ctypes.byref(jid)))
    return jid.value


def server_poll(s: int, job_id: int, n_bits: Optional[int] = None):
    """(done, amplitudes or None, info dict)."""
    info = JobInfo()
    amps = np.zeros(2 * max(n_bits or 0, 1)) if n_bits is not None else None
    rc = _scheck(lib.server_poll(s, job_id, _ptr(amps), ctypes.byref(info)))
    d = {name: getattr(info, name) for name, _ in JobInfo._fields_}
    if rc == SF_PENDING:
        return False, None, d
    return True, (amps.view(np.complex128)[: n_bits] if amps is not None else None), d


def server_release(s: int, job_id: int):
    _scheck(lib.server_release(s, job_id))


def server_drain(s: int):
    _scheck(lib.server_drain(s))


def server_stats(s: int) -> dict:
    st = ServerStats()
    _scheck(lib.server_stats(s, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in ServerStats._fields_}


def server_destroy(s: int):
    _scheck(lib.server_destroy(s))


def server_set_policy(s: int, policy: int):
    _scheck(lib.server_set_policy(s, policy))


# ---------------------------------------------------------------- convenience wrapper

class Circuit:
    """Owns one library circuit; marshals numpy inputs to run_paths."""

    def __init__(self, rows: int, cols: int, gates: np.ndarray, block_a_mask: Optional[int] = None):
        self.rows, self.cols, self.n = rows, cols, rows * cols
        self.handle = create_circuit(rows, cols, gates)
        if block_a_mask is None:
            block_a_mask = choose_cut(self.handle)
        self.mask_a = block_a_mask
        self.k = set_cut(self.handle, block_a_mask)

    def close(self):
        if self.handle:
            destroy_circuit(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def amplitudes(self, bitstrings: np.ndarray, path_ids=None, path_begin: int = 0,
                   n_paths: Optional[int] = None, flags: int = 0, stream=None, workspace=None) -> np.ndarray:
        """complex128 array: sum over the paths of psiA_p(x_A) psiB_p(x_B) per bitstring (host arrays)."""
        bits = np.ascontiguousarray(bitstrings, dtype=np.uint64)
        amps = np.zeros(2 * max(bits.size, 1), dtype=np.float64)
        if path_ids is None and n_paths is None:
            n_paths = 1 << self.k
        ws_bytes = 0
        if workspace is not None:
            ws_bytes = workspace.numel() * workspace.element_size() if hasattr(workspace, "numel") else workspace.nbytes
        run_paths(self.handle, path_ids, path_begin, n_paths or 0, bits, bits.size, amps, flags, stream,
                  workspace, ws_bytes)
        return amps.view(np.complex128)[: bits.size]

    def tune(self, **kw):
        set_tuning(self.handle, **kw)

    def stats(self) -> dict:
        return get_run_stats(self.handle)
