"""Python binding of libgfmc (gfx950 GFMC hot path), argument marshalling only.

Every computation runs in the HIP kernels behind the C ABI of ``include/gfmc.h``.
PyTorch provides device memory (the workspaces) and streams.  Loading fails
loudly when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfmc.so")

GFMC_OK, GFMC_EINVAL, GFMC_ENOMEM, GFMC_EDEVICE, GFMC_EBUSY, GFMC_ESTATE, GFMC_ECANCELED = (
    0, -1, -2, -3, -4, -5, -6)
FP64, FP32_ACC64 = 0, 1
JACKSON, LORENTZ = 0, 1
PROPOSE_SPHERE, PROPOSE_CONE = 0, 1
INIT_RANDOM, INIT_FM, INIT_FM_PLUS_RANDOM = 0, 1, 2
VECTORS_SITES, VECTORS_OV, VECTORS_MIXED = 0, 1, 2
HOP_RECOMPUTE, HOP_STORED = 0, 1


class GfmcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gfmc status {status}: {msg}")
        self.status = status


class ChainParams(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("t", ctypes.c_double), ("beta", ctypes.c_double),
        ("mu", ctypes.c_double), ("M", ctypes.c_int32), ("K", ctypes.c_int32),
        ("kernel", ctypes.c_int32), ("lorentz_lambda", ctypes.c_double),
        ("scale_a", ctypes.c_double), ("scale_b", ctypes.c_double),
        ("precision", ctypes.c_int32), ("proposal", ctypes.c_int32),
        ("cone_angle", ctypes.c_double), ("seed", ctypes.c_uint64), ("chain_id", ctypes.c_uint64),
        ("vectors", ctypes.c_int32), ("hoppings", ctypes.c_int32),
        ("fp32_unvalidated", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("request_id", ctypes.c_uint64), ("status", ctypes.c_int32), ("L", ctypes.c_int32),
        ("M", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("proposals", ctypes.c_int64), ("accepted", ctypes.c_int64),
        ("magnetization", ctypes.c_double), ("magnetization_mean", ctypes.c_double),
        ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
        ("t_first_sweep", ctypes.c_double), ("t_done", ctypes.c_double),
    ]


class StepRecord(ctypes.Structure):
    _fields_ = [
        ("index", ctypes.c_int64), ("site", ctypes.c_int32), ("own", ctypes.c_int32),
        ("accepted", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("theta_old", ctypes.c_double), ("phi_old", ctypes.c_double),
        ("theta_new", ctypes.c_double), ("phi_new", ctypes.c_double),
        ("dseff", ctypes.c_double), ("u", ctypes.c_double), ("phase_top", ctypes.c_double),
    ]


_P = ctypes.POINTER
_d, _i32, _i64, _sz, _vp = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
_SIGS = {
    "gfmc_workspace_bytes": [_P(ChainParams), _P(_sz)],
    "gfmc_chain_create": [_P(ChainParams), _vp, _sz, _vp, _P(_vp)],
    "gfmc_chain_destroy": [_vp],
    "gfmc_set_params": [_vp, _d, _d, _d],
    "gfmc_init_spins": [_vp, _i32, _d],
    "gfmc_set_spins": [_vp, _P(_d), _P(_d)],
    "gfmc_get_spins": [_vp, _P(_d), _P(_d)],
    "gfmc_set_counter": [_vp, _i64],
    "gfmc_get_counter": [_vp, _P(_i64)],
    "gfmc_chain_nonfinite": [_vp, _P(_i64)],
    "gfmc_chain_device_angles": [_vp, _P(_vp), _P(_vp)],
    "gfmc_moments": [_vp, _i32, _P(_d)],
    "gfmc_delta_seff": [_vp, _i32, _d, _d, _P(_d), _P(_d)],
    "gfmc_pair_moments": [_vp, _i32, _d, _d, _P(_d)],
    "gfmc_mixed_moments": [_vp, _i32, _d, _d, _P(_d)],
    "gfmc_step": [_vp, _i32, _P(StepRecord)],
    "gfmc_sweep": [_vp, _i32, _P(_d), _P(_i64)],
    "gfmc_sync": [_vp],
    "gfmc_magnetization": [_vp, _P(_d)],
    "gfmc_chain_step_bytes": [_vp, _P(_d), _P(_i32)],
    "gfmc_batch_workspace_bytes": [_P(_vp), _i32, _P(_sz)],
    "gfmc_batch_create": [_P(_vp), _i32, _vp, _sz, _vp, _P(_vp)],
    "gfmc_batch_destroy": [_vp],
    "gfmc_batch_step": [_vp, _i32, _P(_i32), _P(StepRecord)],
    "gfmc_batch_sweep": [_vp, _i32, _P(_d), _P(_i64)],
    "gfmc_batch_use_graph": [_vp, _i32],
    "gfmc_batch_step_timing": [_vp, _P(_d), _P(_i64)],
    "gfmc_batch_set_tuning": [_vp, _i32],
    "gfmc_batch_set_lanes": [_vp, _i32],
    "gfmc_batch_set_schedule": [_vp, _i32],
    "gfmc_batch_get_form": [_vp, _P(_i32), _P(_i32), _P(_i32), _P(_i32)],
    "gfmc_batch_set_nontemporal": [_vp, _i32],
    "gfmc_batch_set_block_threads": [_vp, _i32],
    "gfmc_batch_get_block_threads": [_vp, _P(_i32)],
    "gfmc_batch_get_tuning": [_vp, _P(_i32), _P(_i32)],
    "gfmc_batch_autotune": [_vp, _i32, _P(_i32)],
    "gfmc_engine_create": [ctypes.c_int, _sz, _i32, _P(_vp)],
    "gfmc_engine_submit": [_vp, _P(ChainParams), _i32, _d, _i32, _P(ctypes.c_uint64)],
    "gfmc_engine_poll": [_vp, _vp, _i32, _P(_i32)],
    "gfmc_engine_cancel": [_vp, ctypes.c_uint64],
    "gfmc_engine_sweep_latencies": [_vp, _P(_d), _P(ctypes.c_uint64), _i32, _P(_i32)],
    "gfmc_engine_status": [_vp, _P(_i32), _P(_i32), _P(_i32), _P(_sz)],
    "gfmc_engine_drain": [_vp, _d],
    "gfmc_engine_destroy": [_vp],
    "gfmc_stream_bandwidth": [_i32, _vp, _vp, _vp, _sz, _i32, _vp, _P(_d)],
    "gfmc_delta_seff_static": [_P(ChainParams), _vp, _vp, _i32, _d, _d, _vp, _vp, _vp],
}
EXPORTS = list(_SIGS) + ["gfmc_status_string", "gfmc_last_error", "gfmc_version"]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libgfmc.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_1303_6016_amd/build.py` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        for name in ("gfmc_status_string",):
            getattr(L, name).argtypes = [ctypes.c_int]
            getattr(L, name).restype = ctypes.c_char_p
        for name in ("gfmc_last_error", "gfmc_version"):
            getattr(L, name).argtypes = []
            getattr(L, name).restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int):
    if status != GFMC_OK:
        raise GfmcError(status, lib().gfmc_last_error().decode())


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params:
    L: int
    t: float = 1.0
    beta: float = 20.0
    mu: float = 0.0
    M: int = 256
    K: int = 0
    kernel: int = JACKSON
    lorentz_lambda: float = 0.0
    scale_a: float = 0.0
    scale_b: float = 0.0
    precision: int = FP64
    proposal: int = PROPOSE_SPHERE
    cone_angle: float = 0.0
    seed: int = 0
    chain_id: int = 0
    vectors: int = VECTORS_SITES
    hoppings: int = HOP_RECOMPUTE
    fp32_unvalidated: int = 0

    def c(self) -> ChainParams:
        return ChainParams(self.L, self.t, self.beta, self.mu, self.M, self.K, self.kernel,
                           self.lorentz_lambda, self.scale_a, self.scale_b, self.precision,
                           self.proposal, self.cone_angle, self.seed & (2**64 - 1),
                           self.chain_id & (2**64 - 1), self.vectors, self.hoppings,
                           self.fp32_unvalidated)

    @property
    def N(self) -> int:
        return self.L ** 3


def gfmc_workspace_bytes(p: Params) -> int:
    n = ctypes.c_size_t()
    cp = p.c()
    _check(lib().gfmc_workspace_bytes(ctypes.byref(cp), ctypes.byref(n)))
    return n.value


def _alloc(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


class Chain:
    """One Markov chain; its workspace is a torch uint8 tensor on the device."""

    def __init__(self, p: Params, device="cuda", stream: Optional[torch.cuda.Stream] = None):
        self.p = p
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.nbytes = gfmc_workspace_bytes(p)
            self.ws = _alloc(self.nbytes, self.device)
            h = ctypes.c_void_p()
            cp = p.c()
            _check(lib().gfmc_chain_create(ctypes.byref(cp), ctypes.c_void_p(self.ws.data_ptr()),
                                           self.nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(h)))
            self.h = h

    def close(self):
        if getattr(self, "h", None):
            _check(lib().gfmc_chain_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def N(self):
        return self.p.N

    def set_params(self, t, beta, mu):
        _check(lib().gfmc_set_params(self.h, t, beta, mu))
        self.p.t, self.p.beta, self.p.mu = t, beta, mu

    def init_spins(self, mode: int, frac: float = 0.0):
        _check(lib().gfmc_init_spins(self.h, mode, frac))

    def set_spins(self, theta, phi):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        ph = np.ascontiguousarray(phi, dtype=np.float64)
        assert th.size == self.N and ph.size == self.N
        _check(lib().gfmc_set_spins(self.h, _dptr(th), _dptr(ph)))

    def get_spins(self):
        th = np.zeros(self.N)
        ph = np.zeros(self.N)
        _check(lib().gfmc_get_spins(self.h, _dptr(th), _dptr(ph)))
        return th, ph

    def set_counter(self, index: int):
        _check(lib().gfmc_set_counter(self.h, index))

    def get_counter(self) -> int:
        v = ctypes.c_int64()
        _check(lib().gfmc_get_counter(self.h, ctypes.byref(v)))
        return v.value

    def nonfinite(self) -> int:
        """Proposals rejected because their Delta S_eff was not finite."""
        v = ctypes.c_int64()
        _check(lib().gfmc_chain_nonfinite(self.h, ctypes.byref(v)))
        return v.value

    def device_angles(self):
        """Device addresses (theta, phi) of the spin angles in the workspace."""
        th, ph = ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().gfmc_chain_device_angles(self.h, ctypes.byref(th), ctypes.byref(ph)))
        return th.value, ph.value

    def moments(self, site: int) -> np.ndarray:
        out = np.zeros((self.p.M, 7, 7, 2))
        _check(lib().gfmc_moments(self.h, site, _dptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def pair_moments(self, site: int, theta_new: float, phi_new: float) -> np.ndarray:
        """(M, 3) complex: <o|T_n|o>, <v|T_n|v>, <o|T_n|v> for the proposed move."""
        out = np.zeros((self.p.M, 3, 2))
        _check(lib().gfmc_pair_moments(self.h, site, theta_new, phi_new, _dptr(out)))
        return out[..., 0] + 1j * out[..., 1]

    def mixed_moments(self, site: int, theta_new: float, phi_new: float) -> np.ndarray:
        """(4, M) real: <a|T_n|a> for a = |o>, |v>, |o>+|v>, |o>+i|v>."""
        out = np.zeros((4, self.p.M))
        _check(lib().gfmc_mixed_moments(self.h, site, theta_new, phi_new, _dptr(out)))
        return out

    def delta_seff(self, site: int, theta_new: float, phi_new: float, with_phase_top=False):
        ds, top = ctypes.c_double(), ctypes.c_double()
        _check(lib().gfmc_delta_seff(self.h, site, theta_new, phi_new, ctypes.byref(ds),
                                     ctypes.byref(top)))
        return (ds.value, top.value) if with_phase_top else ds.value

    def step(self, force: int = -1) -> StepRecord:
        rec = StepRecord()
        _check(lib().gfmc_step(self.h, force, ctypes.byref(rec)))
        return rec

    def sweep(self, nsweeps: int):
        mag = np.zeros(max(nsweeps, 1))
        acc = ctypes.c_int64()
        _check(lib().gfmc_sweep(self.h, nsweeps, _dptr(mag), ctypes.byref(acc)))
        return mag[:nsweeps], acc.value

    def sync(self):
        _check(lib().gfmc_sync(self.h))

    def magnetization(self) -> float:
        v = ctypes.c_double()
        _check(lib().gfmc_magnetization(self.h, ctypes.byref(v)))
        return v.value

    def step_bytes(self):
        b, s = ctypes.c_double(), ctypes.c_int32()
        _check(lib().gfmc_chain_step_bytes(self.h, ctypes.byref(b), ctypes.byref(s)))
        return b.value, s.value


class Batch:
    """Several chains advanced together (one launch per Chebyshev step)."""

    def __init__(self, chains: Sequence[Chain], stream: Optional[torch.cuda.Stream] = None):
        self.chains = list(chains)
        if not self.chains:   # the library rejects an empty batch (GFMC_EINVAL)
            _check(lib().gfmc_batch_workspace_bytes(None, 0, ctypes.byref(ctypes.c_size_t())))
        dev = self.chains[0].device
        with torch.cuda.device(dev):
            # a stream of its own: the legacy default stream cannot be captured
            self.stream = stream if stream is not None else torch.cuda.Stream(dev)
            arr = (ctypes.c_void_p * len(self.chains))(*[c.h.value for c in self.chains])
            n = ctypes.c_size_t()
            _check(lib().gfmc_batch_workspace_bytes(arr, len(self.chains), ctypes.byref(n)))
            self.ws = _alloc(n.value, dev)
            h = ctypes.c_void_p()
            _check(lib().gfmc_batch_create(arr, len(self.chains), ctypes.c_void_p(self.ws.data_ptr()),
                                           n.value, ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(h)))
            self.h = h

    def close(self):
        if getattr(self, "h", None):
            _check(lib().gfmc_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nprop: int = 1, force: Optional[np.ndarray] = None, records: bool = False):
        n = len(self.chains)
        fp = None
        if force is not None:
            f = np.ascontiguousarray(force, dtype=np.int32).reshape(nprop, n)
            fp = f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        recs = (StepRecord * (nprop * n))() if records else None
        _check(lib().gfmc_batch_step(self.h, nprop, fp, recs))
        if records:
            return [[recs[q * n + i] for i in range(n)] for q in range(nprop)]
        return None

    def sweep(self, nsweeps: int):
        n = len(self.chains)
        mag = np.zeros((n, max(nsweeps, 1)))
        acc = np.zeros(n, dtype=np.int64)
        _check(lib().gfmc_batch_sweep(self.h, nsweeps, _dptr(mag),
                                      acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return mag[:, :nsweeps], acc

    def use_graph(self, enable: bool = True):
        _check(lib().gfmc_batch_use_graph(self.h, 1 if enable else 0))

    def set_tuning(self, pairs_per_thread: int):
        _check(lib().gfmc_batch_set_tuning(self.h, pairs_per_thread))

    def set_lanes(self, lanes: int):
        """1 to 4 step lanes (>= 2: the chains' steps on that many forked streams)."""
        _check(lib().gfmc_batch_set_lanes(self.h, lanes))

    def set_schedule(self, step_granular: bool):
        """False: lock-step proposals; True: each chain restarts as soon as its
        proposal ends (chains with fewer steps make more proposals)."""
        _check(lib().gfmc_batch_set_schedule(self.h, 1 if step_granular else 0))

    def form(self):
        """{"resident", "persistent" (working blocks, 0 if off), "step_granular",
        "nontemporal"}."""
        r, p, c, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().gfmc_batch_get_form(self.h, ctypes.byref(r), ctypes.byref(p), ctypes.byref(c),
                                         ctypes.byref(n)))
        return {"resident": r.value, "persistent": p.value, "step_granular": c.value,
                "nontemporal": n.value}

    def set_nontemporal(self, on: bool):
        _check(lib().gfmc_batch_set_nontemporal(self.h, 1 if on else 0))

    def set_block_threads(self, threads: int):
        """Threads per block of the launched step kernel: 256 or 512."""
        _check(lib().gfmc_batch_set_block_threads(self.h, threads))

    def block_threads(self) -> int:
        v = ctypes.c_int32()
        _check(lib().gfmc_batch_get_block_threads(self.h, ctypes.byref(v)))
        return v.value

    def tuning(self):
        """(launch shape, lanes) in effect."""
        ppt, lanes = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().gfmc_batch_get_tuning(self.h, ctypes.byref(ppt), ctypes.byref(lanes)))
        return ppt.value, lanes.value

    def autotune(self, trial_steps: int = 16) -> int:
        v = ctypes.c_int32()
        _check(lib().gfmc_batch_autotune(self.h, trial_steps, ctypes.byref(v)))
        return v.value

    def step_timing(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().gfmc_batch_step_timing(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Engine:
    """Serving engine: continuous batching of chain requests on one device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 1 << 30, max_slots: int = 64):
        h = ctypes.c_void_p()
        _check(lib().gfmc_engine_create(device, hbm_budget_bytes, max_slots, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _check(lib().gfmc_engine_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, p: Params, init: int = INIT_RANDOM, frac: float = 0.0, nsweeps: int = 1) -> int:
        rid = ctypes.c_uint64()
        cp = p.c()
        _check(lib().gfmc_engine_submit(self.h, ctypes.byref(cp), init, frac, nsweeps,
                                        ctypes.byref(rid)))
        return rid.value

    def poll(self, cap: int = 256):
        out = (Result * cap)()
        n = ctypes.c_int32()
        _check(lib().gfmc_engine_poll(self.h, out, cap, ctypes.byref(n)))
        return [out[i] for i in range(n.value)]

    def cancel(self, request_id: int):
        _check(lib().gfmc_engine_cancel(self.h, request_id))

    def sweep_latencies(self, cap: int = 1 << 16):
        sec = np.zeros(cap)
        ids = np.zeros(cap, dtype=np.uint64)
        n = ctypes.c_int32()
        _check(lib().gfmc_engine_sweep_latencies(
            self.h, _dptr(sec), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), cap,
            ctypes.byref(n)))
        return sec[:n.value], ids[:n.value]

    def status(self):
        q, r, f, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        _check(lib().gfmc_engine_status(self.h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(f),
                                        ctypes.byref(b)))
        return {"queued": q.value, "running": r.value, "finished": f.value, "bytes": b.value}

    def drain(self, timeout_s: float = 600.0):
        _check(lib().gfmc_engine_drain(self.h, timeout_s))


def stream_bandwidth(mode: int, nbytes: int, reps: int = 10, device="cuda:0") -> float:
    """Streaming bandwidth (GB/s) of the device: mode 0 read, 1 write, 2 copy,
    3 two reads + one write, over buffers of nbytes each."""
    dev = torch.device(device)
    with torch.cuda.device(dev):
        bufs = [torch.zeros(nbytes, dtype=torch.uint8, device=dev) for _ in range(3)]
        st = torch.cuda.current_stream(dev)
        v = ctypes.c_double()
        _check(lib().gfmc_stream_bandwidth(mode, ctypes.c_void_p(bufs[0].data_ptr()),
                                           ctypes.c_void_p(bufs[1].data_ptr()),
                                           ctypes.c_void_p(bufs[2].data_ptr()), nbytes, reps,
                                           ctypes.c_void_p(st.cuda_stream), ctypes.byref(v)))
        del bufs
        return v.value
