"""Python binding of libpbit (include/pbit.h): argument marshalling only.

Every step of the sampling path runs in the library's HIP kernels; torch
supplies device memory (the instance workspace and output buffers) and the
stream.  The library must be built (paper_2501_04971_amd.build) before use:
loading fails loudly if libpbit.so is missing.
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np

from .generators import KIND_QKP, Params, Problem

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpbit.so")

PBIT_OK, PBIT_NOFEAS = 0, 1
PBIT_EINVAL, PBIT_ERANGE, PBIT_EWORKSPACE, PBIT_EDEVICE, PBIT_ESTATE = -1, -2, -3, -4, -5
THETA_LEN = 4609


class PbitError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libpbit status {status}: {message}")
        self.status = status


class pbit_problem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("profit", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("capacity", ctypes.c_void_p), ("density_num", ctypes.c_int32),
                ("density_den", ctypes.c_int32)]


class pbit_params(ctypes.Structure):
    _fields_ = [("replicas", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("beta_num", ctypes.c_int32), ("beta_den", ctypes.c_int32),
                ("eta_num", ctypes.c_int32), ("eta_den", ctypes.c_int32),
                ("p_q", ctypes.c_int32), ("alpha_num", ctypes.c_int32),
                ("alpha_den", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("instance_id", ctypes.c_uint32), ("fixed_beta", ctypes.c_int32),
                ("eta_decay_rounds", ctypes.c_int32), ("pt_slots", ctypes.c_int32)]


class pbit_batch_layout(ctypes.Structure):
    _fields_ = [("blocks_quad", ctypes.c_int32), ("blocks_linear", ctypes.c_int32),
                ("split_percent", ctypes.c_int32), ("split_members", ctypes.c_int32)]


def make_layout(layout=None, blocks: int = 0) -> pbit_batch_layout:
    """layout: dict with any of blocks_quad, blocks_linear, split_percent
    (missing keys: 0, 0, -1); blocks > 0 caps both families' grids."""
    d = {"blocks_quad": blocks, "blocks_linear": blocks, "split_percent": -1}
    d.update(layout or {})
    return pbit_batch_layout(int(d["blocks_quad"]), int(d["blocks_linear"]), int(d["split_percent"]), 0)


class pbit_plan_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("n_ext", ctypes.c_int32),
                ("n_pad", ctypes.c_int32), ("words", ctypes.c_int32),
                ("s_f", ctypes.c_int64), ("s_g", ctypes.c_int64), ("p_q", ctypes.c_int64),
                ("shift", ctypes.c_int32), ("lq_max", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t),
                ("out_x", ctypes.c_size_t), ("out_g", ctypes.c_size_t),
                ("out_profit", ctypes.c_size_t), ("out_feasible", ctypes.c_size_t),
                ("out_G", ctypes.c_size_t), ("out_lambda", ctypes.c_size_t),
                ("out_round", ctypes.c_size_t), ("out_sat", ctypes.c_size_t),
                ("out_slot", ctypes.c_size_t), ("out_bytes", ctypes.c_size_t)]


EXPORTS = {
    "pbit_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_create_instance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_create_instance_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p]),
    "pbit_static_workspace_bytes": (ctypes.c_size_t, []),
    "pbit_sample_round": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_update_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_set_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_get_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_best_feasible": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_round_outputs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p]),
    "pbit_destroy_instance": (ctypes.c_int, [ctypes.c_void_p]),
    "pbit_last_error": (ctypes.c_char_p, []),
    "pbit_theta_table": (ctypes.c_int, [ctypes.c_void_p]),
    "pbit_exchange_table": (ctypes.c_int, [ctypes.c_void_p]),
    "pbit_instance_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_set_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "pbit_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "pbit_create_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_batch_layout_used": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_batch_sample_round": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_batch_update_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p]),
    "pbit_batch_member": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "pbit_batch_rounds_left": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_batch_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "pbit_destroy_batch": (ctypes.c_int, [ctypes.c_void_p]),
    "pbit_batch_set_lambdas": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_batch_snapshot": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_net_param_count": (ctypes.c_int32, []),
    "pbit_net_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "pbit_net_pack": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_net_cast": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_net_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p]),
    "pbit_net_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "pbit_net_adam_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p]),
    "pbit_net_to_lambda": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p]),
}

SNAPSHOT_BYTES = 176
MAX_M = 32

_LIB = None


def lib() -> ctypes.CDLL:
    """Loads libpbit.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2501_04971_amd.build first")
        # torch brings its own HIP runtime; loading it first makes the library
        # bind to that same runtime instead of a second copy (two runtimes in
        # one process do not see each other's devices)
        import torch  # noqa: F401
        so = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(so, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = so
    return _LIB


def _check(status: int) -> int:
    if status < 0:
        raise PbitError(status, lib().pbit_last_error().decode())
    return status


def _ratio(v) -> tuple:
    f = Fraction(v)
    return int(f.numerator), int(f.denominator)


class _Marshalled:
    """C views of a Problem and Params; keeps the numpy buffers alive."""

    def __init__(self, prob: Problem, par: Params):
        self.profit = np.ascontiguousarray(np.asarray(prob.profit, dtype=np.int32))
        self.weight = np.ascontiguousarray(np.asarray(prob.weight, dtype=np.int32))
        self.capacity = np.ascontiguousarray(np.asarray(prob.capacity, dtype=np.int64))
        dn, dd = _ratio(prob.density)
        self.problem = pbit_problem(int(prob.kind), prob.n, prob.m, self.profit.ctypes.data,
                                    self.weight.ctypes.data, self.capacity.ctypes.data, dn, dd)
        bn, bd = _ratio(par.beta)
        en, ed = _ratio(par.eta)
        an, ad = _ratio(par.alpha)
        self.params = pbit_params(int(par.replicas), int(par.sweeps), bn, bd, en, ed,
                                  -1 if par.p_q is None else int(par.p_q), an, ad,
                                  int(par.seed) & ((1 << 64) - 1),
                                  int(par.instance_id) & 0xFFFFFFFF, 1 if par.fixed_beta else 0,
                                  int(par.eta_decay), int(getattr(par, "pt_slots", 0)))


def pbit_plan(prob: Problem, par: Params) -> pbit_plan_info:
    mp = _Marshalled(prob, par)
    info = pbit_plan_info()
    _check(lib().pbit_plan(ctypes.byref(mp.problem), ctypes.byref(mp.params), ctypes.byref(info)))
    return info


def pbit_workspace_bytes(prob: Problem, par: Params) -> int:
    mp = _Marshalled(prob, par)
    return int(lib().pbit_workspace_bytes(ctypes.byref(mp.problem), ctypes.byref(mp.params)))


def pbit_theta_table() -> np.ndarray:
    out = np.zeros(THETA_LEN, dtype=np.int32)
    _check(lib().pbit_theta_table(out.ctypes.data))
    return out


def pbit_exchange_table() -> np.ndarray:
    out = np.zeros(THETA_LEN, dtype=np.int32)
    _check(lib().pbit_exchange_table(out.ctypes.data))
    return out


def _stream_handle(stream) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def pbit_create_instance(prob: Problem, par: Params, workspace, stream=None) -> int:
    """workspace: a uint8 CUDA tensor of at least pbit_workspace_bytes bytes."""
    mp = _Marshalled(prob, par)
    handle = ctypes.c_void_p()
    _check(lib().pbit_create_instance(ctypes.byref(mp.problem), ctypes.byref(mp.params),
                                      workspace.data_ptr(), workspace.numel(),
                                      _stream_handle(stream), ctypes.byref(handle)))
    return int(handle.value)


def pbit_create_instance_static(prob: Problem, par: Params, stream=None) -> int:
    """As pbit_create_instance, with the library's static per-device workspace."""
    mp = _Marshalled(prob, par)
    handle = ctypes.c_void_p()
    _check(lib().pbit_create_instance_static(ctypes.byref(mp.problem), ctypes.byref(mp.params),
                                             _stream_handle(stream), ctypes.byref(handle)))
    return int(handle.value)


def pbit_static_workspace_bytes() -> int:
    return int(lib().pbit_static_workspace_bytes())


def pbit_sample_round(inst: int, stream=None) -> None:
    _check(lib().pbit_sample_round(inst, _stream_handle(stream)))


def pbit_update_lambda(inst: int, stream=None) -> None:
    _check(lib().pbit_update_lambda(inst, _stream_handle(stream)))


def pbit_set_lambda(inst: int, lambda_q, stream=None) -> None:
    v = np.ascontiguousarray(np.asarray(lambda_q, dtype=np.int32))
    _check(lib().pbit_set_lambda(inst, v.ctypes.data, _stream_handle(stream)))


def pbit_get_lambda(inst: int, m: int, stream=None) -> np.ndarray:
    out = np.zeros(m, dtype=np.int32)
    _check(lib().pbit_get_lambda(inst, out.ctypes.data, _stream_handle(stream)))
    return out


def pbit_best_feasible(inst: int, n: int, stream=None):
    """(profit, x bytes, round, replica) or None when nothing feasible was found."""
    profit = ctypes.c_int64()
    rnd = ctypes.c_int32()
    rep = ctypes.c_int32()
    x = np.zeros(n, dtype=np.uint8)
    st = _check(lib().pbit_best_feasible(inst, ctypes.byref(profit), x.ctypes.data,
                                         ctypes.byref(rnd), ctypes.byref(rep),
                                         _stream_handle(stream)))
    if st == PBIT_NOFEAS:
        return None
    return int(profit.value), x, int(rnd.value), int(rep.value)


def pbit_round_outputs(inst: int, out, stream=None) -> None:
    _check(lib().pbit_round_outputs(inst, out.data_ptr(), out.numel(), _stream_handle(stream)))


def pbit_destroy_instance(inst: int) -> None:
    _check(lib().pbit_destroy_instance(inst))


def pbit_instance_info(inst: int) -> pbit_plan_info:
    info = pbit_plan_info()
    _check(lib().pbit_instance_info(inst, ctypes.byref(info)))
    return info


def pbit_set_tiling(inst: int, waves_per_block: int, lds_resident: int = -1, split: int = -1) -> None:
    _check(lib().pbit_set_tiling(inst, int(waves_per_block), int(lds_resident), int(split)))


class _MarshalledSet:
    """C arrays of problems and params for a batch."""

    def __init__(self, probs, pars):
        self.items = [_Marshalled(p, q) for p, q in zip(probs, pars)]
        n = len(self.items)
        self.problems = (pbit_problem * n)(*[m.problem for m in self.items])
        self.params = (pbit_params * n)(*[m.params for m in self.items])
        self.count = n


def pbit_batch_workspace_bytes(probs, pars) -> int:
    ms = _MarshalledSet(probs, pars)
    return int(lib().pbit_batch_workspace_bytes(ms.problems, ms.params, ms.count))


def pbit_create_batch(probs, pars, rounds, workspace, blocks: int = 0, stream=None, layout=None) -> int:
    ms = _MarshalledSet(probs, pars)
    rv = None if rounds is None else np.ascontiguousarray(np.asarray(rounds, dtype=np.int32))
    lay = make_layout(layout, blocks)
    handle = ctypes.c_void_p()
    _check(lib().pbit_create_batch(ms.problems, ms.params, ms.count,
                                   None if rv is None else rv.ctypes.data, ctypes.byref(lay),
                                   workspace.data_ptr(), workspace.numel(),
                                   _stream_handle(stream), ctypes.byref(handle)))
    return int(handle.value)


def pbit_batch_layout_used(batch: int) -> dict:
    out = pbit_batch_layout()
    _check(lib().pbit_batch_layout_used(batch, ctypes.byref(out)))
    return {"blocks_quad": out.blocks_quad, "blocks_linear": out.blocks_linear,
            "split_percent": out.split_percent, "split_members": out.split_members}


def pbit_batch_sample_round(batch: int, stream=None) -> None:
    _check(lib().pbit_batch_sample_round(batch, _stream_handle(stream)))


def pbit_batch_update_lambda(batch: int, stream=None) -> None:
    _check(lib().pbit_batch_update_lambda(batch, _stream_handle(stream)))


def pbit_batch_run(batch: int, rounds: int, use_graph: bool = True, stream=None) -> None:
    _check(lib().pbit_batch_run(batch, int(rounds), 1 if use_graph else 0, _stream_handle(stream)))


def pbit_batch_member(batch: int, index: int) -> int:
    handle = ctypes.c_void_p()
    _check(lib().pbit_batch_member(batch, int(index), ctypes.byref(handle)))
    return int(handle.value)


def pbit_batch_rounds_left(batch: int, count: int, stream=None) -> np.ndarray:
    out = np.zeros(count, dtype=np.int32)
    _check(lib().pbit_batch_rounds_left(batch, out.ctypes.data, _stream_handle(stream)))
    return out


def pbit_batch_shape(batch: int):
    items, blocks, lds = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    _check(lib().pbit_batch_shape(batch, ctypes.byref(items), ctypes.byref(blocks), ctypes.byref(lds)))
    return int(items.value), int(blocks.value), int(lds.value)


def pbit_destroy_batch(batch: int) -> None:
    _check(lib().pbit_destroy_batch(batch))


class Instance:
    """One compiled instance with its torch-owned workspace on the current device."""

    def __init__(self, prob: Problem, par: Params, stream=None, _member=None, static_workspace=False):
        import torch
        self.problem, self.params, self.stream = prob, par, stream
        self.owned = _member is None
        if self.owned and static_workspace:
            self.info = pbit_plan(prob, par)
            self.workspace = None
            self.handle = pbit_create_instance_static(prob, par, stream)
        elif self.owned:
            self.info = pbit_plan(prob, par)
            # torch's caching allocator hands out blocks aligned to at least 512 bytes
            self.workspace = torch.empty(int(self.info.workspace_bytes), dtype=torch.uint8, device="cuda")
            self.handle = pbit_create_instance(prob, par, self.workspace, stream)
        else:
            self.handle = _member
            self.info = pbit_instance_info(_member)
        self.outbuf = torch.empty(int(self.info.out_bytes), dtype=torch.uint8, device="cuda")

    def set_tiling(self, waves_per_block: int, lds_resident: int = -1, split: int = -1):
        pbit_set_tiling(self.handle, waves_per_block, lds_resident, split)

    def sample_round(self):
        pbit_sample_round(self.handle, self.stream)

    def update_lambda(self):
        pbit_update_lambda(self.handle, self.stream)

    def set_lambda(self, lambda_q):
        pbit_set_lambda(self.handle, lambda_q, self.stream)

    def get_lambda(self) -> np.ndarray:
        return pbit_get_lambda(self.handle, self.info.m, self.stream)

    def best_feasible(self):
        return pbit_best_feasible(self.handle, self.info.n, self.stream)

    def round_outputs(self) -> dict:
        """Last round's per-replica results, copied to host numpy arrays."""
        import torch
        pbit_round_outputs(self.handle, self.outbuf, self.stream)
        torch.cuda.current_stream().synchronize() if self.stream is None else self.stream.synchronize()
        raw = self.outbuf.cpu().numpy()
        i, R, m, w = self.info, self.params.replicas, self.info.m, self.info.words

        def view(off, dtype, count):
            return raw[off:off + count * np.dtype(dtype).itemsize].view(dtype)

        return {
            "x_bits": view(i.out_x, np.uint32, R * w).reshape(R, w).copy(),
            "g": view(i.out_g, np.int32, R * m).reshape(R, m).copy(),
            "profit": view(i.out_profit, np.int64, R).copy(),
            "feasible": view(i.out_feasible, np.int32, R).copy(),
            "G": view(i.out_G, np.int64, m).copy(),
            "lambda_q": view(i.out_lambda, np.int32, m).copy(),
            "round": int(view(i.out_round, np.int32, 1)[0]),
            "lambda_saturated": int(view(i.out_sat, np.uint32, 1)[0]),
            "slot": view(i.out_slot, np.int32, R).copy(),
        }

    def close(self):
        if self.handle and self.owned:
            pbit_destroy_instance(self.handle)
        self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pbit_batch_set_lambdas(batch: int, lambda_q, stream=None) -> None:
    """lambda_q: int32 CUDA tensor [count][32]."""
    _check(lib().pbit_batch_set_lambdas(batch, lambda_q.data_ptr(), _stream_handle(stream)))


def pbit_batch_snapshot(batch: int, out, stream=None) -> None:
    """out: uint8 CUDA tensor of count * SNAPSHOT_BYTES bytes."""
    _check(lib().pbit_batch_snapshot(batch, out.data_ptr(), _stream_handle(stream)))


def decode_snapshot(raw: np.ndarray, count: int) -> dict:
    """Host view of pbit_batch_snapshot records."""
    r = np.asarray(raw, dtype=np.uint8).reshape(count, SNAPSHOT_BYTES)
    head = r[:, 8:32].copy().view(np.int32)
    return {"best": r[:, :8].copy().view(np.int64).reshape(count),
            "best_round": head[:, 0], "has_feasible": head[:, 1].astype(bool),
            "rounds": head[:, 2], "feasible_last": head[:, 3],
            "lambda_saturated": head[:, 4].view(np.uint32),
            "lambda_q": r[:, 32:160].copy().view(np.int32).reshape(count, MAX_M),
            "feasible_profit_sum": r[:, 160:168].copy().view(np.int64).reshape(count),
            "residual_sq_sum": r[:, 168:176].copy().view(np.int64).reshape(count)}


# ---- learned starting multipliers -------------------------------------------

def pbit_net_param_count() -> int:
    return int(lib().pbit_net_param_count())


def pbit_net_workspace_bytes(sets: int, rows: int) -> int:
    return int(lib().pbit_net_workspace_bytes(int(sets), int(rows)))


def pbit_net_pack(probs, pars) -> dict:
    """Host arrays of the packed sets (x and ctx as uint16 bf16 bit patterns)."""
    ms = _MarshalledSet(probs, pars)
    sets, rows = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().pbit_net_pack(ms.problems, ms.params, ms.count, ctypes.byref(sets), ctypes.byref(rows),
                               None, None, None, None, None, None))
    S, R = int(sets.value), int(rows.value)
    out = {"x": np.zeros((R, 16), np.uint16), "ctx": np.zeros((S, 16), np.uint16),
           "set_rows": np.zeros(S + 1, np.int32), "set_n": np.zeros(S, np.int32),
           "scale": np.zeros(S, np.float64), "dest": np.zeros(S, np.int32), "sets": S, "rows": R}
    _check(lib().pbit_net_pack(ms.problems, ms.params, ms.count, ctypes.byref(sets), ctypes.byref(rows),
                               out["x"].ctypes.data, out["ctx"].ctypes.data, out["set_rows"].ctypes.data,
                               out["set_n"].ctypes.data, out["scale"].ctypes.data, out["dest"].ctypes.data))
    return out


def pbit_net_cast(w, w_bf16, stream=None) -> None:
    _check(lib().pbit_net_cast(w.data_ptr(), w_bf16.data_ptr(), _stream_handle(stream)))


def pbit_net_forward(w_bf16, x, ctx, set_rows, set_n, sets, rows, ws, t, stream=None) -> None:
    _check(lib().pbit_net_forward(w_bf16.data_ptr(), x.data_ptr(), ctx.data_ptr(), set_rows.data_ptr(),
                                  set_n.data_ptr(), int(sets), int(rows), ws.data_ptr(), ws.numel(),
                                  t.data_ptr(), _stream_handle(stream)))


def pbit_net_backward(w_bf16, x, set_rows, set_n, sets, rows, t, y, ws, grad, loss, stream=None) -> None:
    _check(lib().pbit_net_backward(w_bf16.data_ptr(), x.data_ptr(), set_rows.data_ptr(), set_n.data_ptr(),
                                   int(sets), int(rows), t.data_ptr(), y.data_ptr(), ws.data_ptr(), ws.numel(),
                                   grad.data_ptr(), loss.data_ptr(), _stream_handle(stream)))


def pbit_net_adam_step(w, m, v, grad, w_bf16, step: int, lr: float, stream=None) -> None:
    _check(lib().pbit_net_adam_step(w.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(),
                                    w_bf16.data_ptr(), int(step), float(lr), _stream_handle(stream)))


def pbit_net_to_lambda(t, scale, dest, sets, lambda_q, stream=None) -> None:
    _check(lib().pbit_net_to_lambda(t.data_ptr(), scale.data_ptr(), dest.data_ptr(), int(sets),
                                    lambda_q.data_ptr(), _stream_handle(stream)))


class Batch:
    """A set of instances run together (one persistent launch per round) in one
    torch-owned workspace.  members[i] is an Instance view of member i (its
    lambda / residual vectors include any padding constraints)."""

    def __init__(self, probs, pars, rounds=None, blocks: int = 0, stream=None, layout=None):
        import torch
        self.problems, self.params, self.stream = list(probs), list(pars), stream
        nbytes = pbit_batch_workspace_bytes(self.problems, self.params)
        if nbytes == 0:
            # re-run through create for the error message
            nbytes = 256
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        self.handle = pbit_create_batch(self.problems, self.params, rounds, self.workspace, blocks, stream, layout)
        self.members = [Instance(p, q, stream, _member=pbit_batch_member(self.handle, i))
                        for i, (p, q) in enumerate(zip(self.problems, self.params))]

    def sample_round(self):
        pbit_batch_sample_round(self.handle, self.stream)

    def update_lambda(self):
        pbit_batch_update_lambda(self.handle, self.stream)

    def run(self, rounds: int, use_graph: bool = True):
        pbit_batch_run(self.handle, rounds, use_graph, self.stream)

    def rounds_left(self) -> np.ndarray:
        return pbit_batch_rounds_left(self.handle, len(self.members), self.stream)

    def set_lambdas(self, lambda_q):
        """lambda_q: int32 CUDA tensor [count][32]."""
        pbit_batch_set_lambdas(self.handle, lambda_q, self.stream)

    def snapshot(self, out):
        """Queues the per-member records into out (uint8 CUDA tensor, count * SNAPSHOT_BYTES)."""
        pbit_batch_snapshot(self.handle, out, self.stream)

    def shape(self):
        """(work items, persistent workgroups, LDS bytes per workgroup)."""
        return pbit_batch_shape(self.handle)

    def layout(self) -> dict:
        """The launch layout in force (grids per family, split rule, split members)."""
        return pbit_batch_layout_used(self.handle)

    def close(self):
        if self.handle:
            for m in self.members:
                m.handle = 0
            pbit_destroy_batch(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def unpack_bits(bits: np.ndarray, count: int) -> np.ndarray:
    """(R, words) uint32 -> (R, count) uint8 with bit i of word i//32 = spin i."""
    b = np.asarray(bits, dtype=np.uint32)
    idx = np.arange(count)
    return ((b[:, idx >> 5] >> (idx & 31).astype(np.uint32)) & 1).astype(np.uint8)
