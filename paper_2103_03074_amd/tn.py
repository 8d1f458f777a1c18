"""Python binding of the C ABI in include/tn.h (argument marshalling only).

Every function here converts Python arguments to the C types of tn.h and
calls the HIP library libtnsim.so; all computation happens in the library.
If the library is missing the import fails loudly -- there is no fallback.

Device buffers are torch CUDA (HIP) tensors; streams are torch streams.
"""

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnsim.so")

TN_C64, TN_C128, TN_SPLIT_FP16, TN_BF16 = 0, 1, 2, 3
PRECISIONS = {"c64": TN_C64, "c128": TN_C128, "split_fp16": TN_SPLIT_FP16, "bf16": TN_BF16}


class TnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tn status {status}: {msg}")
        self.status = status


class Gate(ctypes.Structure):
    _fields_ = [("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("re", ctypes.c_double * 16), ("im", ctypes.c_double * 16)]


class CircuitC(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("gates", ctypes.POINTER(Gate))]


class EdgeC(ctypes.Structure):
    _fields_ = [("qubit", ctypes.c_int32), ("segment", ctypes.c_int32)]


class TreeC(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("lhs", ctypes.POINTER(ctypes.c_int32)),
                ("rhs", ctypes.POINTER(ctypes.c_int32))]


class PlanOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("max_log2_size", ctypes.c_int32),
                ("n_slice_edges", ctypes.c_int32), ("batch_log2", ctypes.c_int32),
                ("branch_merge", ctypes.c_int32), ("bighead", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("cost_model", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("max_workspace_bytes", ctypes.c_int64),
                ("model", ctypes.c_void_p), ("slicing", ctypes.c_int32)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n_slices", ctypes.c_uint64), ("n_sliced", ctypes.c_int32),
                ("batch_log2", ctypes.c_int32), ("n_open", ctypes.c_int32),
                ("n_leaves", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("n_c", ctypes.c_int32), ("max_log2_size", ctypes.c_int32),
                ("acc_log2", ctypes.c_int32),
                ("cmacs_per_slice", ctypes.c_double), ("cmacs_per_slice_unmerged", ctypes.c_double),
                ("cmacs_invariant", ctypes.c_double), ("cmacs_tail", ctypes.c_double),
                ("bytes_per_slice", ctypes.c_double), ("cmacs_per_batch", ctypes.c_double),
                ("bytes_per_batch", ctypes.c_double),
                ("workspace_bytes", ctypes.c_uint64), ("tail_workspace_bytes", ctypes.c_uint64),
                ("n_dense_steps", ctypes.c_int32), ("n_small_steps", ctypes.c_int32),
                ("cost_model_used", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("predicted_ms", ctypes.c_double), ("graph_replays", ctypes.c_uint64),
                ("graph_launches", ctypes.c_uint64), ("lanes", ctypes.c_int32),
                ("lanes_workspace_bytes", ctypes.c_uint64)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class XebResult(ctypes.Structure):
    _fields_ = [("F_unif", ctypes.c_double), ("F_self", ctypes.c_double), ("P_s1", ctypes.c_double),
                ("cond_xeb", ctypes.c_double), ("p_max", ctypes.c_double), ("p_min", ctypes.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MixResult(ctypes.Structure):
    _fields_ = [("P_top", ctypes.c_double), ("F_top", ctypes.c_double), ("F_mix_expected", ctypes.c_double)]


class StepProfile(ctypes.Structure):
    _fields_ = [("m_log", ctypes.c_int32), ("n_log", ctypes.c_int32), ("k_log", ctypes.c_int32),
                ("b_log", ctypes.c_int32), ("kernel", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("cmacs", ctypes.c_double), ("bytes", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("launches", ctypes.c_uint64), ("kernel_name", ctypes.c_char * 48)]

    def to_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["kernel_name"] = self.kernel_name.decode()
        return d


# every symbol tn.h declares, with its ctypes signature
_P = ctypes.c_void_p
_SIGS = {
    "tn_plan": (ctypes.c_int, [ctypes.POINTER(CircuitC), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32,
                               ctypes.POINTER(TreeC), ctypes.POINTER(EdgeC), ctypes.c_int32,
                               ctypes.POINTER(PlanOpts), ctypes.POINTER(_P)]),
    "tn_plan_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(PlanStats)]),
    "tn_plan_sliced_edges": (ctypes.c_int, [_P, ctypes.POINTER(EdgeC), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "tn_plan_export_json": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "tn_contract_slices": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, ctypes.c_uint64, ctypes.c_uint64, _P]),
    "tn_contract_slice_list": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, ctypes.POINTER(ctypes.c_uint64),
                                              ctypes.c_uint64, _P]),
    "tn_amplitudes": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, _P]),
    "tn_xeb": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                              ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(XebResult), _P]),
    "tn_choose_open_qubits": (ctypes.c_int, [ctypes.POINTER(CircuitC), ctypes.c_int32, ctypes.POINTER(PlanOpts),
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "tn_plan_step_candidates": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int32)]),
    "tn_plan_set_step_kernel": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "tn_sample_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "tn_sample": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_uint64, _P, _P, ctypes.c_size_t, _P]),
    "tn_mix_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "tn_mix_topk": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32,
                                   ctypes.c_uint64, _P, ctypes.c_uint64, _P, _P, ctypes.c_size_t,
                                   ctypes.POINTER(MixResult), _P]),
    "tn_sample_noalloc": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_uint64, _P, _P]),
    "tn_plan_set_lanes": (ctypes.c_int, [_P, ctypes.c_int32]),
    "tn_plan_set_profiling": (ctypes.c_int, [_P, ctypes.c_int32]),
    "tn_plan_step_profile": (ctypes.c_int, [_P, ctypes.POINTER(StepProfile), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "tn_plan_autotune": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, ctypes.c_char_p, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32), _P]),
    "tn_step_features": (ctypes.c_int, [ctypes.c_int32] * 5 + [ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
    "tn_plan_step_features": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_int32)]),
    "tn_mlp_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "tn_mlp_num_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "tn_mlp_get_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "tn_mlp_set_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_int64]),
    "tn_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P]),
    "tn_mlp_gradient": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(ctypes.c_float), _P]),
    "tn_mlp_train_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_float,
                                         ctypes.POINTER(ctypes.c_float), _P]),
    "tn_mlp_set_support": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                          ctypes.c_int32, ctypes.c_float]),
    "tn_mlp_destroy": (None, [_P]),
    "tn_plan_destroy": (None, [_P]),
    "tn_last_error": (ctypes.c_char_p, []),
}

_lib = None


def library():
    """Load libtnsim.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_03074_amd.build`")
        # torch ships its own HIP runtime with the same soname; loading torch
        # first makes the library bind to that one runtime, so torch's device
        # memory and stream handles are valid inside the library.
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status):
    if status != 0:
        msg = library().tn_last_error().decode(errors="replace")
        raise TnError(status, msg)


def _circuit_c(circuit):
    gates = (Gate * max(1, len(circuit.gates)))()
    for i, g in enumerate(circuit.gates):
        gates[i].q0 = int(g.qubits[0])
        gates[i].q1 = int(g.qubits[1]) if len(g.qubits) == 2 else -1
        flat = np.asarray(g.matrix, dtype=np.complex128).ravel()
        for j, v in enumerate(flat):
            gates[i].re[j] = float(v.real)
            gates[i].im[j] = float(v.imag)
    c = CircuitC(circuit.n_qubits, len(circuit.gates), gates)
    return c, gates


def plan_options(prec="c64", max_log2_size=30, n_slice_edges=-1, batch_log2=-1, branch_merge=0,
                 bighead=0, restarts=8, cost_model=0, seed=0, max_workspace_bytes=0, model=None, slicing=0):
    return PlanOpts(PRECISIONS[prec] if isinstance(prec, str) else int(prec), max_log2_size, n_slice_edges,
                    batch_log2, branch_merge, bighead, restarts, cost_model, seed, max_workspace_bytes,
                    model.handle if model is not None else None, slicing)


def choose_open_qubits(circuit, n_open, **opts):
    """Open qubits read off a contraction order of the closed network, and the
    head-tail cut they give (host only)."""
    c, keep = _circuit_c(circuit)
    o = plan_options(**opts)
    out = (ctypes.c_int32 * max(1, int(n_open)))()
    cut = ctypes.c_int32()
    _check(library().tn_choose_open_qubits(ctypes.byref(c), int(n_open), ctypes.byref(o), out, ctypes.byref(cut)))
    del keep
    return [out[i] for i in range(int(n_open))], cut.value


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Plan:
    """Owner of a tn_plan_t handle."""

    def __init__(self, circuit, open_q, fixed_q, bits, tree=None, sliced=None, **opts):
        lib = library()
        c, keep = _circuit_c(circuit)
        oq = (ctypes.c_int32 * max(1, len(open_q)))(*[int(q) for q in open_q])
        fq = (ctypes.c_int32 * max(1, len(fixed_q)))(*[int(q) for q in fixed_q])
        fb = (ctypes.c_uint8 * max(1, len(bits)))(*[int(b) for b in bits])
        tree_c = None
        if tree is not None:
            lhs = (ctypes.c_int32 * len(tree))(*[int(a) for a, _ in tree])
            rhs = (ctypes.c_int32 * len(tree))(*[int(b) for _, b in tree])
            tree_c = TreeC(len(tree), lhs, rhs)
        n_sl = -1
        sl = None
        if sliced is not None:
            n_sl = len(sliced)
            sl = (EdgeC * max(1, n_sl))(*[EdgeC(int(q), int(t)) for q, t in sliced])
        o = plan_options(**opts)
        h = ctypes.c_void_p()
        _check(lib.tn_plan(ctypes.byref(c), oq, len(open_q), fq, fb, len(fixed_q),
                           ctypes.byref(tree_c) if tree_c is not None else None,
                           sl, n_sl, ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self.n_qubits = circuit.n_qubits
        self.n_open = len(open_q)
        del keep

    def close(self):
        if getattr(self, "handle", None):
            library().tn_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        s = PlanStats()
        _check(library().tn_plan_stats_get(self.handle, ctypes.byref(s)))
        return s.to_dict()

    def sliced_edges(self):
        n = ctypes.c_int32()
        _check(library().tn_plan_sliced_edges(self.handle, None, 0, ctypes.byref(n)))
        arr = (EdgeC * max(1, n.value))()
        _check(library().tn_plan_sliced_edges(self.handle, arr, n.value, ctypes.byref(n)))
        return [(arr[i].qubit, arr[i].segment) for i in range(n.value)]

    def export(self):
        need = ctypes.c_size_t()
        _check(library().tn_plan_export_json(self.handle, None, 0, ctypes.byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(library().tn_plan_export_json(self.handle, buf, need.value, ctypes.byref(need)))
        return json.loads(buf.value.decode())

    def set_lanes(self, lanes):
        _check(library().tn_plan_set_lanes(self.handle, int(lanes)))

    def set_profiling(self, enable):
        _check(library().tn_plan_set_profiling(self.handle, 1 if enable else 0))

    def step_profile(self):
        n = ctypes.c_int32()
        _check(library().tn_plan_step_profile(self.handle, None, 0, ctypes.byref(n)))
        arr = (StepProfile * max(1, n.value))()
        _check(library().tn_plan_step_profile(self.handle, arr, n.value, ctypes.byref(n)))
        return [arr[i].to_dict() for i in range(n.value)]

    def step_candidates(self, step):
        """(kernel, tile) configurations that can run step `step` (index into
        export()["steps"])."""
        n = ctypes.c_int32()
        _check(library().tn_plan_step_candidates(self.handle, int(step), None, None, 0, ctypes.byref(n)))
        ks = (ctypes.c_int32 * max(1, n.value))()
        ts = (ctypes.c_int32 * max(1, n.value))()
        _check(library().tn_plan_step_candidates(self.handle, int(step), ks, ts, n.value, ctypes.byref(n)))
        return [(ks[i], ts[i]) for i in range(n.value)]

    def set_step_kernel(self, step, kernel, tile):
        _check(library().tn_plan_set_step_kernel(self.handle, int(step), int(kernel), int(tile)))

    def autotune(self, ws, acc_scratch, cache_path=None, reps=5, stream=None):
        n = ctypes.c_int32()
        _check(library().tn_plan_autotune(self.handle, ctypes.c_void_p(ws.data_ptr()),
                                          ws.numel() * ws.element_size(), ctypes.c_void_p(acc_scratch.data_ptr()),
                                          cache_path.encode() if cache_path else None, int(reps),
                                          ctypes.byref(n), _stream_ptr(stream)))
        return n.value

    # -- device calls (torch tensors in, nothing allocated here) ---------

    def contract_slices(self, ws, acc, begin, end, stream=None):
        _check(library().tn_contract_slices(self.handle, ctypes.c_void_p(ws.data_ptr()),
                                            ws.numel() * ws.element_size(), ctypes.c_void_p(acc.data_ptr()),
                                            int(begin), int(end), _stream_ptr(stream)))

    def contract_slice_list(self, ws, acc, ids, stream=None):
        ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
        _check(library().tn_contract_slice_list(
            self.handle, ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
            ctypes.c_void_p(acc.data_ptr()), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            ids.size, _stream_ptr(stream)))

    def amplitudes(self, acc, amps, ws=None, stream=None):
        _check(library().tn_amplitudes(self.handle, ctypes.c_void_p(acc.data_ptr()),
                                       ctypes.c_void_p(amps.data_ptr()),
                                       ctypes.c_void_p(ws.data_ptr()) if ws is not None else None,
                                       (ws.numel() * ws.element_size()) if ws is not None else 0,
                                       _stream_ptr(stream)))


STEP_FEATURES = 12


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def step_features(m, n, k, b, kernel, prec="c64"):
    out = np.zeros(STEP_FEATURES, dtype=np.float32)
    _check(library().tn_step_features(int(m), int(n), int(k), int(b), int(kernel),
                                      PRECISIONS[prec] if isinstance(prec, str) else int(prec), _fptr(out)))
    return out


def plan_step_features(plan):
    n = ctypes.c_int32()
    _check(library().tn_plan_step_features(plan.handle, None, 0, ctypes.byref(n)))
    out = np.zeros((max(1, n.value), STEP_FEATURES), dtype=np.float32)
    _check(library().tn_plan_step_features(plan.handle, _fptr(out), n.value, ctypes.byref(n)))
    return out[:n.value]


class Mlp:
    """Owner of a tn_mlp_t (device weights of the learned step-time model)."""

    def __init__(self, d_in=STEP_FEATURES, hidden=128, seed=0):
        h = ctypes.c_void_p()
        _check(library().tn_mlp_create(int(d_in), int(hidden), int(seed), ctypes.byref(h)))
        self.handle = h
        self.d_in, self.hidden = d_in, hidden

    def close(self):
        if getattr(self, "handle", None):
            library().tn_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self):
        n = ctypes.c_int64()
        _check(library().tn_mlp_num_params(self.handle, ctypes.byref(n)))
        return n.value

    def get_params(self):
        out = np.zeros(self.num_params(), dtype=np.float32)
        _check(library().tn_mlp_get_params(self.handle, _fptr(out), out.size))
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        _check(library().tn_mlp_set_params(self.handle, _fptr(flat), flat.size))

    def forward(self, x, y, stream=None):
        _check(library().tn_mlp_forward(self.handle, ctypes.c_void_p(x.data_ptr()), int(x.shape[0]),
                                        ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)))

    def gradient(self, x, t, stream=None):
        g = np.zeros(self.num_params(), dtype=np.float32)
        loss = ctypes.c_float()
        _check(library().tn_mlp_gradient(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                         int(x.shape[0]), _fptr(g), ctypes.byref(loss), _stream_ptr(stream)))
        return g, loss.value

    def train_step(self, x, t, lr, stream=None):
        loss = ctypes.c_float()
        _check(library().tn_mlp_train_step(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                           int(x.shape[0]), float(lr), ctypes.byref(loss), _stream_ptr(stream)))
        return loss.value

    def set_support(self, fmin, fmax, margin=0.05):
        fmin = np.ascontiguousarray(fmin, dtype=np.float32)
        fmax = np.ascontiguousarray(fmax, dtype=np.float32)
        _check(library().tn_mlp_set_support(self.handle, _fptr(fmin), _fptr(fmax), fmin.size, float(margin)))


def sample_workspace_bytes(n_open):
    return int(library().tn_sample_workspace_bytes(int(n_open)))


def sample(amps, n_open, uniforms, out, ws, stream=None):
    """Inverse-transform samples of P(s2 | s1) from a device tensor of
    2^n_open complex128 amplitudes: uniforms (float64) and out (int64, same
    length) and the workspace ws are caller-owned device tensors."""
    n = int(uniforms.numel())
    if int(out.numel()) != n:
        raise ValueError("out and uniforms must have the same length")
    _check(library().tn_sample(ctypes.c_void_p(amps.data_ptr()), int(n_open), ctypes.c_void_p(uniforms.data_ptr()),
                               n, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel() * ws.element_size(), _stream_ptr(stream)))


def sample_noalloc(amps, n_open, uniforms, out, stream=None):
    """tn_sample with the library's file-scope device workspace (no
    allocation; n_open <= 20; overlapping calls on one GPU race)."""
    n = int(uniforms.numel())
    if int(out.numel()) != n:
        raise ValueError("out and uniforms must have the same length")
    _check(library().tn_sample_noalloc(ctypes.c_void_p(amps.data_ptr()), int(n_open),
                                       ctypes.c_void_p(uniforms.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                                       _stream_ptr(stream)))


def mix_topk(amps, n_qubits, open_q, fixed_q, fixed_bits, k, random_words, out, ws, stream=None):
    """k most probable bitstrings of a device tensor of 2^len(open_q)
    complex128 amplitudes mixed with random ones (random_words: uint64 device
    tensor; out: int64/uint64 device tensor of k + len(random_words) whole
    bitstrings; ws: tn_mix_workspace_bytes bytes).  Returns P_top, F_top and
    F_mix_expected."""
    n_open, n_fixed = len(open_q), len(fixed_q)
    if int(out.numel()) != k + int(random_words.numel()):
        raise ValueError("out must hold k + len(random_words) bitstrings")
    oq = (ctypes.c_int32 * max(1, n_open))(*[int(q) for q in open_q])
    fq = (ctypes.c_int32 * max(1, n_fixed))(*[int(q) for q in fixed_q])
    fb = (ctypes.c_uint8 * max(1, n_fixed))(*[int(b) for b in fixed_bits])
    r = MixResult()
    _check(library().tn_mix_topk(ctypes.c_void_p(amps.data_ptr()), int(n_qubits), oq, n_open, fq, fb, n_fixed,
                                 int(k), ctypes.c_void_p(random_words.data_ptr()), int(random_words.numel()),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel() * ws.element_size(), ctypes.byref(r), _stream_ptr(stream)))
    return {"P_top": r.P_top, "F_top": r.F_top, "F_mix_expected": r.F_mix_expected}


def mix_workspace_bytes(n_open):
    return int(library().tn_mix_workspace_bytes(int(n_open)))


def xeb(amps, n_open, n_qubits, weight=1.0, ks=(), stream=None):
    """Eq. (1) statistics of a device tensor of 2^n_open complex128."""
    lib = library()
    r = XebResult()
    nk = len(ks)
    karr = (ctypes.c_int64 * max(1, nk))(*[int(k) for k in ks])
    out = (ctypes.c_double * max(1, nk))()
    _check(lib.tn_xeb(ctypes.c_void_p(amps.data_ptr()), int(n_open), int(n_qubits), float(weight),
                      karr if nk else None, nk, out if nk else None, ctypes.byref(r), _stream_ptr(stream)))
    d = r.to_dict()
    d["topk"] = [out[i] for i in range(nk)]
    return d
