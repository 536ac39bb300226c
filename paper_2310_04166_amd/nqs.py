"""Thin Python binding of the C ABI in ``include/nqs.h`` (ctypes).

Argument marshalling only: every step of the hot path runs in the HIP library
``libnqs.so``.  Device arrays are torch tensors on the current HIP device;
configurations travel as ``torch.int64`` tensors holding the uint64 bit
strings.  The library must be built (``python -m paper_2310_04166_amd.build``);
loading fails loudly if it is missing.

One VMC step (the paper's loop: sample, local energy, gradient, Adam)::

    ham = ham_compile(h, eri, n_alpha, n_beta)            # FP64 integrals, host
    model = Model(MODEL_TRANSFORMER, dims, params, "bf16")  # or MODEL_NADE, "fp32", ...
    x, counts, lost = sample_unique(model, n_samples, seed)
    la, ph = amp_forward(model, x)
    eloc, sums, n_pairs = local_energy(ham, model, x, counts, la, ph)
    g_la, g_ph = vmc_weights(eloc, counts, sums)
    grad = amp_backward(model, x, g_la, g_ph)
    adam_update(model.params_ptr(), grad, m, v, lr=1e-3, t=step)
    model.sync()

``AmpFn`` puts the same forward and hand-written backward behind
torch.autograd; ``Batch`` runs many molecules through one captured step.
"""
import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NQS_LIB", os.path.join(_HERE, "libnqs.so"))

MODEL_MLP, MODEL_TRANSFORMER, MODEL_NADE, MODEL_TABLE = 1, 2, 3, 4
FP64, FP32, BF16 = 1, 2, 3
MU, DU, MUD = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16}
STRATEGIES = {"MU": MU, "DU": DU, "MUd": MUD}

_STATUS = {-1: "EINVAL", -2: "ECAPACITY", -3: "EUNSUPPORTED", -4: "EHIP", -5: "ENOMEM"}


class NQSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None
_vp, _i64, _i32, _u64, _dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_double
_SIGS = {
    "nqs_last_error": ([], C.c_char_p),
    "ham_compile": ([_vp, _vp, C.c_int, _dbl, C.c_int, C.c_int, C.POINTER(_vp)], C.c_int),
    "ham_info": ([_vp, C.POINTER(_i64), C.POINTER(_i64)], C.c_int),
    "ham_tables": ([_vp, _vp, _vp, _vp, _vp], C.c_int),
    "ham_destroy": ([_vp], None),
    "ham_z2_symmetries": ([_vp, C.c_int, _vp, C.POINTER(_i32)], C.c_int),
    "amp_model_create": ([C.c_int, _vp, C.c_int, _vp, _i64, C.c_int, C.c_int, C.c_int,
                          C.POINTER(_vp)], C.c_int),
    "amp_model_info": ([_vp, C.POINTER(_i64), C.POINTER(_i32)], C.c_int),
    "amp_model_params": ([_vp, C.POINTER(_vp)], C.c_int),
    "amp_model_sync": ([_vp, _vp], C.c_int),
    "amp_model_get_params": ([_vp, _vp], C.c_int),
    "amp_model_set_params": ([_vp, _vp], C.c_int),
    "amp_model_destroy": ([_vp], None),
    "amp_forward": ([_vp, _vp, _i64, _vp, _vp, _vp], C.c_int),
    "amp_backward": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp], C.c_int),
    "sample_unique": ([_vp, _u64, _u64, _vp, _vp, _i64, C.POINTER(_i64), C.POINTER(_u64), _vp],
                      C.c_int),
    "connected_pairs": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp, _i64, C.POINTER(_i64), _vp], C.c_int),
    "connected_pairs_noalloc": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp, _i64, C.POINTER(_i64), _vp],
                                C.c_int),
    "local_energy": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, C.POINTER(_i64), _vp],
                     C.c_int),
    "local_energy_stats": ([_vp, C.POINTER(_i64), C.POINTER(_i64)], C.c_int),
    "vmc_weights": ([_vp, _vp, _i64, _vp, _vp, _vp, _vp], C.c_int),
    "adam_update": ([_vp, _vp, _vp, _vp, _i64, C.c_int, _dbl, _dbl, _dbl, _dbl, _i64, _vp],
                    C.c_int),
    "amp_model_set_sectors": ([_vp, C.c_int, _vp, _vp, _vp], C.c_int),
    "amp_model_set_z2": ([_vp, C.c_int, _vp, _vp], C.c_int),
    "amp_model_set_prefix_sharing": ([_vp, C.c_int], C.c_int),
    "amp_model_tree_rows": ([_vp, C.POINTER(_i64), C.POINTER(_i64)], C.c_int),
    "amp_model_set_mixed_backward": ([_vp, C.c_int], C.c_int),
    "amp_model_set_symmetries": ([_vp, C.c_int, _vp, _vp, C.c_int, _vp, _vp], C.c_int),
    "sample_unique_batch": ([_vp, C.c_int, _vp, _u64, _vp, _vp, _i64, C.POINTER(_i64), _vp,
                             C.POINTER(_u64), _vp], C.c_int),
    "batch_create": ([_vp, C.c_int, _vp, C.POINTER(_vp)], C.c_int),
    "batch_set_table": ([_vp, _i64], C.c_int),
    "batch_destroy": ([_vp], None),
    "batch_info": ([_vp, _vp, _vp], C.c_int),
    "batch_local_energy": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_i64), _vp],
                           C.c_int),
    "batch_set_mode": ([_vp, C.c_int, C.c_int], C.c_int),
    "batch_set_tile": ([_vp, C.c_int, C.c_int, C.c_int], C.c_int),
    "batch_stats": ([_vp, C.POINTER(_i64), C.POINTER(_i64), _vp, C.POINTER(_i64), _vp, _vp,
                     C.c_int], C.c_int),
    "vmc_weights_batch": ([_vp, _vp, _vp, _i64, _vp, C.c_int, _vp, _vp, _vp], C.c_int),
    "nqs_timing_enable": ([C.c_int], C.c_int),
    "nqs_timing_read": ([C.POINTER(_dbl), C.POINTER(_i64), C.POINTER(_i64)], C.c_int),
    "nqs_timing_read_mode": ([C.c_int, C.POINTER(_dbl), C.POINTER(_i64), C.POINTER(_i64)], C.c_int),
    "nqs_sampler_device_walk": ([C.c_int], C.c_int),
}
EXPORTS = tuple(_SIGS)


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2310_04166_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes, f.restype = args, res
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise NQSError(status, lib().nqs_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype):
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
    return t


class Hamiltonian:
    """A compiled Hamiltonian (``ham_compile``)."""

    def __init__(self, h1, eri, n_alpha, n_beta, e_core=0.0):
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        self.n = h1.shape[0]
        self.n_alpha, self.n_beta = n_alpha, n_beta
        h = _vp()
        _check(lib().ham_compile(_ptr(h1), _ptr(eri), self.n, float(e_core), n_alpha, n_beta,
                                 C.byref(h)))
        self.handle = h

    def info(self):
        G, T = _i64(), _i64()
        _check(lib().ham_info(self.handle, C.byref(G), C.byref(T)))
        return G.value, T.value

    def z2_symmetries(self, max_gen=16):
        """Qubit masks of the Hamiltonian's Z2 symmetries beyond the electron
        parities (``ham_z2_symmetries``)."""
        masks = np.zeros(max_gen, np.uint64)
        n = _i32()
        _check(lib().ham_z2_symmetries(self.handle, max_gen, _ptr(masks), C.byref(n)))
        return [int(v) for v in masks[:n.value]]

    def tables(self):
        G, T = self.info()
        flip = np.zeros(G, np.uint64)
        off = np.zeros(G + 1, np.int64)
        z = np.zeros(T, np.uint64)
        c = np.zeros(T, np.float64)
        _check(lib().ham_tables(self.handle, _ptr(flip), _ptr(off), _ptr(z), _ptr(c)))
        return flip, off, z, c

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ham_destroy(self.handle)
            self.handle = None


def ham_compile(h1, eri, n_alpha, n_beta, e_core=0.0):
    return Hamiltonian(h1, eri, n_alpha, n_beta, e_core)


class Model:
    """An amplitude model (``amp_model_create``)."""

    def __init__(self, kind, dims, params, precision="fp32", strategy="MU", d=0):
        dims_a = np.ascontiguousarray(dims, dtype=np.int32)
        p = np.ascontiguousarray(params, dtype=np.float64)
        h = _vp()
        _check(lib().amp_model_create(kind, _ptr(dims_a), len(dims_a), _ptr(p), len(p),
                                      PRECISIONS[precision], STRATEGIES[strategy], d, C.byref(h)))
        self.handle, self.kind, self.dims = h, kind, list(dims)
        self.precision, self.strategy = precision, strategy
        n, bytes_ = _i64(), _i32()
        _check(lib().amp_model_info(h, C.byref(n), C.byref(bytes_)))
        self.n_params, self.param_bytes = n.value, bytes_.value
        self.param_dtype = torch.float64 if self.param_bytes == 8 else torch.float32

    def params_ptr(self):
        p = _vp()
        _check(lib().amp_model_params(self.handle, C.byref(p)))
        return p.value

    def sync(self, stream=None):
        _check(lib().amp_model_sync(self.handle, _stream(stream)))

    def params_tensor(self):
        """The master parameter vector as a torch tensor aliasing the library's
        device buffer (no copy; valid while the model lives).  After writing
        it, call sync() so that the derived (packed) weights follow."""
        class _Buffer:
            pass
        buf = _Buffer()
        buf.__cuda_array_interface__ = {
            "shape": (self.n_params,), "typestr": "<f8" if self.param_bytes == 8 else "<f4",
            "data": (self.params_ptr(), False), "version": 2}
        return torch.as_tensor(buf, device="cuda")

    def get_params(self):
        out = np.zeros(self.n_params, np.float64)
        _check(lib().amp_model_get_params(self.handle, _ptr(out)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float64)
        assert len(p) == self.n_params
        _check(lib().amp_model_set_params(self.handle, _ptr(p)))

    def set_sectors(self, sectors):
        """Serve several molecules: ``sectors`` = [(n, n_alpha, n_beta), ...]
        (empty = back to the model's own sector)."""
        a = np.ascontiguousarray(np.asarray(sectors, dtype=np.int32).reshape(-1, 3).T)
        _check(lib().amp_model_set_sectors(self.handle, a.shape[1], _ptr(a[0].copy()),
                                           _ptr(a[1].copy()), _ptr(a[2].copy())))

    def set_prefix_sharing(self, on, tree=True):
        """bf16 transformer batches by shared prefixes (default; ``tree``: the
        local energy's tree tail where the sector allows it) or configuration
        by configuration (``amp_model_set_prefix_sharing``)."""
        _check(lib().amp_model_set_prefix_sharing(self.handle, (1 if tree else 2) if on else 0))

    def tree_rows(self):
        """Distinct (n-3)- and (n-2)-token prefixes evaluated so far by the
        local energy's tree tail (``amp_model_tree_rows``)."""
        q, q1 = _i64(), _i64()
        _check(lib().amp_model_tree_rows(self.handle, C.byref(q), C.byref(q1)))
        return q.value, q1.value

    def set_mixed_backward(self, on):
        """bf16 transformer backward on split-bf16 MFMA products (default) or
        fp32 library products (``amp_model_set_mixed_backward``)."""
        _check(lib().amp_model_set_mixed_backward(self.handle, 1 if on else 0))

    def set_z2(self, masks, targets=None):
        """Restrict the sector by Z2 symmetries (``amp_model_set_z2``); targets
        default to the Hartree-Fock determinant's parities."""
        m = np.ascontiguousarray([int(v) for v in masks], dtype=np.uint64)
        t = None if targets is None else np.ascontiguousarray(targets, dtype=np.int32)
        _check(lib().amp_model_set_z2(self.handle, len(m), _ptr(m) if len(m) else None, _ptr(t)))

    def set_symmetries(self, eig=(), targets=(), z2=(), z2_targets=None):
        """Sector by general quantum numbers (amp_model_set_symmetries): ``eig``
        a list of additive symmetries, each 4n integers (qubit q holding bit b
        -> entry 2q + b), ``targets`` their sums; ``z2`` qubit masks with target
        parities ``z2_targets`` (default 0).  No arguments: back to the
        (n_alpha, n_beta) sector."""
        e = np.ascontiguousarray(np.asarray(eig, dtype=np.int32).reshape(-1))
        t = np.ascontiguousarray(targets, dtype=np.int32)
        z = np.ascontiguousarray([int(v) for v in z2], dtype=np.uint64)
        zt = None if z2_targets is None else np.ascontiguousarray(z2_targets, dtype=np.int32)
        _check(lib().amp_model_set_symmetries(self.handle, len(t), _ptr(e) if len(t) else None,
                                              _ptr(t) if len(t) else None, len(z),
                                              _ptr(z) if len(z) else None, _ptr(zt)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.amp_model_destroy(self.handle)
            self.handle = None


def amp_model_create(kind, dims, params, precision="fp32", strategy="MU", d=0):
    return Model(kind, dims, params, precision, strategy, d)


def table_model(n, n_alpha, n_beta, basis, logabs, phase, strategy="MU", d=0):
    """NQS_MODEL_TABLE: psi given on an ascending basis of configurations
    (ints); dims carry the basis as (low, high) 32-bit halves."""
    b = np.ascontiguousarray([int(v) for v in basis], dtype=np.uint64)
    halves = b.view(np.uint32).view(np.int32)            # little-endian: low, high
    dims = np.concatenate([np.asarray([n, n_alpha, n_beta], np.int32), halves])
    params = np.concatenate([np.asarray(logabs, np.float64), np.asarray(phase, np.float64)])
    return Model(MODEL_TABLE, dims, params, "fp64", strategy, d)


def amp_forward(model, x, logabs=None, phase=None, stream=None):
    x = _dev(x, torch.int64)
    n = x.numel()
    logabs = torch.empty(n, dtype=torch.float64, device=x.device) if logabs is None else logabs
    phase = torch.empty(n, dtype=torch.float64, device=x.device) if phase is None else phase
    _check(lib().amp_forward(model.handle, _ptr(x), n, _ptr(logabs), _ptr(phase), _stream(stream)))
    return logabs, phase


def amp_backward(model, x, g_logabs, g_phase, grad=None, stream=None):
    x = _dev(x, torch.int64)
    grad = torch.empty(model.n_params, dtype=model.param_dtype, device=x.device) if grad is None else grad
    _check(lib().amp_backward(model.handle, _ptr(x), x.numel(), _ptr(_dev(g_logabs, torch.float64)),
                              _ptr(_dev(g_phase, torch.float64)), _ptr(grad), _stream(stream)))
    return grad


class AmpFn(torch.autograd.Function):
    """(log|psi(x)|, phase(x)) as a differentiable function of a parameter
    vector theta in the canonical layout: forward = amp_forward with theta
    written into the model (unless theta is model.params_tensor() itself) and
    the derived weights repacked; backward = amp_backward, the hand-written
    backward with activations recomputed.  Usage:
        la, ph = AmpFn.apply(theta, model, x)"""

    @staticmethod
    def forward(ctx, theta, model, x):
        view = model.params_tensor()
        if theta.data_ptr() != view.data_ptr():
            view.copy_(theta.detach().reshape(-1).to(view.dtype))
        model.sync()
        x = _dev(x, torch.int64)
        la, ph = amp_forward(model, x)
        ctx.model, ctx.theta_dtype = model, theta.dtype
        ctx.save_for_backward(x)
        return la, ph

    @staticmethod
    def backward(ctx, g_la, g_ph):
        (x,) = ctx.saved_tensors
        zeros = lambda g: torch.zeros(x.numel(), dtype=torch.float64, device=x.device) if g is None \
            else g.contiguous().to(torch.float64)
        grad = amp_backward(ctx.model, x, zeros(g_la), zeros(g_ph))
        return grad.to(ctx.theta_dtype), None, None


def sample_unique(model, n_samples, seed, capacity=None, stream=None, device="cuda"):
    """Returns (configs int64 tensor, counts int64 tensor, lost)."""
    cap = int(capacity if capacity is not None else min(int(n_samples), 1 << 24))
    configs = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
    counts = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
    nu, lost = _i64(), _u64()
    st = lib().sample_unique(model.handle, int(n_samples), int(seed) & ((1 << 64) - 1),
                             _ptr(configs), _ptr(counts), cap, C.byref(nu), C.byref(lost),
                             _stream(stream))
    if st == -2 and capacity is None:
        return sample_unique(model, n_samples, seed, nu.value, stream, device)
    _check(st)
    return configs[:nu.value], counts[:nu.value], lost.value


TAG_SHIFT = 58


def tag(x, mol):
    """Configuration words of molecule ``mol`` (int64 tensor, bits 58..63)."""
    return x | (int(mol) << TAG_SHIFT)


def untag(x):
    """(occupation bits, molecule index) of tagged words."""
    return x & ((1 << TAG_SHIFT) - 1), (x >> TAG_SHIFT) & 63


def sample_unique_batch(model, n_samples, seed, capacity=None, stream=None, device="cuda"):
    """One tree per molecule of a model with sectors.  Returns (configs, counts,
    offsets (numpy, n_mol + 1), lost)."""
    ns = np.ascontiguousarray(n_samples, dtype=np.uint64)
    n_mol = len(ns)
    cap = int(capacity if capacity is not None else min(int(ns.sum()), 1 << 24))
    configs = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
    counts = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
    offsets = np.zeros(n_mol + 1, dtype=np.int64)
    nu, lost = _i64(), _u64()
    st = lib().sample_unique_batch(model.handle, n_mol, _ptr(ns), int(seed) & ((1 << 64) - 1),
                                   _ptr(configs), _ptr(counts), cap, C.byref(nu), _ptr(offsets),
                                   C.byref(lost), _stream(stream))
    if st == -2 and capacity is None:
        return sample_unique_batch(model, n_samples, seed, nu.value, stream, device)
    _check(st)
    return configs[:nu.value], counts[:nu.value], offsets, lost.value


class Batch:
    """Molecules sharing one transformer (``batch_create``)."""

    def __init__(self, hams, model):
        arr = (C.c_void_p * len(hams))(*[h.handle for h in hams])
        h = _vp()
        _check(lib().batch_create(arr, len(hams), model.handle, C.byref(h)))
        self.handle, self.hams, self.model, self.n_mol = h, list(hams), model, len(hams)

    def info(self):
        k = np.zeros(self.n_mol, np.int64)
        g = np.zeros(self.n_mol, np.int64)
        _check(lib().batch_info(self.handle, _ptr(k), _ptr(g)))
        return k, g

    def set_mode(self, use_graph=True, retune=False):
        _check(lib().batch_set_mode(self.handle, int(bool(use_graph)), int(bool(retune))))

    def set_table(self, slots):
        """Distinct-x' table size of the next call (0 = automatic)."""
        _check(lib().batch_set_table(self.handle, int(slots)))

    def set_tile(self, pairs_blocks, fused_pairs, fused_blocks):
        _check(lib().batch_set_tile(self.handle, pairs_blocks, fused_pairs, fused_blocks))

    def local_energy(self, x, counts, offsets, logabs_x=None, phase_x=None, stream=None):
        """Returns (eloc complex128 [U], sums float64 [n_mol, 4], n_pairs)."""
        x = _dev(x, torch.int64)
        n = x.numel()
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        eloc = torch.empty((max(n, 1), 2), dtype=torch.float64, device=x.device)
        sums = torch.empty((self.n_mol, 4), dtype=torch.float64, device=x.device)
        npairs = _i64()
        _check(lib().batch_local_energy(self.handle, _ptr(x), _ptr(counts), _ptr(off),
                                        _ptr(logabs_x), _ptr(phase_x), _ptr(eloc), _ptr(sums),
                                        C.byref(npairs), _stream(stream)))
        return torch.view_as_complex(eloc[:n]), sums, npairs.value

    def stats(self, n_tune=12):
        p, d, c = _i64(), _i64(), _i64()
        per = np.zeros(self.n_mol, np.int64)
        tile = np.zeros(3, np.int32)
        tm = np.zeros(n_tune, np.float64)
        _check(lib().batch_stats(self.handle, C.byref(p), C.byref(d), _ptr(per), C.byref(c),
                                 _ptr(tile), _ptr(tm), n_tune))
        return {"pairs": p.value, "distinct": d.value, "distinct_per_mol": per,
                "captures": c.value, "tile": tile.tolist(), "tune_ms": tm.tolist()}

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.batch_destroy(self.handle)
            self.handle = None


def vmc_weights_batch(eloc, counts, x, sums, stream=None):
    er = torch.view_as_real(eloc).contiguous()
    n = eloc.numel()
    gl = torch.empty(n, dtype=torch.float64, device=eloc.device)
    gp = torch.empty(n, dtype=torch.float64, device=eloc.device)
    _check(lib().vmc_weights_batch(_ptr(er), _ptr(counts), _ptr(x), n, _ptr(sums),
                                   sums.shape[0], _ptr(gl), _ptr(gp), _stream(stream)))
    return gl, gp


def connected_pairs(ham, x, capacity=None, stream=None):
    """Returns (offsets, xp, hval, hdiag) for configurations x."""
    x = _dev(x, torch.int64)
    n = x.numel()
    off = torch.empty(n + 1, dtype=torch.int64, device=x.device)
    total = _i64()
    if capacity is None:
        st = lib().connected_pairs(ham.handle, _ptr(x), n, _ptr(off), None, None, None, 0,
                                   C.byref(total), _stream(stream))
        if st not in (0, -2):
            _check(st)
        capacity = total.value
    xp = torch.empty(max(capacity, 1), dtype=torch.int64, device=x.device)
    hv = torch.empty(max(capacity, 1), dtype=torch.float64, device=x.device)
    hd = torch.empty(max(n, 1), dtype=torch.float64, device=x.device)
    _check(lib().connected_pairs(ham.handle, _ptr(x), n, _ptr(off), _ptr(xp), _ptr(hv), _ptr(hd),
                                 capacity, C.byref(total), _stream(stream)))
    return off, xp[:total.value], hv[:total.value], hd[:n]


NOALLOC_MAX_CONFIGS = 262144


def connected_pairs_noalloc(ham, x, offsets, xp, hval, hdiag, stream=None):
    """connected_pairs into caller-allocated tensors (offsets n+1 int64, xp /
    hval of equal capacity, hdiag n); the library allocates nothing.  Returns
    the number of pairs."""
    x = _dev(x, torch.int64)
    total = _i64()
    _check(lib().connected_pairs_noalloc(ham.handle, _ptr(x), x.numel(), _ptr(offsets), _ptr(xp),
                                         _ptr(hval), _ptr(hdiag), xp.numel(), C.byref(total),
                                         _stream(stream)))
    return total.value


def local_energy(ham, model, x, counts=None, logabs_x=None, phase_x=None, stream=None):
    """Returns (eloc complex128 tensor [n], sums float64 [4], n_pairs)."""
    x = _dev(x, torch.int64)
    n = x.numel()
    eloc = torch.empty((max(n, 1), 2), dtype=torch.float64, device=x.device)
    sums = torch.empty(4, dtype=torch.float64, device=x.device)
    npairs = _i64()
    _check(lib().local_energy(ham.handle, model.handle, _ptr(x), _ptr(counts), n, _ptr(logabs_x),
                              _ptr(phase_x), _ptr(eloc), _ptr(sums), C.byref(npairs),
                              _stream(stream)))
    return torch.view_as_complex(eloc[:n]), sums, npairs.value


def local_energy_stats(ham):
    """(pairs, distinct x') of the last local_energy call on ``ham``."""
    p, d = _i64(), _i64()
    _check(lib().local_energy_stats(ham.handle, C.byref(p), C.byref(d)))
    return p.value, d.value


def vmc_weights(eloc, counts, sums, stream=None):
    er = torch.view_as_real(eloc).contiguous()
    n = eloc.numel()
    gl = torch.empty(n, dtype=torch.float64, device=eloc.device)
    gp = torch.empty(n, dtype=torch.float64, device=eloc.device)
    _check(lib().vmc_weights(_ptr(er), _ptr(counts), n, _ptr(sums), _ptr(gl), _ptr(gp),
                             _stream(stream)))
    return gl, gp


def adam_update(params_ptr, grad, m, v, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, t=1, stream=None):
    n = grad.numel()
    _check(lib().adam_update(C.c_void_p(params_ptr), _ptr(grad), _ptr(m), _ptr(v), n,
                             grad.element_size(), lr, b1, b2, eps, t, _stream(stream)))


def timing_enable(on=True):
    _check(lib().nqs_timing_enable(1 if on else 0))


def timing_read(mode=None):
    """(milliseconds, launches, configurations) of the fused amplitude kernel:
    every launch, or those of one row layout (TIMING_* below)."""
    ms, nl, nc = _dbl(), _i64(), _i64()
    if mode is None:
        _check(lib().nqs_timing_read(C.byref(ms), C.byref(nl), C.byref(nc)))
    else:
        _check(lib().nqs_timing_read_mode(mode, C.byref(ms), C.byref(nl), C.byref(nc)))
    return ms.value, nl.value, nc.value


def sampler_device_walk(on=True):
    """Frontier sizes of bf16 samplers kept on the device (default) or the
    per-level walk (``nqs_sampler_device_walk``)."""
    _check(lib().nqs_sampler_device_walk(1 if on else 0))


TIMING_PLAIN, TIMING_WIDE, TIMING_TRUNK, TIMING_SUFFIX, TIMING_MID, TIMING_TAIL = 0, 1, 2, 3, 4, 5
TIMING_TREE, TIMING_PHASE = 6, 7
TIMING_NADE = -1


# ---------------------------------------------------------------- models ---

def model_dims(cfg):
    """dims vector of amp_model_create for a workload description."""
    if cfg["model"] in ("mlp", "nade"):
        return [cfg["n"], cfg["n_alpha"], cfg["n_beta"], cfg.get("hidden", 64)]
    d = cfg["d"]
    return [cfg["n"], cfg["n_alpha"], cfg["n_beta"], d, cfg["n_layers"], cfg["n_heads"],
            cfg.get("ffn", 4 * d), cfg.get("phase_hidden", 256)]


def model_kind(cfg):
    return {"mlp": MODEL_MLP, "nade": MODEL_NADE}.get(cfg["model"], MODEL_TRANSFORMER)
