"""Seeded initial parameters of the two amplitude networks, and their flat order.

The flat order returned by ``*_param_spec`` is the canonical parameter vector
layout that the C ABI takes (``amp_model_create``) and that ``amp_backward``
writes gradients in.  Matrices are stored row-major with shape (in, out), so a
layer computes ``y = x @ W + b``.

Initial values: weights N(0, std), biases and layer-norm shifts 0 (or
N(0, bias_std) when asked, for tests away from activation kinks), gains 1,
and for the transformer a per-position logit bias that is ``hf_bias`` on the
Hartree-Fock token of each position and 0 elsewhere (the knob that sets how
peaked the initial distribution is).  Every value is representable in float32;
with ``round_to="bf16"`` every weight is also representable in bfloat16.
"""
import numpy as np


def mlp_param_spec(n, hidden=64):
    """Per-token MLP (one subnetwork per spatial orbital, NADE-like).

    Subnetwork p reads the one-hot codes of tokens 0..p-1 (4p inputs) and
    produces 4 logits followed by 4 phases.
    """
    spec = []
    for p in range(n):
        spec += [(f"mlp{p}.w1", (4 * p, hidden)), (f"mlp{p}.b1", (hidden,)),
                 (f"mlp{p}.w2", (hidden, hidden)), (f"mlp{p}.b2", (hidden,)),
                 (f"mlp{p}.w3", (hidden, 8)), (f"mlp{p}.b3", (8,))]
    return spec


def transformer_param_spec(n, d, n_layers, ffn, phase_hidden=256):
    """Decoder-only transformer over n orbital tokens plus a phase MLP."""
    spec = [("tok_emb", (5, d)), ("pos_emb", (n, d))]
    for l in range(n_layers):
        spec += [(f"l{l}.ln1_g", (d,)), (f"l{l}.ln1_b", (d,)),
                 (f"l{l}.wqkv", (d, 3 * d)), (f"l{l}.bqkv", (3 * d,)),
                 (f"l{l}.wo", (d, d)), (f"l{l}.bo", (d,)),
                 (f"l{l}.ln2_g", (d,)), (f"l{l}.ln2_b", (d,)),
                 (f"l{l}.w1", (d, ffn)), (f"l{l}.b1", (ffn,)),
                 (f"l{l}.w2", (ffn, d)), (f"l{l}.b2", (d,))]
    spec += [("lnf_g", (d,)), ("lnf_b", (d,)), ("whead", (d, 4)), ("bhead", (4,)),
             ("logit_bias", (n, 4)),
             ("ph_w1", (4 * n, phase_hidden)), ("ph_b1", (phase_hidden,)),
             ("ph_w2", (phase_hidden, phase_hidden)), ("ph_b2", (phase_hidden,)),
             ("ph_w3", (phase_hidden, 1)), ("ph_b3", (1,))]
    return spec


def _round(a, round_to):
    a = np.asarray(a, dtype=np.float32)
    if round_to == "bf16":
        u = a.view(np.uint32).astype(np.uint64)
        u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16   # round to nearest even
        a = u.astype(np.uint32).view(np.float32)
    return a.astype(np.float64)


def _init(spec, seed, std, round_to, special, bias_std=0.0):
    rng = np.random.default_rng([seed, 0x5EED])
    out = {}
    for name, shape in spec:
        base = name.split(".")[-1]
        if name in special:
            val = special[name]
        elif base.endswith("_g"):
            val = np.ones(shape)
        elif base.startswith("b") or base.endswith("_b") or "_b" in base:
            val = rng.normal(0.0, bias_std, size=shape) if bias_std else np.zeros(shape)
        else:
            val = rng.normal(0.0, std, size=shape)
        out[name] = _round(val, round_to).reshape(shape)
    return out


def make_mlp_params(n, hidden=64, seed=0, std=0.02, round_to=None, bias_std=0.0):
    return _init(mlp_param_spec(n, hidden), seed, std, round_to, {}, bias_std)


def make_transformer_params(n, n_alpha, n_beta, d, n_layers, ffn=None,
                            phase_hidden=256, seed=0, std=0.02, hf_bias=0.0,
                            round_to=None, bias_std=0.0, occ_bias=0.0):
    """``hf_bias`` favours each position's Hartree-Fock token of the sector
    (n_alpha, n_beta).  ``occ_bias`` instead adds ``occ_bias`` per electron of
    the token (0, 1, 1, 2 for tokens 0..3) at every position, which favours
    the Hartree-Fock state of *any* sector under the symmetry mask; it is the
    knob of a model shared by molecules of different electron counts."""
    ffn = 4 * d if ffn is None else ffn
    bias = np.zeros((n, 4))
    for p in range(n):
        hf_tok = int(p < n_alpha) + 2 * int(p < n_beta)
        bias[p, hf_tok] = hf_bias
        bias[p] += occ_bias * np.array([0.0, 1.0, 1.0, 2.0])
    spec = transformer_param_spec(n, d, n_layers, ffn, phase_hidden)
    return _init(spec, seed, std, round_to, {"logit_bias": bias}, bias_std)


def flatten_params(params, spec, dtype=np.float64):
    return np.concatenate([np.asarray(params[k], dtype=dtype).reshape(-1)
                           for k, _ in spec]) if spec else np.zeros(0, dtype)


def unflatten_params(flat, spec):
    out, o = {}, 0
    for name, shape in spec:
        size = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + size]).reshape(shape)
        o += size
    assert o == len(flat), (o, len(flat))
    return out


def nade_param_spec(n, hidden=64):
    """The paper's per-qubit ansatz: one complex-weight MLP per qubit i of the
    2n, reading the i previous bits, two hidden layers of width ``hidden`` and
    two complex outputs.  Real and imaginary parts are separate real tensors,
    matrices (in, out)."""
    spec = []
    for i in range(2 * n):
        for part in ("re", "im"):
            spec.append((f"nade{i}.w1_{part}", (i, hidden)))
        for part in ("re", "im"):
            spec.append((f"nade{i}.b1_{part}", (hidden,)))
        for part in ("re", "im"):
            spec.append((f"nade{i}.w2_{part}", (hidden, hidden)))
        for part in ("re", "im"):
            spec.append((f"nade{i}.b2_{part}", (hidden,)))
        for part in ("re", "im"):
            spec.append((f"nade{i}.w3_{part}", (hidden, 2)))
        for part in ("re", "im"):
            spec.append((f"nade{i}.b3_{part}", (2,)))
    return spec


def make_nade_params(n, hidden=64, seed=0, std=0.1, bias_std=0.0, round_to=None,
                     n_alpha=0, n_beta=0, hf_bias=0.0):
    """Weights N(0, std) (real and imaginary parts drawn independently, in spec
    order), biases N(0, bias_std).  ``hf_bias`` is added to the real output bias
    of each qubit's Hartree-Fock value in the sector (n_alpha, n_beta): qubit
    2p + s is occupied when p < n_alpha (s = 0) or p < n_beta (s = 1)."""
    params = _init(nade_param_spec(n, hidden), seed, std, round_to, {}, bias_std)
    if hf_bias:
        for i in range(2 * n):
            p, s = divmod(i, 2)
            occupied = int(p < (n_alpha if s == 0 else n_beta))
            params[f"nade{i}.b3_re"][occupied] += hf_bias
    return params
