"""The bf16 transformer's backward on split-bf16 MFMA products (every fp32
operand split into bf16 hi + lo parts, three products with fp32 accumulation,
bias / residual / GELU and its derivative in the products' epilogues) against
the same backward on fp32 library products and against the FP64 oracle's
gradient of the surrogate sum_l g_l log|psi_l| + h_l phi_l (Variational Monte
Carlo gradient)."""
import numpy as np
import pytest
import torch

from oracle.model import TransformerModel
from oracle.sector import Sector
from synth import flatten_params, make_transformer_params, transformer_param_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    mod.lib()
    return mod


def log(msg):
    print(msg, flush=True)


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.uint64).view(np.int64)).cuda()


def sector_configs(n, na, nb, count, seed):
    """Up to `count` distinct configurations of the sector, sorted."""
    rng = np.random.default_rng(seed)
    out = set()
    for _ in range(count):
        a = rng.choice(n, na, replace=False)
        b = rng.choice(n, nb, replace=False)
        out.add(int(sum(1 << (2 * int(p)) for p in a) | sum(1 << (2 * int(p) + 1) for p in b)))
    return sorted(out)


# (n, n_alpha, n_beta, d, layers, configurations drawn): several 128-row
# blocks of token rows with a ragged tail; at d 64 the QKV product's 192
# columns end in a partial 128-column chunk; a batch of a few configurations
@pytest.mark.parametrize("n,na,nb,d,L,count", [(15, 7, 7, 128, 4, 3001), (10, 5, 5, 64, 2, 777),
                                               (6, 2, 2, 64, 1, 5)])
def test_mixed_backward_vs_fp32_products_and_oracle(nqs, n, na, nb, d, L, count):
    H = d // 16
    params = make_transformer_params(n, na, nb, d, L, seed=31, std=0.05, round_to="bf16",
                                     bias_std=0.02)
    spec = transformer_param_spec(n, d, L, 4 * d, 256)
    m = nqs.Model(nqs.MODEL_TRANSFORMER, [n, na, nb, d, L, H, 4 * d, 256],
                  flatten_params(params, spec), "bf16")
    xs = sector_configs(n, na, nb, count, 7)
    x = dev(xs)
    rng = np.random.default_rng(3)
    gl = rng.normal(size=len(xs))
    gp = rng.normal(size=len(xs))
    gl_d, gp_d = torch.tensor(gl).cuda(), torch.tensor(gp).cuda()
    g_mx = nqs.amp_backward(m, x, gl_d, gp_d).double().cpu().numpy()
    m.set_mixed_backward(False)
    g32 = nqs.amp_backward(m, x, gl_d, gp_d).double().cpu().numpy()
    m.set_mixed_backward(True)
    scale = np.max(np.abs(g32))
    err = np.max(np.abs(g_mx - g32))
    log(f"n={n} d={d} L={L}: {len(xs)} configurations, max|g| {scale:.3e}, "
        f"max|g_mixed - g_fp32| {err:.3e} ({err / scale:.2e} of max|g|)")
    assert np.all(np.isfinite(g_mx))
    # about 2^-16 relative per product, summed over rows with mixed signs
    assert err <= 1e-4 * scale
    # the FP64 oracle on up to 64 of the configurations
    k = min(64, len(xs))
    ref = TransformerModel(params, Sector(n, na, nb), H, requires_grad=True)
    la, ph = ref.amplitudes(xs[:k])
    (torch.sum(torch.tensor(gl[:k]) * la) + torch.sum(torch.tensor(gp[:k]) * ph)).backward()
    g_ref = ref.flat_grad(spec)
    g_mk = nqs.amp_backward(m, x[:k].contiguous(), gl_d[:k].contiguous(),
                            gp_d[:k].contiguous()).double().cpu().numpy()
    e_ref = np.max(np.abs(g_mk - g_ref))
    log(f"  vs oracle ({k} configurations): max err {e_ref:.3e} "
        f"({e_ref / np.max(np.abs(g_ref)):.2e} of max|g|)")
    assert e_ref <= 1e-4 * np.max(np.abs(g_ref))
