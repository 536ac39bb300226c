"""The hand-written backward behind torch.autograd (nqs.AmpFn): gradients of
(log|psi|, phase) with respect to the canonical parameter vector, checked by
torch.autograd.gradcheck (FP64 central differences of the library's own
forward) and against amp_backward called directly."""
import numpy as np
import pytest
import torch

from oracle.sector import Sector
from synth import (flatten_params, make_mlp_params, make_nade_params, make_transformer_params,
                   mlp_param_spec, nade_param_spec, transformer_param_spec)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    mod.lib()
    return mod


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.uint64).view(np.int64)).cuda()


def test_params_tensor_aliases_the_model(nqs):
    params = make_mlp_params(3, 8, seed=1, std=0.3)
    flat = flatten_params(params, mlp_param_spec(3, 8))
    m = nqs.Model(nqs.MODEL_MLP, [3, 1, 1, 8], flat, "fp64")
    view = m.params_tensor()
    assert view.numel() == m.n_params and view.dtype == torch.float64
    assert np.array_equal(view.cpu().numpy(), flat)
    view.mul_(2.0)
    m.sync()
    assert np.array_equal(m.get_params(), 2.0 * flat)


@pytest.mark.parametrize("kind", ["mlp", "nade"])
def test_gradcheck_fp64(nqs, kind):
    if kind == "mlp":
        n, na, nb, hid = 3, 1, 1, 8
        params = make_mlp_params(n, hid, seed=2, std=0.3, bias_std=0.1)
        flat, k = flatten_params(params, mlp_param_spec(n, hid)), nqs.MODEL_MLP
    else:
        n, na, nb, hid = 2, 1, 1, 4
        params = make_nade_params(n, hid, seed=3, std=0.3, bias_std=0.1)
        flat, k = flatten_params(params, nade_param_spec(n, hid)), nqs.MODEL_NADE
    m = nqs.Model(k, [n, na, nb, hid], flat, "fp64")
    x = dev(Sector(n, na, nb).enumerate())
    theta = torch.tensor(flat, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda th: nqs.AmpFn.apply(th, m, x), (theta,), eps=1e-6,
                                    atol=1e-7, rtol=1e-5)


def test_autograd_equals_amp_backward_bf16_transformer(nqs):
    """A bf16 transformer through autograd: the gradient of a weighted sum of
    log|psi| and phase equals amp_backward with the same weights."""
    n, na, nb, d = 6, 2, 2, 64
    params = make_transformer_params(n, na, nb, d, 1, seed=4, std=0.05, round_to="bf16")
    flat = flatten_params(params, transformer_param_spec(n, d, 1, 4 * d, 256))
    m = nqs.Model(nqs.MODEL_TRANSFORMER, [n, na, nb, d, 1, 4, 4 * d, 256], flat, "bf16")
    x = dev(Sector(n, na, nb).enumerate())
    rng = np.random.default_rng(0)
    gl = torch.tensor(rng.normal(size=x.numel()), device="cuda")
    gp = torch.tensor(rng.normal(size=x.numel()), device="cuda")
    theta = m.params_tensor().clone().requires_grad_(True)
    la, ph = nqs.AmpFn.apply(theta, m, x)
    ((gl * la).sum() + (gp * ph).sum()).backward()
    want = nqs.amp_backward(m, x, gl, gp)
    assert torch.equal(theta.grad, want)
