"""Lost and unique samples of the pruning strategies during optimisation.

A synthetic analogue of the paper's comparison of Mask-Unphysical on all but
the last two levels (MU-2) with Discard-Unphysical (DU) ("Experiments",
pruning strategies): from the same initial parameters, each strategy drives its
own optimisation (library step, Adam in its default configuration, 1e5 samples
per iteration as in the first iterations of the paper's schedule) on the
20-spin-orbital, 5+5-electron system with the fp32 transformer.  The energy
and gradient use the paper's estimator, which divides by N_s (its energy
equation): lost samples count as zero, so probability outside the sector costs
energy.  The reducer divides by the sum of the counts W; replacing W by N_s in
the sums before vmc_weights gives the paper's form (identical under MU).  The
paper's finding is that MU-2 loses fewer samples and produces more unique
samples than DU; both are asserted over the run.  Parity with the oracle of
the sampler under DU and MU-d is covered by test_gpu_parity.py.
"""
import numpy as np
import pytest
import torch

from synth import flatten_params, transformer_param_spec, workload

pytestmark = pytest.mark.gpu

ITERATIONS = 150


def run(nqs, strategy, d):
    cfg, h, eri, params = workload("fp32")
    ham = nqs.ham_compile(h, eri, cfg["n_alpha"], cfg["n_beta"])
    spec = transformer_param_spec(cfg["n"], cfg["d"], cfg["n_layers"], 4 * cfg["d"], 256)
    model = nqs.Model(nqs.MODEL_TRANSFORMER, nqs.model_dims(cfg), flatten_params(params, spec),
                      "fp32", strategy, d)
    grad = torch.zeros(model.n_params, dtype=torch.float32, device="cuda")
    m, v = torch.zeros_like(grad), torch.zeros_like(grad)
    lost, unique, energy = [], [], []
    for t in range(1, ITERATIONS + 1):
        x, c, n_lost = nqs.sample_unique(model, cfg["n_samples"], t)
        assert int(c.sum()) + n_lost == cfg["n_samples"]
        la, ph = nqs.amp_forward(model, x)
        eloc, sums, _ = nqs.local_energy(ham, model, x, c, la, ph)
        w = float(sums[0])
        sums[0] = float(cfg["n_samples"])       # the paper's normalisation by N_s
        gl, gp = nqs.vmc_weights(eloc, c, sums)
        grad = nqs.amp_backward(model, x, gl, gp, grad=grad)
        nqs.adam_update(model.params_ptr(), grad, m, v, lr=1e-3, t=t)
        model.sync()
        s = sums.cpu().numpy()
        lost.append(n_lost)
        unique.append(x.numel())
        energy.append(s[1] / w)                 # energy of the in-sector part
    return np.array(lost), np.array(unique), np.array(energy)


def test_mu2_loses_fewer_and_keeps_more_unique_samples():
    from paper_2310_04166_amd import nqs
    nqs.lib()
    assert torch.cuda.is_available()
    du = run(nqs, "DU", 0)
    mu2 = run(nqs, "MUd", 2)
    for name, (lost, unique, energy) in (("DU", du), ("MU-2", mu2)):
        for t in (0, 9, 49, 99, ITERATIONS - 1):
            print(f"{name:5s} iteration {t + 1:4d}: lost {lost[t]:6d} of 1e5, unique {unique[t]:5d}, "
                  f"E {energy[t]:.5f}", flush=True)
        print(f"{name:5s} total lost {lost.sum()}, mean unique {unique.mean():.0f}", flush=True)
    assert du[0][0] > 0                          # DU loses samples from the start
    assert mu2[0].sum() < du[0].sum()            # MU-2 loses fewer samples
    assert mu2[1].mean() > du[1].mean()          # and keeps more unique ones
    # both optimisations lower the energy
    assert du[2][-10:].mean() < du[2][:10].mean()
    assert mu2[2][-10:].mean() < mu2[2][:10].mean()
