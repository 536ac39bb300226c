"""The six synthetic workloads, shaped like the paper's molecules.

* ``tiny``      - 12 spin-orbitals, 2+2 electrons (LiH-sized sector of 225), MLP.
* ``fp32``      - 20 spin-orbitals, 5+5 electrons (sector 63,504), small transformer.
* ``precision`` - 30 spin-orbitals, 7+7 electrons (Li2O-sized sector 41,409,225),
                  d_model 128 / 4 layers / 8 heads transformer, bf16 GEMMs.
* ``batching``  - 64 molecules of 12..28 spin-orbitals sharing one d_model 64 model.
* ``grad``      - the ``precision`` system, full step plus gradient check.
* ``nade``      - the ``precision`` system with the paper's per-qubit ansatz
                  (complex weights, hidden width 64, 30 qubits), bf16 fused forward.

``hf_bias`` is the initial logit bias on each position's Hartree-Fock token.  It
sets how peaked the initial Born distribution is and therefore how many unique
samples a batch of ``n_samples`` produces; its values were chosen with the CPU
oracle's sampler (``oracle/calibrate_hf_bias.py``) to give about 3e3 unique
samples at ``fp32`` and about 2e4 at ``precision``.  The batching workload's
shared model uses the per-electron ``occ_bias`` instead (same script), chosen
so that the molecules' unique counts spread over roughly 1e2 .. 3e3.
"""
import numpy as np

from .integrals import make_integrals
from .params import make_mlp_params, make_nade_params, make_transformer_params

WORKLOADS = {
    "tiny": dict(n=6, n_alpha=2, n_beta=2, rank=12, seed=1, model="mlp",
                 hidden=64, n_samples=10_000, precision="fp64"),
    "fp32": dict(n=10, n_alpha=5, n_beta=5, rank=20, seed=2, model="transformer",
                 d=64, n_layers=2, n_heads=4, n_samples=100_000, precision="fp32",
                 hf_bias=2.7),
    "precision": dict(n=15, n_alpha=7, n_beta=7, rank=30, seed=3, model="transformer",
                      d=128, n_layers=4, n_heads=8, n_samples=1_000_000,
                      precision="bf16", hf_bias=3.3, round_to="bf16"),
    "nade": dict(n=15, n_alpha=7, n_beta=7, rank=30, seed=3, model="nade", hidden=64,
                 std=0.1, n_samples=1_000_000, precision="bf16", hf_bias=1.5,
                 round_to="bf16"),
    "grad": dict(n=15, n_alpha=7, n_beta=7, rank=30, seed=3, model="transformer",
                 d=128, n_layers=4, n_heads=8, n_samples=1_000_000,
                 precision="bf16", hf_bias=3.3, round_to="bf16", fd_params=100,
                 fd_seed=5),
}


def workload(name):
    """Return ``(cfg, h, eri, params)`` for a named single-molecule workload."""
    cfg = dict(WORKLOADS[name])
    h, eri = make_integrals(cfg["n"], cfg["rank"], cfg["seed"])
    if cfg["model"] == "mlp":
        params = make_mlp_params(cfg["n"], cfg["hidden"], seed=cfg["seed"])
    elif cfg["model"] == "nade":
        params = make_nade_params(cfg["n"], cfg["hidden"], seed=cfg["seed"], std=cfg["std"],
                                  n_alpha=cfg["n_alpha"], n_beta=cfg["n_beta"],
                                  hf_bias=cfg["hf_bias"], round_to=cfg.get("round_to"))
    else:
        params = make_transformer_params(
            cfg["n"], cfg["n_alpha"], cfg["n_beta"], cfg["d"], cfg["n_layers"],
            seed=cfg["seed"], hf_bias=cfg["hf_bias"], round_to=cfg.get("round_to"))
    return cfg, h, eri, params


BATCHING_MODEL = dict(n=14, d=64, n_layers=2, n_heads=4, ffn=256, phase_hidden=256,
                      seed=4, occ_bias=2.0, round_to="bf16")


def batching_params():
    """Shared transformer of the batching workload: 14 positions (the largest
    molecule), d_model 64, 2 layers, 4 heads, electron-count logit bias."""
    c = BATCHING_MODEL
    return make_transformer_params(c["n"], 0, 0, c["d"], c["n_layers"], ffn=c["ffn"],
                                   phase_hidden=c["phase_hidden"], seed=c["seed"],
                                   occ_bias=c["occ_bias"], round_to=c["round_to"])


def batching_workload(count=64, base_seed=1000):
    """``(molecules, params)``: each molecule dict also carries its integrals
    ``h``, ``eri``; ``params`` is the shared model."""
    mols = batching_molecules(count, base_seed)
    for m in mols:
        m["h"], m["eri"] = make_integrals(m["n"], m["rank"], m["seed"])
    return mols, batching_params()


def batching_molecules(count=64, base_seed=1000):
    """Molecule list of the batching workload.

    Molecule i uses seed ``base_seed + i``; its spin-orbital count is uniform
    over {12, 16, 20, 24, 28}; electrons per spin are drawn independently and
    uniformly from {n/2 - 1, n/2, n/2 + 1} (n = spatial orbitals); the sample
    count is log-uniform in [1e4, 1e5].
    """
    mols = []
    for i in range(count):
        rng = np.random.default_rng([base_seed + i, 0xBA7C])
        n = int(rng.choice([6, 8, 10, 12, 14]))
        na = int(n // 2 + rng.integers(-1, 2))
        nb = int(n // 2 + rng.integers(-1, 2))
        ns = int(round(10 ** rng.uniform(4.0, 5.0)))
        mols.append(dict(n=n, n_alpha=na, n_beta=nb, rank=2 * n,
                         seed=base_seed + i, n_samples=ns))
    return mols
