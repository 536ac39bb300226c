"""Choose the initial Hartree-Fock logit bias of a workload.

Runs the oracle's tree sampler on the workload's model for a few bias values
and prints the number of unique samples each gives.  The workloads' ``hf_bias``
values were picked from this output (target: about 3e3 unique samples at 20
spin-orbitals / 1e5 samples, about 2e4 at 30 spin-orbitals / 1e6 samples, for
the transformer and for the paper's per-qubit ansatz alike).

    python -m oracle.calibrate_hf_bias fp32 2.5 3.0 3.5
    python -m oracle.calibrate_hf_bias batching 1.5 2.0 2.5
    python -m oracle.calibrate_hf_bias nade 1.0 1.5 2.0

For ``batching`` the value is the shared model's per-electron bias and the
output lists the unique counts of the first eight molecules.
"""
import sys
import time

from oracle.model import TransformerModel, build_model
from oracle.sampler import sample_tree
from oracle.sector import Sector
from synth import (BATCHING_MODEL, batching_molecules, make_nade_params,
                   make_transformer_params, workload)


def unique_count(name, bias, seed=0):
    cfg, _, _, _ = workload(name)
    if cfg["model"] == "nade":
        params = make_nade_params(cfg["n"], cfg["hidden"], seed=cfg["seed"], std=cfg["std"],
                                  n_alpha=cfg["n_alpha"], n_beta=cfg["n_beta"], hf_bias=bias,
                                  round_to=cfg.get("round_to"))
        configs, _, _ = sample_tree(build_model(cfg, params), cfg["n_samples"], seed)
        return len(configs)
    params = make_transformer_params(cfg["n"], cfg["n_alpha"], cfg["n_beta"], cfg["d"],
                                     cfg["n_layers"], seed=cfg["seed"], hf_bias=bias,
                                     round_to=cfg.get("round_to"))
    model = build_model(cfg, params)
    configs, counts, _ = sample_tree(model, cfg["n_samples"], seed)
    return len(configs)


def batching_unique_counts(bias, count=8, seed=0):
    c = BATCHING_MODEL
    params = make_transformer_params(c["n"], 0, 0, c["d"], c["n_layers"], ffn=c["ffn"],
                                     phase_hidden=c["phase_hidden"], seed=c["seed"],
                                     occ_bias=bias, round_to=c["round_to"])
    out = []
    for i, m in enumerate(batching_molecules()[:count]):
        model = TransformerModel(params, Sector(m["n"], m["n_alpha"], m["n_beta"]), c["n_heads"])
        configs, _, _ = sample_tree(model, m["n_samples"], seed, stream=i)
        out.append(len(configs))
    return out


if __name__ == "__main__":
    name = sys.argv[1]
    for b in sys.argv[2:]:
        if name == "batching":
            print(name, b, batching_unique_counts(float(b)), flush=True)
            continue
        t = time.time()
        print(name, b, unique_count(name, float(b)), f"{time.time() - t:.1f}s", flush=True)
