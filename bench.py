"""Benchmark: full VMC steps of the 30-spin-orbital workload on one MI355X.

A step is one pass of the whole hot path over one batch:
    sample_unique (1e6 samples -> ~2e4 unique, Mask-Unphysical tree on the GPU)
    amp_forward   (log|psi|, phase of the unique samples)
    local_energy  (bit kernel -> ~9e7 connected (x, x') pairs -> fused bf16
                   amplitude kernel on every x' -> ratios, double accumulation)
    vmc_weights + amp_backward (hand-written backward, activations recomputed)
    adam_update + repack of the bf16 weights
Inputs are seeded synthetic integrals and a random-initialised transformer
(d_model 128, 4 layers, 8 heads), resident in HBM before the timed region.

Prints one JSON line.  `value` = connected (x, x') pairs per second of the
whole step (the E_loc evals/s metric measured over complete steps).

--workload nade: the same system and step with the paper's per-qubit
complex-weight ansatz (hidden width 64) and its fused bf16 kernel; the roofline
is then the VALU bound of that kernel.  --workload batching: 64 molecules in
one graph-captured step (run_batching).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic multiply-adds of one amplitude evaluation of the 30-qubit model:
# 15 tokens x 4 layers x 12 d^2 + causal attention 4 x 2 x d T(T+1)/2
# + head 15 x 4 d + phase MLP 256^2 + 256
FLOP_PER_CONFIG = 2 * (15 * 4 * 12 * 128 ** 2 + 4 * 2 * 128 * 120 + 15 * 4 * 128 + 256 * 256 + 256)
BF16_PEAK_TFLOPS = 2500.0
# positions of a shared prefix (the library evaluates positions 0..7 once per
# distinct 8-token prefix, positions 8.. per configuration)
TRUNK = 8


def rows_flop(t0, t1, d, n_layers, ffn, ph, phase):
    """Multiply-adds x 2 of positions t0 .. t1 - 1 of one configuration: per
    position and layer 4 d^2 + 2 d ffn, causal attention 2 d (t + 1) per query t
    and layer, the head 4 d per position; the phase MLP ph^2 + ph if asked for.
    rows_flop(0, n, ...) with the phase MLP is one whole evaluation."""
    pos = t1 - t0
    keys = sum(t + 1 for t in range(t0, t1))
    return 2 * (pos * n_layers * (4 * d * d + 2 * d * ffn) + n_layers * 2 * d * keys
                + pos * 4 * d + ((ph * ph + ph) if phase else 0))

# The per-qubit ansatz (workload "nade") is bound by its elementwise VALU work.
# Peak VALU issue of MI355X without packed fp32 (the library is compiled without it):
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per second, a
# transcendental (exp2, log2, sin, cos, reciprocal) taking 4 issue slots.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic slots per evaluation: complex tanh = 4 transcendentals + 11 plain
# operations; split leaky ReLU = 2 per real value; normaliser of one qubit =
# 3 transcendentals + 6 plain.
NADE_SLOTS = {"ctanh": 4 * 4 + 11, "lerelu": 2, "normaliser": 3 * 4 + 6}


def tf_valu_slots(n, d, n_layers, n_heads, ffn, ph, t0=0, phase=True):
    """Algorithmic VALU slots of one transformer evaluation of an n-token
    configuration (same accounting as NADE_SLOTS): per layer and token two layer
    norms (5 per feature + a reciprocal square root), two residual additions
    per feature and a tanh-form GELU per hidden value (3 plain operations, exp2,
    1 plain, reciprocal, 1 plain: 13 slots); per layer and head the causal
    softmax (8 slots per score: max, scaled subtraction, exp2, sum, scale; a
    reciprocal per row); the embedding sum, the final layer norm, the masked
    log-softmax of 4 logits per token (28); the phase MLP (its first layer a sum
    of n rows, two GELU layers, the final dot product).  Bias additions ride in
    the MFMA accumulators and are not counted; neither are bf16 conversions.
    With t0 > 0: positions t0 .. n - 1 only (a suffix over a shared prefix);
    phase=False leaves the phase MLP out."""
    ln = 5 * d + 4
    pos = n - t0
    keys = sum(t + 1 for t in range(t0, n))
    per_layer = pos * (2 * ln + 2 * d + 13 * ffn) + n_heads * keys * 8 + n_heads * pos * 4
    return (n_layers * per_layer + pos * d + pos * ln + pos * 28
            + ((n * ph + 2 * 13 * ph + ph) if phase else 0))


def nade_work(n_qubits, hidden):
    """Per configuration: (multiply-adds x 2 of the three complex layers as real
    block GEMMs, qubit i: i x 2H, 2H x 2H, 2H x 4; VALU slots of the
    elementwise work: H complex tanh, 2H leaky ReLU values, one normaliser)."""
    h2 = 2 * hidden
    flop = sum(2 * (i * h2 + h2 * h2 + h2 * 4) for i in range(n_qubits))
    slots = n_qubits * (hidden * NADE_SLOTS["ctanh"] + h2 * NADE_SLOTS["lerelu"]
                        + NADE_SLOTS["normaliser"])
    return flop, slots

# The precision check at trained weights: this many VMC steps at this Adam step
# size on a copy of the model before comparing with the oracle.
TRAIN_STEPS, TRAIN_LR = 5, 1e-3

# HBM bytes per launch of the dominant fused kernel (TREE: positions 12 and 13
# once per distinct prefix, the mean of a step's six launches) on this workload, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by the same counters on a 1 GiB copy
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0); valid only for the kernel source they were
# taken on (sha256 prefix), otherwise the roofline reports null.
FUSED_TRAFFIC = {"source_sha256_prefix": "daa55938af7f22c4", "bytes_per_launch": 3.818e9,
                 "profile": "profiles/fused_kernel_precision_traffic.md"}


# The same for the per-qubit ansatz's fused kernel on workload "nade" (mean of a
# step's two launches, the samples and the distinct x').
NADE_TRAFFIC = {"source_sha256_prefix": "8824cc1e65180fb8", "bytes_per_launch": 84.03e6,
                "profile": "profiles/nade_fused_kernel_traffic.md"}


def fused_traffic(entry=None, source="tf_fused.hip"):
    import hashlib
    entry = entry or FUSED_TRAFFIC
    src = os.path.join(ROOT, "paper_2310_04166_amd", "csrc", source)
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return entry["bytes_per_launch"] if sha == entry["source_sha256_prefix"] else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def param_spec(cfg):
    from synth import nade_param_spec, transformer_param_spec
    if cfg["model"] == "nade":
        return nade_param_spec(cfg["n"], cfg["hidden"])
    return transformer_param_spec(cfg["n"], cfg["d"], cfg["n_layers"], 4 * cfg["d"], 256)


def setup(workload_name, precision):
    from paper_2310_04166_amd import nqs
    from synth import flatten_params, workload
    cfg, h, eri, params = workload(workload_name)
    ham = nqs.ham_compile(h, eri, cfg["n_alpha"], cfg["n_beta"])
    model = nqs.Model(nqs.model_kind(cfg), nqs.model_dims(cfg),
                      flatten_params(params, param_spec(cfg)), precision)
    return cfg, ham, model, params


def trained_check(nqs, torch, args, cfg):
    """A separate copy of the model after TRAIN_STEPS full VMC steps at Adam lr
    TRAIN_LR, so that the fp32 master weights have left the bf16 grid; the
    local energies of its cpu_sample highest-count samples on the bf16 and the
    fp32 GPU paths, and the energy estimator of both paths over its fp32_sample
    highest-count samples plus as many drawn uniformly.  Returns
    (configurations, counts, bf16 E_loc, fp32 E_loc, the trained parameters as
    a dict, unique samples per training step, the estimator comparison)."""
    from synth import unflatten_params
    _, ham, m, _ = setup(args.workload, "bf16")
    dev = torch.device("cuda:0")
    st = {"grad": torch.empty(m.n_params, dtype=torch.float32, device=dev),
          "m": torch.zeros(m.n_params, dtype=torch.float32, device=dev),
          "v": torch.zeros(m.n_params, dtype=torch.float32, device=dev), "lr": TRAIN_LR}
    unique = []
    for t in range(1, TRAIN_STEPS + 1):
        unique.append(vmc_step(nqs, ham, m, cfg, 100 + t, st, t)[0].numel())
    x, c, _ = nqs.sample_unique(m, cfg["n_samples"], 11)
    top = torch.argsort(c, descending=True)[:args.cpu_sample]
    xs, cs = x[top].contiguous(), c[top].contiguous()
    e16, _, _ = nqs.local_energy(ham, m, xs, cs)
    params = m.get_params()
    m32 = nqs.Model(nqs.model_kind(cfg), nqs.model_dims(cfg), params, "fp32")
    e32, _, _ = nqs.local_energy(ham, m32, xs, cs)
    order = torch.argsort(c, descending=True)
    rng = np.random.default_rng(0)
    pick = np.unique(np.concatenate([order[:args.fp32_sample].cpu().numpy(),
                                     rng.choice(x.numel(), min(args.fp32_sample, x.numel()),
                                                replace=False)]))
    idx = torch.as_tensor(pick, device=x.device)
    xe, ce = x[idx].contiguous(), c[idx].contiguous()
    w = ce.cpu().numpy().astype(np.float64)
    E = {}
    for name, mm in (("bf16", m), ("fp32", m32)):
        e, _, _ = nqs.local_energy(ham, mm, xe, ce)
        E[name] = float(np.real(np.sum(w * e.cpu().numpy()) / np.sum(w)))
    est = {"estimator_samples": int(xe.numel()), "estimator_counts": int(w.sum()),
           "E_bf16_estimator": E["bf16"], "E_fp32_estimator": E["fp32"],
           "abs_diff_bf16_fp32_estimator_ha": abs(E["bf16"] - E["fp32"])}
    return ([int(v) for v in xs.cpu().numpy().view(np.uint64)], cs.cpu().numpy().astype(np.float64),
            e16.cpu().numpy(), e32.cpu().numpy(), unflatten_params(params, param_spec(cfg)), unique,
            est)


def vmc_step(nqs, ham, model, cfg, seed, state, t, events=None):
    x, cnt, lost = nqs.sample_unique(model, cfg["n_samples"], seed)
    la, ph = nqs.amp_forward(model, x)
    if events:
        events[0].record()
    eloc, sums, npairs = nqs.local_energy(ham, model, x, cnt, la, ph)
    if events:
        events[1].record()
    gl, gp = nqs.vmc_weights(eloc, cnt, sums)
    grad = nqs.amp_backward(model, x, gl, gp, grad=state["grad"])
    nqs.adam_update(model.params_ptr(), grad, state["m"], state["v"], lr=state["lr"], t=t)
    model.sync()
    return x, cnt, eloc, sums, npairs


def precision_check(nqs, torch, args, cfg, ham, model):
    """bf16 vs fp32 GPU paths on the same samples at the same (initial) parameters:
    the 1024 unique samples with the largest counts plus 1024 drawn uniformly.
    Returns the comparison and, for the oracle, the args.cpu_sample samples with
    the largest counts: (configurations, counts, bf16 E_loc, fp32 E_loc)."""
    x, c, _ = nqs.sample_unique(model, cfg["n_samples"], 7)
    order = torch.argsort(c, descending=True)
    rng = np.random.default_rng(0)
    pick = np.unique(np.concatenate([order[:args.fp32_sample].cpu().numpy(),
                                     rng.choice(x.numel(), min(args.fp32_sample, x.numel()),
                                                replace=False)]))
    idx = torch.as_tensor(pick, device=x.device)
    xs, cs = x[idx].contiguous(), c[idx].contiguous()
    _, _, m32, _ = setup(args.workload, "fp32")
    m32.set_params(model.get_params())
    out = {}
    for name, m in (("fp32", m32), ("bf16", model)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        e, s, npairs = nqs.local_energy(ham, m, xs, cs)
        torch.cuda.synchronize()
        out[name] = (e, s.cpu().numpy(), npairs, time.perf_counter() - a)
    e32, s32, np32, t32 = out["fp32"]
    e16, s16, np16, t16 = out["bf16"]
    d = (e16 - e32).abs().cpu().numpy()
    w = cs.cpu().numpy().astype(np.float64)
    # the highest-count samples, for the oracle's energy on the same samples
    top = np.argsort(-w, kind="stable")[:args.cpu_sample]
    cplx = lambda e: e[..., 0] + 1j * e[..., 1] if e.ndim == 2 else e
    top_samples = ([int(v) for v in xs.cpu().numpy().view(np.uint64)[top]], w[top],
                   cplx(e16.cpu().numpy())[top], cplx(e32.cpu().numpy())[top])
    return top_samples, {"samples": len(pick), "counts_covered": int(w.sum()), "pairs": int(np32),
            "E_bf16": float(s16[1] / s16[0]), "E_fp32": float(s32[1] / s32[0]),
            "abs_diff_ha": float(abs(s16[1] / s16[0] - s32[1] / s32[0])),
            "count_weighted_mean_abs_eloc_diff": float((w * d).sum() / w.sum()),
            "fp32_pairs_per_s": np32 / t32, "bf16_pairs_per_s": np16 / t16,
            "speedup_bf16_over_fp32": (np16 / t16) / (np32 / t32)}


def cpu_baseline(cfg, params, x_sample, where):
    """The FP64 oracle's local energy on a bounded sample of unique configurations."""
    import torch
    from oracle.model import build_model
    from oracle.vmc import local_energy
    from synth import make_integrals
    h, eri = make_integrals(cfg["n"], cfg["rank"], cfg["seed"])
    model = build_model(cfg, params)
    pairs, elocs = 0, []
    t0 = time.perf_counter()
    with torch.no_grad():
        for x in x_sample:
            e, xs, _ = local_energy(model, h, eri, int(x))
            pairs += len(xs) - 1
            elocs.append(complex(e))
    dt = time.perf_counter() - t0
    cpu_model, nproc = cpu_info()
    return {"value": round(pairs / dt, 1), "unit": "pairs/s", "cores": torch.get_num_threads(),
            "cpu_model": cpu_model, "nproc": nproc, "kind": "oracle",
            "sample": f"{len(x_sample)} unique configurations ({where}, largest counts) with all "
                      f"their {pairs} connected x' (FP64 torch CPU forward + Slater-Condon "
                      f"matrix elements), {dt:.1f} s"}, np.array(elocs)


def tf_roofline(flop, slots, k_ms, executed_flop=None):
    """Roofline of the transformer kernel against the bf16 dense MFMA peak (the
    amplitude network is a dense contraction): achieved = algorithmic FLOP /
    kernel time.  Beside it, the MFMA rate counting the executed products (the
    hi/lo operand pairs, padded rows and causal halves included) and the
    model-based VALU-issue fraction (algorithmic elementwise slots at
    VALU_PEAK_TOPS)."""
    sec = k_ms * 1e-3 if k_ms > 0 else float("inf")
    mfma = flop / sec / 1e12
    out = {"bound": "mfma", "achieved": round(mfma, 2), "peak": BF16_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(mfma / BF16_PEAK_TFLOPS, 4),
           "valu_frac_model": round(slots / sec / 1e12 / VALU_PEAK_TOPS, 4)}
    if executed_flop is not None:
        out["executed_mfma_frac"] = round(executed_flop / sec / 1e12 / BF16_PEAK_TFLOPS, 4)
    return out


def executed_flop_per_config(n_layers, d, ph, mode="plain"):
    """MFMA FLOP the fused kernel issues per configuration (or prefix): per
    32-row tile and layer, with the attention weight products taken on the hi
    and lo weight sets, the feed-forward ones on one set, and the attention
    probabilities and output as hi + lo pairs, in 32x32x16 MFMAs of 32768 FLOP;
    the phase MLP's 256 x 256 layer as hi + lo per 32 configurations.  A tile
    holds 2 configurations of 16 padded positions ("plain"), 4 prefixes of 8
    positions ("trunk", no phase MLP), 4 configurations of 8 positions that also
    attend to their prefix's 8 keys ("suffix": per head pair two more score and
    eight more probability-value products), 8 prefixes of 4 positions that also
    attend to the 8-token prefix ("mid": two more scores and four more
    probability-value products, no phase MLP), 8 configurations of 4 positions
    that attend to both levels ("tail": four more scores, twelve more
    probability-value products) or 8 slots of 4 rows that attend to both levels
    ("tree", per slot, no phase MLP); "phase" is the phase MLP alone."""
    nb, ks, fb = d // 32, d // 16, 4 * d // 32
    phase = 2 * (ph // 32) * (ph // 16) * 32768 / 32
    if mode == "phase":
        return phase
    extra = {"plain": 0, "trunk": 0, "suffix": 2 + 8, "mid": 2 + 4, "tail": 4 + 12,
             "tree": 4 + 12}[mode]
    per_head_pair = 2 * (3 * ks) + 2 + 2 * 4 + 3 * ks + extra   # QKV hi+lo, S, PV, O-proj
    per_layer = nb * per_head_pair + 2 * fb * ks                # + FFN W1, W2
    tile = n_layers * per_layer * 32768
    phase = 0 if mode in ("trunk", "mid", "tree") else phase
    per_tile = {"plain": 2, "trunk": 4, "suffix": 4, "mid": 8, "tail": 8, "tree": 8}[mode]
    return tile / per_tile + phase


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def flop_per_config(n, d, n_layers, ffn, ph):
    """Multiply-adds x 2 of one amplitude evaluation of an n-token configuration:
    n tokens x layers x (4 d^2 + 2 d ffn) + causal attention layers x 2 d n(n+1)/2
    + head n x 4 d + phase MLP ph^2 + ph (its first layer is a row lookup)."""
    return 2 * (n * n_layers * (4 * d * d + 2 * d * ffn) + n_layers * 2 * d * n * (n + 1) // 2
                + n * 4 * d + ph * ph + ph)


def run_batching(args, torch, nqs):
    """64 molecules (12..28 spin-orbitals) sharing one d_model 64 transformer;
    one step = sample_unique_batch + batch_local_energy (graph-captured) +
    vmc_weights_batch + amp_backward + Adam + repack."""
    from synth import BATCHING_MODEL as C, batching_workload, flatten_params, transformer_param_spec
    mols, params = batching_workload()
    spec = transformer_param_spec(C["n"], C["d"], C["n_layers"], C["ffn"], C["phase_hidden"])
    dims = [C["n"], 0, 0, C["d"], C["n_layers"], C["n_heads"], C["ffn"], C["phase_hidden"]]
    model = nqs.Model(nqs.MODEL_TRANSFORMER, dims, flatten_params(params, spec), "bf16")
    hams = [nqs.ham_compile(m["h"], m["eri"], m["n_alpha"], m["n_beta"]) for m in mols]
    batch = nqs.Batch(hams, model)
    ns = [m["n_samples"] for m in mols]
    dev = torch.device("cuda:0")
    state = {"grad": torch.empty(model.n_params, dtype=torch.float32, device=dev),
             "m": torch.zeros(model.n_params, dtype=torch.float32, device=dev),
             "v": torch.zeros(model.n_params, dtype=torch.float32, device=dev)}

    def step(seed, t):
        x, c, off, _ = nqs.sample_unique_batch(model, ns, seed)
        eloc, sums, npairs = batch.local_energy(x, c, off)
        gl, gp = nqs.vmc_weights_batch(eloc, c, x, sums)
        grad = nqs.amp_backward(model, x, gl, gp, grad=state["grad"])
        nqs.adam_update(model.params_ptr(), grad, state["m"], state["v"], lr=args.lr, t=t)
        model.sync()
        return x, c, off, eloc, sums, npairs

    log(f"batching: {len(mols)} molecules, params={model.n_params}")
    t = 1
    for w in range(args.warmup):
        out = step(1000 + w, t)
        t += 1
        log(f"warmup {w}: unique={out[0].numel()} pairs={out[5]} {batch.stats()['tile']}")
    torch.cuda.synchronize()
    nqs.timing_read()
    total_pairs, total_unique, flops, slots, step_ms, energies = 0, 0, 0, 0, [], []
    executed = 0
    first = None
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    t_start = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        nqs.timing_enable(False)        # roofline: only the launch on the distinct x'
        x, c, off = nqs.sample_unique_batch(model, ns, k)[:3]
        nqs.timing_enable(True)
        eloc, sums, npairs = batch.local_energy(x, c, off)
        nqs.timing_enable(False)
        gl, gp = nqs.vmc_weights_batch(eloc, c, x, sums)
        grad = nqs.amp_backward(model, x, gl, gp, grad=state["grad"])
        nqs.adam_update(model.params_ptr(), grad, state["m"], state["v"], lr=args.lr, t=t)
        model.sync()
        t += 1
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - s0) * 1e3)
        st = batch.stats()
        flops += sum(int(st["distinct_per_mol"][i]) *
                     flop_per_config(m["n"], C["d"], C["n_layers"], C["ffn"], C["phase_hidden"])
                     for i, m in enumerate(mols))
        slots += sum(int(st["distinct_per_mol"][i]) *
                     tf_valu_slots(m["n"], C["d"], C["n_layers"], C["n_heads"], C["ffn"],
                                   C["phase_hidden"]) for i, m in enumerate(mols))
        executed += st["distinct"] * executed_flop_per_config(C["n_layers"], C["d"],
                                                              C["phase_hidden"])
        s = sums.cpu().numpy()
        energies.append(float(np.sum(s[:, 1] / s[:, 0])))
        total_pairs += npairs
        total_unique += x.numel()
        if first is None:
            first = (x.clone(), c.clone(), off.copy())
        log(f"step {k}: unique={x.numel()} pairs={npairs} distinct={st['distinct']} "
            f"sum E={energies[-1]:.6f} {step_ms[-1]:.0f} ms")
    ev1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    gpu_ms = ev0.elapsed_time(ev1)
    k_ms, k_launches, k_cfgs = nqs.timing_read()
    nqs.timing_enable(False)
    st = batch.stats()
    roofline = tf_roofline(flops, slots, k_ms, executed)
    roofline.update({"traffic": None,
                     "kernel": "fused_kernel<64> on the distinct x' (inside the captured step)",
                     "avg_launch_ms": round(k_ms / max(k_launches, 1), 3),
                     "launches": k_launches, "configs": k_cfgs, "algorithmic_flop": flops,
                     "algorithmic_valu_slots": slots, "executed_flop": executed,
                     "kernel_share_of_steps": round(k_ms / max(gpu_ms, 1e-9), 4)})
    cpu = None
    if not args.no_cpu:
        cpu = batching_cpu_baseline(mols, params, first, args.cpu_sample_batching)
    out = {"metric": "connected-config E_loc evals/s over full VMC steps "
                     "(64 molecules, 12..28 spin-orbitals, one graph-captured step)",
           "value": round(total_pairs / elapsed, 1), "unit": "pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(elapsed * 1e3 / args.steps, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "batching: 64 molecules, 12..28 spin-orbitals, electrons "
                                  "n/2 +/- 1 per spin, 1e4..1e5 samples each, shared "
                                  "transformer d64 L2 h4 + phase MLP 256",
                      "unique_per_step": total_unique / args.steps,
                      "pairs_per_step": total_pairs / args.steps,
                      "distinct_xprime_last_step": st["distinct"],
                      "tile": st["tile"], "graph_captures": st["captures"],
                      "gpu_ms_per_step": round(gpu_ms / args.steps, 2),
                      "step_ms": [round(v, 1) for v in step_ms],
                      "step_ms_median": round(float(np.median(step_ms)), 2),
                      "sum_energy_per_step": energies},
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def batching_cpu_baseline(mols, params, first, per_mol):
    """The FP64 oracle's local energy on the most frequent samples of a few molecules."""
    import torch
    from oracle.model import TransformerModel
    from oracle.sector import Sector
    from oracle.vmc import local_energy
    from synth import BATCHING_MODEL as C
    x, c, off = first
    pairs, picked = 0, []
    t0 = time.perf_counter()
    for i in range(0, len(mols), 16):
        m = mols[i]
        model = TransformerModel(params, Sector(m["n"], m["n_alpha"], m["n_beta"]), C["n_heads"])
        cc = c[off[i]:off[i + 1]].cpu().numpy()
        xs = (x[off[i]:off[i + 1]] & ((1 << 58) - 1)).cpu().numpy().view(np.uint64)
        for j in np.argsort(-cc)[:per_mol]:
            _, xp, _ = local_energy(model, m["h"], m["eri"], int(xs[j]))
            pairs += len(xp) - 1
            picked.append(i)
    dt = time.perf_counter() - t0
    cpu_model, nproc = cpu_info()
    return {"value": round(pairs / dt, 1), "unit": "pairs/s", "cores": torch.get_num_threads(),
            "cpu_model": cpu_model, "nproc": nproc, "kind": "oracle",
            "sample": f"{len(picked)} samples (the {per_mol} most frequent of molecules "
                      f"{sorted(set(picked))}) with all their {pairs} connected x' (FP64 torch "
                      f"CPU forward + Slater-Condon matrix elements), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="precision", choices=["precision", "nade", "batching"],
                    help="precision: the 30-spin-orbital transformer step (default); nade: the "
                         "same system with the paper's per-qubit ansatz; batching: 64 molecules")
    ap.add_argument("--cpu-sample", type=int, default=8,
                    help="samples (largest counts) whose local energies the oracle computes")
    ap.add_argument("--cpu-sample-batching", type=int, default=100,
                    help="batching workload: samples per sampled molecule for the oracle")
    ap.add_argument("--fp32-sample", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the steps, copy a MIB-MiB buffer once (a plain copy kernel of "
                         "known size, to scale HBM byte counters)")
    ap.add_argument("--lr", type=float, default=1e-6,
                    help="Adam step size; small so every timed step sees the calibrated workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; "
              "run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_04166_amd import nqs
    if args.workload == "batching":
        run_batching(args, torch, nqs)
        return
    cfg, ham, model, params = setup(args.workload, "bf16")
    dev = torch.device("cuda:0")
    log(f"workload {args.workload}: n={cfg['n']} N_s={cfg['n_samples']} params={model.n_params}")
    top_samples, precision = (None, None) if args.no_fp32 else \
        precision_check(nqs, torch, args, cfg, ham, model)
    if precision:
        log(f"precision: {precision}")
    trained = None if (args.no_fp32 or args.no_cpu) else trained_check(nqs, torch, args, cfg)

    state = {"grad": torch.empty(model.n_params, dtype=torch.float32, device=dev),
             "m": torch.zeros(model.n_params, dtype=torch.float32, device=dev),
             "v": torch.zeros(model.n_params, dtype=torch.float32, device=dev), "lr": args.lr}
    t = 1
    for w in range(args.warmup):
        out = vmc_step(nqs, ham, model, cfg, 1000 + w, state, t)
        t += 1
        log(f"warmup {w}: unique={out[0].numel()} pairs={out[4]}")
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written")
        del src, dst
    torch.cuda.synchronize()
    nqs.timing_enable(True)
    nqs.timing_read()
    total_pairs, total_unique, total_distinct, step_ms, energies = 0, 0, 0, [], []
    eloc_ms, eloc_pairs = [], []
    first = None
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    tree0 = model.tree_rows()
    ev0.record()
    t_start = time.perf_counter()
    for k in range(args.steps):
        s0 = time.perf_counter()
        evs = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        x, cnt, eloc, sums, npairs = vmc_step(nqs, ham, model, cfg, k, state, t, evs)
        t += 1
        torch.cuda.synchronize()
        eloc_ms.append(evs[0].elapsed_time(evs[1]))
        eloc_pairs.append(npairs)
        step_ms.append((time.perf_counter() - s0) * 1e3)
        s = sums.cpu().numpy()
        energies.append(float(s[1] / s[0]))
        total_pairs += npairs
        total_unique += x.numel()
        total_distinct += nqs.local_energy_stats(ham)[1]
        if first is None:
            first = (x.clone(), cnt.clone())
        log(f"step {k}: unique={x.numel()} pairs={npairs} E={s[1] / s[0]:.6f} "
            f"{step_ms[-1]:.0f} ms")
    ev1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    gpu_ms = ev0.elapsed_time(ev1)
    # launches by row layout: the last positions of every configuration (TAIL
    # with three levels, SUFFIX with two), the shared levels, every other
    # launch (the sampler's, and the samples' own forward without sharing)
    rec = {k: nqs.timing_read(getattr(nqs, "TIMING_" + k.upper()))
           for k in ("tail", "tree", "phase", "mid", "suffix", "trunk")}
    rec["rest"] = nqs.timing_read()
    nqs.timing_enable(False)
    tree_q, tree_q1 = (b - a for a, b in zip(tree0, model.tree_rows()))

    value = total_pairs / elapsed
    nade = cfg["model"] == "nade"
    if nade:
        k_ms, k_launches, k_cfgs = rec["rest"]
        flop, slots = nade_work(2 * cfg["n"], cfg["hidden"])
        achieved = (k_cfgs * slots) / (k_ms * 1e-3) / 1e12 if k_ms > 0 else 0.0
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TOPS,
                    "unit": "T VALU lane-op/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                    "traffic": fused_traffic(NADE_TRAFFIC, "nade_fused.hip"),
                    "traffic_unit": "bytes per launch",
                    "kernel": "nade_fused_kernel (bf16 per-qubit ansatz)",
                    "avg_launch_ms": round(k_ms / max(k_launches, 1), 3),
                    "launches": k_launches, "configs": k_cfgs, "valu_slots_per_config": slots,
                    "flop_per_config": flop,
                    "mfma_tflops": round(k_cfgs * flop / (k_ms * 1e-3) / 1e12, 2) if k_ms else 0,
                    "kernel_share_of_steps": round(k_ms / max(gpu_ms, 1e-9), 4)}
    else:
        n, d, nl, nh = cfg["n"], cfg["d"], cfg["n_layers"], cfg["n_heads"]
        # middle split of the three-level forward: the models here mask every
        # level (MU), so the sector fixes the last token (its conditional is a
        # membership test).  With the tree tail (13..15 tokens) the middle level
        # covers positions 8 .. n-4 per (n-4)-token prefix and TREE positions
        # n-3 and n-2 once per distinct prefix; otherwise from 14 tokens on TAIL
        # evaluates positions n-5 .. n-2, the middle level (n-5)-token prefixes
        tree = rec["tree"][1] > 0
        q = n - 3
        pm = q if tree else n - 5 if n >= 14 else n - 4
        # rows each layout evaluates: (first position, last + 1, phase MLP, executed kind)
        rows = {"tail": (pm, pm + 4, True, "tail"), "mid": (TRUNK, pm, False, "mid"),
                "tree": (q, q + 2, False, "tree"), "phase": (0, 0, True, "phase"),
                "suffix": (TRUNK, n, True, "suffix"), "trunk": (0, TRUNK, False, "trunk"),
                "rest": (0, n, True, "plain")}
        names = {"tail": f"fused_kernel<128, TAIL> (bf16 amplitude network, positions "
                         f"{pm}..{pm + 3} of each configuration)",
                 "mid": f"fused_kernel<128, MID> (positions 8..{pm - 1} once per distinct "
                        f"{pm if not tree else pm - 1}-token prefix)",
                 "tree": f"fused_kernel<128, TREE> (bf16 amplitude network: position {q} once "
                         f"per distinct {q}-token prefix, {q + 1} once per distinct "
                         f"{q + 1}-token prefix, slots of four rows)",
                 "phase": "fused_kernel<128, PHASE> (the phase MLP of each configuration)",
                 "suffix": "fused_kernel<128, SUFFIX> (positions 8..15 of each configuration)",
                 "trunk": "fused_kernel<128, TRUNK> (positions 0..7 once per distinct "
                          "8-token prefix)",
                 "rest": "fused_kernel<128, PLAIN> (bf16 amplitude network)"}
        dom = "tree" if tree else max(("tail", "suffix", "rest"), key=lambda k: rec[k][0])
        k_ms, k_launches, k_cfgs = rec[dom]
        t0, t1, ph, kind = rows[dom]
        exe_cfg = executed_flop_per_config(nl, d, 256, kind)
        if tree:
            # algorithmic work: one row per distinct q- and (q+1)-token prefix
            f_q, f_q1 = (rows_flop(t, t + 1, d, nl, 4 * d, 256, False) for t in (q, q + 1))
            s_q, s_q1 = (tf_valu_slots(t + 1, d, nl, nh, 4 * d, 256, t, phase=False)
                         for t in (q, q + 1))
            roofline = tf_roofline(tree_q * f_q + tree_q1 * f_q1, tree_q * s_q + tree_q1 * s_q1,
                                   k_ms, k_cfgs * exe_cfg)
            flop_cfg = {"row_q": f_q, "row_q1": f_q1, "rows_q": tree_q, "rows_q1": tree_q1}
            slots_cfg = {"row_q": s_q, "row_q1": s_q1}
        else:
            slots_cfg = tf_valu_slots(t1, d, nl, nh, 4 * d, 256, t0)
            flop_cfg = rows_flop(t0, t1, d, nl, 4 * d, 256, ph)
            roofline = tf_roofline(k_cfgs * flop_cfg, k_cfgs * slots_cfg, k_ms, k_cfgs * exe_cfg)
        roofline.update({"traffic": fused_traffic() if args.workload == "precision" else None,
                         "traffic_unit": "bytes per launch",
                         "kernel": names[dom],
                         "avg_launch_ms": round(k_ms / max(k_launches, 1), 3),
                         "launches": k_launches, "configs": k_cfgs,
                         "flop_per_config": flop_cfg,
                         "network_flop_per_config": FLOP_PER_CONFIG,
                         "executed_flop_per_config": int(exe_cfg),
                         "valu_slots_per_config": slots_cfg,
                         "kernel_share_of_steps": round(k_ms / max(gpu_ms, 1e-9), 4)})
        others = {}
        for k in ("mid", "trunk", "suffix", "tail", "tree", "phase", "rest"):
            ms, nlaunch, cfgs = rec[k]
            if k == dom or nlaunch == 0:
                continue
            t0, t1, ph, kind = rows[k]
            f = rows_flop(t0, t1, d, nl, 4 * d, 256, ph)
            others[k] = {"kernel": names[k], "launches": nlaunch, "items": cfgs,
                         "ms": round(ms, 3), "flop_per_item": f,
                         "mfma_frac": round(cfgs * f / max(ms, 1e-9) / 1e9 / BF16_PEAK_TFLOPS, 4),
                         "executed_mfma_frac": round(cfgs * executed_flop_per_config(
                             nl, d, 256, kind) / max(ms, 1e-9) / 1e9 / BF16_PEAK_TFLOPS, 4),
                         "share_of_steps": round(ms / max(gpu_ms, 1e-9), 4)}
        roofline["other_launches"] = others

    cpu = None
    if not args.no_cpu and precision:
        # the oracle at the initial parameters on the precision check's
        # highest-count samples: its energy there against both GPU paths
        xs_cpu, w, e16, e32 = top_samples
        _, e_or = cpu_baseline(cfg, params, xs_cpu, "the precision check's samples")
        E = lambda e, w=w: float(np.real(np.sum(w * e) / np.sum(w)))
        precision.update({"oracle_samples": len(xs_cpu), "oracle_counts": int(w.sum()),
                          "E_oracle_top": E(e_or), "E_bf16_top": E(e16), "E_fp32_top": E(e32),
                          "abs_diff_bf16_oracle_top_ha": abs(E(e16) - E(e_or)),
                          "abs_diff_fp32_oracle_top_ha": abs(E(e32) - E(e_or))})
        # and after TRAIN_STEPS steps at lr TRAIN_LR (master weights off the bf16
        # grid), where the CPU baseline is timed
        xs_t, w_t, e16_t, e32_t, p_t, unique_t, est_t = trained
        cpu, e_or_t = cpu_baseline(cfg, p_t, xs_t, "the trained model's samples")
        Et = lambda e: float(np.real(np.sum(w_t * e) / np.sum(w_t)))
        precision["trained"] = {
            "steps": TRAIN_STEPS, "lr": TRAIN_LR, "unique_per_step": unique_t,
            "oracle_samples": len(xs_t), "oracle_counts": int(w_t.sum()),
            "E_oracle_top": Et(e_or_t), "E_bf16_top": Et(e16_t), "E_fp32_top": Et(e32_t),
            "abs_diff_bf16_oracle_top_ha": abs(Et(e16_t) - Et(e_or_t)),
            "abs_diff_fp32_oracle_top_ha": abs(Et(e32_t) - Et(e_or_t)),
            "max_abs_eloc_diff_bf16_oracle_ha": float(np.max(np.abs(e16_t - e_or_t))),
            # the noise of that energy: the standard error of its per-sample errors
            "std_err_bf16_oracle_top_ha": float(np.sqrt(np.sum(w_t ** 2 * np.real(e16_t - e_or_t) ** 2))
                                                / np.sum(w_t)),
            **est_t}
    elif not args.no_cpu:
        x0, c0 = first
        top = torch.argsort(c0, descending=True)[:args.cpu_sample]
        xs_cpu = [int(v) for v in x0[top].cpu().numpy().view(np.uint64)]
        cpu, _ = cpu_baseline(cfg, params, xs_cpu, "step 0")

    out = {"metric": "connected-config E_loc evals/s over full VMC steps (30 qubits)",
           "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 2),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": f"{args.workload}: 30 spin-orbitals 7a+7b, sector 41,409,225, "
                                  "1e6 samples/step, " +
                                  ("the paper's per-qubit ansatz (complex weights, hidden 64, "
                                   "30 qubits)" if nade else
                                   "transformer d128 L4 h8 + phase MLP 256"),
                      "unique_per_step": total_unique / args.steps,
                      "pairs_per_step": total_pairs / args.steps,
                      "distinct_xprime_per_step": total_distinct / args.steps,
                      "gpu_ms_per_step": round(gpu_ms / args.steps, 2),
                      "step_ms": [round(v, 1) for v in step_ms],
                      "step_ms_median": round(float(np.median(step_ms)), 2),
                      "local_energy_pairs_per_s": round(sum(eloc_pairs) / (sum(eloc_ms) * 1e-3), 1),
                      "local_energy_pairs_per_s_median": round(float(np.median(
                          [p / (ms * 1e-3) for p, ms in zip(eloc_pairs, eloc_ms)])), 1),
                      "local_energy_ms": [round(v, 2) for v in eloc_ms],
                      "energy_per_step": energies},
           "roofline": roofline, "cpu_baseline": cpu, "precision": precision}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
