"""The premise of the prefix-shared forward, measured on the 30-spin-orbital
workload (ANQS product rule: the transformer is causal, so positions 0..7 of
a configuration depend on its first 8 tokens only).  One step's distinct
connected x' share few 8-token prefixes; the table of distinct k-token
prefixes shows where sharing stops paying (a 14-token prefix fixes the
configuration: the last token is forced by the electron counts).  And the
energies of both evaluations agree with each other."""
import numpy as np
import pytest
import torch

from synth import flatten_params, transformer_param_spec, workload

pytestmark = pytest.mark.gpu


def test_distinct_prefixes_of_one_step():
    from paper_2310_04166_amd import nqs
    nqs.lib()
    cfg, h, eri, params = workload("precision")
    spec = transformer_param_spec(15, 128, 4, 512, 256)
    m = nqs.Model(nqs.MODEL_TRANSFORMER, nqs.model_dims(cfg), flatten_params(params, spec), "bf16")
    H = nqs.ham_compile(h, eri, 7, 7)
    x, c, _ = nqs.sample_unique(m, cfg["n_samples"], 11)
    _, xp, _, _ = nqs.connected_pairs(H, x)
    u = torch.unique(xp)
    print(f"unique samples {x.numel()}, pairs {xp.numel()}, distinct x' {u.numel()}", flush=True)
    counts = {}
    for k in range(4, 16):
        counts[k] = torch.unique(u & ((1 << (2 * k)) - 1)).numel()
        print(f"  {k:2d}-token prefixes: {counts[k]:9d} ({counts[k] / u.numel():.4f} of the x')",
              flush=True)
    assert counts[8] <= 4 ** 8 and counts[8] < 0.02 * u.numel()
    assert counts[14] == counts[15] == u.numel()
    # both evaluations of the step's local energies (bf16 amplitudes)
    e_sh, s_sh, _ = nqs.local_energy(H, m, x, c)
    m.set_prefix_sharing(False)
    e_un, s_un, _ = nqs.local_energy(H, m, x, c)
    s_sh, s_un = s_sh.cpu().numpy(), s_un.cpu().numpy()
    d = np.abs(e_sh.cpu().numpy() - e_un.cpu().numpy())
    print(f"  energy shared {s_sh[1] / s_sh[0]:.8f} unshared {s_un[1] / s_un[0]:.8f}; per-sample "
          f"|difference| median {np.median(d):.1e} max {d.max():.1e} Ha", flush=True)
    # The two use the same bf16 operands and differ in the order of fp32 sums
    # only, but a configuration has ~1e5 activations rounded to bf16, so a few
    # of them land on the other side of a rounding boundary (one bf16 ulp,
    # 2^-9 relative): per sample the two evaluations are two draws of the
    # bf16 error itself (against the oracle 3e-5 .. 4e-4 Ha on the
    # highest-count samples of this model, the first-order bound 2 eps A(x)
    # larger where A(x) is large), which average out in the energy.
    w = c.cpu().numpy().astype(np.float64)
    wmean = float(np.sum(w * d) / w.sum())
    print(f"  count-weighted mean |difference| {wmean:.1e} Ha", flush=True)
    assert abs(s_sh[1] / s_sh[0] - s_un[1] / s_un[0]) < 1e-5
    assert np.median(d) < 1e-3 and wmean < 1e-3


@pytest.mark.parametrize("n,na,nb,d,L,samples", [
    (13, 3, 3, 64, 2, 20_000),     # the shortest sequence of three levels (middle: position 8)
    (14, 2, 3, 128, 2, 50_000),
    (16, 3, 2, 64, 1, 20_000),     # every position a token (middle: positions 8..11)
])
def test_three_levels_vs_unshared_and_oracle(n, na, nb, d, L, samples):
    """13..16 tokens: the local energy evaluates positions 0..7 once per 8-token
    prefix, 8 .. pm-1 once per pm-token prefix and pm .. pm+3 per configuration
    (slices, passes of 8 items holding up to two 8-token prefixes; pm = n - 4 at 13
    tokens, n - 5 from 14 on, where the sector fixes the last token).  Its
    energy against the per-configuration evaluation (same bf16 operands) and,
    on the four highest-count samples, every local energy against the FP64
    oracle within 1.5 x its first-order bound (tests/eloc_bound.py)."""
    import eloc_bound
    from oracle.model import TransformerModel
    from oracle.sector import Sector
    from paper_2310_04166_amd import nqs
    from synth import make_integrals, make_transformer_params
    nqs.lib()
    h, eri = make_integrals(n, n, 40 + n)
    params = make_transformer_params(n, na, nb, d, L, seed=n, std=0.05, hf_bias=1.0,
                                     round_to="bf16", bias_std=0.02)
    spec = transformer_param_spec(n, d, L, 4 * d, 256)
    m = nqs.Model(nqs.MODEL_TRANSFORMER, [n, na, nb, d, L, d // 16, 4 * d, 256],
                  flatten_params(params, spec), "bf16")
    H = nqs.ham_compile(h, eri, na, nb)
    x, c, _ = nqs.sample_unique(m, samples, 3)
    e3, s3, npairs = nqs.local_energy(H, m, x, c)
    distinct = nqs.local_energy_stats(H)[1]
    m.set_prefix_sharing(False)
    eu, su, _ = nqs.local_energy(H, m, x, c)
    m.set_prefix_sharing(True)
    s3, su = s3.cpu().numpy(), su.cpu().numpy()
    E3, Eu = s3[1] / s3[0], su[1] / su[0]
    d_e = np.abs(e3.cpu().numpy() - eu.cpu().numpy())
    print(f"n={n}: unique {x.numel()}, pairs {npairs}, distinct {distinct}; energy three levels "
          f"{E3:.8f} unshared {Eu:.8f}; per-sample |difference| median {np.median(d_e):.1e}",
          flush=True)
    assert abs(E3 - Eu) < 1e-5
    ref = TransformerModel(params, Sector(n, na, nb), d // 16)
    cv = c.cpu().numpy()
    top = list(np.argsort(-cv, kind="stable")[:4])
    xv = x.cpu().numpy().view(np.uint64)
    e = e3.cpu().numpy()
    res = eloc_bound.check(ref, h, eri, [int(xv[i]) for i in top], eloc_bound.gpu_amplitudes(nqs, m))
    for i, (want, A, eps) in zip(top, res):
        err = abs(e[i] - want)
        print(f"  x={int(xv[i]):#x} count={cv[i]} err {err:.2e} bound {2 * eps * A:.2e}", flush=True)
        assert err <= 1.5 * 2 * eps * A + 1e-9


# the lists: groups in ascending order (the 8-token prefix is the most
# significant part of the sort key), following each other unless the pass
# of 8 a group would start in already holds two groups (one slice)
def list_end(counts):
    pos, held = 0, 0
    for k in counts:
        if pos % 8 and held >= 2:
            pos, held = (pos + 7) // 8 * 8, 0
        end = pos + int(k)
        held = (1 if pos % 8 == 0 else held + 1) if (end - 1) // 8 == pos // 8 else 1
        pos = end
        if pos % 8 == 0:
            held = 0
    return pos


def slice_cuts(k_mid, entry_bytes):
    """First group of every slice: whole groups whose middle entries
    (entry_bytes each) fit in 2 GiB, then the number of groups."""
    cap = min(int(np.sum(k_mid)), (1 << 31) // entry_bytes)
    cuts, g0, G = [], 0, len(k_mid)
    while g0 < G:
        g1, tot = g0 + 1, int(k_mid[g0])
        while g1 < G and tot + int(k_mid[g1]) <= cap:
            tot += int(k_mid[g1])
            g1 += 1
        cuts.append(g0)
        g0 = g1
    return cuts + [G]


def sliced_items(counts, cuts):
    """Items over all slices: each slice's list starts a new pass."""
    return sum(list_end(counts[a:b]) for a, b in zip(cuts[:-1], cuts[1:]))


def expected_items(u, pm, entry_bytes):
    """Items of the MID and TAIL launches over the distinct x' u: per 8-token
    prefix its distinct pm-token prefixes (MID) and its configurations (TAIL),
    a pass of 8 holding at most two 8-token prefixes, slice by slice."""
    u = np.unique(np.asarray(u, dtype=np.uint64))
    gm = np.unique(u & np.uint64((1 << (2 * pm)) - 1))
    _, k_mid = np.unique(gm & np.uint64(0xFFFF), return_counts=True)
    _, k_tail = np.unique(u & np.uint64(0xFFFF), return_counts=True)
    cuts = slice_cuts(k_mid, entry_bytes)
    return sliced_items(k_mid, cuts), sliced_items(k_tail, cuts)


# (n, n_alpha, n_beta, strategy, general symmetries, middle split): the split
# moves to n - 5 exactly when every level is masked and the sector leaves one
# token at the last position - particle numbers (table or general symmetries)
# do; masks that stop 2 levels early (MU-d) or 2 S_z alone (an empty and a
# doubly occupied orbital add the same) do not
@pytest.mark.parametrize("n,na,nb,strategy,general,pm", [
    (14, 3, 3, "MU", None, 9),
    (14, 3, 3, "MUd", None, 10),
    (15, 3, 2, "MU", "n_sz", 10),
    (15, 3, 2, "MU", "sz", 11),
])
def test_three_level_split_follows_the_sector(n, na, nb, strategy, general, pm):
    """The middle split the library takes (counted from the MID launches'
    items) and the local energy it gives, against the per-configuration
    evaluation and the FP64 oracle (as above)."""
    import eloc_bound
    from oracle.model import TransformerModel
    from oracle.sector import GeneralSector, Sector, particle_number_eigs, two_sz_eigs
    from paper_2310_04166_amd import nqs
    from synth import make_integrals, make_transformer_params
    nqs.lib()
    d, L = 64, 1
    h, eri = make_integrals(n, n, 70 + n)
    params = make_transformer_params(n, na, nb, d, L, seed=n + 1, std=0.05, hf_bias=1.0,
                                     round_to="bf16", bias_std=0.02)
    spec = transformer_param_spec(n, d, L, 4 * d, 256)
    m = nqs.Model(nqs.MODEL_TRANSFORMER, [n, na, nb, d, L, d // 16, 4 * d, 256],
                  flatten_params(params, spec), "bf16", strategy, 2 if strategy == "MUd" else 0)
    m.set_prefix_sharing(True, tree=False)    # the middle split of the TAIL layout
    sec = Sector(n, na, nb)
    if general is not None:
        eig = [two_sz_eigs(n)] if general == "sz" else [particle_number_eigs(n), two_sz_eigs(n)]
        tgt = [na - nb] if general == "sz" else [na + nb, na - nb]
        m.set_symmetries(eig, tgt)
        sec = GeneralSector(n, eig, tgt)
    H = nqs.ham_compile(h, eri, na, nb)
    x, c, _ = nqs.sample_unique(m, 20_000, 5)
    _, xp, _, _ = nqs.connected_pairs(H, x)
    u = torch.unique(xp).cpu().numpy().view(np.uint64)
    mid_want, tail_want = expected_items(u, pm, L * (d // 32) * 512)
    nqs.timing_read()                       # drop older records
    nqs.timing_enable(True)
    try:
        e3, s3, _ = nqs.local_energy(H, m, x, c)
        torch.cuda.synchronize()
        assert nqs.local_energy_stats(H)[1] == len(u)
        _, _, mid_items = nqs.timing_read(nqs.TIMING_MID)
        _, _, tail_items = nqs.timing_read(nqs.TIMING_TAIL)
    finally:
        nqs.timing_enable(False)
        nqs.timing_read()
    print(f"n={n} {strategy} {general}: {x.numel()} samples, {len(u)} distinct x'; MID items "
          f"{mid_items} (split {pm}: {mid_want}), TAIL items {tail_items} ({tail_want})", flush=True)
    assert (mid_items, tail_items) == (mid_want, tail_want)
    m.set_prefix_sharing(False)
    eu, su, _ = nqs.local_energy(H, m, x, c)
    m.set_prefix_sharing(True, tree=False)
    s3, su = s3.cpu().numpy(), su.cpu().numpy()
    assert abs(s3[1] / s3[0] - su[1] / su[0]) < 1e-5
    ref = TransformerModel(params, sec, d // 16)
    cv = c.cpu().numpy()
    top = list(np.argsort(-cv, kind="stable")[:4])
    xv = x.cpu().numpy().view(np.uint64)
    e = e3.cpu().numpy()
    res = eloc_bound.check(ref, h, eri, [int(xv[i]) for i in top], eloc_bound.gpu_amplitudes(nqs, m))
    for i, (want, A, eps) in zip(top, res):
        err = abs(e[i] - want)
        print(f"  x={int(xv[i]):#x} count={cv[i]} err {err:.2e} bound {2 * eps * A:.2e}", flush=True)
        assert err <= 1.5 * 2 * eps * A + 1e-9


def expected_tree_items(u, n):
    """Items of the MID and TREE launches of the tree tail over the distinct x'
    u (q = n - 3): per 8-token prefix its distinct (q-1)-token prefixes (MID)
    and their slots (TREE), a pass of 8 holding at most two 8-token prefixes.
    The slots of a
    (q-1)-token prefix: its q-token prefixes in token order, each a root row
    with its distinct (q+1)-token extensions; with two of the current slot's
    four rows free or more, the root and as many extensions as fit go in (the
    rest follow under a repeated root), else the next slot opens."""
    q = n - 3
    u = np.unique(np.asarray(u, dtype=np.uint64))
    gm = np.unique(u & np.uint64((1 << (2 * (q - 1))) - 1))
    _, k_mid = np.unique(gm & np.uint64(0xFFFF), return_counts=True)
    g1 = np.unique(u & np.uint64((1 << (2 * (q + 1))) - 1))
    nq, ext = np.unique(g1 & np.uint64((1 << (2 * q)) - 1), return_counts=True)
    parent = nq & np.uint64((1 << (2 * (q - 1))) - 1)
    token = (nq >> np.uint64(2 * (q - 1))) & np.uint64(3)
    order = np.lexsort((token, parent))
    slots = {}
    used = {}
    for k in order:
        j = int(parent[k])
        c = int(ext[k])
        while c > 0:
            if used.get(j, 4) > 2:
                slots[j] = slots.get(j, 0) + 1
                used[j] = 0
            take = min(c, 3 - used[j])
            used[j] += 1 + take
            c -= take
    groups = {}
    for j, ns in slots.items():
        groups[j & 0xFFFF] = groups.get(j & 0xFFFF, 0) + ns
    return list_end(k_mid), list_end([groups[g] for g in sorted(groups)])


# (n, n_alpha, n_beta, d, layers, samples, strategy, general symmetries, tree):
# the tree tail where every level is masked and the last token is fixed (13..15
# tokens, particle-number tables or general symmetries), not otherwise
@pytest.mark.parametrize("n,na,nb,d,L,samples,strategy,general,tree", [
    (13, 3, 3, 64, 2, 20_000, "MU", None, True),
    (14, 2, 3, 128, 2, 50_000, "MU", None, True),
    (15, 3, 2, 64, 1, 20_000, "MU", "n_sz", True),
    (15, 3, 2, 64, 1, 20_000, "MU", "sz", False),
    (14, 3, 3, 64, 1, 20_000, "MUd", None, False),
])
def test_tree_tail_vs_tail_unshared_and_oracle(n, na, nb, d, L, samples, strategy, general, tree):
    """The local energy through the tree tail (each of positions n-3 and n-2
    once per distinct prefix, their masked conditionals gathered per x')
    against the per-configuration tail rows and the unshared evaluation (same
    bf16 operands), its launches' items against the prefix counts, and on the
    four highest-count samples against the FP64 oracle."""
    import eloc_bound
    from oracle.model import TransformerModel
    from oracle.sector import GeneralSector, Sector, particle_number_eigs, two_sz_eigs
    from paper_2310_04166_amd import nqs
    from synth import make_integrals, make_transformer_params
    nqs.lib()
    h, eri = make_integrals(n, n, 90 + n)
    params = make_transformer_params(n, na, nb, d, L, seed=n + 7, std=0.05, hf_bias=1.0,
                                     round_to="bf16", bias_std=0.02)
    spec = transformer_param_spec(n, d, L, 4 * d, 256)
    m = nqs.Model(nqs.MODEL_TRANSFORMER, [n, na, nb, d, L, d // 16, 4 * d, 256],
                  flatten_params(params, spec), "bf16", strategy, 2 if strategy == "MUd" else 0)
    sec = Sector(n, na, nb)
    if general is not None:
        eig = [two_sz_eigs(n)] if general == "sz" else [particle_number_eigs(n), two_sz_eigs(n)]
        tgt = [na - nb] if general == "sz" else [na + nb, na - nb]
        m.set_symmetries(eig, tgt)
        sec = GeneralSector(n, eig, tgt)
    H = nqs.ham_compile(h, eri, na, nb)
    x, c, _ = nqs.sample_unique(m, samples, 9)
    _, xp, _, _ = nqs.connected_pairs(H, x)
    u = torch.unique(xp).cpu().numpy().view(np.uint64)
    nqs.timing_read()
    nqs.timing_enable(True)
    try:
        et, st, _ = nqs.local_energy(H, m, x, c)
        torch.cuda.synchronize()
        assert nqs.local_energy_stats(H)[1] == len(u)
        _, _, mid_items = nqs.timing_read(nqs.TIMING_MID)
        _, _, tree_items = nqs.timing_read(nqs.TIMING_TREE)
        _, _, tail_items = nqs.timing_read(nqs.TIMING_TAIL)
        _, _, phase_items = nqs.timing_read(nqs.TIMING_PHASE)
    finally:
        nqs.timing_enable(False)
        nqs.timing_read()
    print(f"n={n} {strategy} {general}: {x.numel()} samples, {len(u)} distinct x'; items MID "
          f"{mid_items} TREE {tree_items} TAIL {tail_items} PHASE {phase_items}", flush=True)
    if tree:
        want_mid, want_tree = expected_tree_items(u, n)
        print(f"  expected MID {want_mid} TREE {want_tree}", flush=True)
        assert (mid_items, tree_items, tail_items, phase_items) == (want_mid, want_tree, 0, len(u))
    else:
        assert tree_items == 0 and tail_items > 0
    m.set_prefix_sharing(True, tree=False)
    e3, s3, _ = nqs.local_energy(H, m, x, c)
    m.set_prefix_sharing(False)
    eu, su, _ = nqs.local_energy(H, m, x, c)
    m.set_prefix_sharing(True)
    st, s3, su = st.cpu().numpy(), s3.cpu().numpy(), su.cpu().numpy()
    Et, E3, Eu = st[1] / st[0], s3[1] / s3[0], su[1] / su[0]
    d_t = np.abs(et.cpu().numpy() - eu.cpu().numpy())
    print(f"  energy tree {Et:.8f} tail {E3:.8f} unshared {Eu:.8f}; per-sample |tree - "
          f"unshared| median {np.median(d_t):.1e} max {d_t.max():.1e}", flush=True)
    assert abs(Et - Eu) < 1e-5 and abs(Et - E3) < 1e-5
    ref = TransformerModel(params, sec, d // 16)
    cv = c.cpu().numpy()
    top = list(np.argsort(-cv, kind="stable")[:4])
    xv = x.cpu().numpy().view(np.uint64)
    e = et.cpu().numpy()
    res = eloc_bound.check(ref, h, eri, [int(xv[i]) for i in top], eloc_bound.gpu_amplitudes(nqs, m))
    for i, (want, A, eps) in zip(top, res):
        err = abs(e[i] - want)
        print(f"  x={int(xv[i]):#x} count={cv[i]} err {err:.2e} bound {2 * eps * A:.2e}", flush=True)
        assert err <= 1.5 * 2 * eps * A + 1e-9
