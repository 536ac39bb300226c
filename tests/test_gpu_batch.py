"""Many molecules sharing one transformer: parity of the batched path (tagged
configuration words, one sampler tree per molecule, bit kernel with hash-table
dedupe, graph-captured bf16 step) against the FP64 CPU oracle, molecule by
molecule."""
import numpy as np
import pytest
import torch

from oracle.hamiltonian import slater_condon_row
from oracle.model import TransformerModel
from oracle.sampler import sample_tree
from oracle.sector import Sector
from oracle.vmc import energy_stats, gradient, local_energies, surrogate_weights
from synth import (BATCHING_MODEL, batching_molecules, batching_params, flatten_params,
                   make_integrals, transformer_param_spec)

pytestmark = pytest.mark.gpu

C4 = BATCHING_MODEL
SPEC = transformer_param_spec(C4["n"], C4["d"], C4["n_layers"], C4["ffn"], C4["phase_hidden"])
DIMS = [C4["n"], 0, 0, C4["d"], C4["n_layers"], C4["n_heads"], C4["ffn"], C4["phase_hidden"]]


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    mod.lib()
    return mod


def small_molecules():
    """Five molecules of the batching workload with n <= 10, fewer samples."""
    mols = [m for m in batching_molecules() if m["n"] <= 10][:5]
    for m in mols:
        m["h"], m["eri"] = make_integrals(m["n"], m["rank"], m["seed"])
        m["n_samples"] = 3000
    return mols


def k_closed_form(n, na, nb):
    c2 = lambda a: a * (a - 1) // 2
    return (na * (n - na) + nb * (n - nb) + c2(na) * c2(n - na) + c2(nb) * c2(n - nb)
            + na * (n - na) * nb * (n - nb))


def make(nqs, mols, precision, params=None):
    params = batching_params() if params is None else params
    m = nqs.Model(nqs.MODEL_TRANSFORMER, DIMS, flatten_params(params, SPEC), precision)
    hams = [nqs.ham_compile(mm["h"], mm["eri"], mm["n_alpha"], mm["n_beta"]) for mm in mols]
    b = nqs.Batch(hams, m)
    return m, b, params


def oracle_model(params, mm):
    return TransformerModel(params, Sector(mm["n"], mm["n_alpha"], mm["n_beta"]), C4["n_heads"])


def split(x, offsets):
    occ = (x & ((1 << 58) - 1)).cpu().numpy().view(np.uint64)
    return [[int(v) for v in occ[offsets[i]:offsets[i + 1]]] for i in range(len(offsets) - 1)]


def test_batch_sampler_replay_fp64(nqs):
    """FP64 conditionals, one Philox stream per molecule: every molecule's
    unique samples and counts equal the oracle tree sampler's, bit for bit."""
    mols = small_molecules()
    m, b, params = make(nqs, mols, "fp64")
    x, c, off, lost = nqs.sample_unique_batch(m, [mm["n_samples"] for mm in mols], 21)
    assert lost == 0
    mol_of = ((x >> 58) & 63).cpu().numpy()
    assert np.all(np.diff(mol_of) >= 0)
    for i, mm in enumerate(mols):
        cfg_o, cnt_o, _ = sample_tree(oracle_model(params, mm), mm["n_samples"], 21, stream=i)
        got = split(x, off)[i]
        log(f"molecule {i} n={mm['n']} ({mm['n_alpha']},{mm['n_beta']}): {len(got)} unique")
        assert got == cfg_o
        assert c[off[i]:off[i + 1]].cpu().tolist() == cnt_o


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 3e-5), ("bf16", 3e-2)])
def test_batch_forward(nqs, precision, tol):
    """Amplitudes of tagged configurations of molecules of 6..10 tokens."""
    mols = small_molecules()
    m, b, params = make(nqs, mols, precision)
    rng = np.random.default_rng(5)
    words, refs = [], []
    for i, mm in enumerate(mols):
        basis = Sector(mm["n"], mm["n_alpha"], mm["n_beta"]).enumerate()
        xs = [basis[k] for k in rng.choice(len(basis), 40, replace=False)]
        la, ph = oracle_model(params, mm).amplitudes(xs)
        refs.append((la.detach().numpy(), ph.detach().numpy()))
        words += [x | (i << 58) for x in xs]
    xw = torch.as_tensor(np.asarray(words, dtype=np.uint64).view(np.int64)).cuda()
    la, ph = nqs.amp_forward(m, xw)
    la, ph = la.cpu().numpy(), ph.cpu().numpy()
    want_la = np.concatenate([r[0] for r in refs])
    want_ph = np.concatenate([r[1] for r in refs])
    err = max(np.max(np.abs(la - want_la)), np.max(np.abs(ph - want_ph)))
    log(f"batch forward {precision}: max err {err:.2e}")
    assert err < tol


def test_batch_local_energy_fp64(nqs):
    """FP64 model: per-sample E_loc 1e-10 relative, pairs = sum U_i K_i with
    the closed-form K_i, distinct x' = the union of the oracle's connected
    sets (integer, exact), per-molecule sums."""
    mols = small_molecules()[:3]
    m, b, params = make(nqs, mols, "fp64")
    k, _ = b.info()
    assert [int(v) for v in k] == [k_closed_form(mm["n"], mm["n_alpha"], mm["n_beta"]) for mm in mols]
    x, c, off, _ = nqs.sample_unique_batch(m, [mm["n_samples"] for mm in mols], 3)
    eloc, sums, npairs = b.local_energy(x, c, off)
    st = b.stats()
    assert npairs == sum((off[i + 1] - off[i]) * k[i] for i in range(len(mols)))
    occ = split(x, off)
    got = eloc.cpu().numpy()
    s = sums.cpu().numpy()
    distinct = 0
    for i, mm in enumerate(mols):
        ref = oracle_model(params, mm)
        xs = occ[i]
        want = local_energies(ref, mm["h"], mm["eri"], xs)
        g = got[off[i]:off[i + 1]]
        err = np.max(np.abs(g - want) / np.abs(want))
        log(f"molecule {i}: {len(xs)} samples, E_loc max rel err {err:.2e}")
        assert err < 1e-10
        cnt = c[off[i]:off[i + 1]].cpu().numpy()
        W, E, _ = energy_stats(want, cnt)
        assert s[i, 0] == W
        assert abs(s[i, 1] / W - E.real) < 1e-10 * abs(E)
        conn = set()
        for xx in xs:
            conn.update(slater_condon_row(mm["h"], mm["eri"], xx)[0][1:])
        distinct += len(conn)
        assert st["distinct_per_mol"][i] == len(conn)
    assert st["distinct"] == distinct


@pytest.fixture(scope="module")
def bf16_step(nqs):
    mols = small_molecules()
    m, b, params = make(nqs, mols, "bf16")
    x, c, off, _ = nqs.sample_unique_batch(m, [mm["n_samples"] for mm in mols], 8)
    return dict(m=m, b=b, params=params, mols=mols, x=x, c=c, off=off)


def test_batch_graph_replays_match_direct_launches(nqs, bf16_step):
    """The captured step, replayed three times with other GPU work in between,
    gives bit-identical results to launching the same kernels directly."""
    b, x, c, off = bf16_step["b"], bf16_step["x"], bf16_step["c"], bf16_step["off"]
    b.set_mode(use_graph=False)
    e0, s0, _ = b.local_energy(x, c, off)
    e0, s0 = e0.clone(), s0.clone()
    b.set_mode(use_graph=True)
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        e, s, _ = b.local_energy(x, c, off)
        assert torch.equal(e, e0) and torch.equal(s, s0), rep
        assert torch.isfinite(junk)
    st = b.stats()
    log(f"graph: captures {st['captures']}, tile {st['tile']}, distinct {st['distinct']}")
    assert st["captures"] >= 1


def test_batch_tile_invariance(nqs, bf16_step):
    """Launch shapes change only the speed: results are bitwise equal."""
    b, x, c, off = bf16_step["b"], bf16_step["x"], bf16_step["c"], bf16_step["off"]
    out = []
    for tile in [(512, 2, 512), (2048, 16, 1024), (1024, 8, 256)]:
        b.set_tile(*tile)
        e, s, _ = b.local_energy(x, c, off)
        out.append((e.clone(), s.clone()))
    for e, s in out[1:]:
        assert torch.equal(e, out[0][0]) and torch.equal(s, out[0][1])


def test_batch_empty_molecule_and_empty_step(nqs, bf16_step):
    """A molecule with no samples between molecules that have some, then a step
    with no samples at all, through the captured step: the other molecules'
    E_loc, sums and weights are bitwise those of the full step (a sample's E_loc
    and a molecule's sums depend only on its own samples), the empty molecule's
    sums are zero, and the full step run again is unchanged."""
    b, x, c, off = bf16_step["b"], bf16_step["x"], bf16_step["c"], bf16_step["off"]
    b.set_mode(use_graph=True)
    e_full, s_full, p_full = b.local_energy(x, c, off)
    e_full, s_full = e_full.clone(), s_full.clone()
    gl, gp = nqs.vmc_weights_batch(e_full, c, x, s_full)
    n_mol = len(off) - 1
    k, _ = b.info()
    drop = 1
    keep = torch.cat([torch.arange(int(off[i]), int(off[i + 1])) for i in range(n_mol)
                      if i != drop]).to(x.device)
    sizes = [0 if i == drop else int(off[i + 1] - off[i]) for i in range(n_mol)]
    off2 = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    x2, c2 = x[keep].contiguous(), c[keep].contiguous()
    e2, s2, p2 = b.local_energy(x2, c2, off2)
    assert p2 == p_full - int(off[drop + 1] - off[drop]) * int(k[drop])
    assert torch.equal(e2, e_full[keep])
    for i in range(n_mol):
        if i == drop:
            assert torch.all(s2[i] == 0)
        else:
            assert torch.equal(s2[i], s_full[i]), i
    gl2, gp2 = nqs.vmc_weights_batch(e2, c2, x2, s2)
    assert torch.equal(gl2, gl[keep]) and torch.equal(gp2, gp[keep])
    # no samples in any molecule
    e0, s0, p0 = b.local_energy(x[:0], c[:0], np.zeros(n_mol + 1, np.int64))
    assert e0.numel() == 0 and p0 == 0 and bool(torch.all(s0 == 0))
    gl0, gp0 = nqs.vmc_weights_batch(e0, c[:0], x[:0], s0)
    assert gl0.numel() == 0 and gp0.numel() == 0
    e3, s3, _ = b.local_energy(x, c, off)
    assert torch.equal(e3, e_full) and torch.equal(s3, s_full)


def test_batch_bf16_energy_vs_oracle(nqs, bf16_step):
    """Mixed precision against the FP64 oracle on the same samples: every
    molecule's energy within 1e-4 Ha, and every sample's E_loc within the
    first-order bound 2 eps A(x) of its log-amplitude error
    (tests/eloc_bound.py)."""
    import eloc_bound
    b, x, c, off = bf16_step["b"], bf16_step["x"], bf16_step["c"], bf16_step["off"]
    params, mols = bf16_step["params"], bf16_step["mols"]
    m = bf16_step["m"]
    eloc, sums, _ = b.local_energy(x, c, off)
    occ = split(x, off)
    got = eloc.cpu().numpy()
    s = sums.cpu().numpy()
    amps = eloc_bound.gpu_amplitudes(nqs, m)
    for i, mm in enumerate(mols):
        res = eloc_bound.check(oracle_model(params, mm), mm["h"], mm["eri"], occ[i], amps,
                               tag=lambda v, i=i: int(v) | (i << 58))
        want = np.array([r[0] for r in res])
        bound = np.array([2 * r[2] * r[1] for r in res])
        g = got[off[i]:off[i + 1]]
        cnt = c[off[i]:off[i + 1]].cpu().numpy()
        _, E, _ = energy_stats(want, cnt)
        e_gpu = s[i, 1] / s[i, 0]
        log(f"molecule {i}: E bf16 {e_gpu:.6f} oracle {E.real:.6f} (|d| {abs(e_gpu - E.real):.1e}); "
            f"max |dE_loc| {np.max(np.abs(g - want)):.2e}, max |dE_loc| / bound "
            f"{np.max(np.abs(g - want) / (bound + 1e-30)):.2f}")
        assert np.all(np.abs(g - want) <= 1.5 * bound + 1e-9)
        assert abs(e_gpu - E.real) <= 1e-4


def test_batch_weights_and_backward_fp64(nqs):
    """Per-molecule upstream weights and the shared model's gradient of the sum
    of the molecules' energies, against the oracle's autograd."""
    mols = small_molecules()[:3]
    params = batching_params()
    m, b, _ = make(nqs, mols, "fp64", params)
    x, c, off, _ = nqs.sample_unique_batch(m, [400, 300, 500], 4)
    eloc, sums, _ = b.local_energy(x, c, off)
    gl, gp = nqs.vmc_weights_batch(eloc, c, x, sums)
    g = nqs.amp_backward(m, x, gl, gp).double().cpu().numpy()
    occ = split(x, off)
    el = eloc.cpu().numpy()
    g_ref = np.zeros_like(g)
    for i, mm in enumerate(mols):
        cnt = c[off[i]:off[i + 1]].cpu().numpy()
        e = el[off[i]:off[i + 1]]
        rl, rp = surrogate_weights(cnt, e)
        assert np.max(np.abs(gl[off[i]:off[i + 1]].cpu().numpy() - rl)) < 1e-14
        assert np.max(np.abs(gp[off[i]:off[i + 1]].cpu().numpy() - rp)) < 1e-14
        ref = TransformerModel(params, Sector(mm["n"], mm["n_alpha"], mm["n_beta"]),
                               C4["n_heads"], requires_grad=True)
        g_ref += gradient(ref, occ[i], cnt, e, SPEC)
    err = np.max(np.abs(g - g_ref))
    log(f"batch backward: max|g| {np.max(np.abs(g_ref)):.3e} err {err:.3e}")
    assert err < 1e-10 * np.max(np.abs(g_ref))


def test_batch_backward_bf16_split_products(nqs):
    """The shared bf16 model's backward over three molecules of different
    lengths (tagged configurations) on split-bf16 MFMA products, against the
    same backward on fp32 library products and against the oracle's autograd
    of the sum of the molecules' surrogates (bound 1e-4 of max |g| for both)."""
    mols = small_molecules()[:3]
    params = batching_params()
    m, b, _ = make(nqs, mols, "bf16", params)
    x, c, off, _ = nqs.sample_unique_batch(m, [400, 300, 500], 4)
    eloc, sums, _ = b.local_energy(x, c, off)
    gl, gp = nqs.vmc_weights_batch(eloc, c, x, sums)
    g = nqs.amp_backward(m, x, gl, gp).double().cpu().numpy()
    m.set_mixed_backward(False)
    g32 = nqs.amp_backward(m, x, gl, gp).double().cpu().numpy()
    m.set_mixed_backward(True)
    occ = split(x, off)
    el = eloc.cpu().numpy()
    g_ref = np.zeros_like(g)
    for i, mm in enumerate(mols):
        cnt = c[off[i]:off[i + 1]].cpu().numpy()
        ref = TransformerModel(params, Sector(mm["n"], mm["n_alpha"], mm["n_beta"]),
                               C4["n_heads"], requires_grad=True)
        g_ref += gradient(ref, occ[i], cnt, el[off[i]:off[i + 1]], SPEC)
    scale = np.max(np.abs(g_ref))
    e32, eor = np.max(np.abs(g - g32)), np.max(np.abs(g - g_ref))
    log(f"batch bf16 backward: max|g| {scale:.3e}, split vs fp32 products {e32:.2e}, "
        f"vs oracle {eor:.2e}")
    assert e32 <= 1e-4 * np.max(np.abs(g32))
    assert eor <= 1e-4 * scale


def test_batch_full_workload(nqs):
    """All 64 molecules (12..28 spin-orbitals) in one graph-captured bf16 step:
    sizes exact, every molecule's energy finite and variational-looking, and a
    few samples of every fifth molecule against the FP64 oracle."""
    from synth import batching_workload
    mols, params = batching_workload()
    m, b, _ = make(nqs, mols, "bf16", params)
    x, c, off, lost = nqs.sample_unique_batch(m, [mm["n_samples"] for mm in mols], 1)
    assert lost == 0
    k, _ = b.info()
    eloc, sums, npairs = b.local_energy(x, c, off)
    e2, s2, _ = b.local_energy(x, c, off)           # a replay of the captured step
    assert torch.equal(eloc, e2) and torch.equal(sums, s2)
    u = np.diff(off)
    assert npairs == int(np.sum(u * k))
    for i, mm in enumerate(mols):
        assert int(c[off[i]:off[i + 1]].sum()) == mm["n_samples"]
    st = b.stats()
    log(f"64 molecules: unique {off[-1]} (min {u.min()}, max {u.max()}), pairs {npairs}, "
        f"distinct {st['distinct']}, tile {st['tile']}")
    s = sums.cpu().numpy()
    assert np.all(np.isfinite(s))
    occ = split(x, off)
    got = eloc.cpu().numpy()
    import eloc_bound
    amps = eloc_bound.gpu_amplitudes(nqs, m)
    for i in range(0, len(mols), 5):
        mm = mols[i]
        pick = np.argsort(-c[off[i]:off[i + 1]].cpu().numpy())[:2]
        xs = [occ[i][j] for j in pick]
        res = eloc_bound.check(oracle_model(params, mm), mm["h"], mm["eri"], xs, amps,
                               tag=lambda v, i=i: int(v) | (i << 58))
        g = got[off[i]:off[i + 1]][pick]
        for gj, (want, A, eps) in zip(g, res):
            assert abs(gj - want) <= 1.5 * 2 * eps * A + 1e-9, i


def test_batch_table_enlarge_and_rerun(nqs, bf16_step):
    """A distinct-x' table of 1024 slots (batch_set_table) overflows on this
    step's ~1e4 distinct x': the step is run again with an enlarged table (two
    more graph captures) and gives bit-identical local energies and sums."""
    b, x, c, off = bf16_step["b"], bf16_step["x"], bf16_step["c"], bf16_step["off"]
    b.set_mode(use_graph=True)
    e0, s0, _ = b.local_energy(x, c, off)
    e0, s0 = e0.clone(), s0.clone()
    st0 = b.stats()
    assert st0["distinct"] > 4096
    b.set_table(1024)
    e1, s1, _ = b.local_energy(x, c, off)
    st1 = b.stats()
    log(f"table 1024: distinct {st1['distinct']} (auto {st0['distinct']}), captures "
        f"{st0['captures']} -> {st1['captures']}")
    assert st1["captures"] >= st0["captures"] + 2
    assert st1["distinct"] == st0["distinct"]
    assert torch.equal(e1, e0) and torch.equal(s1, s0)
    e2, s2, _ = b.local_energy(x, c, off)          # automatic size from here on
    assert b.stats()["captures"] == st1["captures"]
    assert torch.equal(e2, e0) and torch.equal(s2, s0)


def test_batch_model_shared_by_batches(nqs):
    """A second batch_create on the same model reinstalls its sector tables: a
    batch whose molecules the model no longer serves is refused, and once the
    model serves them again (a batch of the same molecules) the first batch
    runs again with its captured step rebuilt, with unchanged results."""
    mols = small_molecules()
    m, bA, params = make(nqs, mols, "bf16")
    x, c, off, _ = nqs.sample_unique_batch(m, [mm["n_samples"] for mm in mols], 8)
    eA, sA, _ = bA.local_energy(x, c, off)
    eA, sA = eA.clone(), sA.clone()
    other = mols[::-1]
    assert [(mm["n"], mm["n_alpha"], mm["n_beta"]) for mm in other] != \
        [(mm["n"], mm["n_alpha"], mm["n_beta"]) for mm in mols]
    hams = [nqs.ham_compile(mm["h"], mm["eri"], mm["n_alpha"], mm["n_beta"]) for mm in other]
    bB = nqs.Batch(hams, m)
    with pytest.raises(nqs.NQSError) as e:
        bA.local_energy(x, c, off)
    assert e.value.status == -1
    hams2 = [nqs.ham_compile(mm["h"], mm["eri"], mm["n_alpha"], mm["n_beta"]) for mm in mols]
    bC = nqs.Batch(hams2, m)
    cap0 = bA.stats()["captures"]
    e2, s2, _ = bA.local_energy(x, c, off)
    assert bA.stats()["captures"] == cap0 + 1
    assert torch.equal(e2, eA) and torch.equal(s2, sA)
    del bB, bC
