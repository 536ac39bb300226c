"""The algorithmic work counts behind bench.py's roofline (host arithmetic, no
GPU): the constants agree with the per-configuration formulas, the formulas
with sums written out by hand, and the roofline is the MFMA one."""
import bench


def test_transformer_flops_constant_matches_the_formula():
    # 15 tokens, d 128, 4 layers, ffn 512, phase MLP 256
    assert bench.FLOP_PER_CONFIG == bench.flop_per_config(15, 128, 4, 512, 256)


def test_transformer_flops_by_hand():
    # per token and layer: q, k, v, o (4 d^2) + ffn (2 d f) multiply-adds;
    # attention: per layer 2 d (scores and P V) per causal (query, key) pair
    n, d, L, f, ph = 3, 8, 2, 16, 4
    macs = n * L * (4 * d * d + 2 * d * f) + L * 2 * d * (1 + 2 + 3) + n * 4 * d + ph * ph + ph
    assert bench.flop_per_config(n, d, L, f, ph) == 2 * macs


def test_transformer_valu_slots_by_hand():
    n, d, L, H, f, ph = 2, 4, 1, 2, 8, 4
    ln = 5 * d + 4                                    # one layer norm of one token
    per_layer = n * (2 * ln + 2 * d + 13 * f) + H * 3 * 8 + H * n * 4
    total = per_layer + n * d + n * ln + n * 28 + n * ph + 2 * 13 * ph + ph
    assert bench.tf_valu_slots(n, d, L, H, f, ph) == total
    # the 30-qubit model of the precision workload
    assert bench.tf_valu_slots(15, 128, 4, 8, 512, 256) == 547392


def test_nade_work_by_hand():
    flop, slots = bench.nade_work(3, 2)               # 3 qubits, hidden 2 (4 real features)
    assert flop == 2 * sum(i * 4 + 16 + 16 for i in range(3))
    assert slots == 3 * (2 * 27 + 4 * 2 + 18)
    assert bench.nade_work(30, 64) == (1125120, 60060)


def test_roofline_is_the_mfma_bound():
    # the amplitude network is a dense contraction: frac = algorithmic FLOP / time
    # / bf16 peak; the VALU fraction and the executed-MFMA fraction ride along
    r = bench.tf_roofline(flop=1e14, slots=1e13, k_ms=1000.0, executed_flop=2.5e14)
    assert r["bound"] == "mfma" and abs(r["frac"] - 100.0 / bench.BF16_PEAK_TFLOPS) < 5e-5
    assert abs(r["valu_frac_model"] - 10.0 / bench.VALU_PEAK_TOPS) < 5e-5
    assert abs(r["executed_mfma_frac"] - 250.0 / bench.BF16_PEAK_TFLOPS) < 5e-5


def test_executed_mfma_count_by_hand():
    # per 32-row tile and layer at d 128: per head pair Q, K, V (8 k-steps each,
    # hi + lo weights) 48, scores 2, P V (hi + lo P) 8, output projection (hi
    # weights x O hi + lo, lo weights x O hi) 24; per hidden block of 32 (16 of
    # them) W1 and W2 on one weight set 16 -> 4 * 82 + 16 * 16 = 584 MFMAs
    per_tile = 4 * 584 * 32768
    phase = 2 * 8 * 16 * 32768 / 32
    assert bench.executed_flop_per_config(4, 128, 256) == per_tile / 2 + phase


def test_valu_peak_from_unit_counts():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9


def test_prefix_split_work_adds_up():
    # positions 0..7 (once per prefix) and 8..n-1 (per configuration, with the
    # phase MLP) make one whole evaluation
    for n in (9, 15, 16):
        whole = bench.flop_per_config(n, 128, 4, 512, 256)
        assert bench.rows_flop(0, n, 128, 4, 512, 256, True) == whole
        assert (bench.rows_flop(0, 8, 128, 4, 512, 256, False)
                + bench.rows_flop(8, n, 128, 4, 512, 256, True)) == whole
    # suffix of the 30-qubit model by hand: 7 positions, queries 8..14 see 9..15 keys
    macs = 7 * 4 * (4 * 128 ** 2 + 2 * 128 * 512) + 4 * 2 * 128 * sum(range(9, 16)) \
        + 7 * 4 * 128 + 256 * 256 + 256
    assert bench.rows_flop(8, 15, 128, 4, 512, 256, True) == 2 * macs
    # the VALU model of the suffix: the same per-position terms over 7 positions
    n, d, L, H, f, ph = 15, 128, 4, 8, 512, 256
    ln = 5 * d + 4
    per_layer = 7 * (2 * ln + 2 * d + 13 * f) + H * sum(range(9, 16)) * 8 + H * 7 * 4
    total = L * per_layer + 7 * d + 7 * ln + 7 * 28 + n * ph + 2 * 13 * ph + ph
    assert bench.tf_valu_slots(n, d, L, H, f, ph, 8) == total


def test_executed_mfma_count_shared_prefix_by_hand():
    # suffix tile: 4 configurations x 8 positions; per head pair also the
    # scores against the prefix's 8 keys (2) and their P V products (hi + lo
    # P, 2 k-steps, 2 heads: 8) -> 4 * 92 + 256 = 624 MFMAs per layer
    phase = 2 * 8 * 16 * 32768 / 32
    assert bench.executed_flop_per_config(4, 128, 256, "suffix") == 4 * 624 * 32768 / 4 + phase
    # trunk tile: 4 prefixes x 8 positions, the plain count, no phase MLP
    assert bench.executed_flop_per_config(4, 128, 256, "trunk") == 4 * 584 * 32768 / 4


def test_executed_mfma_count_three_levels_by_hand():
    # mid tile: 8 prefixes x 4 positions; per head pair scores against the own and
    # the 8-token prefix's keys (4), probability-value products own (2 k-steps x
    # hi + lo x 2 heads = 8) and prefix (1 k-step: 4) -> 48 + 4 + 12 + 24 = 88
    assert bench.executed_flop_per_config(4, 128, 256, "mid") == 4 * (4 * 88 + 256) * 32768 / 8
    # tail tile: 8 configurations x 4 positions, also the middle level's keys:
    # scores 6, probability-value products 8 + 4 + 8 = 20 -> 98 per head pair
    phase = 2 * 8 * 16 * 32768 / 32
    assert bench.executed_flop_per_config(4, 128, 256, "tail") == \
        4 * (4 * 98 + 256) * 32768 / 8 + phase
