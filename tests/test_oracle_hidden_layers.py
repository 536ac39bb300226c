"""Pins of the hidden layers of the oracle's per-token MLP and of the paper's
per-qubit complex ansatz (Appendix "ANQS architecture": tanh, then leaky ReLU,
then the normalising third activation).

Each network is hand-built so that every hidden value follows from an identity
of the elementary functions, not from the code under test:
    tanh(atanh(y)) = y,   tanh(i y) = i tan(y),   tanh(x + i pi/2) = coth(x),
    coth(ln 2) = 5/3,     leaky ReLU(z) = 0.01 z for z < 0,
so the expected outputs are numbers written down by hand.  The inputs put the
leaky ReLU on its negative branch and the complex tanh on arguments where it
differs from tanh applied to the real and imaginary parts separately; a swapped
activation order, another slope or a split tanh changes the outputs by far more
than the 1e-13 tolerance."""
import cmath
import math

import numpy as np
import torch

from oracle.model import MLPModel
from oracle.nade import NADEModel
from oracle.sector import Sector


def mlp_params(hidden=2):
    """Two tokens.  Token 0's network has no input (biases only); token 1's
    reads the one-hot code of token 0."""
    H = hidden
    p = {}
    # token 0: h1 = tanh(b1) = (0.5, -0.25); z2 = h1 W2 + b2 = (-0.5, 1.0) -> (-0.005, 1.0)
    p["mlp0.w1"] = np.zeros((0, H))
    p["mlp0.b1"] = np.array([math.atanh(0.5), -math.atanh(0.25)])
    p["mlp0.w2"] = np.array([[2.0, 0.0], [0.0, 4.0]])
    p["mlp0.b2"] = np.array([-1.5, 2.0])
    w3 = np.zeros((H, 8))
    w3[0, 0], w3[1, 1] = 100.0, 1.0       # logits (-0.5, 1.0, 0, 0)
    w3[1, 5], w3[0, 6] = 0.25, 10.0       # phases of tokens 1 and 2: 0.25, -0.05
    p["mlp0.w3"] = w3
    p["mlp0.b3"] = np.zeros(8)
    # token 1 after token 0 = 1 (one-hot row 1):
    #   h1 = tanh(atanh(0.8) + 0, 0 - atanh(0.6)) = (0.8, -0.6)
    #   z2 = (0.8 * 1 - 0.6 * 3 - 1, 0.8 * 5 + 0) = (-2.0, 4.0) -> (-0.02, 4.0)
    w1 = np.zeros((4, H))
    w1[1] = [math.atanh(0.8), -math.atanh(0.6)]
    p["mlp1.w1"] = w1
    p["mlp1.b1"] = np.zeros(H)
    p["mlp1.w2"] = np.array([[1.0, 5.0], [3.0, 0.0]])
    p["mlp1.b2"] = np.array([-1.0, 0.0])
    w3 = np.zeros((H, 8))
    w3[0, 3], w3[1, 2] = 50.0, 0.5        # logits (0, 0, 2.0, -1.0)
    w3[1, 5] = -0.125                     # phase of token 1: -0.5
    p["mlp1.w3"] = w3
    p["mlp1.b3"] = np.array([0.3, 0, 0, 0, 0, 0, 0, 0.0])   # logit 0 -> 0.3
    # token 1 after token 0 = 2 (one-hot row 2, a zero row of w1): h1 = 0,
    #   z2 = b2 = (-1, 0) -> (-0.01, 0): logits (0.3, 0, 0, -0.5), phases 0
    return p


def log_softmax(v):
    m = max(v)
    return [x - m - math.log(sum(math.exp(y - m) for y in v)) for x in v]


def test_mlp_hidden_layers_closed_form():
    """Unmasked conditionals (mask_levels = 0) of both tokens and the phase."""
    m = MLPModel(mlp_params(), Sector(2, 1, 1), mask_levels=0)
    toks = torch.tensor([[1, 1], [2, 3]])
    lc = m.log_cond(toks).numpy()
    want0 = log_softmax([-0.5, 1.0, 0.0, 0.0])
    assert np.max(np.abs(lc[0, 0] - want0)) < 1e-13
    assert np.max(np.abs(lc[1, 0] - want0)) < 1e-13
    assert np.max(np.abs(lc[0, 1] - log_softmax([0.3, 0.0, 2.0, -1.0]))) < 1e-13
    assert np.max(np.abs(lc[1, 1] - log_softmax([0.3, 0.0, 0.0, -0.5]))) < 1e-13
    # phi = phi_0[x_0] + phi_1[x_1]: (1, 1) -> 0.25 - 0.125 * 4.0; (2, 3) -> -0.05 + 0
    ph = m.phase(toks).numpy()
    assert abs(ph[0] - (-0.25)) < 1e-13
    assert abs(ph[1] - (-0.05)) < 1e-13


def test_mlp_pin_detects_wrong_activations():
    """Token 0's first logit (-0.5 pinned above) from a slope of 0.1, or from
    the activations in the other order, is far from the pinned value."""
    b1 = (math.atanh(0.5), -math.atanh(0.25))
    leaky = lambda v, a: v if v >= 0 else a * v
    good = 100 * leaky(2 * math.tanh(b1[0]) - 1.5, 0.01)
    slope = 100 * leaky(2 * math.tanh(b1[0]) - 1.5, 0.1)
    swapped = 100 * math.tanh(2 * leaky(b1[0], 0.01) - 1.5)
    assert abs(good - (-0.5)) < 1e-13
    assert abs(slope - good) > 1.0 and abs(swapped - good) > 1.0


def nade_params(hidden=2):
    """One spatial orbital = two qubits.  Qubit 0's network has no input; qubit
    1's reads bit x_0."""
    H = hidden
    z = lambda *s: np.zeros(s)
    p = {}
    # qubit 0: h1 = tanh(b1) with b1 = (i pi/4, 0) -> (i, 0); z2 = h1 W2 + b2,
    # W2 = [[1, 0], [0, 0]] -> (i + b2_0); b2_0 = -1 + i -> z2_0 = -1 + 2i -> h2_0 = -0.01 + 2i
    p["nade0.w1_re"], p["nade0.w1_im"] = z(0, H), z(0, H)
    p["nade0.b1_re"], p["nade0.b1_im"] = np.array([0.0, 0.0]), np.array([math.pi / 4, 0.0])
    p["nade0.w2_re"], p["nade0.w2_im"] = np.array([[1.0, 0.0], [0.0, 0.0]]), z(H, H)
    p["nade0.b2_re"], p["nade0.b2_im"] = np.array([-1.0, 0.0]), np.array([1.0, 0.0])
    # z = h2 W3 + b3 with W3 column 0 = (50, 0), column 1 = (0, 0), b3 = (0, 0.25i)
    #   -> z = (-0.5 + 100i, 0.25i)
    p["nade0.w3_re"], p["nade0.w3_im"] = np.array([[50.0, 0.0], [0.0, 0.0]]), z(H, 2)
    p["nade0.b3_re"], p["nade0.b3_im"] = np.array([0.0, 0.0]), np.array([0.0, 0.25])
    # qubit 1 with x_0 = 1: z1 = W1 + b1 = (ln 2 + i pi/2, i pi/4)
    #   h1 = (coth(ln 2), tanh(i pi/4)) = (5/3, i)
    #   z2 = h1 W2 + b2, W2 = [[0.6, 0], [0, 1]], b2 = (-3 + 2i, 1 - 3i)
    #      = (1 - 3 + 2i, i + 1 - 3i) = (-2 + 2i, 1 - 2i) -> h2 = (-0.02 + 2i, 1 - 0.02i)
    #   z = h2 W3 + b3, W3 = identity, b3 = 0 -> (-0.02 + 2i, 1 - 0.02i)
    p["nade1.w1_re"], p["nade1.w1_im"] = np.array([[math.log(2.0), 0.0]]), \
        np.array([[math.pi / 2, math.pi / 4]])
    p["nade1.b1_re"], p["nade1.b1_im"] = z(H), z(H)
    p["nade1.w2_re"], p["nade1.w2_im"] = np.array([[0.6, 0.0], [0.0, 1.0]]), z(H, H)
    p["nade1.b2_re"], p["nade1.b2_im"] = np.array([-3.0, 1.0]), np.array([2.0, -3.0])
    p["nade1.w3_re"], p["nade1.w3_im"] = np.eye(H), z(H, 2)
    p["nade1.b3_re"], p["nade1.b3_im"] = z(2), z(2)
    return p


def normalised(z0, z1):
    lse = 0.5 * math.log(math.exp(2 * z0.real) + math.exp(2 * z1.real))
    return [z0 - lse, z1 - lse]


def test_nade_hidden_layers_closed_form():
    """Unmasked (mask_levels = 0) log psi_i(v | x_<i) of both qubits."""
    m = NADEModel(nade_params(), Sector(1, 1, 1), mask_levels=0)
    xs = [0b01, 0b11]                       # x_0 = 1 in both
    bits = NADEModel.bits_of(xs, 2)
    lc = m.log_cond(bits, xs).numpy()       # (B, 2 qubits, 2 values), complex
    want0 = normalised(complex(-0.5, 100.0), complex(0.0, 0.25))
    want1 = normalised(complex(-0.02, 2.0), complex(1.0, -0.02))
    for b in range(2):
        assert max(abs(lc[b, 0, v] - want0[v]) for v in range(2)) < 1e-13
        assert max(abs(lc[b, 1, v] - want1[v]) for v in range(2)) < 1e-13
    # the identities the hand values rest on
    assert abs(cmath.tanh(complex(math.log(2.0), math.pi / 2)) - 5.0 / 3.0) < 1e-14
    assert abs(cmath.tanh(complex(0.0, math.pi / 4)) - 1j) < 1e-15


def test_nade_pin_detects_split_tanh():
    """tanh applied to the real and imaginary parts separately gives a first
    hidden value 0.6 + 0.917i instead of 5/3, so qubit 1's outputs move."""
    split = complex(math.tanh(math.log(2.0)), math.tanh(math.pi / 2))
    assert abs(split - 5.0 / 3.0) > 0.5
    z2_split = split * 0.6 + complex(-3.0, 2.0)
    assert abs(z2_split - complex(-2.0, 2.0)) > 0.5
