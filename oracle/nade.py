"""The paper's autoregressive ansatz, per qubit, with complex weights (paper:
Appendix "ANQS architecture"; "Pruning strategies" for the masks), in
float64 / complex128 PyTorch CPU ops.

Qubit i (spin-orbital i = 2p + s, 0-based) has its own MLP: input the i
previous bits x_0 .. x_{i-1} (as reals), two complex hidden layers of width H
and two complex outputs z = (z_0, z_1):

    h1 = tanh(x W1 + b1)                    (complex tanh)
    h2 = LeReLU(Re(h1 W2 + b2)) + i LeReLU(Im(h1 W2 + b2))
    z  = h2 W3 + b3
    log psi_i(v | x_<i) = z_v - 1/2 LogSumExp(2 Re z)

so |psi_i(0)|^2 + |psi_i(1)|^2 = 1; the phase is Im z_v.  LeReLU is read as
the usual leaky ReLU (slope 0.01 below 0).  Mask-Unphysical, qubit by qubit
(Algorithm 1 on the binary tree): when only one value v of qubit i keeps the
prefix physical, psi_i(v) = 1 and psi_i(1 - v) = 0; when both do, the
conditional is the network's; after an unphysical prefix both are 0.  Levels
of tokens p >= ``mask_levels`` (qubits 2p, 2p + 1) are left unmasked
(Discard-Unphysical / MU-d, d counted in tokens as for the other models).

The library's sampler splits samples over a token's four children at
once, so the model also gives token log-probabilities
    log p(a, b | x_<2p) = 2 Re log psi_2p(a) + 2 Re log psi_2p+1(b | a)
and token phases Im log psi_2p(a) + Im log psi_2p+1(b | a); the product of the
two binary splits has the same distribution as one four-way split.
"""
import numpy as np
import torch
import torch.nn.functional as F

from .sector import Sector, compose, eigs, local_eigs


class NADEModel:
    def __init__(self, params, sector: Sector, mask_levels=None, requires_grad=False):
        self.sector, self.n = sector, sector.n
        self.N = 2 * self.n
        self.mask_levels = self.n if mask_levels is None else mask_levels
        self.t = {k: torch.tensor(np.asarray(v), dtype=torch.float64,
                                  requires_grad=requires_grad) for k, v in params.items()}
        self.hidden = self.t["nade0.b1_re"].shape[0]

    def _w(self, i, name):
        return torch.complex(self.t[f"nade{i}.{name}_re"], self.t[f"nade{i}.{name}_im"])

    def subnet(self, i, bits):
        """Complex outputs z (B, 2) of qubit i's network for prefix bits (B, i)."""
        B = bits.shape[0]
        x = bits[:, :i].to(torch.float64)
        z1 = torch.complex(x, torch.zeros_like(x)) @ self._w(i, "w1") if i > 0 else \
            torch.zeros((B, self.hidden), dtype=torch.complex128)
        h1 = torch.tanh(z1 + self._w(i, "b1"))
        z2 = h1 @ self._w(i, "w2") + self._w(i, "b2")
        h2 = torch.complex(F.leaky_relu(z2.real, 0.01), F.leaky_relu(z2.imag, 0.01))
        return h2 @ self._w(i, "w3") + self._w(i, "b3")

    @staticmethod
    def normalise(z):
        """Third activation: z - 1/2 LogSumExp(2 Re z) over the two outputs."""
        return z - 0.5 * torch.logsumexp(2.0 * z.real, dim=1, keepdim=True)

    def qubit_allowed(self, x, i):
        """Which values of qubit i keep the prefix x_<i physical (Algorithm 1 on
        the binary tree, at qubit level i + 1 counted from 1)."""
        sec = self.sector
        s = eigs(x & ((1 << i) - 1), sec.N, sec.z2)
        return [sec.isphys(i + 2, compose(s, local_eigs(i + 1, v, sec.z2))) for v in (0, 1)]

    def log_cond(self, bits, xs):
        """Masked log psi_i(v | x_<i), complex (B, N, 2)."""
        B = bits.shape[0]
        out = []
        for i in range(self.N):
            lz = self.normalise(self.subnet(i, bits))
            if i // 2 < self.mask_levels:
                ok = torch.tensor([self.qubit_allowed(int(x), i) for x in xs], dtype=torch.bool)
                one = ok.sum(1) == 1
                neg = torch.full_like(lz.real, float("-inf"))
                re = torch.where(ok, torch.where(one[:, None], torch.zeros_like(lz.real), lz.real), neg)
                im = torch.where(ok & ~one[:, None], lz.imag, torch.zeros_like(lz.imag))
                lz = torch.complex(re, im)
            out.append(lz)
        return torch.stack(out, 1)

    @staticmethod
    def bits_of(xs, N):
        x = np.asarray(xs, dtype=np.uint64)
        return torch.from_numpy(((x[:, None] >> np.arange(N, dtype=np.uint64)) &
                                 np.uint64(1)).astype(np.int64))

    def amplitudes(self, xs):
        """(log|psi|, phase) of configurations ``xs`` (ints)."""
        xs = [int(v) for v in xs]
        bits = self.bits_of(xs, self.N)
        lc = self.log_cond(bits, xs)
        sel = torch.gather(lc.real, 2, bits.unsqueeze(-1)).squeeze(-1)
        ph = torch.gather(lc.imag, 2, bits.unsqueeze(-1)).squeeze(-1)
        return sel.sum(1), ph.sum(1)

    def token_logits(self, xs, p):
        """Token log-probabilities (B, 4) at token level p for prefixes xs
        (bits of tokens >= p ignored); token k = a + 2b, a the alpha bit."""
        xs = [int(v) & ((1 << (2 * p)) - 1) for v in xs]
        out = torch.zeros((len(xs), 4), dtype=torch.float64)
        lpa = self._masked(xs, 2 * p)                       # (B, 2) log-modulus of the alpha qubit
        for a in (0, 1):
            xa = [x | (a << (2 * p)) for x in xs]
            lpb = self._masked(xa, 2 * p + 1)
            for b in (0, 1):
                out[:, a + 2 * b] = 2.0 * (lpa[:, a] + lpb[:, b])
        return out

    def _masked(self, xs, i):
        bits = self.bits_of(xs, self.N)
        lz = self.normalise(self.subnet(i, bits)).real
        if i // 2 < self.mask_levels:
            ok = torch.tensor([self.qubit_allowed(x, i) for x in xs], dtype=torch.bool)
            one = ok.sum(1) == 1
            lz = torch.where(ok, torch.where(one[:, None], torch.zeros_like(lz), lz),
                             torch.full_like(lz, float("-inf")))
        return lz

    def flat_grad(self, spec):
        return np.concatenate([
            (self.t[k].grad if self.t[k].grad is not None else torch.zeros_like(self.t[k]))
            .detach().numpy().reshape(-1) for k, _ in spec])
