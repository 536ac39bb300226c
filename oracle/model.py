"""Amplitude networks in float64 PyTorch CPU ops (paper: the ANQS product rule;
"Pruning strategies" for Mask-Unphysical; Appendix B for the network).

log psi(x) = sum_p log psi_p(x_p | x_<p) over the n orbital tokens, with
|psi_p|^2 the conditional probability.  Readings of the paper:

* One token per spatial orbital (4 states), not one per qubit.  A prefix of p
  tokens is the qubit prefix of length 2p, so Algorithm 1 applies unchanged.
* Mask-Unphysical with 4 children: the conditional is the softmax of the
  logits over the physical tokens only; unphysical tokens get probability 0.
  With one physical child this is the paper's psi(0)=0, psi(1)=1 rule.  Levels
  p >= ``mask_levels`` are left unmasked (Discard-Unphysical / MU-d).
* The logits play the role of 2 Re z in the paper's third activation, so the
  normaliser is a log-softmax.
* The phase is carried separately from the masked modulus: the MLP gives one
  phase per (position, token) and phi = sum_p phi_p[x_p]; the transformer
  has a phase MLP over the one-hot code of the whole configuration.
* One transformer may serve molecules of different sizes (its position
  tables cover the largest): a molecule of n tokens reads rows 0..n-1 of the
  position embedding and of the per-position logit bias, and its phase-MLP
  input is its one-hot code followed by zeros for the absent positions.
* MLP activations: tanh, then leaky ReLU with slope 0.01 for x < 0 (the
  printed "-0.01 x" is read as the usual leaky ReLU).
"""
import math

import numpy as np
import torch
import torch.nn.functional as F

from .sector import Sector


def tokens_from_ints(xs, n):
    x = np.asarray(xs, dtype=np.uint64)
    toks = np.zeros((len(x), n), dtype=np.int64)
    for p in range(n):
        toks[:, p] = ((x >> np.uint64(2 * p)) & np.uint64(1)).astype(np.int64) \
            + 2 * ((x >> np.uint64(2 * p + 1)) & np.uint64(1)).astype(np.int64)
    return torch.from_numpy(toks)


class AmplitudeModel:
    def __init__(self, params, sector: Sector, mask_levels=None, requires_grad=False):
        self.sector, self.n = sector, sector.n
        self.mask_levels = self.n if mask_levels is None else mask_levels
        self.names = list(params.keys())
        self.t = {k: torch.tensor(np.asarray(v), dtype=torch.float64,
                                  requires_grad=requires_grad) for k, v in params.items()}
        self.phys = None
        if getattr(sector, "general", False):     # masks walked per configuration
            return
        n, K = self.n, len(sector.z2)
        # child masks by (position, alpha, beta, Z2 partial eigenvalues of the
        # prefix as a K-bit index: bit j set when eigenvalue j is -1)
        tab = torch.zeros((n + 1, n + 1, n + 1, 1 << K, 4), dtype=torch.bool)
        for p in range(n):
            for a in range(n + 1):
                for b in range(n + 1):
                    for zi in range(1 << K):
                        z = tuple(-1 if (zi >> j) & 1 else 1 for j in range(K))
                        tab[p, a, b, zi] = torch.tensor(sector.child_mask(p, a, b, z))
        self.phys = tab
        # K-bit Z2 index contribution of token t at position p
        self.z2_flip = torch.zeros((max(n, 1), 4), dtype=torch.long)
        for p in range(n):
            for t in range(4):
                v = 0
                for j, m in enumerate(sector.z2):
                    v |= ((((m >> (2 * p)) & 1) & (t & 1)) ^
                          (((m >> (2 * p + 1)) & 1) & (t >> 1))) << j
                self.z2_flip[p, t] = v

    # -- to be provided by subclasses
    def logits(self, toks):
        raise NotImplementedError

    def phase(self, toks):
        raise NotImplementedError

    def masks(self, toks):
        """[B, n, 4] bool: which tokens keep each prefix physical."""
        B, n = toks.shape
        if self.phys is None:                     # general sector: Algorithm 1 per prefix
            sec = self.sector
            m = torch.zeros((B, n, 4), dtype=torch.bool)
            for r in range(B):
                s = sec.root()
                for p in range(n):
                    m[r, p] = torch.tensor(sec.child_mask_state(p, s))
                    t = int(toks[r, p])
                    s = sec.compose(sec.compose(s, sec.local_eigs(2 * p, t & 1)),
                                    sec.local_eigs(2 * p + 1, t >> 1))
            m[:, self.mask_levels:, :] = True
            return m
        alpha = (toks & 1)
        beta = (toks >> 1)
        a = torch.cat([torch.zeros((B, 1), dtype=torch.long), alpha.cumsum(1)[:, :-1]], 1)
        b = torch.cat([torch.zeros((B, 1), dtype=torch.long), beta.cumsum(1)[:, :-1]], 1)
        p = torch.arange(n).expand(B, n)
        flips = self.z2_flip[p, toks]                      # [B, n]
        zi = torch.zeros((B, n), dtype=torch.long)
        for q in range(1, n):
            zi[:, q] = zi[:, q - 1] ^ flips[:, q - 1]
        m = self.phys[p, a, b, zi]
        m[:, self.mask_levels:, :] = True
        return m

    def log_cond(self, toks):
        """Masked log conditional probabilities, [B, n, 4] (-inf where masked).
        After an unphysical prefix no token is physical: the whole row is -inf
        (probability zero), so a configuration outside the sector has
        log|psi| = -inf."""
        lg = self.logits(toks)
        m = self.masks(toks)
        lp = torch.log_softmax(lg.masked_fill(~m, float("-inf")), dim=-1)
        return lp.masked_fill(~m.any(-1, keepdim=True), float("-inf"))

    def log_abs(self, toks):
        lp = self.log_cond(toks)
        return 0.5 * torch.gather(lp, 2, toks.unsqueeze(-1)).squeeze(-1).sum(1)

    def amplitudes(self, xs):
        toks = tokens_from_ints(xs, self.n)
        return self.log_abs(toks), self.phase(toks)

    def flat_grad(self, spec):
        return np.concatenate([
            (self.t[k].grad if self.t[k].grad is not None else torch.zeros_like(self.t[k]))
            .detach().numpy().reshape(-1) for k, _ in spec])


class MLPModel(AmplitudeModel):
    """One MLP per token: one-hot(x_<p) -> 64 tanh -> 64 leaky ReLU -> 4 logits, 4 phases."""

    def _outputs(self, toks):
        B = toks.shape[0]
        outs = []
        for p in range(self.n):
            inp = F.one_hot(toks[:, :p], 4).to(torch.float64).reshape(B, 4 * p)
            t = self.t
            h1 = torch.tanh(inp @ t[f"mlp{p}.w1"] + t[f"mlp{p}.b1"])
            z = h1 @ t[f"mlp{p}.w2"] + t[f"mlp{p}.b2"]
            h2 = torch.where(z >= 0, z, 0.01 * z)     # the x >= 0 branch owns x = 0
            outs.append(h2 @ t[f"mlp{p}.w3"] + t[f"mlp{p}.b3"])
        return torch.stack(outs, 1)          # [B, n, 8]

    def logits(self, toks):
        return self._outputs(toks)[:, :, :4]

    def phase(self, toks):
        ph = self._outputs(toks)[:, :, 4:]
        return torch.gather(ph, 2, toks.unsqueeze(-1)).squeeze(-1).sum(1)


def layer_norm(x, g, b, eps=1e-5):
    mu = x.mean(-1, keepdim=True)
    var = ((x - mu) ** 2).mean(-1, keepdim=True)
    return (x - mu) / torch.sqrt(var + eps) * g + b


def gelu_tanh(x):
    return 0.5 * x * (1.0 + torch.tanh(math.sqrt(2.0 / math.pi) * (x + 0.044715 * x ** 3)))


class TransformerModel(AmplitudeModel):
    """Pre-LN decoder over [BOS, x_0 .. x_{n-2}]; output p predicts token p."""

    def __init__(self, params, sector, n_heads, **kw):
        super().__init__(params, sector, **kw)
        self.n_heads = n_heads
        self.n_layers = sum(1 for k in params if k.endswith(".wqkv"))

    def logits(self, toks):
        t, B, n = self.t, toks.shape[0], self.n
        d = t["tok_emb"].shape[1]
        H = self.n_heads
        dh = d // H
        inp = torch.cat([torch.full((B, 1), 4, dtype=torch.long), toks[:, :n - 1]], 1)
        h = t["tok_emb"][inp] + t["pos_emb"][None, :n]
        causal = torch.ones((n, n), dtype=torch.bool).tril()
        for l in range(self.n_layers):
            a = layer_norm(h, t[f"l{l}.ln1_g"], t[f"l{l}.ln1_b"])
            qkv = a @ t[f"l{l}.wqkv"] + t[f"l{l}.bqkv"]
            q, k, v = qkv.split(d, dim=-1)
            q = q.reshape(B, n, H, dh).transpose(1, 2)
            k = k.reshape(B, n, H, dh).transpose(1, 2)
            v = v.reshape(B, n, H, dh).transpose(1, 2)
            s = (q @ k.transpose(-1, -2)) / math.sqrt(dh)
            s = s.masked_fill(~causal, float("-inf"))
            o = (torch.softmax(s, -1) @ v).transpose(1, 2).reshape(B, n, d)
            h = h + o @ t[f"l{l}.wo"] + t[f"l{l}.bo"]
            a = layer_norm(h, t[f"l{l}.ln2_g"], t[f"l{l}.ln2_b"])
            h = h + gelu_tanh(a @ t[f"l{l}.w1"] + t[f"l{l}.b1"]) @ t[f"l{l}.w2"] + t[f"l{l}.b2"]
        hf = layer_norm(h, t["lnf_g"], t["lnf_b"])
        return hf @ t["whead"] + t["bhead"] + t["logit_bias"][None, :n]

    def phase(self, toks):
        t, B, n = self.t, toks.shape[0], self.n
        oh = F.one_hot(toks, 4).to(torch.float64).reshape(B, 4 * n)
        rows = t["ph_w1"].shape[0]
        if rows > 4 * n:     # model shared with larger molecules: absent positions are zero
            oh = torch.cat([oh, torch.zeros((B, rows - 4 * n), dtype=torch.float64)], 1)
        z = gelu_tanh(oh @ t["ph_w1"] + t["ph_b1"])
        z = gelu_tanh(z @ t["ph_w2"] + t["ph_b2"])
        return (z @ t["ph_w3"] + t["ph_b3"])[:, 0]


def build_model(cfg, params, sector=None, requires_grad=False, mask_levels=None):
    sector = sector or Sector(cfg["n"], cfg["n_alpha"], cfg["n_beta"])
    if cfg["model"] == "mlp":
        return MLPModel(params, sector, mask_levels=mask_levels, requires_grad=requires_grad)
    if cfg["model"] == "nade":
        from .nade import NADEModel
        return NADEModel(params, sector, mask_levels=mask_levels, requires_grad=requires_grad)
    return TransformerModel(params, sector, cfg["n_heads"], mask_levels=mask_levels,
                            requires_grad=requires_grad)


class TableModel:
    """Explicit amplitudes over an enumerated basis (no network): psi(x) is
    looked up; used to test the local energy independently of any network."""

    def __init__(self, basis, psi):
        self.index = {int(x): k for k, x in enumerate(basis)}
        self.psi = np.asarray(psi, dtype=np.complex128)

    def amplitudes(self, xs):
        v = self.psi[[self.index[int(x)] for x in xs]]
        return torch.from_numpy(np.log(np.abs(v))), torch.from_numpy(np.angle(v))
