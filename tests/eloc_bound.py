"""First-order error bound of a mixed-precision local energy (test helper).

Local-energy equation: E_loc(x) = sum_x' H_xx' psi(x') / psi(x).  If the GPU's
log psi carries a complex error Delta (log|psi| and phase), then

    |dE_loc(x)| <= sum_{x' != x} |H_xx'| |psi(x') / psi(x)| |Delta(x') - Delta(x)|
                <= 2 eps(x) A(x),   A(x) = sum_{x' != x} |H_xx' psi(x') / psi(x)|,

with eps(x) the largest |Delta| over x and its connected x' (terms of second
order in eps are below eps^2 A(x)).  ``check`` evaluates the oracle's E_loc,
A(x) and eps(x) for each sample, from the GPU's amplitudes of the same x'."""
import numpy as np
import torch

from oracle.hamiltonian import slater_condon_row


def check(oracle_model, h, eri, xs, gpu_amplitudes, tag=None):
    """For configurations ``xs`` (ints): oracle E_loc, A(x) and eps(x).
    ``gpu_amplitudes(list of ints) -> (logabs, phase)`` numpy arrays; ``tag``
    (optional) maps an occupation int to the word the GPU model takes."""
    rows = [slater_condon_row(h, eri, int(x)) for x in xs]
    flat = [xp for r in rows for xp in r[0]]
    with torch.no_grad():
        la_r, ph_r = (v.numpy() for v in oracle_model.amplitudes(flat))
    words = flat if tag is None else [tag(v) for v in flat]
    la_g, ph_g = gpu_amplitudes(words)
    out, o = [], 0
    for xp, vals in rows:
        k = len(xp)
        lr, pr = la_r[o:o + k], ph_r[o:o + k]
        delta = (la_g[o:o + k] - lr) + 1j * (ph_g[o:o + k] - pr)
        ratio = np.exp((lr - lr[0]) + 1j * (pr - pr[0]))
        v = np.asarray(vals)
        eloc = complex(np.sum(v * ratio))
        A = float(np.sum(np.abs(v[1:] * ratio[1:])))
        out.append((eloc, A, float(np.max(np.abs(delta)))))
        o += k
    return out


def gpu_amplitudes(nqs, model):
    def f(words):
        x = torch.as_tensor(np.asarray(words, dtype=np.uint64).view(np.int64)).cuda()
        la, ph = nqs.amp_forward(model, x)
        return la.cpu().numpy(), ph.cpu().numpy()
    return f
