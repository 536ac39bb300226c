"""Symmetry sector and physicality (paper: "Physicality evaluation algorithm",
Algorithm 1; Appendix A; "System description" for the HF sector).

The quantum-number symmetries are the particle number, s(x) = sum_i x_i, and
the spin projection, s(x) = 1/2 sum_i (-1)^(i-1) x_i with i counted from 1
(Appendix A).  Both are additive, so the composition operation of Algorithm 1
is addition.  The spin projection is carried as the integer 2 S_z to keep the
arithmetic exact.  The target sector is that of the Hartree-Fock determinant.

Tokens: the sampler moves one spatial orbital (two qubits) per level, token
t_p = x_{2p} + 2 x_{2p+1} in {0: empty, 1: alpha, 2: beta, 3: both}.  Token
level p of the 4-ary tree is qubit level 2p + 1 (counted from 1) of the binary
tree, so the token-level physicality table is read off Algorithm 1.
"""
from itertools import combinations


def hf_config(n, n_alpha, n_beta):
    """x_HF: alpha spin-orbitals 2p for p < n_alpha, beta 2p+1 for p < n_beta."""
    x = 0
    for p in range(n_alpha):
        x |= 1 << (2 * p)
    for p in range(n_beta):
        x |= 1 << (2 * p + 1)
    return x


def local_eigs(i, bit):
    """(particle number, 2 S_z) of qubit i (counted from 1) holding ``bit``."""
    return (bit, bit if (i - 1) % 2 == 0 else -bit)


def eigs(x, N):
    s = (0, 0)
    for i in range(1, N + 1):
        e = local_eigs(i, (x >> (i - 1)) & 1)
        s = (s[0] + e[0], s[1] + e[1])
    return s


class IsPhys:
    """Algorithm 1 with its lookup table, over the N-qubit binary tree."""

    def __init__(self, N, s_ref):
        self.N, self.s_ref, self.lookup = N, s_ref, {}

    def __call__(self, i, s):
        key = (i, s)
        if key not in self.lookup:
            if i == self.N + 1:
                self.lookup[key] = (s == self.s_ref)
            else:
                children = []
                for bit in (0, 1):
                    e = local_eigs(i, bit)
                    children.append(self(i + 1, (s[0] + e[0], s[1] + e[1])))
                self.lookup[key] = children[0] or children[1]
        return self.lookup[key]


class Sector:
    """The (N_alpha, N_beta) sector of an n-spatial-orbital system."""

    def __init__(self, n, n_alpha, n_beta):
        self.n, self.n_alpha, self.n_beta = n, n_alpha, n_beta
        self.N = 2 * n
        self.x_hf = hf_config(n, n_alpha, n_beta)
        self.s_ref = eigs(self.x_hf, self.N)
        self.isphys = IsPhys(self.N, self.s_ref)

    def token_phys(self, p, a, b):
        """Physicality of a token prefix of length p holding a alpha and b beta
        electrons: Algorithm 1 at qubit level 2p + 1."""
        return self.isphys(2 * p + 1, (a + b, a - b))

    def child_mask(self, p, a, b):
        """Which of the 4 tokens at position p keep the prefix physical."""
        return [self.token_phys(p + 1, a + (k & 1), b + (k >> 1)) for k in range(4)]

    def contains(self, x):
        return eigs(x, self.N) == self.s_ref and x >> self.N == 0

    def enumerate(self):
        """Every basis vector of the sector, ascending as integers."""
        alpha = [sum(1 << (2 * p) for p in c) for c in combinations(range(self.n), self.n_alpha)]
        beta = [sum(1 << (2 * p + 1) for p in c) for c in combinations(range(self.n), self.n_beta)]
        return sorted(a | b for a in alpha for b in beta)


def tokens_of(x, n):
    return [((x >> (2 * p)) & 1) + 2 * ((x >> (2 * p + 1)) & 1) for p in range(n)]


def config_of(tokens):
    x = 0
    for p, t in enumerate(tokens):
        x |= (int(t) & 1) << (2 * p)
        x |= ((int(t) >> 1) & 1) << (2 * p + 1)
    return x
