"""Symmetry sector and physicality (paper: "Physicality evaluation algorithm",
Algorithm 1; Appendix A; "System description" for the HF sector).

The quantum-number symmetries are the particle number, s(x) = sum_i x_i, and
the spin projection, s(x) = 1/2 sum_i (-1)^(i-1) x_i with i counted from 1
(Appendix A).  Both are additive, so the composition operation of Algorithm 1
is addition.  The spin projection is carried as the integer 2 S_z to keep the
arithmetic exact.  Optional Z2 symmetries ("Molecular symmetries"): Z on the
qubits of a mask m, eigenvalue s(x) = prod over qubits i in m of (-1)^x_i,
composed by multiplication.  The target sector is that of the Hartree-Fock
determinant.

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


def local_eigs(i, bit, z2=()):
    """(particle number, 2 S_z, Z2 eigenvalues ...) of qubit i (counted from 1)
    holding ``bit``."""
    zs = tuple(-1 if bit and (m >> (i - 1)) & 1 else 1 for m in z2)
    return (bit, bit if (i - 1) % 2 == 0 else -bit) + zs


def compose(s, e):
    """The composition of Algorithm 1: addition for the particle number and
    2 S_z, multiplication for the Z2 eigenvalues."""
    return (s[0] + e[0], s[1] + e[1]) + tuple(u * v for u, v in zip(s[2:], e[2:]))


def eigs(x, N, z2=()):
    s = (0, 0) + (1,) * len(z2)
    for i in range(1, N + 1):
        s = compose(s, local_eigs(i, (x >> (i - 1)) & 1, z2))
    return s


class IsPhys:
    """Algorithm 1 with its lookup table, over the N-qubit binary tree."""

    def __init__(self, N, s_ref, z2=()):
        self.N, self.s_ref, self.z2, self.lookup = N, s_ref, tuple(z2), {}

    def __call__(self, i, s):
        key = (i, s)
        if key not in self.lookup:
            if i == self.N + 1:
                self.lookup[key] = (s == self.s_ref)
            else:
                children = []
                for bit in (0, 1):
                    children.append(self(i + 1, compose(s, local_eigs(i, bit, self.z2))))
                self.lookup[key] = children[0] or children[1]
        return self.lookup[key]


class Sector:
    """The (N_alpha, N_beta) sector of an n-spatial-orbital system, optionally
    restricted by Z2 symmetries (qubit masks ``z2``) to the eigenvalues of the
    HF determinant."""

    def __init__(self, n, n_alpha, n_beta, z2=()):
        self.n, self.n_alpha, self.n_beta = n, n_alpha, n_beta
        self.N = 2 * n
        self.z2 = tuple(int(m) for m in z2)
        self.x_hf = hf_config(n, n_alpha, n_beta)
        self.s_ref = eigs(self.x_hf, self.N, self.z2)
        self.isphys = IsPhys(self.N, self.s_ref, self.z2)

    def prefix_z2(self, x, p):
        """Z2 partial eigenvalues of the first p tokens of x."""
        return eigs(x & ((1 << (2 * p)) - 1), self.N, self.z2)[2:]

    def token_phys(self, p, a, b, z=()):
        """Physicality of a token prefix of length p holding a alpha and b beta
        electrons (and Z2 partial eigenvalues z): Algorithm 1 at qubit level
        2p + 1."""
        return self.isphys(2 * p + 1, (a + b, a - b) + (tuple(z) or (1,) * len(self.z2)))

    def child_mask(self, p, a, b, z=()):
        """Which of the 4 tokens at position p keep the prefix physical."""
        z = tuple(z) or (1,) * len(self.z2)
        out = []
        for k in range(4):
            e = compose(compose((0, 0) + z, local_eigs(2 * p + 1, k & 1, self.z2)),
                        local_eigs(2 * p + 2, k >> 1, self.z2))
            out.append(self.token_phys(p + 1, a + (k & 1), b + (k >> 1), e[2:]))
        return out

    def contains(self, x):
        return eigs(x, self.N, self.z2) == self.s_ref and x >> self.N == 0

    def enumerate(self):
        """Every basis vector of the sector, ascending as integers."""
        alpha = [sum(1 << (2 * p) for p in c) for c in combinations(range(self.n), self.n_alpha)]
        beta = [sum(1 << (2 * p + 1) for p in c) for c in combinations(range(self.n), self.n_beta)]
        out = sorted(a | b for a in alpha for b in beta)
        if self.z2:
            out = [x for x in out if eigs(x, self.N, self.z2)[2:] == self.s_ref[2:]]
        return out


def tokens_of(x, n):
    return [((x >> (2 * p)) & 1) + 2 * ((x >> (2 * p + 1)) & 1) for p in range(n)]


def config_of(tokens):
    x = 0
    for p, t in enumerate(tokens):
        x |= (int(t) & 1) << (2 * p)
        x |= ((int(t) >> 1) & 1) << (2 * p + 1)
    return x


class GeneralSector:
    """A sector fixed by any additive quantum numbers plus optional Z2 parities
    (paper: "Physicality evaluation algorithm", Algorithm 1 for N_sym
    symmetries, Appendix A): additive symmetry s gives qubit i (0-based here)
    holding bit b the integer eigenvalue ``eig[s][2 i + b]``, and the
    eigenvalue of a configuration is the sum over qubits (composition by
    addition); Z2 symmetry j gives (-1)^(x_i) on the qubits of ``z2[j]``
    (composition by multiplication, carried as a parity bit).  The sector is
    every configuration whose sums equal ``targets`` and whose parities equal
    ``z2_targets`` (0 = eigenvalue +1).

    The particle number is eig[2i + b] = b, 2 S_z is (-1)^i b, and any
    combination of them is another instance.  Tokens as in Sector."""

    general = True

    def __init__(self, n, eig, targets, z2=(), z2_targets=None):
        self.n, self.N = n, 2 * n
        self.eig = [tuple(int(v) for v in e) for e in eig]
        assert all(len(e) == 2 * self.N for e in self.eig)
        self.targets = tuple(int(t) for t in targets)
        self.z2 = tuple(int(m) for m in z2)
        zt = [0] * len(self.z2) if z2_targets is None else [int(v) for v in z2_targets]
        self.s_ref = self.targets + tuple(-1 if t else 1 for t in zt)
        self.lookup = {}

    def local_eigs(self, i, bit):
        """Eigenvalues of qubit i (0-based) holding ``bit``."""
        return tuple(e[2 * i + bit] for e in self.eig) + \
            tuple(-1 if bit and (m >> i) & 1 else 1 for m in self.z2)

    def compose(self, s, e):
        k = len(self.eig)
        return tuple(a + b for a, b in zip(s[:k], e[:k])) + \
            tuple(a * b for a, b in zip(s[k:], e[k:]))

    def root(self):
        return (0,) * len(self.eig) + (1,) * len(self.z2)

    def isphys(self, i, s):
        """Algorithm 1 over the binary tree: can the prefix of qubits 0..i-1 with
        eigenvalues s be completed into the sector?"""
        key = (i, s)
        if key not in self.lookup:
            if i == self.N:
                self.lookup[key] = s == self.s_ref
            else:
                self.lookup[key] = any(self.isphys(i + 1, self.compose(s, self.local_eigs(i, b)))
                                       for b in (0, 1))
        return self.lookup[key]

    def prefix_state(self, x, p):
        s = self.root()
        for i in range(2 * p):
            s = self.compose(s, self.local_eigs(i, (x >> i) & 1))
        return s

    def child_mask_state(self, p, s):
        """Which of the 4 tokens at position p keep a prefix with eigenvalues s
        physical."""
        out = []
        for k in range(4):
            e = self.compose(self.compose(s, self.local_eigs(2 * p, k & 1)),
                             self.local_eigs(2 * p + 1, k >> 1))
            out.append(self.isphys(2 * p + 2, e))
        return out

    def contains(self, x):
        return x >> self.N == 0 and self.prefix_state(x, self.n) == self.s_ref

    def enumerate(self):
        """Every configuration of the sector, ascending, by walking the token
        tree through physical prefixes."""
        out = []

        def walk(p, x, s):
            if p == self.n:
                out.append(x)
                return
            for k, ok in enumerate(self.child_mask_state(p, s)):
                if ok:
                    e = self.compose(self.compose(s, self.local_eigs(2 * p, k & 1)),
                                     self.local_eigs(2 * p + 1, k >> 1))
                    walk(p + 1, x | (k << (2 * p)), e)

        if self.isphys(0, self.root()):
            walk(0, 0, self.root())
        return sorted(out)


def particle_number_eigs(n):
    return [b for i in range(2 * n) for b in (0, 1)]


def two_sz_eigs(n):
    return [b if i % 2 == 0 else -b for i in range(2 * n) for b in (0, 1)]
