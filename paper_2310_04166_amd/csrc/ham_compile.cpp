// Hamiltonian compiler (host): molecular integrals -> Jordan-Wigner Pauli
// strings grouped by X/Y flip mask.  Paper: "System description" (the H_SQ
// equation; Jordan-Wigner keeps the occupation-number interpretation).
//
// Each creation/annihilation product is mapped exactly.  Acting on |x>, an
// operator a_j or a+_j flips bit j, requires the bit's current value (1 for a,
// 0 for a+), and contributes the Jordan-Wigner string prod_{k<j} Z_k, i.e. the
// sign (-1)^popcount(current & below(j)).  Writing current = x ^ F (F = flips
// already applied) splits that sign into a fixed part (-1)^popcount(F & below)
// and an x-dependent part (-1)^popcount(x & below).  The occupation
// requirements are projectors [x_j = r] = (1 + (-1)^r (-1)^x_j) / 2, which
// expand into Z strings.  So every term becomes a sum of
//     c (-1)^popcount(x & z) |x ^ f>,
// which is the Pauli string with X/Y on f and Z/Y on z, the i-factors of its
// Y's folded into the real coefficient c.  Strings with an odd number of Y's
// (odd popcount(f & z)) cancel for a real symmetric H and are dropped.
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "ham.h"

namespace {

struct Key {
  uint64_t f, z;
  bool operator==(const Key &o) const { return f == o.f && z == o.z; }
};
struct KeyHash {
  size_t operator()(const Key &k) const {
    uint64_t h = k.f * 0x9E3779B97F4A7C15ull ^ (k.z + 0x632BE59BD9B4E019ull + (k.f << 6));
    return static_cast<size_t>(h ^ (h >> 29));
  }
};

using TermMap = std::unordered_map<Key, double, KeyHash>;

struct Op {
  bool create;
  int j;
};

inline uint64_t below(int j) { return (j == 0) ? 0ull : ((~0ull) >> (64 - j)); }

// Adds the Pauli expansion of c * (ops[0] ops[1] ... ops[k-1]) to the map.
void add_product(TermMap &map, double c, const Op *ops, int k) {
  uint64_t F = 0, z = 0, cond_mask = 0, cond_val = 0;
  double sgn = 1.0;
  for (int t = k - 1; t >= 0; --t) {  // rightmost acts first
    const int j = ops[t].j;
    const uint64_t bit = 1ull << j;
    const uint64_t req = (ops[t].create ? 0ull : 1ull) ^ ((F >> j) & 1ull);
    if (cond_mask & bit) {
      if (((cond_val >> j) & 1ull) != req) return;  // contradictory: term is zero
    } else {
      cond_mask |= bit;
      cond_val |= req << j;
    }
    z ^= below(j);
    if (__builtin_popcountll(F & below(j)) & 1) sgn = -sgn;
    F ^= bit;
  }
  // expand prod over conditioned bits of (1 + (-1)^r Z_j) / 2
  int idx[8];
  int nc = 0;
  for (int j = 0; j < 64; ++j)
    if ((cond_mask >> j) & 1ull) idx[nc++] = j;
  const double scale = c * sgn / double(1u << nc);
  for (uint32_t s = 0; s < (1u << nc); ++s) {
    uint64_t zz = z;
    double v = scale;
    for (int b = 0; b < nc; ++b) {
      if ((s >> b) & 1u) {
        zz ^= 1ull << idx[b];
        if ((cond_val >> idx[b]) & 1ull) v = -v;
      }
    }
    map[Key{F, zz}] += v;
  }
}

}  // namespace

extern "C" int ham_compile(const double *h1, const double *eri, int n, double e_core,
                           int n_alpha, int n_beta, nqs_ham **out) {
  return nqs::guarded([&] {
    NQS_REQUIRE(out && h1 && eri, NQS_EINVAL, "ham_compile: null argument");
    *out = nullptr;
    NQS_REQUIRE(n >= 1, NQS_EINVAL, "ham_compile: n_spatial < 1");
    NQS_REQUIRE(n <= 32, NQS_EUNSUPPORTED, "ham_compile: more than 64 spin-orbitals");
    NQS_REQUIRE(n_alpha >= 0 && n_alpha <= n && n_beta >= 0 && n_beta <= n, NQS_EINVAL,
                "ham_compile: electron counts out of range");
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q)
        NQS_REQUIRE(h1[p * n + q] == h1[q * n + p], NQS_EINVAL, "ham_compile: h1 not symmetric");

    TermMap map;
    map.reserve(size_t(1) << 20);
    map[Key{0, 0}] += e_core;
    Op ops[4];
    for (int s = 0; s < 2; ++s)
      for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
          const double v = h1[p * n + q];
          if (v == 0.0) continue;
          ops[0] = {true, 2 * p + s};
          ops[1] = {false, 2 * q + s};
          add_product(map, v, ops, 2);
        }
    for (int s = 0; s < 2; ++s)
      for (int t = 0; t < 2; ++t)
        for (int p = 0; p < n; ++p)
          for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
              for (int u = 0; u < n; ++u) {
                const double v = eri[((size_t(p) * n + q) * n + r) * n + u];
                if (v == 0.0) continue;
                ops[0] = {true, 2 * p + s};
                ops[1] = {true, 2 * r + t};
                ops[2] = {false, 2 * u + t};
                ops[3] = {false, 2 * q + s};
                add_product(map, 0.5 * v, ops, 4);
              }

    struct Entry {
      uint64_t f, z;
      double c;
    };
    std::vector<Entry> kept;
    kept.reserve(map.size());
    double cmax = 0.0, odd_max = 0.0;
    for (const auto &kv : map) cmax = std::max(cmax, std::fabs(kv.second));
    for (const auto &kv : map) {
      const bool odd = __builtin_popcountll(kv.first.f & kv.first.z) & 1;
      if (odd) {
        odd_max = std::max(odd_max, std::fabs(kv.second));
        continue;
      }
      if (kv.second == 0.0) continue;
      kept.push_back({kv.first.f, kv.first.z, kv.second});
    }
    NQS_REQUIRE(odd_max <= 1e-12 * std::max(cmax, 1e-300), NQS_EINVAL,
                "ham_compile: integrals are not symmetric (imaginary Pauli terms remain)");
    std::sort(kept.begin(), kept.end(), [](const Entry &a, const Entry &b) {
      return a.f != b.f ? a.f < b.f : a.z < b.z;
    });

    auto *H = new nqs_ham();
    H->n = n;
    H->N = 2 * n;
    H->n_alpha = n_alpha;
    H->n_beta = n_beta;
    H->e_core = e_core;
    H->flip.push_back(0);  // the diagonal group comes first, even if empty
    H->off.push_back(0);
    for (const Entry &e : kept) {
      if (e.f != H->flip.back()) {
        H->flip.push_back(e.f);
        H->off.push_back(int64_t(H->zmask.size()));
      }
      H->zmask.push_back(e.z);
      H->coef.push_back(e.c);
    }
    H->off.push_back(int64_t(H->zmask.size()));
    *out = H;
  });
}

extern "C" int ham_info(const nqs_ham *H, int64_t *G, int64_t *T) {
  return nqs::guarded([&] {
    NQS_REQUIRE(H, NQS_EINVAL, "ham_info: null handle");
    if (G) *G = int64_t(H->flip.size());
    if (T) *T = int64_t(H->zmask.size());
  });
}

extern "C" int ham_tables(const nqs_ham *H, uint64_t *flip, int64_t *off, uint64_t *zmask,
                          double *coef) {
  return nqs::guarded([&] {
    NQS_REQUIRE(H, NQS_EINVAL, "ham_tables: null handle");
    if (flip) std::copy(H->flip.begin(), H->flip.end(), flip);
    if (off) std::copy(H->off.begin(), H->off.end(), off);
    if (zmask) std::copy(H->zmask.begin(), H->zmask.end(), zmask);
    if (coef) std::copy(H->coef.begin(), H->coef.end(), coef);
  });
}

// Z2 symmetries (paper: "Molecular symmetries"): Z on the qubits of m commutes
// with a Pauli string iff m and the string's X/Y support f share an even number
// of qubits, so the symmetries of H are the null space over GF(2) of its flip
// masks.  Elimination column by column: each pivot row owns its lowest set
// bit, which the other rows do not contain; every free column c then gives the
// null vector e_c + sum of the pivot columns whose row contains c.  Returned:
// the null vectors that are independent modulo the parities of the alpha and
// beta electron numbers (which the electron counts already fix).
extern "C" int ham_z2_symmetries(const nqs_ham *H, int max_gen, uint64_t *masks, int *n_gen) {
  return nqs::guarded([&] {
    NQS_REQUIRE(H && n_gen, NQS_EINVAL, "ham_z2_symmetries: null argument");
    NQS_REQUIRE(max_gen >= 0 && (max_gen == 0 || masks), NQS_EINVAL,
                "ham_z2_symmetries: null mask array");
    const int N = H->N;
    std::vector<uint64_t> rows;             // reduced rows, pivot = lowest set bit
    std::vector<int> pivot_of(N, -1);       // column -> row index
    for (uint64_t f : H->flip) {
      for (size_t r = 0; r < rows.size(); ++r) {
        const int c = __builtin_ctzll(rows[r]);
        if ((f >> c) & 1ull) f ^= rows[r];
      }
      if (f == 0) continue;
      const int c = __builtin_ctzll(f);
      for (auto &r : rows)
        if ((r >> c) & 1ull) r ^= f;
      pivot_of[c] = int(rows.size());
      rows.push_back(f);
    }
    // null vectors, kept when independent of the alpha / beta parity masks
    // and of the vectors kept before (the electron counts fix those parities)
    uint64_t alpha = 0;
    for (int p = 0; p < H->n; ++p) alpha |= 1ull << (2 * p);
    std::vector<uint64_t> span = {alpha, alpha << 1};   // reduced, pivot = highest bit
    auto reduce = [&](uint64_t v) {
      for (uint64_t b : span)
        if ((v >> (63 - __builtin_clzll(b))) & 1ull) v ^= b;
      return v;
    };
    {
      std::vector<uint64_t> echelon;
      for (uint64_t b : span) {
        for (uint64_t e : echelon)
          if ((b >> (63 - __builtin_clzll(e))) & 1ull) b ^= e;
        if (b) echelon.push_back(b);
      }
      span = echelon;
    }
    int count = 0;
    for (int c = 0; c < N; ++c) {
      if (pivot_of[c] >= 0) continue;
      uint64_t m = 1ull << c;
      for (int p = 0; p < N; ++p)
        if (pivot_of[p] >= 0 && ((rows[size_t(pivot_of[p])] >> c) & 1ull)) m |= 1ull << p;
      const uint64_t r = reduce(m);
      if (r == 0) continue;
      for (auto &b : span)                 // keep the span reduced on the new pivot
        if ((b >> (63 - __builtin_clzll(r))) & 1ull) b ^= r;
      span.push_back(r);
      if (count < max_gen) masks[count] = m;
      ++count;
    }
    *n_gen = count;
    NQS_REQUIRE(count <= max_gen, NQS_ECAPACITY,
                "ham_z2_symmetries: more symmetries than max_gen (n_gen holds the count)");
  });
}

extern "C" void ham_destroy(nqs_ham *H) { delete H; }

void nqs_ham::upload() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (device == dev && d_flip.ptr) return;
  const size_t G = flip.size(), T = zmask.size();
  HIP_OK(hipMemcpy(d_flip.reserve(G * 8), flip.data(), G * 8, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_off.reserve((G + 1) * 8), off.data(), (G + 1) * 8, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_zmask.reserve(T * 8), zmask.data(), T * 8, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_coef.reserve(T * 8), coef.data(), T * 8, hipMemcpyHostToDevice));
  device = dev;
}
