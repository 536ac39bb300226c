// C-ABI entry points: model handles, amplitudes, local energy, reducer, Adam.
#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ham.h"
#include "model.h"
#include "ops.h"

namespace nqs {

namespace {
thread_local std::string g_last_error;
}  // namespace

void set_last_error(const std::string &msg) { g_last_error = msg; }

// defined in eloc.hip
// fp32_ratio: psi(x') / psi(x) from the log-amplitude differences in fp32 (bf16 mode),
// the n_amp distinct amplitudes packed as fp32 pairs into lp2_ws first (when given)
void launch_accumulate(int64_t n, const int64_t *off, const double *hval, const uint32_t *uid,
                       const double *la_p, const double *ph_p, const double *la_x,
                       const double *ph_x, const double *hdiag, double *eloc, hipStream_t s,
                       bool fp32_ratio, int64_t n_amp = 0, float2 *lp2_ws = nullptr);
// defined in dedupe.hip
int64_t dedupe_pairs(uint64_t *xp, int64_t n, int key_bits, int pm, uint64_t *keys_sorted,
                     uint32_t *vals_in, uint32_t *vals_sorted, uint32_t *head, uint32_t *run,
                     uint64_t *ukeys, uint32_t *pair_uid, DevBuf &tmp, hipStream_t s);
void launch_reduce(const double *eloc, const uint64_t *counts, int64_t n, double *sums,
                   hipStream_t s);
void launch_weights(const double *eloc, const uint64_t *counts, int64_t n, const double *sums,
                    double *gl, double *gp, hipStream_t s);
void launch_adam(void *p, const void *g, void *m, void *v, int64_t n, int elem, double lr,
                 double b1, double b2, double eps, int64_t t, hipStream_t s);

namespace {

void check_device() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
    throw Error(NQS_EHIP, "no HIP device available");
}

// Algorithm 1 evaluated bottom-up over token levels: phys[p][a][b][z] holds
// the 4-bit set of tokens k whose child prefix at level p+1 - a + k&1 alpha,
// b + k>>1 beta electrons, Z2 parities z ^ dz(p, k) - can still reach
// (n_alpha, n_beta) and the target parities at level n.  The partial Z2
// eigenvalues (+-1, composed by multiplication) are carried as parity bits
// (composed by XOR); without Z2 symmetries z has the single value 0.
std::vector<uint8_t> physical_children(int n, int na, int nb, const std::vector<uint64_t> &z2,
                                       uint32_t target) {
  const int S = n + 1, Z = 1 << int(z2.size());
  std::vector<uint8_t> reach(size_t(S + 1) * S * S * Z, 0);  // reach[p][a][b][z]
  auto at = [&](int p, int a, int b, int z) { return ((size_t(p) * S + a) * S + b) * Z + z; };
  for (int a = 0; a <= n; ++a)
    for (int b = 0; b <= n; ++b)
      for (int z = 0; z < Z; ++z) reach[at(n, a, b, z)] = (a == na && b == nb && uint32_t(z) == target);
  std::vector<uint8_t> kids(size_t(S) * S * S * Z, 0);
  for (int p = n - 1; p >= 0; --p) {
    int dz[4];                                       // parity change of token k at level p
    for (int k = 0; k < 4; ++k) {
      dz[k] = 0;
      for (size_t j = 0; j < z2.size(); ++j) {
        const int bit = int(((z2[j] >> (2 * p)) & 1ull) & uint64_t(k & 1)) ^
                        int(((z2[j] >> (2 * p + 1)) & 1ull) & uint64_t(k >> 1));
        dz[k] |= bit << j;
      }
    }
    for (int a = 0; a <= n; ++a)
      for (int b = 0; b <= n; ++b)
        for (int z = 0; z < Z; ++z) {
          uint8_t mask = 0;
          for (int k = 0; k < 4; ++k) {
            const int a2 = a + (k & 1), b2 = b + (k >> 1);
            if (a2 <= n && b2 <= n && reach[at(p + 1, a2, b2, z ^ dz[k])]) mask |= uint8_t(1u << k);
          }
          kids[at(p, a, b, z)] = mask;
          reach[at(p, a, b, z)] = mask != 0;
        }
  }
  return kids;
}

// Algorithm 1 for general quantum numbers: n_add additive symmetries (qubit q
// holding bit b contributes eig[s][2 q + b] to symmetry s; composition by
// addition) and Z2 parities (composition by XOR), as a table of prefix states.
// Level p holds the states (partial sums, parities) of the physical prefixes of
// p tokens: those reachable from the empty prefix from which some completion
// reaches the targets.  Layout (int32): n + 1 level offsets, then four children
// per state (the child's index within level p + 1, or -1).
std::vector<int32_t> general_children(int n, int n_add, const std::vector<int32_t> &eig,
                                      const std::vector<int32_t> &target,
                                      const std::vector<uint64_t> &z2, uint32_t z2_target) {
  using State = std::vector<int64_t>;     // n_add partial sums, then the parity bits
  const int W = 4 * n;                     // eig entries per symmetry (2 per qubit)
  auto child = [&](const State &s, int p, int k) {
    State c = s;
    for (int a = 0; a < n_add; ++a)
      c[size_t(a)] += eig[size_t(a) * W + 2 * (2 * p) + (k & 1)] +
                      eig[size_t(a) * W + 2 * (2 * p + 1) + (k >> 1)];
    int64_t dz = 0;
    for (size_t j = 0; j < z2.size(); ++j)
      dz |= int64_t((((z2[j] >> (2 * p)) & 1ull) & uint64_t(k & 1)) ^
                    (((z2[j] >> (2 * p + 1)) & 1ull) & uint64_t(k >> 1))) << j;
    c[size_t(n_add)] ^= dz;
    return c;
  };
  // forward: every state reachable at each level
  std::vector<std::vector<State>> level(size_t(n) + 1);
  level[0].push_back(State(size_t(n_add) + 1, 0));
  for (int p = 0; p < n; ++p) {
    std::vector<State> next;
    for (const State &st : level[size_t(p)])
      for (int k = 0; k < 4; ++k) next.push_back(child(st, p, k));
    std::sort(next.begin(), next.end());
    next.erase(std::unique(next.begin(), next.end()), next.end());
    NQS_REQUIRE(next.size() <= (size_t(1) << 22), NQS_EUNSUPPORTED,
                "amp_model_set_symmetries: more than 2^22 prefix states in a level");
    level[size_t(p) + 1] = std::move(next);
  }
  // backward (Algorithm 1): a state is physical when a child is
  State goal(target.begin(), target.end());
  goal.push_back(int64_t(z2_target));
  std::vector<std::vector<State>> phys(size_t(n) + 1);
  for (const State &st : level[size_t(n)])
    if (st == goal) phys[size_t(n)].push_back(st);
  for (int p = n - 1; p >= 0; --p)
    for (const State &st : level[size_t(p)]) {
      bool ok = false;
      for (int k = 0; k < 4 && !ok; ++k)
        ok = std::binary_search(phys[size_t(p) + 1].begin(), phys[size_t(p) + 1].end(),
                                child(st, p, k));
      if (ok) phys[size_t(p)].push_back(st);   // level states are sorted, so phys is too
    }
  NQS_REQUIRE(!phys[0].empty(), NQS_EINVAL, "amp_model_set_symmetries: the sector is empty");
  std::vector<int32_t> out(size_t(n) + 1, 0);
  int64_t total = 0;
  for (int p = 0; p <= n; ++p) {
    out[size_t(p)] = int32_t(total);
    total += int64_t(phys[size_t(p)].size());
  }
  out.resize(size_t(n) + 1 + 4 * size_t(total), -1);
  for (int p = 0; p < n; ++p) {
    const auto &cur = phys[size_t(p)], &nxt = phys[size_t(p) + 1];
    for (size_t i = 0; i < cur.size(); ++i)
      for (int k = 0; k < 4; ++k) {
        const auto it = std::lower_bound(nxt.begin(), nxt.end(), child(cur[i], p, k));
        if (it != nxt.end() && *it == child(cur[i], p, k))
          out[size_t(n) + 1 + 4 * (size_t(out[size_t(p)]) + i) + size_t(k)] =
              int32_t(it - nxt.begin());
      }
  }
  return out;
}

// Sector tables of a model: one per molecule, physical-children table of each
// from Algorithm 1, masked levels from the model's pruning strategy.
void install_sectors(nqs_model &m, const std::vector<std::array<int, 3>> &secs, bool tagged) {
  std::vector<uint8_t> phys;
  std::vector<nqs_sector_info> info;
  for (const auto &sc : secs) {
    const int n = sc[0];
    nqs_sector_info si{};
    si.n = n;
    si.na = sc[1];
    si.nb = sc[2];
    si.mask_levels = m.strategy == NQS_MU ? n : m.strategy == NQS_DU ? 0 : std::max(n - m.dlev, 0);
    si.phys_off = int64_t(phys.size());
    // Z2 symmetries only for the model's own sector (untagged words)
    const std::vector<uint64_t> none;
    const std::vector<uint64_t> &z2 = tagged ? none : m.z2;
    si.nz2 = int32_t(z2.size());
    for (size_t j = 0; j < z2.size(); ++j) si.z2[j] = z2[j];
    const std::vector<uint8_t> t = physical_children(n, si.na, si.nb, z2, tagged ? 0u : m.z2_target);
    phys.insert(phys.end(), t.begin(), t.end());
    info.push_back(si);
  }
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(m.phys.reserve(phys.size()), phys.data(), phys.size(), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(m.sec.reserve(info.size() * sizeof(nqs_sector_info)), info.data(),
                   info.size() * sizeof(nqs_sector_info), hipMemcpyHostToDevice));
  m.phys_host = std::move(phys);
  m.sec_host = std::move(info);
  m.tagged = tagged ? 1 : 0;
  m.gen_nadd = 0;
  m.gen_eig.clear();
  m.gen_target.clear();
  ++m.sec_gen;   // device tables may have moved: captured launch sequences are stale
}

// The model's own sector from general symmetries (one sector, untagged words).
void install_general(nqs_model &m, int n_add, const std::vector<int32_t> &eig,
                     const std::vector<int32_t> &target, const std::vector<uint64_t> &z2,
                     uint32_t z2_target) {
  const std::vector<int32_t> table = general_children(m.n, n_add, eig, target, z2, z2_target);
  nqs_sector_info si{};
  si.n = m.n;
  si.na = m.na;
  si.nb = m.nb;
  si.mask_levels = m.mask_levels;
  si.phys_off = 0;
  si.general = 1;
  const size_t bytes = table.size() * 4;
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(m.phys.reserve(bytes), table.data(), bytes, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(m.sec.reserve(sizeof(nqs_sector_info)), &si, sizeof(nqs_sector_info),
                   hipMemcpyHostToDevice));
  m.phys_host.assign(reinterpret_cast<const uint8_t *>(table.data()),
                     reinterpret_cast<const uint8_t *>(table.data()) + bytes);
  m.sec_host.assign(1, si);
  m.tagged = 0;
  m.z2.clear();
  m.gen_nadd = n_add;
  m.gen_eig = eig;
  m.gen_target = target;
  ++m.sec_gen;
}

}  // namespace
}  // namespace nqs

using namespace nqs;

extern "C" const char *nqs_last_error(void) { return g_last_error.c_str(); }

// derived weights from the canonical parameters: fp32 / fp64 block matrices of
// the per-qubit ansatz, then the bf16 fragments of the fused forward
static void repack(nqs_model &m, hipStream_t s) {
  if (m.kind == NQS_MODEL_TABLE) {
    table_pack(m, s);
  } else if (m.kind == NQS_MODEL_NADE) {
    nade_pack(m, s);
    if (m.precision == NQS_BF16) nade_fused_pack(m, s);
  } else if (m.precision == NQS_BF16) {
    fused_pack(m, s);
  }
}

extern "C" int amp_model_create(int kind, const int32_t *dims, int n_dims, const double *params,
                                int64_t n_params, int precision, int strategy, int dlev,
                                nqs_model **out) {
  return guarded([&] {
    NQS_REQUIRE(out && dims && params, NQS_EINVAL, "amp_model_create: null argument");
    *out = nullptr;
    NQS_REQUIRE(kind == NQS_MODEL_MLP || kind == NQS_MODEL_TRANSFORMER ||
                    kind == NQS_MODEL_NADE || kind == NQS_MODEL_TABLE,
                NQS_EUNSUPPORTED, "amp_model_create: unknown model kind");
    NQS_REQUIRE(precision == NQS_FP64 || precision == NQS_FP32 || precision == NQS_BF16,
                NQS_EUNSUPPORTED, "amp_model_create: unknown precision");
    NQS_REQUIRE(strategy == NQS_MU || strategy == NQS_DU || strategy == NQS_MUD, NQS_EUNSUPPORTED,
                "amp_model_create: unknown strategy");
    if (kind == NQS_MODEL_TABLE)
      NQS_REQUIRE(n_dims >= 5 && (n_dims - 3) % 2 == 0, NQS_EINVAL,
                  "amp_model_create: a table needs dims {n, n_alpha, n_beta} and two words "
                  "per basis configuration");
    else
      NQS_REQUIRE(n_dims == (kind == NQS_MODEL_TRANSFORMER ? 8 : 4), NQS_EINVAL,
                  "amp_model_create: wrong number of dims");
    auto m = std::make_unique<nqs_model>();
    m->kind = kind;
    m->precision = precision;
    m->strategy = strategy;
    m->dlev = dlev;
    m->n = dims[0];
    m->na = dims[1];
    m->nb = dims[2];
    const int n = m->n;
    NQS_REQUIRE(n >= 1, NQS_EINVAL, "amp_model_create: n < 1");
    NQS_REQUIRE(n <= 32, NQS_EUNSUPPORTED, "amp_model_create: more than 32 tokens");
    NQS_REQUIRE(m->na >= 0 && m->na <= n && m->nb >= 0 && m->nb <= n, NQS_EINVAL,
                "amp_model_create: electron counts out of range");
    NQS_REQUIRE(strategy != NQS_MUD || (dlev >= 0 && dlev <= n), NQS_EINVAL,
                "amp_model_create: d out of range");
    m->mask_levels = strategy == NQS_MU ? n : strategy == NQS_DU ? 0 : n - dlev;
    int64_t o = 0;
    auto add = [&](int64_t size) {
      m->off.push_back(o);
      o += size;
    };
    std::vector<uint64_t> basis;
    if (kind == NQS_MODEL_TABLE) {
      NQS_REQUIRE(precision == NQS_FP64, NQS_EUNSUPPORTED, "amp_model_create: a table is FP64");
      const int64_t M = (n_dims - 3) / 2;
      basis.resize(size_t(M));
      for (int64_t j = 0; j < M; ++j)
        basis[size_t(j)] = uint64_t(uint32_t(dims[3 + 2 * j])) |
                           (uint64_t(uint32_t(dims[4 + 2 * j])) << 32);
      add(M);    // log|psi|
      add(M);    // phase
    } else if (kind == NQS_MODEL_NADE) {
      m->hid = dims[3];
      NQS_REQUIRE(m->hid >= 1, NQS_EINVAL, "amp_model_create: hidden < 1");
      NQS_REQUIRE(precision != NQS_BF16 || nade_fused_supported(*m), NQS_EUNSUPPORTED,
                  "amp_model_create: bf16 mode of the per-qubit ansatz needs hidden width 64");
      const int h = m->hid;
      for (int i = 0; i < 2 * n; ++i) {
        add(int64_t(i) * h); add(int64_t(i) * h); add(h); add(h);
        add(int64_t(h) * h); add(int64_t(h) * h); add(h); add(h);
        add(int64_t(h) * 2); add(int64_t(h) * 2); add(2); add(2);
      }
    } else if (kind == NQS_MODEL_MLP) {
      m->hid = dims[3];
      NQS_REQUIRE(m->hid >= 1, NQS_EINVAL, "amp_model_create: hidden < 1");
      NQS_REQUIRE(precision != NQS_BF16, NQS_EUNSUPPORTED, "amp_model_create: MLP has no bf16 mode");
      const int h = m->hid;
      for (int p = 0; p < n; ++p) {
        add(int64_t(4) * p * h); add(h); add(int64_t(h) * h); add(h); add(int64_t(h) * 8); add(8);
      }
    } else {
      m->d = dims[3];
      m->L = dims[4];
      m->H = dims[5];
      m->F = dims[6];
      m->PH = dims[7];
      NQS_REQUIRE(m->d >= 1 && m->L >= 1 && m->H >= 1 && m->F >= 1 && m->PH >= 1, NQS_EINVAL,
                  "amp_model_create: non-positive transformer dimension");
      NQS_REQUIRE(m->d % m->H == 0 && m->d / m->H <= 64, NQS_EUNSUPPORTED,
                  "amp_model_create: d_model must split into heads of at most 64");
      const int d = m->d, F = m->F, PH = m->PH;
      add(5 * d); add(int64_t(n) * d);
      for (int l = 0; l < m->L; ++l) {
        add(d); add(d); add(int64_t(d) * 3 * d); add(3 * d); add(int64_t(d) * d); add(d);
        add(d); add(d); add(int64_t(d) * F); add(F); add(int64_t(F) * d); add(d);
      }
      add(d); add(d); add(int64_t(d) * 4); add(4); add(int64_t(n) * 4);
      add(int64_t(4) * n * PH); add(PH); add(int64_t(PH) * PH); add(PH); add(PH); add(1);
      if (precision == NQS_BF16)
        NQS_REQUIRE(fused_supported(*m), NQS_EUNSUPPORTED,
                    "amp_model_create: bf16 mode needs d_model 64 or 128, ffn 4 d_model, "
                    "head dim 16, at most 16 tokens");
    }
    m->P = o;
    NQS_REQUIRE(n_params == m->P, NQS_EINVAL,
                "amp_model_create: n_params does not match the dimensions (expected " +
                    std::to_string(m->P) + ")");
    check_device();
    size_t free_b = 0, total_b = 0;
    HIP_OK(hipMemGetInfo(&free_b, &total_b));
    m->act_budget = std::min<int64_t>(std::max<int64_t>(int64_t(free_b / 8), int64_t(1) << 30),
                                      int64_t(16) << 30);
    install_sectors(*m, {{n, m->na, m->nb}}, false);
    if (kind == NQS_MODEL_TABLE) table_install(*m, basis.data(), int64_t(basis.size()));
    if (m->fp64()) {
      HIP_OK(hipMemcpy(m->master.reserve(size_t(m->P) * 8), params, size_t(m->P) * 8,
                       hipMemcpyHostToDevice));
    } else {
      std::vector<float> f(params, params + m->P);
      HIP_OK(hipMemcpy(m->master.reserve(size_t(m->P) * 4), f.data(), size_t(m->P) * 4,
                       hipMemcpyHostToDevice));
    }
    repack(*m, nullptr);
    HIP_OK(hipDeviceSynchronize());
    *out = m.release();
  });
}

extern "C" int amp_model_set_sectors(nqs_model *m, int n_mol, const int32_t *n,
                                     const int32_t *n_alpha, const int32_t *n_beta) {
  return guarded([&] {
    NQS_REQUIRE(m, NQS_EINVAL, "amp_model_set_sectors: null handle");
    NQS_REQUIRE(n_mol >= 0 && n_mol <= 64, NQS_EINVAL,
                "amp_model_set_sectors: between 0 and 64 molecules");
    if (n_mol == 0) {
      install_sectors(*m, {{m->n, m->na, m->nb}}, false);
      return;
    }
    NQS_REQUIRE(n && n_alpha && n_beta, NQS_EINVAL, "amp_model_set_sectors: null array");
    NQS_REQUIRE(m->kind == NQS_MODEL_TRANSFORMER, NQS_EUNSUPPORTED,
                "amp_model_set_sectors: only the transformer serves several molecules");
    NQS_REQUIRE(m->z2.empty(), NQS_EUNSUPPORTED,
                "amp_model_set_sectors: a model with Z2 symmetries serves one molecule");
    NQS_REQUIRE(2 * m->n <= kTagShift, NQS_EUNSUPPORTED,
                "amp_model_set_sectors: more than 29 tokens leave no room for the molecule index");
    std::vector<std::array<int, 3>> secs;
    for (int i = 0; i < n_mol; ++i) {
      NQS_REQUIRE(n[i] >= 1 && n[i] <= m->n, NQS_EINVAL,
                  "amp_model_set_sectors: molecule has more tokens than the model's positions");
      NQS_REQUIRE(n_alpha[i] >= 0 && n_alpha[i] <= n[i] && n_beta[i] >= 0 && n_beta[i] <= n[i],
                  NQS_EINVAL, "amp_model_set_sectors: electron counts out of range");
      secs.push_back({n[i], n_alpha[i], n_beta[i]});
    }
    install_sectors(*m, secs, true);
  });
}

extern "C" int amp_model_set_z2(nqs_model *m, int n_gen, const uint64_t *masks,
                                const int32_t *targets) {
  return guarded([&] {
    NQS_REQUIRE(m, NQS_EINVAL, "amp_model_set_z2: null handle");
    NQS_REQUIRE(m->kind != NQS_MODEL_TABLE, NQS_EUNSUPPORTED,
                "amp_model_set_z2: a table's support is its basis");
    NQS_REQUIRE(!m->tagged, NQS_EUNSUPPORTED,
                "amp_model_set_z2: the model serves several molecules");
    NQS_REQUIRE(n_gen >= 0 && n_gen <= 4, NQS_EINVAL, "amp_model_set_z2: between 0 and 4 masks");
    NQS_REQUIRE(n_gen == 0 || masks, NQS_EINVAL, "amp_model_set_z2: null mask array");
    const uint64_t qubits = 2 * m->n >= 64 ? ~0ull : ((1ull << (2 * m->n)) - 1);
    // the Hartree-Fock determinant fixes the target eigenvalues unless given
    uint64_t hf = 0;
    for (int p = 0; p < m->na; ++p) hf |= 1ull << (2 * p);
    for (int p = 0; p < m->nb; ++p) hf |= 1ull << (2 * p + 1);
    std::vector<uint64_t> z2;
    uint32_t target = 0;
    for (int j = 0; j < n_gen; ++j) {
      NQS_REQUIRE(masks[j] != 0 && (masks[j] & ~qubits) == 0, NQS_EINVAL,
                  "amp_model_set_z2: a mask is empty or names qubits beyond the model's");
      NQS_REQUIRE(!targets || targets[j] == 0 || targets[j] == 1, NQS_EINVAL,
                  "amp_model_set_z2: target parities are 0 or 1");
      const uint32_t t = targets ? uint32_t(targets[j]) : uint32_t(__builtin_popcountll(hf & masks[j]) & 1);
      target |= t << j;
      z2.push_back(masks[j]);
    }
    m->z2 = std::move(z2);
    m->z2_target = target;
    install_sectors(*m, {{m->n, m->na, m->nb}}, false);
  });
}

extern "C" int amp_model_set_symmetries(nqs_model *m, int n_add, const int32_t *eig,
                                        const int32_t *targets, int n_z2, const uint64_t *z2_masks,
                                        const int32_t *z2_targets) {
  return guarded([&] {
    NQS_REQUIRE(m, NQS_EINVAL, "amp_model_set_symmetries: null handle");
    NQS_REQUIRE(!m->tagged, NQS_EUNSUPPORTED,
                "amp_model_set_symmetries: the model serves several molecules");
    NQS_REQUIRE(n_add >= 0 && n_add <= 8 && n_z2 >= 0 && n_z2 <= 4, NQS_EINVAL,
                "amp_model_set_symmetries: 0..8 additive and 0..4 Z2 symmetries");
    if (n_add == 0 && n_z2 == 0) {                 // back to the (n_alpha, n_beta) sector
      m->z2.clear();
      m->z2_target = 0;
      install_sectors(*m, {{m->n, m->na, m->nb}}, false);
      return;
    }
    NQS_REQUIRE(n_add == 0 || (eig && targets), NQS_EINVAL,
                "amp_model_set_symmetries: null eigenvalues or targets");
    NQS_REQUIRE(n_z2 == 0 || z2_masks, NQS_EINVAL, "amp_model_set_symmetries: null Z2 masks");
    const int N = 2 * m->n;
    const uint64_t qubits = N >= 64 ? ~0ull : ((1ull << N) - 1);
    std::vector<int32_t> e(eig, eig + size_t(n_add) * 2 * N), t(targets, targets + n_add);
    for (int32_t v : e)
      NQS_REQUIRE(v >= -(1 << 20) && v <= (1 << 20), NQS_EINVAL,
                  "amp_model_set_symmetries: eigenvalue out of range");
    std::vector<uint64_t> z(z2_masks, z2_masks + n_z2);
    uint32_t zt = 0;
    for (int j = 0; j < n_z2; ++j) {
      NQS_REQUIRE(z[size_t(j)] != 0 && (z[size_t(j)] & ~qubits) == 0, NQS_EINVAL,
                  "amp_model_set_symmetries: Z2 mask empty or beyond the qubits");
      const int32_t tj = z2_targets ? z2_targets[j] : 0;
      NQS_REQUIRE(tj == 0 || tj == 1, NQS_EINVAL, "amp_model_set_symmetries: Z2 target not 0/1");
      zt |= uint32_t(tj) << j;
    }
    install_general(*m, n_add, e, t, z, zt);
  });
}

extern "C" int amp_model_info(const nqs_model *m, int64_t *n_params, int32_t *param_bytes) {
  return guarded([&] {
    NQS_REQUIRE(m, NQS_EINVAL, "amp_model_info: null handle");
    if (n_params) *n_params = m->P;
    if (param_bytes) *param_bytes = int32_t(m->elem());
  });
}

extern "C" int amp_model_params(nqs_model *m, void **dev_params) {
  return guarded([&] {
    NQS_REQUIRE(m && dev_params, NQS_EINVAL, "amp_model_params: null argument");
    *dev_params = m->master.ptr;
  });
}

extern "C" int amp_model_sync(nqs_model *m, nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(m, NQS_EINVAL, "amp_model_sync: null handle");
    repack(*m, as_stream(stream));
  });
}

extern "C" int amp_model_get_params(const nqs_model *m, double *host_out) {
  return guarded([&] {
    NQS_REQUIRE(m && host_out, NQS_EINVAL, "amp_model_get_params: null argument");
    HIP_OK(hipDeviceSynchronize());
    if (m->fp64()) {
      HIP_OK(hipMemcpy(host_out, m->master.ptr, size_t(m->P) * 8, hipMemcpyDeviceToHost));
    } else {
      std::vector<float> f(size_t(m->P));
      HIP_OK(hipMemcpy(f.data(), m->master.ptr, size_t(m->P) * 4, hipMemcpyDeviceToHost));
      std::copy(f.begin(), f.end(), host_out);
    }
  });
}

extern "C" int amp_model_set_params(nqs_model *m, const double *host_in) {
  return guarded([&] {
    NQS_REQUIRE(m && host_in, NQS_EINVAL, "amp_model_set_params: null argument");
    HIP_OK(hipDeviceSynchronize());
    if (m->fp64()) {
      HIP_OK(hipMemcpy(m->master.ptr, host_in, size_t(m->P) * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> f(host_in, host_in + m->P);
      HIP_OK(hipMemcpy(m->master.ptr, f.data(), size_t(m->P) * 4, hipMemcpyHostToDevice));
    }
    repack(*m, nullptr);
    HIP_OK(hipDeviceSynchronize());
  });
}

extern "C" void amp_model_destroy(nqs_model *m) { delete m; }

extern "C" int amp_model_set_prefix_sharing(nqs_model *m, int on) {
  return guarded([&] {
    NQS_REQUIRE(m, NQS_EINVAL, "amp_model_set_prefix_sharing: null handle");
    NQS_REQUIRE(on >= 0 && on <= 2, NQS_EINVAL, "amp_model_set_prefix_sharing: on not 0..2");
    m->prefix_share = on != 0;
    m->tail_tree = on == 1;
  });
}

extern "C" int amp_model_tree_rows(const nqs_model *m, int64_t *rows_q, int64_t *rows_q1) {
  return guarded([&] {
    NQS_REQUIRE(m && rows_q && rows_q1, NQS_EINVAL, "amp_model_tree_rows: null pointer");
    *rows_q = m->tree_rows_q;
    *rows_q1 = m->tree_rows_q1;
  });
}

extern "C" int amp_model_set_mixed_backward(nqs_model *m, int on) {
  return guarded([&] {
    NQS_REQUIRE(m, NQS_EINVAL, "amp_model_set_mixed_backward: null handle");
    m->mixed_backward = on != 0;
  });
}

namespace {
// bf16 forward of a batch: prefix-shared where the model allows it
void bf16_forward(nqs_model &m, const uint64_t *x, int64_t n, double *logabs, double *phase,
                  hipStream_t s) {
  if (fused_shared_supported(m)) fused_forward_shared(m, x, n, logabs, phase, s);
  else fused_forward(m, x, n, logabs, phase, nullptr, -1, s);
}
}  // namespace

extern "C" int amp_forward(nqs_model *m, const uint64_t *x, int64_t n, double *logabs,
                           double *phase, nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(m, NQS_EINVAL, "amp_forward: null handle");
    NQS_REQUIRE(n >= 0, NQS_EINVAL, "amp_forward: negative n");
    if (n == 0) return;
    NQS_REQUIRE(x && (logabs || phase), NQS_EINVAL, "amp_forward: null pointer");
    if (m->precision == NQS_BF16)
      bf16_forward(*m, x, n, logabs, phase, as_stream(stream));
    else
      model_forward(*m, x, n, logabs, phase, nullptr, as_stream(stream));
  });
}

extern "C" int amp_backward(nqs_model *m, const uint64_t *x, int64_t n, const double *g_logabs,
                            const double *g_phase, void *grad, nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(m && grad, NQS_EINVAL, "amp_backward: null argument");
    NQS_REQUIRE(n >= 0, NQS_EINVAL, "amp_backward: negative n");
    NQS_REQUIRE(n == 0 || (x && g_logabs && g_phase), NQS_EINVAL, "amp_backward: null pointer");
    model_backward(*m, x, n, g_logabs, g_phase, grad, as_stream(stream));
  });
}

extern "C" int connected_pairs(nqs_ham *H, const uint64_t *x, int64_t n, int64_t *offsets,
                               uint64_t *xp, double *hval, double *hdiag, int64_t capacity,
                               int64_t *n_pairs, nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(H && offsets && n_pairs, NQS_EINVAL, "connected_pairs: null argument");
    NQS_REQUIRE(n >= 0, NQS_EINVAL, "connected_pairs: negative n");
    hipStream_t s = as_stream(stream);
    check_device();
    H->upload();
    int64_t *cnt = static_cast<int64_t *>(H->w_cnt.reserve(size_t(n > 0 ? n : 1) * 8));
    if (n > 0) launch_count_pairs(*H, x, n, cnt, s);
    launch_exclusive_scan(cnt, offsets, n, s, H->w_scan);
    int64_t total = 0;
    HIP_OK(hipMemcpyAsync(&total, offsets + n, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *n_pairs = total;
    NQS_REQUIRE(total <= capacity, NQS_ECAPACITY, "connected_pairs: capacity too small");
    if (n > 0) launch_emit_pairs(*H, x, n, offsets, xp, hval, nullptr, hdiag, 0, s);
  });
}

// ---- connected_pairs_noalloc: the scratch of connected_pairs (the pair count
// of every configuration and the multi-block scan's tile totals) in a fixed
// device array.  Every device the library runs on holds its own copy until the
// process ends; host code reaches it only through the address returned by
// hipGetSymbolAddress on that device (the array's name is a host-side stand-in).
namespace nqs {
namespace {
constexpr int64_t kNoallocScanWs = 2 * (NQS_NOALLOC_MAX_CONFIGS / 1024) + 1;
constexpr int64_t kNoallocEntries = NQS_NOALLOC_MAX_CONFIGS + kNoallocScanWs;
static __device__ __align__(256) int64_t scratch[kNoallocEntries];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call there.
int64_t *device_scratch() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  NQS_REQUIRE(dev >= 0 && dev < kMaxDevices, NQS_EHIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    NQS_REQUIRE(p != nullptr, NQS_EHIP, "scratch: no device address");
    g_scratch[dev] = static_cast<int64_t *>(p);
  }
  return g_scratch[dev];
}
}  // namespace
}  // namespace nqs

extern "C" int connected_pairs_noalloc(const nqs_ham *H, const uint64_t *x, int64_t n,
                                       int64_t *offsets, uint64_t *xp, double *hval,
                                       double *hdiag, int64_t capacity, int64_t *n_pairs,
                                       nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(H && offsets && n_pairs, NQS_EINVAL, "connected_pairs_noalloc: null argument");
    NQS_REQUIRE(n >= 0, NQS_EINVAL, "connected_pairs_noalloc: negative n");
    NQS_REQUIRE(n <= NQS_NOALLOC_MAX_CONFIGS, NQS_EUNSUPPORTED,
                "connected_pairs_noalloc: more than NQS_NOALLOC_MAX_CONFIGS configurations");
    NQS_REQUIRE(n == 0 || x, NQS_EINVAL, "connected_pairs_noalloc: null x");
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    NQS_REQUIRE(H->device == dev && H->d_flip.ptr, NQS_EINVAL,
                "connected_pairs_noalloc: the Hamiltonian's tables are not on this device "
                "(any other call with it uploads them)");
    hipStream_t s = as_stream(stream);
    int64_t *cnt = device_scratch();
    int64_t *ws = cnt + NQS_NOALLOC_MAX_CONFIGS;
    static_assert(kNoallocScanWs >= 2 * ((NQS_NOALLOC_MAX_CONFIGS + 1023) / 1024) + 1,
                  "scan workspace of the largest call");
    if (n > 0) launch_count_pairs(*H, x, n, cnt, s);
    launch_exclusive_scan(cnt, offsets, n, s, ws);
    int64_t total = 0;
    HIP_OK(hipMemcpyAsync(&total, offsets + n, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *n_pairs = total;
    NQS_REQUIRE(total <= capacity, NQS_ECAPACITY, "connected_pairs_noalloc: capacity too small");
    if (n > 0) launch_emit_pairs(*H, x, n, offsets, xp, hval, nullptr, hdiag, 0, s);
  });
}

extern "C" int local_energy(nqs_ham *H, nqs_model *m, const uint64_t *x, const uint64_t *counts,
                            int64_t n, const double *logabs_x, const double *phase_x,
                            double *eloc, double *sums, int64_t *n_pairs, nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(H && m && sums, NQS_EINVAL, "local_energy: null argument");
    NQS_REQUIRE(n >= 0, NQS_EINVAL, "local_energy: negative n");
    NQS_REQUIRE(n == 0 || (x && eloc), NQS_EINVAL, "local_energy: null array");
    NQS_REQUIRE((logabs_x == nullptr) == (phase_x == nullptr), NQS_EINVAL,
                "local_energy: give both or neither of logabs_x, phase_x");
    NQS_REQUIRE(H->n == m->n && H->n_alpha == m->na && H->n_beta == m->nb && !m->tagged,
                NQS_EINVAL, "local_energy: Hamiltonian and model describe different systems");
    hipStream_t s = as_stream(stream);
    check_device();
    H->upload();
    if (n_pairs) *n_pairs = 0;
    if (n == 0) {
      zero_async(sums, 4 * 8, s);
      return;
    }
    int64_t *cnt = static_cast<int64_t *>(H->w_cnt.reserve(size_t(n) * 8));
    int64_t *off = static_cast<int64_t *>(H->w_off.reserve(size_t(n + 1) * 8));
    launch_count_pairs(*H, x, n, cnt, s);
    launch_exclusive_scan(cnt, off, n, s, H->w_scan);
    std::vector<int64_t> off_h(size_t(n) + 1);
    HIP_OK(hipMemcpyAsync(off_h.data(), off, size_t(n + 1) * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (n_pairs) *n_pairs = off_h[n];
    H->last_pairs = off_h[n];
    double *hdiag = static_cast<double *>(H->w_diag.reserve(size_t(n) * 8));
    const double *lax = logabs_x, *phx = phase_x;
    if (!lax) {
      double *a = static_cast<double *>(H->w_lax.reserve(size_t(n) * 8));
      double *b = static_cast<double *>(H->w_phx.reserve(size_t(n) * 8));
      if (m->precision == NQS_BF16) bf16_forward(*m, x, n, a, b, s);
      else model_forward(*m, x, n, a, b, nullptr, s);
      lax = a;
      phx = b;
    }
    // Pairs are processed in slices of whole configurations (at most 2^27
    // pairs); inside a slice the amplitude network runs once per distinct x'.
    const int64_t cap = int64_t(1) << 27;
    int64_t maxk = 0;
    for (int64_t i = 0; i < n; ++i) maxk = std::max(maxk, off_h[i + 1] - off_h[i]);
    const int64_t slice = std::min(std::max(cap, maxk), std::max<int64_t>(off_h[n], 1));
    auto *xp = static_cast<uint64_t *>(H->w_xp.reserve(size_t(slice) * 8));
    auto *hv = static_cast<double *>(H->w_h.reserve(size_t(slice) * 8));
    auto *la = static_cast<double *>(H->w_la.reserve(size_t(slice) * 8));
    auto *ph = static_cast<double *>(H->w_ph.reserve(size_t(slice) * 8));
    auto *lp2 = m->precision == NQS_BF16 ? static_cast<float2 *>(H->w_lp2.reserve(size_t(slice) * 8))
                                         : nullptr;
    auto *keys = static_cast<uint64_t *>(H->w_keys.reserve(size_t(slice) * 8));
    auto *ukeys = static_cast<uint64_t *>(H->w_ukeys.reserve(size_t(slice) * 8));
    auto *u32 = static_cast<uint32_t *>(H->w_u32.reserve(size_t(slice) * 4 * 5));
    uint32_t *vin = u32, *vsort = u32 + slice, *head = u32 + 2 * slice,
             *run = u32 + 3 * slice, *uid = u32 + 4 * slice;
    int64_t i0 = 0;
    H->last_distinct = 0;
    while (i0 < n) {
      int64_t i1 = i0 + 1;
      while (i1 < n && off_h[i1 + 1] - off_h[i0] <= slice) ++i1;
      const int64_t np = off_h[i1] - off_h[i0];
      launch_emit_pairs(*H, x + i0, i1 - i0, off + i0, xp, hv, nullptr, hdiag + i0, 0, s);
      // grouped by the prefixes of the prefix-shared forward
      const int levels = fused_shared_levels(*m);
      const bool tree = levels == 3 && fused_tree(*m);
      const int pm = tree ? -1 : levels == 3 ? 2 * fused_shared_pm(*m) : levels == 2 ? 16 : 0;
      const int64_t nu = dedupe_pairs(xp, np, H->N, pm, keys, vin, vsort, head, run, ukeys, uid,
                                      H->w_tmp, s);
      H->last_distinct += nu;
      if (nu > 0) {
        if (tree) fused_forward_tree(*m, ukeys, nu, la, ph, s);
        else if (levels == 3) fused_forward_shared3(*m, ukeys, nu, la, ph, s);
        else if (m->precision == NQS_BF16) bf16_forward(*m, ukeys, nu, la, ph, s);
        else model_forward(*m, ukeys, nu, la, ph, nullptr, s);
      }
      launch_accumulate(i1 - i0, off + i0, hv, np > 0 ? uid : nullptr, la, ph, lax + i0,
                        phx + i0, hdiag + i0, eloc + 2 * i0, s, m->precision == NQS_BF16, nu, lp2);
      i0 = i1;
    }
    launch_reduce(eloc, counts, n, sums, s);
  });
}

extern "C" int local_energy_stats(const nqs_ham *H, int64_t *n_pairs, int64_t *n_distinct) {
  return guarded([&] {
    NQS_REQUIRE(H, NQS_EINVAL, "local_energy_stats: null handle");
    if (n_pairs) *n_pairs = H->last_pairs;
    if (n_distinct) *n_distinct = H->last_distinct;
  });
}

extern "C" int vmc_weights(const double *eloc, const uint64_t *counts, int64_t n,
                           const double *sums, double *g_logabs, double *g_phase,
                           nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(n >= 0, NQS_EINVAL, "vmc_weights: negative n");
    if (n == 0) return;
    NQS_REQUIRE(eloc && sums && g_logabs && g_phase, NQS_EINVAL, "vmc_weights: null pointer");
    launch_weights(eloc, counts, n, sums, g_logabs, g_phase, as_stream(stream));
  });
}

extern "C" int adam_update(void *params, const void *grad, void *mom, void *vel, int64_t n,
                           int elem_bytes, double lr, double b1, double b2, double eps, int64_t t,
                           nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(n >= 0 && t >= 1, NQS_EINVAL, "adam_update: n < 0 or t < 1");
    NQS_REQUIRE(elem_bytes == 4 || elem_bytes == 8, NQS_EINVAL, "adam_update: elem_bytes not 4/8");
    if (n == 0) return;
    NQS_REQUIRE(params && grad && mom && vel, NQS_EINVAL, "adam_update: null pointer");
    launch_adam(params, grad, mom, vel, n, elem_bytes, lr, b1, b2, eps, t, as_stream(stream));
  });
}
