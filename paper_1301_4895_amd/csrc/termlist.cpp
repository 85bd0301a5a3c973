// Term list of the recursive multibaryon method (host side, integer exact).
//
// Builds, once per nucleus and spin request (Sec. 3-5, 7):
//   * G of each nucleon type antisymmetrised in its same-flavour slots;
//   * L on sorted index sets by L^(n+1) = L^(n) . G (eq. recr_L), with the
//     antisymmetric product of eq. antis_product_2 over the proton-spin,
//     neutron-spin, u and d index groups;
//   * the final required components (requested sink sets times every quark
//     index set with a nonzero L for a requested source set), and backwards
//     the required components of every stage (Sec. 3, pruning);
//   * the operation list of every step in factorised form: the split of a
//     component into (previous component, block component) is a split of
//     its quark part times a split of its baryon-index part, and the sign of
//     eq. antis_product_2 is the product of the per-group signs.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <unordered_map>

#include "internal.h"

namespace mb {

static thread_local std::string g_err;
void set_error(const std::string &m) { g_err = m; }
int fail(int code, const std::string &m) {
  g_err = m;
  return code;
}

int binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long long r = 1;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return int(r);
}

int factorial(int n) {
  int r = 1;
  for (int i = 2; i <= n; i++) r *= i;
  return r;
}

int subset_rank(uint32_t pos, int m) {
  int rem = __builtin_popcount(pos), r = 0;
  for (int i = m - 1; i >= 0; i--)
    if (pos >> i & 1) {
      r += binom(i, rem);
      rem--;
    }
  return r;
}

uint32_t to_positions(uint32_t sub, uint32_t base) {
  uint32_t out = 0;
  int p = 0;
  for (int i = 0; i < 32; i++)
    if (base >> i & 1) {
      if (sub >> i & 1) out |= 1u << p;
      p++;
    }
  return out;
}

uint32_t from_positions(uint32_t pos, uint32_t base) {
  uint32_t out = 0;
  int p = 0;
  for (int i = 0; i < 32; i++)
    if (base >> i & 1) {
      if (pos >> p & 1) out |= 1u << i;
      p++;
    }
  return out;
}

// (-1)^(number of pairs i in x, j in y with i > j): the sign of the
// permutation that sorts the indices of x followed by those of y.
static inline int split_sign(uint32_t x, uint32_t y) {
  int s = 0;
  for (uint32_t t = y; t; t &= t - 1) {
    int j = __builtin_ctz(t);
    s += j >= 31 ? 0 : __builtin_popcount(x >> (j + 1));
  }
  return (s & 1) ? -1 : 1;
}

static inline uint32_t pair_rank(int a, int b) { return uint32_t(b * (b - 1) / 2 + a); }

// Block quark index of a block component (see mbcontract.h).
static inline uint32_t block_qidx(int type, uint32_t yu, uint32_t yd, int nxi) {
  if (type == PROTON) {
    int a = __builtin_ctz(yu), b = 31 - __builtin_clz(yu), c = __builtin_ctz(yd);
    return pair_rank(a, b) * uint32_t(nxi) + uint32_t(c);
  }
  int c = __builtin_ctz(yu), a = __builtin_ctz(yd), b = 31 - __builtin_clz(yd);
  return uint32_t(c) * uint32_t(nxi * (nxi - 1) / 2) + pair_rank(a, b);
}

// Block quark index of a Lambda block component: s index e, u index c, d
// index f (one-bit masks) -> (e*n_xi + c)*n_xi + f.
static inline uint32_t lambda_qidx(uint32_t ys, uint32_t yu, uint32_t yd, int nxi) {
  return (uint32_t(__builtin_ctz(ys)) * uint32_t(nxi) + uint32_t(__builtin_ctz(yu))) * uint32_t(nxi) +
         uint32_t(__builtin_ctz(yd));
}

// ---------------------------------------------------------------------------
// Gamma matrices restricted to the active spins (Sec. 7).  On the spins that
// enter (all four relativistically, the upper two nonrelativistically in the
// Dirac representation) Gamma_1 is the identity in both cases and Gamma_2 is
// C gamma_5 = [[0,-1,0,0],[1,0,0,0],[0,0,0,-1],[0,0,1,0]] (C = i g^2 g^0).
static int cg5(int a, int b) {
  if ((a == 0 && b == 1) || (a == 2 && b == 3)) return -1;
  if ((a == 1 && b == 0) || (a == 3 && b == 2)) return 1;
  return 0;
}

static int levi(int a, int b, int c) {
  if (a == b || b == c || a == c) return 0;
  return ((b - a + 3) % 3 == 1) ? 1 : -1;
}

struct GEnt {
  int chi;
  uint32_t u, d;
  int64_t c;
};

// G-tilde(chi; xi1, xi2, xi3) of eq. def_g / eq. G_tilde over active indices.
static int g_value(int chi, int x1, int x2, int x3, int nsrc) {
  int s = chi % nsrc, alpha = chi / nsrc;
  if (x1 % nsrc != s || x2 % nsrc != s || x3 % nsrc != s) return 0;
  int k1 = x1 / nsrc, k2 = x2 / nsrc, k3 = x3 / nsrc;
  if (k1 / 3 != alpha) return 0;
  return cg5(k2 / 3, k3 / 3) * levi(k1 % 3, k2 % 3, k3 % 3);
}

// Nonzero entries of G antisymmetrised (without normalisation) in the two
// same-flavour slots: proton slots (u,u,d), neutron slots (d,u,d).
static std::vector<GEnt> g_antisym(int type, int nsrc, int npsi, int nxi, uint32_t allowed) {
  std::vector<GEnt> out;
  for (int chi = 0; chi < npsi; chi++) {
    if (!(allowed >> chi & 1)) continue;
    for (int a = 0; a < nxi; a++)
      for (int b = a + 1; b < nxi; b++)
        for (int c = 0; c < nxi; c++) {
          int v;
          if (type == PROTON)
            v = g_value(chi, a, b, c, nsrc) - g_value(chi, b, a, c, nsrc);
          else
            v = g_value(chi, a, c, b, nsrc) - g_value(chi, b, c, a, nsrc);
          if (!v) continue;
          GEnt e;
          e.chi = chi;
          e.c = v;
          if (type == PROTON) {
            e.u = (1u << a) | (1u << b);
            e.d = 1u << c;
          } else {
            e.u = 1u << c;
            e.d = (1u << a) | (1u << b);
          }
          out.push_back(e);
        }
  }
  return out;
}

// Nonzero entries of G of the Lambda, slots (s, u, d): no two slots share a
// flavour, so nothing is antisymmetrised.
struct GEntL {
  int chi;
  uint32_t s, u, d;
  int64_t c;
};
static std::vector<GEntL> g_lambda(int nsrc, int npsi, int nxi, uint32_t allowed) {
  std::vector<GEntL> out;
  for (int chi = 0; chi < npsi; chi++) {
    if (!(allowed >> chi & 1)) continue;
    for (int a = 0; a < nxi; a++)
      for (int b = 0; b < nxi; b++)
        for (int c = 0; c < nxi; c++) {
          const int v = g_value(chi, a, b, c, nsrc);
          if (v) out.push_back({chi, 1u << a, 1u << b, 1u << c, v});
        }
  }
  return out;
}

// Component key for L: proton set (8 bits), neutron set (8), u (24), d (24).
static inline uint64_t lkey(uint32_t p, uint32_t n, uint32_t u, uint32_t d) {
  return (uint64_t(p) << 56) | (uint64_t(n) << 48) | (uint64_t(u) << 24) | uint64_t(d);
}

// Open-addressing set of uint64 keys (insert only), for the required sets.
struct KeySet {
  std::vector<uint64_t> slot;
  std::vector<uint8_t> used;
  size_t n = 0, mask = 0;
  explicit KeySet(size_t cap = 1024) { reset(cap); }
  void reset(size_t cap) {
    size_t c = 64;
    while (c < 2 * cap) c <<= 1;
    slot.assign(c, 0);
    used.assign(c, 0);
    mask = c - 1;
    n = 0;
  }
  static inline uint64_t mix(uint64_t h) {
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    return h;
  }
  void insert(uint64_t k) {
    if (2 * (n + 1) > slot.size()) grow();
    size_t i = mix(k) & mask;
    while (used[i]) {
      if (slot[i] == k) return;
      i = (i + 1) & mask;
    }
    used[i] = 1;
    slot[i] = k;
    n++;
  }
  void grow() {
    std::vector<uint64_t> s2;
    s2.reserve(n);
    for (size_t i = 0; i < slot.size(); i++)
      if (used[i]) s2.push_back(slot[i]);
    reset(2 * slot.size());
    for (uint64_t k : s2) insert(k);
  }
  std::vector<uint64_t> sorted() const {
    std::vector<uint64_t> v;
    v.reserve(n);
    for (size_t i = 0; i < slot.size(); i++)
      if (used[i]) v.push_back(slot[i]);
    std::sort(v.begin(), v.end());
    return v;
  }
};

// Processing (and storage) order of a stage's quark parts.  A step that adds
// a proton splits off a u pair and one d index; its outputs are ordered d set
// major so that consecutive outputs share previous components (and a neutron
// step, which splits off one u index, u set major).  The order only affects
// memory locality.
static inline uint64_t order_key(uint64_t q, bool d_major) {
  return d_major ? ((q << 32) | (q >> 32)) : q;
}

static void sort_stage(std::vector<uint64_t> &v, bool d_major) {
  std::sort(v.begin(), v.end(),
            [d_major](uint64_t a, uint64_t b) { return order_key(a, d_major) < order_key(b, d_major); });
}

static uint32_t find_stage(const std::vector<uint64_t> &v, bool d_major, uint64_t k) {
  auto it = std::lower_bound(v.begin(), v.end(), k, [d_major](uint64_t a, uint64_t b) {
    return order_key(a, d_major) < order_key(b, d_major);
  });
  return uint32_t(it - v.begin());
}

// Enumerates the quark splits of quark part (u, d) for the added species:
// proton: u pair (colex order of pairs) x d single; neutron: u single x d
// pair.  f(yu, yd) is called for every split in this canonical order.
template <class F>
static inline void for_quark_splits(int type, uint32_t u, uint32_t d, F &&f) {
  // Both species: the single index of the added baryon (d for a proton, u
  // for a neutron) varies slowest, then the same-flavour pair (a < b) in
  // increasing b, then a, i.e. in increasing pair rank.
  if (type == PROTON) {
    for (uint32_t tc = d; tc; tc &= tc - 1)
      for (uint32_t tb = u; tb; tb &= tb - 1) {
        int b = __builtin_ctz(tb);
        for (uint32_t ta = u & ((1u << b) - 1); ta; ta &= ta - 1) {
          int a = __builtin_ctz(ta);
          f((1u << a) | (1u << b), tc & (~tc + 1));
        }
      }
  } else {
    for (uint32_t tc = u; tc; tc &= tc - 1)
      for (uint32_t tb = d; tb; tb &= tb - 1) {
        int b = __builtin_ctz(tb);
        for (uint32_t ta = d & ((1u << b) - 1); ta; ta &= ta - 1) {
          int a = __builtin_ctz(ta);
          f(tc & (~tc + 1), (1u << a) | (1u << b));
        }
      }
  }
}

// The quark splits of a Lambda step: the Lambda takes one u index (slowest)
// and one d index of the output; its s index is the output's whole s set.
template <class F>
static inline void for_lambda_splits(uint32_t uf, uint32_t d, F &&f) {
  for (uint32_t tu = ufield_u(uf); tu; tu &= tu - 1)
    for (uint32_t td = d; td; td &= td - 1) f(tu & (~tu + 1), td & (~td + 1));
}

// c_alpha(q) = L^(n)(alpha; q) / (k_P! k_N!) on sorted sets for the nucleus
// of the first n baryons of the path (k_P protons, k_N neutrons), for every
// source set alpha in `alphas` (eq. recr_L).  The recursion antisymmetrises
// the baryon indices too, which multiplies L on sorted sets by k_P! k_N!.
static int source_coefficients(const mb_term_list *tl, int n, const std::vector<std::array<uint32_t, 2>> &alphas,
                               std::vector<std::vector<std::pair<uint64_t, int64_t>>> &per_alpha) {
  const int nsrc = tl->nsrc, npsi = tl->npsi, nxi = tl->nxi;
  uint32_t allowP = 0, allowN = 0;
  for (auto &a : alphas) {
    allowP |= a[0];
    allowN |= a[1];
  }
  const std::vector<GEnt> gP = g_antisym(PROTON, nsrc, npsi, nxi, allowP);
  const std::vector<GEnt> gN = g_antisym(NEUTRON, nsrc, npsi, nxi, allowN);
  auto wanted_spins = [&](uint32_t p, uint32_t nm) {
    for (auto &a : alphas)
      if (!(p & ~a[0]) && !(nm & ~a[1])) return true;
    return false;
  };
  std::unordered_map<uint64_t, int64_t> L, L2;
  for (const GEnt &g : (tl->path[0] == PROTON ? gP : gN)) {
    uint32_t p = tl->path[0] == PROTON ? (1u << g.chi) : 0, nm = tl->path[0] == PROTON ? 0 : (1u << g.chi);
    L[lkey(p, nm, g.u, g.d)] += g.c;
  }
  for (int s = 1; s < n; s++) {
    const int T = tl->path[s];
    const std::vector<GEnt> &G = T == PROTON ? gP : gN;
    L2.clear();
    L2.reserve(L.size() * 8);
    for (auto &kv : L) {
      uint64_t k = kv.first;
      uint32_t p = uint32_t(k >> 56), nm = uint32_t(k >> 48) & 0xff, u = uint32_t(k >> 24) & 0xffffff,
               d = uint32_t(k) & 0xffffff;
      for (const GEnt &g : G) {
        uint32_t sb = 1u << g.chi;
        uint32_t xs = T == PROTON ? p : nm;
        if ((xs & sb) || (u & g.u) || (d & g.d)) continue;
        uint32_t p2 = T == PROTON ? (p | sb) : p, n2 = T == PROTON ? nm : (nm | sb);
        if (!wanted_spins(p2, n2)) continue;
        int sg = split_sign(xs, sb) * split_sign(u, g.u) * split_sign(d, g.d);
        L2[lkey(p2, n2, u | g.u, d | g.d)] += sg * kv.second * g.c;
      }
    }
    L.clear();
    for (auto &kv : L2)
      if (kv.second != 0) L.insert(kv);
  }
  int kP = 0, kN = 0;
  for (int s = 0; s < n; s++) (tl->path[s] == PROTON ? kP : kN)++;
  const int64_t norm = int64_t(factorial(kP)) * factorial(kN);
  per_alpha.assign(alphas.size(), {});
  std::unordered_map<uint64_t, int> aidx;
  for (size_t i = 0; i < alphas.size(); i++) aidx[(uint64_t(alphas[i][0]) << 32) | alphas[i][1]] = int(i);
  for (auto &kv : L) {
    uint64_t k = kv.first;
    uint32_t p = uint32_t(k >> 56), nm = uint32_t(k >> 48) & 0xff, u = uint32_t(k >> 24) & 0xffffff,
             d = uint32_t(k) & 0xffffff;
    auto it = aidx.find((uint64_t(p) << 32) | nm);
    if (it == aidx.end()) continue;
    if (kv.second % norm != 0) return fail(MB_EINVAL, "internal: L not divisible by k_P! k_N!");
    per_alpha[it->second].push_back({qkey(u, d), kv.second / norm});
  }
  return MB_OK;
}

// Extends the nucleon coefficients by the Lambda (eq. recr_L with G of the
// Lambda as the last factor): for column i, with nucleon source sets
// nalphas[nidx[i]] and Lambda source index chi_i,
//   c_i(U, D, s) = sum over nucleon parts (U', D') and Lambda entries
//                  g = (s, u, d) with U = U' + u, D = D' + d of
//                  sgn(U'|u) sgn(D'|d) c_nuc(U', D') g,
// keyed qkey(U | s << S_SHIFT, D).  One Lambda: its spin split and the
// normalisation (1!) are trivial.
static void lambda_coefficients(const mb_term_list *tl, const std::vector<std::vector<std::pair<uint64_t, int64_t>>> &nuc,
                                const std::vector<int> &nidx,
                                std::vector<std::vector<std::pair<uint64_t, int64_t>>> &per_alpha) {
  uint32_t allow = 0;
  for (uint32_t l : tl->alphaL) allow |= l;
  const std::vector<GEntL> g = g_lambda(tl->nsrc, tl->npsi, tl->nxi, allow);
  per_alpha.assign(tl->alphaL.size(), {});
  for (size_t i = 0; i < tl->alphaL.size(); i++) {
    const int chi = __builtin_ctz(tl->alphaL[i]);
    std::unordered_map<uint64_t, int64_t> m;
    for (const auto &e : nuc[size_t(nidx[i])]) {
      const uint32_t u = qkey_u(e.first), d = qkey_d(e.first);
      for (const GEntL &ge : g) {
        if (ge.chi != chi || (u & ge.u) || (d & ge.d)) continue;
        const int sg = split_sign(u, ge.u) * split_sign(d, ge.d);
        m[qkey((u | ge.u) | (ge.s << S_SHIFT), d | ge.d)] += sg * e.second * ge.c;
      }
    }
    for (auto &kv : m)
      if (kv.second != 0) per_alpha[i].push_back(kv);
  }
}

// Source sets of `n` baryons of one species with all spins: every n-subset
// of the D*N_s indices with one source; with several sources, min(n, D) on
// source 0, min(rest, D) on source 1 and so on, any spins on each (the
// convention of Tables 1-3 for two sources, continued source by source).
static std::vector<uint32_t> all_source_sets(int n, int D, int nsrc) {
  const uint32_t all = (1u << (D * nsrc)) - 1;
  std::vector<uint32_t> v;
  if (nsrc == 1) {
    for (uint32_t m = 0; m <= all; m++)
      if (__builtin_popcount(m) == n) v.push_back(m);
    return v;
  }
  // counts per source, then every choice of spins on each source
  int cnt[8] = {};
  for (int s = 0, left = n; s < nsrc; s++) {
    cnt[s] = std::min(left, D);
    left -= cnt[s];
  }
  v.push_back(0);
  for (int s = 0; s < nsrc; s++) {
    std::vector<uint32_t> next;
    for (uint32_t base : v)
      for (uint32_t ms = 0; ms < (1u << D); ms++) {
        if (__builtin_popcount(ms) != cnt[s]) continue;
        uint32_t m = base;
        for (int a = 0; a < D; a++)
          if (ms >> a & 1) m |= 1u << (nsrc * a + s);
        next.push_back(m);
      }
    v.swap(next);
  }
  std::sort(v.begin(), v.end());
  return v;
}

// Operations of every step for the recursion order `path`, counted from the
// final quark parts backwards (the required sets of each stage are the
// sub-tuples of the next one's), without operation tables.
static int64_t path_operations(const std::vector<uint64_t> &U, const int *path, int A, uint32_t SP, uint32_t SN) {
  int kP[MB_MAX_STAGES], kN[MB_MAX_STAGES];
  for (int s = 0, p = 0, n = 0; s < A; s++) {
    (path[s] == PROTON ? p : n)++;
    kP[s] = p;
    kN[s] = n;
  }
  std::vector<uint64_t> cur = U;
  int64_t total = 0;
  for (int s = A - 1; s >= 1; s--) {
    const int T = path[s];
    const int ku = 2 * kP[s] + kN[s], kd = kP[s] + 2 * kN[s];
    const int64_t Sq = T == PROTON ? int64_t(binom(ku, 2)) * kd : int64_t(ku) * binom(kd, 2);
    const int64_t nspin = int64_t(binom(__builtin_popcount(SP), kP[s])) * binom(__builtin_popcount(SN), kN[s]);
    total += nspin * int64_t(cur.size()) * (T == PROTON ? kP[s] : kN[s]) * Sq;
    KeySet X(cur.size() * 4 + 16);
    for (uint64_t q : cur) {
      const uint32_t u = qkey_u(q), d = qkey_d(q);
      for_quark_splits(T, u, d, [&](uint32_t yu, uint32_t yd) { X.insert(qkey(u & ~yu, d & ~yd)); });
    }
    cur = X.sorted();
  }
  return total;
}

static int build(const mb_nucleus *nuc, const mb_spin_request *req, int n_side, const mb_side_request *side,
                 bool counts_only, mb_term_list **out) {
  if (!nuc || !req || !out) return fail(MB_EINVAL, "null argument");
  if (n_side < 0 || (n_side > 0 && !side)) return fail(MB_EINVAL, "bad side requests");
  if (nuc->n_P < 0 || nuc->n_N < 0 || nuc->n_Lambda < 0) return fail(MB_EINVAL, "baryon counts must not be negative");
  if (nuc->n_Lambda > 1) return fail(MB_EUNSUPPORTED, "at most one Lambda");
  if (nuc->n_Lambda && (nuc->path == MB_PATH_BEST || n_side > 0 || req->proj))
    return fail(MB_EUNSUPPORTED, "a Lambda with MB_PATH_BEST, side requests or a projection");
  if (nuc->path == MB_PATH_BEST) {
    // the final required quark parts do not depend on the order (only signs
    // of L do): take them from the AUTO order, count every order, then build
    // the best one
    if (n_side > 0) return fail(MB_EUNSUPPORTED, "order search with side requests");
    mb_nucleus n2 = *nuc;
    n2.path = MB_PATH_AUTO;
    mb_term_list *probe = nullptr;
    int rc = build(&n2, req, 0, nullptr, true, &probe);
    if (rc) return rc;
    std::unique_ptr<mb_term_list> pg(probe);
    const int A = probe->A;
    uint32_t auto_mask = 0;
    for (int i = 0; i < A; i++)
      if (probe->path[i] == PROTON) auto_mask |= 1u << i;
    int path[MB_MAX_STAGES];
    auto ops = [&](uint32_t m) {
      for (int i = 0; i < A; i++) path[i] = (m >> i & 1) ? PROTON : NEUTRON;
      return path_operations(probe->st[A - 1].quark, path, A, probe->SP, probe->SN);
    };
    uint32_t best = auto_mask;
    int64_t best_ops = ops(auto_mask);
    for (uint32_t m = 0; m < (1u << A); m++) {
      if (__builtin_popcount(m) != nuc->n_P || m == auto_mask) continue;
      const int64_t o = ops(m);
      if (o < best_ops) {
        best_ops = o;
        best = m;
      }
    }
    n2.path = MB_PATH_EXPLICIT;
    n2.order = best;
    rc = build(&n2, req, 0, nullptr, counts_only, out);
    if (rc == MB_OK) (*out)->nuc.path = MB_PATH_BEST;
    return rc;
  }
  *out = nullptr;
  const int nP = nuc->n_P, nN = nuc->n_N, nLam = nuc->n_Lambda, An = nP + nN;
  if (An + nLam < 1) return fail(MB_EINVAL, "need at least one baryon");
  if (An + nLam > MB_MAX_STAGES) return fail(MB_EUNSUPPORTED, "more than 16 baryons");
  if (nuc->rel != 0 && nuc->rel != 1) return fail(MB_EINVAL, "rel must be 0 or 1");
  if (nuc->n_src < 1 || nuc->n_src > 3) return fail(MB_EUNSUPPORTED, "n_src must be 1, 2 or 3");
  // quark index sets are 24-bit fields of the packed keys: 3 D N_s <= 24
  if (nuc->n_src == 3 && nuc->rel) return fail(MB_EUNSUPPORTED, "three sources need nonrelativistic operators");
  if (nuc->path < 0 || nuc->path > MB_PATH_EXPLICIT) return fail(MB_EINVAL, "bad path");
  const int D = nuc->rel ? 4 : 2, nsrc = nuc->n_src;
  const int npsi = D * nsrc, nxi = 3 * D * nsrc;
  const int nu = 2 * nP + nN + nLam, nd = nP + 2 * nN + nLam;
  if (nP > npsi || nN > npsi)
    return fail(MB_EPAULI, "more baryons of one species than baryon indices");
  if (nu > nxi || nd > nxi) return fail(MB_EPAULI, "more quarks of one flavour than quark indices");
  // the s set of the Lambda's stage is packed above the u set (bit S_SHIFT)
  if (nLam && nxi > S_SHIFT - 4) return fail(MB_EUNSUPPORTED, "a Lambda needs at most 12 quark indices per flavour");

  mb_term_list *tl = new (std::nothrow) mb_term_list();
  if (!tl) return fail(MB_ENOMEM, "out of host memory");
  std::unique_ptr<mb_term_list> guard(tl);
  tl->nuc = *nuc;
  tl->D = D;
  tl->nsrc = nsrc;
  tl->npsi = npsi;
  tl->nxi = nxi;
  tl->A = An + nLam;
  tl->nLam = nLam;
  tl->counts_only = counts_only;
  const int A = tl->A;

  // path (Sec. 7)
  int first = nuc->path == MB_PATH_PROTONS_FIRST ? PROTON
              : nuc->path == MB_PATH_NEUTRONS_FIRST ? NEUTRON
              : (nN >= nP ? NEUTRON : PROTON);
  if (first == PROTON && nP == 0) first = NEUTRON;
  if (first == NEUTRON && nN == 0) first = PROTON;
  if (nuc->path == MB_PATH_EXPLICIT) {
    if ((An < 32 && (nuc->order >> An) != 0) || __builtin_popcount(nuc->order) != nP)
      return fail(MB_EINVAL, "order must mark n_P of the first n_P + n_N baryons as protons");
    for (int i = 0; i < An; i++) tl->path[i] = (nuc->order >> i & 1) ? PROTON : NEUTRON;
  } else {
    int nf = first == PROTON ? nP : nN;
    for (int i = 0; i < An; i++) tl->path[i] = i < nf ? first : 1 - first;
  }
  if (nLam) tl->path[A - 1] = LAMBDA;   // the Lambda after the nucleons
  tl->nstages = A;

  // spin request
  const uint32_t all = (1u << npsi) - 1;
  if (req->all_components) {
    tl->SP = nP ? all : 0;
    tl->SN = nN ? all : 0;
    tl->SL = nLam ? all : 0;
    const std::vector<uint32_t> lsets = nLam ? all_source_sets(1, D, nsrc) : std::vector<uint32_t>{0u};
    for (uint32_t p : all_source_sets(nP, D, nsrc))
      for (uint32_t n : all_source_sets(nN, D, nsrc))
        for (uint32_t l : lsets) {
          tl->alphas.push_back({p, n});
          if (nLam) tl->alphaL.push_back(l);
        }
  } else {
    if ((req->sink_P & ~all) || (req->sink_N & ~all))
      return fail(MB_EINVAL, "sink set has indices beyond D*N_s");
    if (__builtin_popcount(req->sink_P) < nP || __builtin_popcount(req->sink_N) < nN)
      return fail(MB_EINVAL, "sink base set smaller than the number of baryons");
    if (req->n_alpha < 1 || !req->alpha) return fail(MB_EINVAL, "no source sets");
    tl->SP = req->sink_P;
    tl->SN = req->sink_N;
    for (int i = 0; i < req->n_alpha; i++) {
      uint32_t p = req->alpha[2 * i], n = req->alpha[2 * i + 1];
      if ((p & ~all) || (n & ~all) || __builtin_popcount(p) != nP || __builtin_popcount(n) != nN)
        return fail(MB_EINVAL, "source set with wrong indices or size");
      tl->alphas.push_back({p, n});
    }
    if (nLam) {
      if ((req->sink_L & ~all) || !req->sink_L) return fail(MB_EINVAL, "Lambda sink set empty or beyond D*N_s");
      if (!req->alpha_L) return fail(MB_EINVAL, "no Lambda source sets");
      tl->SL = req->sink_L;
      for (int i = 0; i < req->n_alpha; i++) {
        const uint32_t l = req->alpha_L[i];
        if ((l & ~all) || __builtin_popcount(l) != 1) return fail(MB_EINVAL, "Lambda source set must be one index");
        tl->alphaL.push_back(l);
      }
    }
  }
  if (nP == 0) tl->SP = 0;
  if (nN == 0) tl->SN = 0;

  // ---- L by the recursion L^(n+1) = L^(n) . G (eq. recr_L); c_alpha per source set
  std::vector<std::vector<std::pair<uint64_t, int64_t>>> per_alpha;
  if (!nLam) {
    const int rc = source_coefficients(tl, A, tl->alphas, per_alpha);
    if (rc) return rc;
  } else {
    // the nucleons' coefficients for their distinct source sets, then the
    // Lambda as the last factor
    std::vector<std::array<uint32_t, 2>> nal;
    std::vector<int> nidx;
    for (auto &a : tl->alphas) {
      size_t j = 0;
      while (j < nal.size() && nal[j] != a) j++;
      if (j == nal.size()) nal.push_back(a);
      nidx.push_back(int(j));
    }
    std::vector<std::vector<std::pair<uint64_t, int64_t>>> nucc;
    if (An > 0) {
      const int rc = source_coefficients(tl, An, nal, nucc);
      if (rc) return rc;
    } else {
      nucc.assign(nal.size(), {{qkey(0, 0), 1}});
    }
    lambda_coefficients(tl, nucc, nidx, per_alpha);
  }

  const bool last_d_major = tl->path[A - 1] == PROTON && A > 1;
  std::vector<uint64_t> U;
  // Projection (Sec. 5): L_M(delta; q) = sum_alpha w[delta][alpha] c_alpha(q)
  // for every sink set delta (proton rank major, as the final stage's spin
  // parts), summed in alpha order; the final quark parts are those with a
  // nonzero L_M for some delta.
  std::vector<std::vector<std::pair<uint64_t, double>>> lm;
  tl->projected = req->proj != nullptr;
  if (tl->projected) {
    const int64_t ndel = int64_t(binom(__builtin_popcount(tl->SP), nP)) * binom(__builtin_popcount(tl->SN), nN);
    const size_t nal = tl->alphas.size();
    for (size_t i = 0; i < size_t(ndel) * nal; i++)
      if (!std::isfinite(req->proj[i])) return fail(MB_EINVAL, "projection weight not finite");
    lm.resize(size_t(ndel));
    for (int64_t dl = 0; dl < ndel; dl++) {
      std::unordered_map<uint64_t, double> m;
      for (size_t al = 0; al < nal; al++) {
        const double w = req->proj[size_t(dl) * nal + al];
        if (w == 0.0) continue;
        for (auto &e : per_alpha[al]) m[e.first] += w * double(e.second);
      }
      for (auto &kv : m)
        if (kv.second != 0.0) {   // entries that cancel exactly leave the list
          lm[dl].push_back(kv);
          U.push_back(kv.first);
        }
    }
  } else {
    for (auto &v : per_alpha)
      for (auto &e : v) U.push_back(e.first);
  }
  sort_stage(U, last_d_major);
  U.erase(std::unique(U.begin(), U.end()), U.end());
  tl->nU = int64_t(U.size());
  auto kept = [&](uint64_t q) {
    const uint32_t i = find_stage(U, last_d_major, q);
    return i < U.size() && U[i] == q;
  };
  if (tl->projected) {
    tl->prow.assign(1, 0);
    for (auto &v : lm) {
      std::vector<std::pair<uint32_t, double>> row;
      for (auto &e : v) row.push_back({find_stage(U, last_d_major, e.first), e.second});
      std::sort(row.begin(), row.end());
      for (auto &e : row) {
        tl->pcol.push_back(e.first);
        tl->pval.push_back(e.second);
      }
      tl->prow.push_back(int64_t(tl->pcol.size()));
    }
  }
  tl->crow.assign(1, 0);
  for (auto &v : per_alpha) {
    std::vector<std::pair<uint32_t, int64_t>> row;
    for (auto &e : v)
      if (!tl->projected || kept(e.first)) row.push_back({find_stage(U, last_d_major, e.first), e.second});
    std::sort(row.begin(), row.end());
    for (auto &e : row) {
      tl->ccol.push_back(e.first);
      tl->cval.push_back(e.second);
    }
    tl->crow.push_back(int64_t(tl->ccol.size()));
  }
  tl->nL = int64_t(tl->ccol.size());

  // ---- smaller nuclei on the path (Sec. 7): the nucleus of the first
  // stage+1 baryons, read from that stage with its own coefficients
  if (n_side > 0 && tl->projected) return fail(MB_EUNSUPPORTED, "side requests with a projection");
  std::vector<std::vector<std::vector<std::pair<uint64_t, int64_t>>>> side_coef(static_cast<size_t>(n_side));
  for (int i = 0; i < n_side; i++) {
    const mb_side_request &r = side[i];
    if (r.stage < 0 || r.stage >= A - 1) return fail(MB_EINVAL, "side stage must lie before the last stage");
    int kP = 0, kN = 0;
    for (int s = 0; s <= r.stage; s++) (tl->path[s] == PROTON ? kP : kN)++;
    Side sd;
    sd.stage = r.stage;
    if (r.all_components) {
      for (uint32_t p : all_source_sets(kP, D, nsrc))
        for (uint32_t n : all_source_sets(kN, D, nsrc)) sd.alphas.push_back({p, n});
    } else {
      if (r.n_alpha < 1 || !r.alpha) return fail(MB_EINVAL, "side request without source sets");
      for (int j = 0; j < r.n_alpha; j++) {
        uint32_t p = r.alpha[2 * j], n = r.alpha[2 * j + 1];
        if ((p & ~all) || (n & ~all) || __builtin_popcount(p) != kP || __builtin_popcount(n) != kN)
          return fail(MB_EINVAL, "side source set with wrong indices or size");
        sd.alphas.push_back({p, n});
      }
    }
    const int rc = source_coefficients(tl, r.stage + 1, sd.alphas, side_coef[i]);
    if (rc) return rc;
    tl->sides.push_back(std::move(sd));
  }

  // ---- stages
  tl->st.resize(A);
  {
    int kp = 0, kn = 0, kl = 0;
    for (int s = 0; s < A; s++) {
      Stage &S = tl->st[s];
      S.type = tl->path[s];
      (S.type == PROTON ? kp : S.type == NEUTRON ? kn : kl)++;
      S.kP = kp;
      S.kN = kn;
      S.kL = kl;
      S.ku = 2 * kp + kn + kl;
      S.kd = kp + 2 * kn + kl;
      S.nPsets = binom(__builtin_popcount(tl->SP), kp);
      S.nNsets = binom(__builtin_popcount(tl->SN), kn);
      S.nLsets = binom(__builtin_popcount(tl->SL), kl);
    }
  }
  tl->st[A - 1].quark = U;
  for (int s = A - 1; s >= 1; s--) {
    Stage &S = tl->st[s], &P = tl->st[s - 1];
    const int T = S.type;
    KeySet X(S.quark.size() * 4 + 16);
    for (uint64_t q : S.quark) {
      uint32_t u = qkey_u(q), d = qkey_d(q);
      if (T == LAMBDA)
        for_lambda_splits(u, d, [&](uint32_t yu, uint32_t yd) { X.insert(qkey(ufield_u(u) & ~yu, d & ~yd)); });
      else
        for_quark_splits(T, u, d, [&](uint32_t yu, uint32_t yd) { X.insert(qkey(u & ~yu, d & ~yd)); });
    }
    // the quark parts that side nuclei read from stage s - 1
    for (size_t i = 0; i < tl->sides.size(); i++)
      if (tl->sides[i].stage == s - 1)
        for (auto &v : side_coef[i])
          for (auto &e : v) X.insert(e.first);
    P.quark = X.sorted();
    const bool pd = P.type == PROTON && s - 1 > 0;
    sort_stage(P.quark, pd);
    S.Sq = T == PROTON ? binom(S.ku, 2) * S.kd : T == NEUTRON ? S.ku * binom(S.kd, 2) : S.ku * S.kd;
    const int kT = T == PROTON ? S.kP : T == NEUTRON ? S.kN : S.kL;
    S.n_lambda = S.nreq() * kT * S.Sq;
    if (!counts_only) {
      try {
        S.qsplit.resize(S.quark.size() * size_t(S.Sq) * 2);
      } catch (...) {
        return fail(MB_ENOMEM, "out of host memory for the operation tables");
      }
      size_t o = 0;
      for (uint64_t q : S.quark) {
        uint32_t u = qkey_u(q), d = qkey_d(q);
        if (T == LAMBDA) {
          const uint32_t uu = ufield_u(u), ys = ufield_s(u);
          for_lambda_splits(u, d, [&](uint32_t yu, uint32_t yd) {
            uint32_t xu = uu & ~yu, xd = d & ~yd;
            uint32_t xi = find_stage(P.quark, pd, qkey(xu, xd));
            int sg = split_sign(xu, yu) * split_sign(xd, yd);
            S.qsplit[o++] = xi;
            S.qsplit[o++] = lambda_qidx(ys, yu, yd, nxi) | (sg < 0 ? 0x80000000u : 0u);
          });
          continue;
        }
        for_quark_splits(T, u, d, [&](uint32_t yu, uint32_t yd) {
          uint32_t xu = u & ~yu, xd = d & ~yd;
          uint32_t xi = find_stage(P.quark, pd, qkey(xu, xd));
          int sg = split_sign(xu, yu) * split_sign(xd, yd);
          S.qsplit[o++] = xi;
          S.qsplit[o++] = block_qidx(T, yu, yd, nxi) | (sg < 0 ? 0x80000000u : 0u);
        });
      }
    }
  }
  // side coefficients as CSR over their source sets, columns in the order of
  // their stage
  for (size_t i = 0; i < tl->sides.size(); i++) {
    Side &sd = tl->sides[i];
    const int j = sd.stage;
    const bool dm = tl->path[j] == PROTON && j > 0;
    sd.crow.assign(1, 0);
    for (auto &v : side_coef[i]) {
      std::vector<std::pair<uint32_t, int64_t>> row;
      for (auto &e : v) row.push_back({find_stage(tl->st[j].quark, dm, e.first), e.second});
      std::sort(row.begin(), row.end());
      for (auto &e : row) {
        sd.ccol.push_back(e.first);
        sd.cval.push_back(e.second);
      }
      sd.crow.push_back(int64_t(sd.ccol.size()));
    }
  }
  {
    Stage &S0 = tl->st[0];
    if (!counts_only) {
      S0.first.resize(S0.quark.size());
      for (size_t i = 0; i < S0.quark.size(); i++) {
        const uint32_t u = qkey_u(S0.quark[i]), d = qkey_d(S0.quark[i]);
        S0.first[i] = S0.type == LAMBDA ? lambda_qidx(ufield_s(u), ufield_u(u), d, nxi)
                                        : block_qidx(S0.type, u, d, nxi);
      }
    }
  }
  *out = guard.release();
  set_error("");
  return MB_OK;
}

}  // namespace mb

size_t mb_term_list::image_bytes() const {
  if (counts_only) return 0;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t o = 0;
  for (int s = 1; s < nstages; s++)
    o += al(st[s].qsplit.size() * 4) + al(st[s].quark.size() * 8) + al(st[s].quark.size() * st[s].nsingle() * 4);
  o += al(st[0].first.size() * 4);
  if (projected) o += al(prow.size() * 8) + al(pcol.size() * 4) + al(pval.size() * 8);
  else o += al(crow.size() * 8) + al(ccol.size() * 4) + al(cval.size() * 8);
  for (const mb::Side &sd : sides) o += al(sd.crow.size() * 8) + al(sd.ccol.size() * 4) + al(sd.cval.size() * 8);
  return o + 256;
}

int64_t mb_term_list::main_outputs() const {
  return projected ? 1 : st.back().nspin() * int64_t(alphas.size());
}

int64_t mb_term_list::side_offset(size_t i) const {
  int64_t o = main_outputs();
  for (size_t j = 0; j < i; j++) o += st[sides[j].stage].nspin() * int64_t(sides[j].alphas.size());
  return o;
}

using namespace mb;

extern "C" {

int mb_build_term_list(const mb_nucleus *nuc, const mb_spin_request *req, mb_term_list **out) {
  try {
    return build(nuc, req, 0, nullptr, false, out);
  } catch (const std::bad_alloc &) {
    return fail(MB_ENOMEM, "out of host memory");
  }
}

int mb_build_term_list_counts_only(const mb_nucleus *nuc, const mb_spin_request *req,
                                   mb_term_list **out) {
  try {
    return build(nuc, req, 0, nullptr, true, out);
  } catch (const std::bad_alloc &) {
    return fail(MB_ENOMEM, "out of host memory");
  }
}

int mb_build_term_list_path(const mb_nucleus *nuc, const mb_spin_request *req, int n_side,
                            const mb_side_request *side, mb_term_list **out) {
  try {
    return build(nuc, req, n_side, side, false, out);
  } catch (const std::bad_alloc &) {
    return fail(MB_ENOMEM, "out of host memory");
  }
}

void mb_term_list_free(mb_term_list *tl) { delete tl; }

int mb_term_list_counts(const mb_term_list *tl, mb_counts *c) {
  if (!tl || !c) return fail(MB_EINVAL, "null argument");
  std::memset(c, 0, sizeof *c);
  c->n_stages = tl->nstages;
  for (int s = 0; s < tl->nstages; s++) {
    const Stage &S = tl->st[s];
    c->path[s] = tl->path[s];
    c->n_lambda_step[s] = S.n_lambda;
    c->n_lambda += S.n_lambda;
    c->n_req[s] = S.nreq();
    c->n_quark[s] = int64_t(S.quark.size());
    c->n_spin[s] = int32_t(S.nspin());
  }
  c->n_L = tl->nL;
  c->n_U = tl->nU;
  c->n_delta = int32_t(tl->st[tl->nstages - 1].nspin());
  c->n_alpha = int32_t(tl->alphas.size());
  c->n_psi = tl->npsi;
  c->n_xi = tl->nxi;
  c->device_bytes = int64_t(tl->image_bytes());
  c->projected = tl->projected ? 1 : 0;
  c->n_LM = int64_t(tl->pcol.size());
  c->n_side = int32_t(tl->sides.size());
  c->n_out = tl->side_offset(tl->sides.size());
  c->rel = tl->nuc.rel;
  c->n_src = tl->nsrc;
  c->n_Lambda = tl->nLam;
  return MB_OK;
}

int mb_term_list_export(const mb_term_list *tl, int what, int stage, void *buf, size_t *bytes) {
  if (!tl || !bytes) return fail(MB_EINVAL, "null argument");
  if (what == MB_EXPORT_SIDE) {
    if (stage < 0 || size_t(stage) >= tl->sides.size()) return fail(MB_EINVAL, "no such side request");
  } else if (stage < 0 || stage >= tl->nstages) {
    return fail(MB_EINVAL, "bad stage");
  }
  const Stage &S = tl->st[what == MB_EXPORT_SIDE ? 0 : stage];
  std::vector<uint8_t> tmp;
  auto put = [&](const void *p, size_t n) {
    size_t o = tmp.size();
    tmp.resize(o + n);
    if (n) std::memcpy(tmp.data() + o, p, n);
  };
  switch (what) {
    case MB_EXPORT_QUARK:
      for (uint64_t q : S.quark) {
        uint32_t v[2] = {tl->nLam ? ufield_u(qkey_u(q)) : qkey_u(q), qkey_d(q)};
        put(v, 8);
      }
      break;
    case MB_EXPORT_QUARK_S:
      for (uint64_t q : S.quark) {
        const uint32_t v = tl->nLam ? ufield_s(qkey_u(q)) : 0u;
        put(&v, 4);
      }
      break;
    case MB_EXPORT_SPIN:
    case MB_EXPORT_SPIN_L: {
      int mP = __builtin_popcount(tl->SP), mN = __builtin_popcount(tl->SN), mL = __builtin_popcount(tl->SL);
      std::vector<uint32_t> ps, ns, ls;
      for (uint32_t m = 0; m < (1u << mP); m++)
        if (__builtin_popcount(m) == S.kP) ps.push_back(from_positions(m, tl->SP));
      for (uint32_t m = 0; m < (1u << mN); m++)
        if (__builtin_popcount(m) == S.kN) ns.push_back(from_positions(m, tl->SN));
      for (uint32_t m = 0; m < (1u << mL); m++)
        if (__builtin_popcount(m) == S.kL) ls.push_back(from_positions(m, tl->SL));
      for (uint32_t p : ps)
        for (uint32_t n : ns)
          for (uint32_t l : ls) {
            uint32_t v[2] = {p, n};
            if (what == MB_EXPORT_SPIN) put(v, 8);
            else put(&l, 4);
          }
      break;
    }
    case MB_EXPORT_QSPLIT:
      if (stage < 1 || tl->counts_only) return fail(MB_EINVAL, "no split table for this stage");
      put(S.qsplit.data(), S.qsplit.size() * 4);
      break;
    case MB_EXPORT_SSPLIT: {
      if (stage < 1) return fail(MB_EINVAL, "no split table for stage 0");
      const Stage &Pv = tl->st[stage - 1];
      const int T = S.type;
      if (T == LAMBDA) {
        // one split per output: the Lambda takes its index, the nucleon
        // spin part passes through (sign +1)
        for (int rpn = 0; rpn < S.nPsets * S.nNsets; rpn++)
          for (uint32_t t = tl->SL; t; t &= t - 1) {
            int32_t v[3] = {rpn, __builtin_ctz(t), 1};
            put(v, 12);
          }
        break;
      }
      int mP = __builtin_popcount(tl->SP), mN = __builtin_popcount(tl->SN);
      for (int rp = 0; rp < S.nPsets; rp++)
        for (int rn = 0; rn < S.nNsets; rn++) {
          // unrank
          uint32_t pp = 0, np = 0;
          int c = 0;
          for (uint32_t m = 0; m < (1u << mP); m++)
            if (__builtin_popcount(m) == S.kP && c++ == rp) pp = m;
          c = 0;
          for (uint32_t m = 0; m < (1u << mN); m++)
            if (__builtin_popcount(m) == S.kN && c++ == rn) np = m;
          uint32_t act = T == PROTON ? pp : np, base = T == PROTON ? tl->SP : tl->SN;
          for (uint32_t t = act; t; t &= t - 1) {
            uint32_t bit = t & (~t + 1);
            uint32_t rest = act & ~bit;
            int32_t sg = split_sign(rest, bit);
            int32_t psi = __builtin_ctz(from_positions(bit, base));
            int32_t idx = T == PROTON ? subset_rank(rest, mP) * Pv.nNsets + rn
                                      : rp * Pv.nNsets + subset_rank(rest, mN);
            int32_t v[3] = {idx, psi, sg};
            put(v, 12);
          }
        }
      break;
    }
    case MB_EXPORT_COEF:
      put(tl->crow.data(), tl->crow.size() * 8);
      put(tl->ccol.data(), tl->ccol.size() * 8);
      put(tl->cval.data(), tl->cval.size() * 8);
      break;
    case MB_EXPORT_DELTA: {
      size_t n = 0;
      mb_term_list_export(tl, MB_EXPORT_SPIN, tl->nstages - 1, nullptr, &n);
      tmp.resize(n);
      mb_term_list_export(tl, MB_EXPORT_SPIN, tl->nstages - 1, tmp.data(), &n);
      break;
    }
    case MB_EXPORT_ALPHA:
      for (auto &a : tl->alphas) put(a.data(), 8);
      break;
    case MB_EXPORT_DELTA_L: {
      size_t n = 0;
      mb_term_list_export(tl, MB_EXPORT_SPIN_L, tl->nstages - 1, nullptr, &n);
      tmp.resize(n);
      mb_term_list_export(tl, MB_EXPORT_SPIN_L, tl->nstages - 1, tmp.data(), &n);
      break;
    }
    case MB_EXPORT_ALPHA_L:
      for (size_t i = 0; i < tl->alphas.size(); i++) {
        const uint32_t l = tl->nLam ? tl->alphaL[i] : 0u;
        put(&l, 4);
      }
      break;
    case MB_EXPORT_SIDE: {
      const Side &sd = tl->sides[size_t(stage)];
      const int64_t hd[2] = {sd.stage, int64_t(sd.alphas.size())};
      put(hd, 16);
      for (auto &a : sd.alphas) put(a.data(), 8);
      put(sd.crow.data(), sd.crow.size() * 8);
      put(sd.ccol.data(), sd.ccol.size() * 8);
      put(sd.cval.data(), sd.cval.size() * 8);
      break;
    }
    case MB_EXPORT_PROJ:
      if (!tl->projected) return fail(MB_EINVAL, "not a projected term list");
      put(tl->prow.data(), tl->prow.size() * 8);
      put(tl->pcol.data(), tl->pcol.size() * 8);
      put(tl->pval.data(), tl->pval.size() * 8);
      break;
    default:
      return fail(MB_EINVAL, "unknown export item");
  }
  if (!buf) {
    *bytes = tmp.size();
    return MB_OK;
  }
  if (*bytes < tmp.size()) return fail(MB_ENOWORKSPACE, "export buffer too small");
  std::memcpy(buf, tmp.data(), tmp.size());
  *bytes = tmp.size();
  return MB_OK;
}

const char *mb_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Saving and loading term lists: a magic word and format version, then every
// field of the host list in a fixed order; vectors as a 64-bit length
// followed by their elements.
namespace {

constexpr uint64_t kFileMagic = 0x3153494c4d524554ull;   // "TERMLIS1"
constexpr uint32_t kFileVersion = 2;

struct Writer {
  FILE *f;
  bool ok = true;
  void raw(const void *p, size_t n) {
    if (ok && n) ok = std::fwrite(p, 1, n, f) == n;
  }
  template <typename T> void val(const T &v) { raw(&v, sizeof v); }
  void val(const bool &v) {
    const uint8_t b = v ? 1 : 0;
    raw(&b, 1);
  }
  template <typename T> void vec(const std::vector<T> &v) {
    val(uint64_t(v.size()));
    raw(v.data(), v.size() * sizeof(T));
  }
};

struct Reader {
  FILE *f;
  bool ok = true;
  void raw(void *p, size_t n) {
    if (ok && n) ok = std::fread(p, 1, n, f) == n;
  }
  template <typename T> void val(T &v) { raw(&v, sizeof v); }
  void val(bool &v) {
    uint8_t b = 0;
    raw(&b, 1);
    if (b > 1) ok = false;
    v = b == 1;
  }
  template <typename T> void vec(std::vector<T> &v) {
    uint64_t n = 0;
    val(n);
    // a length beyond what is left in the file marks a corrupt file
    const long here = std::ftell(f);
    std::fseek(f, 0, SEEK_END);
    const long end = std::ftell(f);
    std::fseek(f, here, SEEK_SET);
    if (!ok || here < 0 || end < here || n > uint64_t(end - here) / sizeof(T)) {
      ok = false;
      return;
    }
    v.resize(size_t(n));
    raw(v.data(), v.size() * sizeof(T));
  }
};

template <typename IO, typename TL, typename STAGE, typename SIDE>
void fields(IO &io, TL &tl, std::vector<STAGE> &st, std::vector<SIDE> &sides) {
  io.val(tl.nuc);
  io.val(tl.D);
  io.val(tl.nsrc);
  io.val(tl.npsi);
  io.val(tl.nxi);
  io.val(tl.A);
  io.val(tl.nstages);
  io.val(tl.path);
  io.val(tl.SP);
  io.val(tl.SN);
  io.vec(tl.alphas);
  io.vec(tl.crow);
  io.vec(tl.ccol);
  io.vec(tl.cval);
  io.val(tl.nL);
  io.val(tl.nU);
  io.val(tl.projected);
  io.vec(tl.prow);
  io.vec(tl.pcol);
  io.vec(tl.pval);
  io.val(tl.counts_only);
  for (auto &S : st) {
    io.val(S.type);
    io.val(S.kP);
    io.val(S.kN);
    io.val(S.ku);
    io.val(S.kd);
    io.val(S.nPsets);
    io.val(S.nNsets);
    io.vec(S.quark);
    io.val(S.Sq);
    io.vec(S.qsplit);
    io.vec(S.first);
    io.val(S.n_lambda);
  }
  for (auto &sd : sides) {
    io.val(sd.stage);
    io.vec(sd.alphas);
    io.vec(sd.crow);
    io.vec(sd.ccol);
    io.vec(sd.cval);
  }
}

// Structural checks of a loaded list: every size follows from the nucleus,
// the path and the sink base sets as in a built list, and every index the
// kernels follow (split tables, gather indices, coefficient lists) stays
// inside the table it points into.
bool valid_loaded(const mb_term_list &t) {
  const mb_nucleus &n = t.nuc;
  if (n.n_Lambda != 0 || t.nLam != 0) return false;   // not saved (mb_term_list_save)
  if (n.n_P < 0 || n.n_N < 0 || n.n_P + n.n_N < 1 || n.n_P + n.n_N > MB_MAX_STAGES) return false;
  if ((n.rel != 0 && n.rel != 1) || n.n_src < 1 || n.n_src > 3 || (n.n_src == 3 && n.rel)) return false;
  const int D = n.rel ? 4 : 2, A = n.n_P + n.n_N;
  if (t.D != D || t.nsrc != n.n_src || t.npsi != D * n.n_src || t.nxi != 3 * D * n.n_src) return false;
  if (t.A != A || t.nstages != A || int(t.st.size()) != A) return false;
  const uint32_t allpsi = (1u << t.npsi) - 1, allxi = (1u << t.nxi) - 1;
  if ((t.SP & ~allpsi) || (t.SN & ~allpsi)) return false;
  int kP = 0, kN = 0;
  for (int s = 0; s < A; s++) {
    const Stage &S = t.st[size_t(s)];
    if (t.path[s] != PROTON && t.path[s] != NEUTRON) return false;
    (t.path[s] == PROTON ? kP : kN)++;
    if (S.type != t.path[s] || S.kP != kP || S.kN != kN || S.ku != 2 * kP + kN || S.kd != kP + 2 * kN) return false;
    if (S.nPsets != binom(__builtin_popcount(t.SP), kP) || S.nNsets != binom(__builtin_popcount(t.SN), kN)) return false;
    if (S.nPsets < 1 || S.nNsets < 1) return false;
    for (uint64_t q : S.quark)
      if ((qkey_u(q) & ~allxi) || (qkey_d(q) & ~allxi) || __builtin_popcount(qkey_u(q)) != S.ku ||
          __builtin_popcount(qkey_d(q)) != S.kd)
        return false;
    // quark parts strictly increasing in the stage's order (lookups bisect)
    const bool dm = S.type == PROTON && s > 0;
    for (size_t i = 1; i < S.quark.size(); i++)
      if (order_key(S.quark[i - 1], dm) >= order_key(S.quark[i], dm)) return false;
    if (s == 0) {
      if (!t.counts_only && S.first.size() != S.quark.size()) return false;
      for (size_t i = 0; i < S.first.size(); i++)
        if (S.first[i] != block_qidx(S.type, qkey_u(S.quark[i]), qkey_d(S.quark[i]), t.nxi)) return false;
      continue;
    }
    const Stage &P = t.st[size_t(s) - 1];
    const bool pdm = P.type == PROTON && s - 1 > 0;
    const int64_t Sq = S.type == PROTON ? int64_t(binom(S.ku, 2)) * S.kd : int64_t(S.ku) * binom(S.kd, 2);
    if (S.Sq != Sq || S.n_lambda != S.nreq() * (S.type == PROTON ? kP : kN) * Sq) return false;
    if (S.qsplit.size() != (t.counts_only ? 0 : S.quark.size() * size_t(S.Sq) * 2)) return false;
    // every split entry is the one the builder derives from the quark parts
    bool same = true;
    for (size_t qi = 0; same && qi < S.quark.size(); qi++) {
      const uint32_t u = qkey_u(S.quark[qi]), d = qkey_d(S.quark[qi]);
      size_t o = qi * size_t(S.Sq) * 2;
      for_quark_splits(S.type, u, d, [&](uint32_t yu, uint32_t yd) {
        if (!same || S.qsplit.empty()) return;
        const uint64_t xk = qkey(u & ~yu, d & ~yd);
        const uint32_t xi = find_stage(P.quark, pdm, xk);
        const int sg = split_sign(u & ~yu, yu) * split_sign(d & ~yd, yd);
        const uint32_t y = block_qidx(S.type, yu, yd, t.nxi) | (sg < 0 ? 0x80000000u : 0u);
        if (xi >= P.quark.size() || P.quark[xi] != xk || S.qsplit[o] != xi || S.qsplit[o + 1] != y) same = false;
        o += 2;
      });
    }
    if (!same) return false;
  }
  if (kP != n.n_P || kN != n.n_N) return false;
  auto csr_ok = [](const std::vector<int64_t> &row, size_t nrows, const std::vector<int64_t> &col, size_t nval,
                   size_t ncols) {
    if (row.size() != nrows + 1 || row[0] != 0 || uint64_t(row.back()) != col.size() || nval != col.size())
      return false;
    for (size_t i = 0; i < nrows; i++)
      if (row[i + 1] < row[i]) return false;
    for (int64_t c : col)
      if (c < 0 || uint64_t(c) >= ncols) return false;
    return true;
  };
  const size_t nfinal = t.st.back().quark.size();
  for (auto &a : t.alphas)
    if ((a[0] & ~allpsi) || (a[1] & ~allpsi) || __builtin_popcount(a[0]) != n.n_P || __builtin_popcount(a[1]) != n.n_N)
      return false;
  if (!csr_ok(t.crow, t.alphas.size(), t.ccol, t.cval.size(), nfinal)) return false;
  if (t.projected && !csr_ok(t.prow, size_t(t.st.back().nspin()), t.pcol, t.pval.size(), nfinal)) return false;
  if (!t.projected && (!t.prow.empty() || !t.pcol.empty() || !t.pval.empty())) return false;
  if (t.projected && !t.sides.empty()) return false;
  for (const Side &sd : t.sides) {
    if (sd.stage < 0 || sd.stage >= A - 1) return false;
    if (!csr_ok(sd.crow, sd.alphas.size(), sd.ccol, sd.cval.size(), t.st[size_t(sd.stage)].quark.size())) return false;
  }
  return true;
}

}  // namespace

extern "C" {

int mb_term_list_save(const mb_term_list *tl, const char *path) {
  if (!tl || !path) return fail(MB_EINVAL, "null argument");
  if (tl->nLam) return fail(MB_EUNSUPPORTED, "saving a term list with a Lambda");
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(MB_EINVAL, std::string("cannot open ") + path + " for writing");
  Writer w{f};
  w.val(kFileMagic);
  w.val(kFileVersion);
  w.val(uint64_t(tl->st.size()));
  w.val(uint64_t(tl->sides.size()));
  // the field walk takes non-const references; the writer only reads them
  mb_term_list &t = const_cast<mb_term_list &>(*tl);
  fields(w, t, t.st, t.sides);
  const bool ok = w.ok && std::fclose(f) == 0;
  if (!ok) return fail(MB_EINVAL, std::string("write to ") + path + " failed");
  set_error("");
  return MB_OK;
}

int mb_term_list_load(const char *path, mb_term_list **out) {
  if (!path || !out) return fail(MB_EINVAL, "null argument");
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(MB_EINVAL, std::string("cannot open ") + path);
  std::unique_ptr<FILE, int (*)(FILE *)> fg(f, std::fclose);
  try {
    Reader r{f};
    uint64_t magic = 0, nst = 0, nside = 0;
    uint32_t version = 0;
    r.val(magic);
    if (!r.ok || magic != kFileMagic) return fail(MB_EINVAL, std::string(path) + " is not a term list file");
    r.val(version);
    if (!r.ok || version != kFileVersion) return fail(MB_EUNSUPPORTED, "term list file of another format version");
    r.val(nst);
    r.val(nside);
    if (!r.ok || nst < 1 || nst > MB_MAX_STAGES || nside > MB_MAX_STAGES)
      return fail(MB_EINVAL, std::string(path) + " is corrupt");
    std::unique_ptr<mb_term_list> tl(new mb_term_list());
    tl->st.resize(size_t(nst));
    tl->sides.resize(size_t(nside));
    fields(r, *tl, tl->st, tl->sides);
    char extra;
    if (!r.ok || std::fread(&extra, 1, 1, f) != 0 || tl->nstages != int(nst) || tl->A != int(nst))
      return fail(MB_EINVAL, std::string(path) + " is truncated or corrupt");
    if (!valid_loaded(*tl)) return fail(MB_EINVAL, std::string(path) + " is corrupt");
    *out = tl.release();
    set_error("");
    return MB_OK;
  } catch (const std::bad_alloc &) {
    return fail(MB_ENOMEM, "out of host memory");
  }
}

}  // extern "C"
