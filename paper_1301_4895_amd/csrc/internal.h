// Internal structures of libmbcontract shared by the host builder, the C ABI
// and the kernel launchers.  Not part of the public interface.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mbcontract.h"

namespace mb {

// Quark part of a component: (u index set, d index set) as bit masks,
// packed as (u << 32) | d so that sorting the packed value sorts by (u, d).
inline uint64_t qkey(uint32_t u, uint32_t d) { return (uint64_t(u) << 32) | d; }
inline uint32_t qkey_u(uint64_t k) { return uint32_t(k >> 32); }
inline uint32_t qkey_d(uint64_t k) { return uint32_t(k); }
// In a system with a Lambda (at most 12 quark indices per flavour) the s
// index set of the Lambda's stage sits above the u set: u field = u | s << 16.
constexpr int S_SHIFT = 16;
inline uint32_t ufield_u(uint32_t f) { return f & ((1u << S_SHIFT) - 1u); }
inline uint32_t ufield_s(uint32_t f) { return f >> S_SHIFT; }

enum { PROTON = 0, NEUTRON = 1, LAMBDA = 2 };

// One stage of the recursion: the components holding the first s+1 baryons
// of the path.  Required components are (spin part) x (quark part); the spin
// parts are every kP-subset of the sink proton base set times every
// kN-subset of the neutron base set (times, at the Lambda's stage, every
// index of the Lambda's sink base set), ordered (proton rank, neutron rank,
// Lambda rank) with subsets ranked by mask value.
struct Stage {
  int type = 0;                  // species of the baryon added to reach this stage
  int kP = 0, kN = 0, ku = 0, kd = 0;
  int kL = 0;                    // 1 at the Lambda's stage
  int nPsets = 0, nNsets = 0;    // C(|SP|, kP), C(|SN|, kN)
  int nLsets = 1;                // C(|SL|, kL)
  std::vector<uint64_t> quark;   // sorted quark parts
  int Sq = 0;                    // quark splits per output quark part (s >= 1)
  std::vector<uint32_t> qsplit;  // [nq][Sq][2]: x index, y block index | sign<<31
  std::vector<uint32_t> first;   // stage 0: block quark index of every quark part
  int64_t n_lambda = 0;
  int tune_pg = 0, tune_lds = 0, tune_tile = 64;  // launch tuning (see mb_term_list_tune)
  int tune_kernel = 0;                            // 0 direct gather, 1 blocks staged in LDS
  int tune_unroll = 0;                            // splits in flight per wavefront (0 automatic)
  int tune_group = 1;                             // outputs per wavefront (grouped kernel when > 1)
  int tune_paired = 1;                            // input stage in the paired layout when possible
  int tune_two_phase = 0;                         // 1: partial sums per single index, then their sum
  int64_t nspin() const { return int64_t(nPsets) * nNsets * nLsets; }
  // quark indices of the added baryon's single flavour in an output quark
  // part (d for a proton step, u for a neutron step): the splits of an
  // output come in that many groups of Sq / nsingle() pair splits (a
  // Lambda step, which has no pair, counts as one group)
  int nsingle() const { return type == PROTON ? kd : type == NEUTRON ? ku : 1; }
  // spin parts of the other species that a step passes through
  int npass() const { return type == PROTON ? nNsets : type == NEUTRON ? nPsets : nPsets * nNsets; }
  int64_t nreq() const { return nspin() * int64_t(quark.size()); }
};

// A smaller nucleus on the path (Sec. 7), read from stage `stage`.
struct Side {
  int stage = 0;
  std::vector<std::array<uint32_t, 2>> alphas;   // source sets
  std::vector<int64_t> crow, ccol, cval;         // c_alpha(q) on the stage's quark parts, CSR over alpha
  size_t off_crow = 0, off_ccol = 0, off_cval = 0;
};

}  // namespace mb

struct mb_term_list {
  mb_nucleus nuc{};
  int D = 0, nsrc = 0, npsi = 0, nxi = 0, A = 0;
  int nstages = 0;
  int path[MB_MAX_STAGES] = {};
  uint32_t SP = 0, SN = 0;                      // sink base sets
  std::vector<std::array<uint32_t, 2>> alphas;   // requested source sets
  int blocks_kernel = 0;                         // MB_TUNE_BLOCKS: 0 automatic, 1 matrix cores, 2 vector units
  int nLam = 0;                                  // 1: one Lambda, added last
  uint32_t SL = 0;                               // the Lambda's sink base set
  std::vector<uint32_t> alphaL;                  // the Lambda's source set per column
  std::vector<mb::Stage> st;
  // final coefficients c_alpha(q) = L(alpha; q) on sorted sets, CSR over alpha
  std::vector<int64_t> crow, ccol, cval;
  int64_t nL = 0, nU = 0;
  // projection (Sec. 5): L_M(delta; q) = sum_alpha w[delta][alpha] c_alpha(q),
  // CSR over the sink sets delta; the final sum uses it in place of c
  bool projected = false;
  std::vector<int64_t> prow, pcol;
  std::vector<double> pval;
  std::vector<mb::Side> sides;
  // complex outputs per lane of the main request, and before side request i
  int64_t main_outputs() const;
  int64_t side_offset(size_t i) const;
  bool counts_only = false;
  // device image
  void *dev = nullptr;
  size_t dev_bytes = 0;
  std::vector<size_t> off_qsplit;  // per stage (s >= 1)
  std::vector<size_t> off_masks;   // per stage (s >= 1): (u mask, d mask) of every quark part
  std::vector<size_t> off_items;   // per stage (s >= 1): two-phase items q * nsingle + j, ordered by
                                   // the single-flavour set of the previous-stage part they read
  size_t off_first = 0, off_crow = 0, off_ccol = 0, off_cval = 0;
  size_t image_bytes() const;
};

namespace mb {
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int binom(int n, int k);
int factorial(int n);
// rank of a k-subset (mask over positions 0..m-1) among the k-subsets of
// 0..m-1 ordered by mask value
int subset_rank(uint32_t posmask, int m);
// the positions of the bits of `sub` within base set `base`, as a mask
uint32_t to_positions(uint32_t sub, uint32_t base);
uint32_t from_positions(uint32_t pos, uint32_t base);
// Blocks (capi.cpp): the launches of mb_make_blocks with the site-chunk
// partial sums in ws, and the size of that workspace.
int check_blocks_problem(const mb_term_list *tl, const mb_problem *p);
size_t blocks_workspace_bytes(const mb_term_list *tl, const mb_problem *p);
int make_blocks_with(const mb_term_list *tl, const mb_problem *p, void *blocks, size_t blocks_bytes, void *ws,
                     size_t ws_bytes, void *stream);
}  // namespace mb
