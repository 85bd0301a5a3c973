// C ABI of libmbcontract: device image of the term list, workspace sizes and
// the two device calls (blocks, contraction).  Arguments are validated on the
// host before anything is launched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"
#include "kernels.h"

using namespace mb;

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

#define HIP_CHECK(expr)                                                          \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) return fail(MB_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

int64_t lanes_padded(int64_t B) { return (B + 63) / 64 * 64; }


int nchunks_for(int64_t B, int64_t V) {
  int64_t want = std::max<int64_t>(1, (4096 + B - 1) / B);
  int64_t maxc = std::max<int64_t>(1, (V + 63) / 64);
  return int(std::min(want, maxc));
}

int check_problem(const mb_term_list *tl, const mb_problem *p) {
  if (!tl || !p) return fail(MB_EINVAL, "null argument");
  if (p->batch < 1 || p->V < 1) return fail(MB_EINVAL, "batch and V must be positive");
  if (p->batch > MB_MAX_BATCH) return fail(MB_EUNSUPPORTED, "batch above MB_MAX_BATCH lanes");
  if (p->in_dtype != MB_C64 && p->in_dtype != MB_C128) return fail(MB_EINVAL, "bad in_dtype");
  if (p->precision != MB_FP64 && p->precision != MB_MIXED && p->precision != MB_MIXED_F32B)
    return fail(MB_EINVAL, "bad precision");
  if (tl->counts_only) return fail(MB_EINVAL, "counts-only term list");
  if (tl->nxi > 18) return fail(MB_EUNSUPPORTED, "blocks support at most 18 quark indices");
  return MB_OK;
}

size_t elem_bytes(const mb_problem *p) { return p->precision == MB_FP64 ? 16 : 8; }

// Blocks are stored in double in every precision mode (they are small and
// every block entry enters every component), followed by the per-lane block
// exponents (int32, padded lanes) and, with MB_MIXED_F32B, float copies of
// the entries for the recursion steps.
// Block quark indices of both nucleon blocks, then of the Lambda's (n_xi^3).
int64_t block_rows(const mb_term_list *tl) {
  const int64_t nyq = int64_t(tl->nxi) * (tl->nxi - 1) / 2 * tl->nxi;
  return 2 * nyq + (tl->nLam ? int64_t(tl->nxi) * tl->nxi * tl->nxi : 0);
}
size_t blocks_entry_bytes(const mb_term_list *tl, const mb_problem *p) {
  return size_t(tl->npsi * block_rows(tl)) * size_t(lanes_padded(p->batch)) * 16;
}

// The sink base set of a species.
uint32_t base_of(const mb_term_list *tl, int type) {
  return type == PROTON ? tl->SP : type == NEUTRON ? tl->SN : tl->SL;
}
// Float block copies of MB_MIXED_F32B after the exponents: per species
// (proton, neutron, Lambda) the positions of its sink base set, two per
// lane side by side (16 bytes per lane and position pair).
size_t blocks_f32_offset(const mb_term_list *tl, const mb_problem *p) {
  return blocks_entry_bytes(tl, p) + al256(size_t(lanes_padded(p->batch)) * 4);
}
int64_t species_rows(const mb_term_list *tl, int type) {
  const int64_t nyq = int64_t(tl->nxi) * (tl->nxi - 1) / 2 * tl->nxi;
  return type == LAMBDA ? (tl->nLam ? int64_t(tl->nxi) * tl->nxi * tl->nxi : 0) : nyq;
}
size_t f32_species_bytes(const mb_term_list *tl, const mb_problem *p, int type) {
  const int npair = (__builtin_popcount(base_of(tl, type)) + 1) / 2;
  return al256(size_t(species_rows(tl, type)) * size_t(lanes_padded(p->batch)) * size_t(npair) * 16);
}
size_t blocks_bytes_of(const mb_term_list *tl, const mb_problem *p) {
  size_t f32 = 0;
  if (p->precision == MB_MIXED_F32B)
    for (int type = PROTON; type <= LAMBDA; type++) f32 += f32_species_bytes(tl, p, type);
  return blocks_f32_offset(tl, p) + f32;
}

// Site-chunk partial sums: one set per nucleon block (one with u = d), then
// the Lambda's (all ordered (u, d) pairs) in the same space after the
// nucleon blocks are finished.
size_t blocks_ws_of(const mb_term_list *tl, const mb_problem *p) {
  const bool sym = p->prop_u == p->prop_d;
  auto part = [&](int npair) {
    return al256(size_t(nchunks_for(p->batch, p->V)) * tl->npsi * tl->nxi * npair * 16 * size_t(p->batch));
  };
  const size_t nuc = part(sym ? tl->nxi * (tl->nxi + 1) / 2 : tl->nxi * tl->nxi) * (sym ? 1 : 2);
  return tl->nLam ? std::max(nuc, part(tl->nxi * tl->nxi)) : nuc;
}

// Per-sink-set sums of a projected final sum: complex double [Bp][n_delta].
size_t proj_bytes_of(const mb_term_list *tl, const mb_problem *p) {
  return tl->projected ? al256(size_t(lanes_padded(p->batch)) * size_t(tl->st.back().nspin()) * 16) : 0;
}

void stage_buffer_sizes(const mb_term_list *tl, const mb_problem *p, size_t *even, size_t *odd) {
  size_t e = 0, o = 0;
  for (int s = 0; s < tl->nstages; s++) {
    size_t n = size_t(tl->st[s].nreq()) * size_t(lanes_padded(p->batch)) * elem_bytes(p);
    if (s % 2 == 0) e = std::max(e, n);
    else o = std::max(o, n);
  }
  *even = al256(e);
  *odd = al256(o);
}

// Partials of the two-phase steps (one set at a time): nsingle partial
// stages of the step's output, in the stage type.
size_t h_bytes_of(const mb_term_list *tl, const mb_problem *p) {
  size_t h = 0;
  for (int s = 1; s < tl->nstages; s++) {
    const Stage &S = tl->st[s];
    if (!S.tune_two_phase || S.tune_kernel != 0) continue;
    h = std::max(h, size_t(S.nsingle()) * size_t(S.nreq()) * size_t(lanes_padded(p->batch)) * elem_bytes(p));
  }
  return al256(h);
}

// The error-estimate area of a mixed contraction: two error stages (float2
// (E, S) per component, plain layout) and, for a projected list, the
// per-sink-set estimates.
void err_stage_sizes(const mb_term_list *tl, const mb_problem *p, size_t *even, size_t *odd) {
  size_t e = 0, o = 0;
  for (int s = 0; s < tl->nstages; s++) {
    size_t n = size_t(tl->st[s].nreq()) * size_t(lanes_padded(p->batch)) * 8;
    if (s % 2 == 0) e = std::max(e, n);
    else o = std::max(o, n);
  }
  *even = al256(e);
  *odd = al256(o);
}
size_t err_bytes_of(const mb_term_list *tl, const mb_problem *p) {
  size_t e, o;
  err_stage_sizes(tl, p, &e, &o);
  return e + o + proj_bytes_of(tl, p);
}

void psi_positions(uint32_t base, int *out) {
  int k = 0;
  for (int i = 0; i < 32 && k < 8; i++)
    if (base >> i & 1) out[k++] = i;
  for (; k < 8; k++) out[k] = 0;
}

}  // namespace

namespace mb {

size_t blocks_workspace_bytes(const mb_term_list *tl, const mb_problem *p) { return blocks_ws_of(tl, p); }
int check_blocks_problem(const mb_term_list *tl, const mb_problem *p) { return check_problem(tl, p); }

// The launches of mb_make_blocks with the site-chunk partial sums in `ws`
// (the caller's workspace, or the no-allocation entry point's scratch).
int make_blocks_with(const mb_term_list *tl, const mb_problem *p, void *blocks, size_t blocks_bytes, void *ws,
                     size_t ws_bytes, void *stream) {
  int rc = check_problem(tl, p);
  if (rc) return rc;
  if (!p->prop_u || !p->prop_d || !blocks || !ws) return fail(MB_EINVAL, "null device buffer");
  if (tl->nLam && !p->prop_s) return fail(MB_EINVAL, "null strange propagator for a term list with a Lambda");
  if (blocks_bytes < blocks_bytes_of(tl, p)) return fail(MB_ENOWORKSPACE, "blocks buffer too small");
  if (ws_bytes < blocks_ws_of(tl, p)) return fail(MB_ENOWORKSPACE, "blocks workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool sym = p->prop_u == p->prop_d;
  const bool mixed = p->precision != MB_FP64;
  BlocksArgs a{};
  a.prop_u = p->prop_u;
  a.prop_d = p->prop_d;
  a.sink_w = p->sink_w;
  a.scale_exp = p->scale_exp;
  a.B = p->batch;
  a.V = p->V;
  a.nsrc = tl->nsrc;
  a.D = tl->D;
  a.nchunk = nchunks_for(p->batch, p->V);
  a.sites_per_chunk = (p->V + a.nchunk - 1) / a.nchunk;
  a.in_c128 = p->in_dtype == MB_C128;
  a.kernel = tl->blocks_kernel == 2 ? 2 : 0;
  const int npair_n = sym ? tl->nxi * (tl->nxi + 1) / 2 : tl->nxi * tl->nxi;
  const size_t half =
      al256(size_t(a.nchunk) * tl->npsi * tl->nxi * npair_n * 16 * size_t(p->batch));
  double *partP = static_cast<double *>(ws);
  double *partN = sym ? partP : reinterpret_cast<double *>(static_cast<char *>(ws) + half);
  a.prop_q1 = p->prop_u;
  a.partial = partP;
  HIP_CHECK(launch_blocks_partial(a, mixed, sym, s));
  if (!sym) {
    a.prop_q1 = p->prop_d;
    a.partial = partN;
    HIP_CHECK(launch_blocks_partial(a, mixed, sym, s));
  }
  FinishArgs f{};
  f.partP = partP;
  f.partN = partN;
  f.blocks = blocks;
  f.B = p->batch;
  f.Bp = lanes_padded(p->batch);
  f.nsrc = tl->nsrc;
  f.D = tl->D;
  f.nchunk = a.nchunk;
  f.sym = sym;
  HIP_CHECK(launch_blocks_finish(f, mixed, s));
  const int nyq = tl->nxi * (tl->nxi - 1) / 2 * tl->nxi;
  if (tl->nLam) {
    // the Lambda (s, u, d): every ordered (u, d) pair, no antisymmetrisation;
    // with S_u = S_d on the matrix cores only the pairs u <= d (the diquark
    // is symmetric; the vector-unit kernel's symmetric form takes slot 1 to
    // be u, so it forms every pair).  Its partials reuse the workspace (the
    // finish above has read it).
    const bool lsym = sym && a.kernel != 2;
    a.prop_q1 = p->prop_s;
    a.partial = partP;
    HIP_CHECK(launch_blocks_partial(a, mixed, lsym, s));
    f.partP = partP;
    f.sym = lsym;
    HIP_CHECK(launch_blocks_finish_lambda(f, tl->nxi, tl->npsi, int64_t(2) * nyq, s));
  }
  // the per-chunk exponents go to the workspace (the finish kernels have read
  // the partial sums)
  HIP_CHECK(launch_blocks_scale(blocks, reinterpret_cast<int32_t *>(static_cast<char *>(blocks) +
                                                                     blocks_entry_bytes(tl, p)),
                                f.Bp, tl->npsi, int(block_rows(tl)), ws, ws_bytes, s));
  if (p->precision == MB_MIXED_F32B) {
    // float copies of the base-set positions of every species, for the steps
    const char *src = static_cast<const char *>(blocks);
    char *dst = static_cast<char *>(blocks) + blocks_f32_offset(tl, p);
    for (int type = PROTON; type <= LAMBDA; type++) {
      int pos[8];
      psi_positions(base_of(tl, type), pos);
      HIP_CHECK(launch_blocks_to_f32(src, dst, species_rows(tl, type), f.Bp, tl->npsi,
                                     __builtin_popcount(base_of(tl, type)), pos, s));
      src += size_t(species_rows(tl, type)) * tl->npsi * f.Bp * 16;
      dst += f32_species_bytes(tl, p, type);
    }
  }
  return MB_OK;
}

}  // namespace mb

extern "C" {

int mb_term_list_upload(mb_term_list *tl, void *dev, size_t bytes, void *stream) {
  if (!tl || !dev) return fail(MB_EINVAL, "null argument");
  if (tl->counts_only) return fail(MB_EINVAL, "counts-only term list has no device image");
  const size_t need = tl->image_bytes();
  if (bytes < need) return fail(MB_ENOWORKSPACE, "device buffer smaller than device_bytes");
  if (reinterpret_cast<uintptr_t>(dev) % 256) return fail(MB_EINVAL, "device buffer not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // a failed copy still waits for the copies already queued: their host
  // sources are locals of this function
#define UPLOAD_CHECK(expr)                                                        \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      (void)hipStreamSynchronize(s);                                              \
      return fail(MB_EHIP, std::string(#expr ": ") + hipGetErrorString(e_));      \
    }                                                                             \
  } while (0)
  char *base = static_cast<char *>(dev);
  size_t o = 0;
  tl->off_qsplit.assign(tl->nstages, 0);
  tl->off_masks.assign(tl->nstages, 0);
  tl->off_items.assign(tl->nstages, 0);
  std::vector<std::vector<uint32_t>> masks(tl->nstages);   // kept alive until the copies finish
  std::vector<std::vector<uint32_t>> items(tl->nstages);
  for (int st = 1; st < tl->nstages; st++) {
    tl->off_qsplit[st] = o;
    const auto &v = tl->st[st].qsplit;
    if (!v.empty()) UPLOAD_CHECK(hipMemcpyAsync(base + o, v.data(), v.size() * 4, hipMemcpyHostToDevice, s));
    o += al256(v.size() * 4);
    tl->off_masks[st] = o;
    auto &m = masks[st];
    m.resize(tl->st[st].quark.size() * 2);
    for (size_t i = 0; i < tl->st[st].quark.size(); i++) {
      m[2 * i] = qkey_u(tl->st[st].quark[i]);
      m[2 * i + 1] = qkey_d(tl->st[st].quark[i]);
    }
    if (!m.empty()) UPLOAD_CHECK(hipMemcpyAsync(base + o, m.data(), m.size() * 4, hipMemcpyHostToDevice, s));
    o += al256(m.size() * 4);
    // two-phase items (q, j): the j-th group of pair splits of output q reads
    // previous-stage parts whose single-flavour set is the output's minus its
    // j-th single index.  Ordered by that set, so that the items reading one
    // group of previous-stage parts run together; then by the output's
    // pair-flavour set, so that neighbouring items read the same rows at
    // every split position; then by the single index.
    tl->off_items[st] = o;
    const Stage &S = tl->st[st];
    const int ns1 = S.nsingle();
    std::vector<std::array<uint32_t, 4>> keyed;
    keyed.reserve(S.quark.size() * ns1);
    for (size_t q = 0; q < S.quark.size(); q++) {
      const uint32_t single = S.type == PROTON ? qkey_d(S.quark[q]) : qkey_u(S.quark[q]);
      const uint32_t pairset = S.type == PROTON ? qkey_u(S.quark[q]) : qkey_d(S.quark[q]);
      uint32_t rest = single;
      for (int j = 0; j < ns1; j++) {
        const uint32_t c = rest & (~rest + 1u);   // j-th smallest single index
        rest &= rest - 1u;
        keyed.push_back({single & ~c, pairset, c, uint32_t(q * ns1 + j)});
      }
    }
    std::sort(keyed.begin(), keyed.end());
    auto &it = items[st];
    it.resize(keyed.size());
    for (size_t i = 0; i < keyed.size(); i++) it[i] = keyed[i][3];
    if (!it.empty()) UPLOAD_CHECK(hipMemcpyAsync(base + o, it.data(), it.size() * 4, hipMemcpyHostToDevice, s));
    o += al256(it.size() * 4);
  }
  tl->off_first = o;
  {
    const auto &v = tl->st[0].first;
    if (!v.empty()) UPLOAD_CHECK(hipMemcpyAsync(base + o, v.data(), v.size() * 4, hipMemcpyHostToDevice, s));
    o += al256(v.size() * 4);
  }
  // the coefficients of the final sum: c over the source sets, or the
  // projected list L_M over the sink sets
  const std::vector<int64_t> &row = tl->projected ? tl->prow : tl->crow;
  tl->off_crow = o;
  UPLOAD_CHECK(hipMemcpyAsync(base + o, row.data(), row.size() * 8, hipMemcpyHostToDevice, s));
  o += al256(row.size() * 8);
  tl->off_ccol = o;
  std::vector<int32_t> col;
  std::vector<double> val;
  if (tl->projected) {
    col.assign(tl->pcol.begin(), tl->pcol.end());
    val = tl->pval;
  } else {
    col.assign(tl->ccol.begin(), tl->ccol.end());
    val.assign(tl->cval.begin(), tl->cval.end());
  }
  if (!col.empty()) UPLOAD_CHECK(hipMemcpyAsync(base + o, col.data(), col.size() * 4, hipMemcpyHostToDevice, s));
  o += al256(col.size() * 4);
  tl->off_cval = o;
  if (!val.empty()) UPLOAD_CHECK(hipMemcpyAsync(base + o, val.data(), val.size() * 8, hipMemcpyHostToDevice, s));
  o += al256(val.size() * 8);
  // the coefficients of every side nucleus, laid out the same way
  std::vector<std::vector<int32_t>> side_col(tl->sides.size());
  std::vector<std::vector<double>> side_val(tl->sides.size());
  for (size_t i = 0; i < tl->sides.size(); i++) {
    mb::Side &sd = tl->sides[i];
    sd.off_crow = o;
    UPLOAD_CHECK(hipMemcpyAsync(base + o, sd.crow.data(), sd.crow.size() * 8, hipMemcpyHostToDevice, s));
    o += al256(sd.crow.size() * 8);
    sd.off_ccol = o;
    side_col[i].assign(sd.ccol.begin(), sd.ccol.end());
    if (!side_col[i].empty())
      UPLOAD_CHECK(hipMemcpyAsync(base + o, side_col[i].data(), side_col[i].size() * 4, hipMemcpyHostToDevice, s));
    o += al256(sd.ccol.size() * 4);
    sd.off_cval = o;
    side_val[i].assign(sd.cval.begin(), sd.cval.end());
    if (!side_val[i].empty())
      UPLOAD_CHECK(hipMemcpyAsync(base + o, side_val[i].data(), side_val[i].size() * 8, hipMemcpyHostToDevice, s));
    o += al256(sd.cval.size() * 8);
  }
#undef UPLOAD_CHECK
  HIP_CHECK(hipStreamSynchronize(s));
  tl->dev = dev;
  tl->dev_bytes = bytes;
  return MB_OK;
}

int mb_term_list_tune(mb_term_list *tl, int step, int what, int value) {
  if (!tl) return fail(MB_EINVAL, "null argument");
  if (what == MB_TUNE_BLOCKS) {
    if (step != 0 && step != -1) return fail(MB_EINVAL, "the blocks kernel is set with step 0");
    if (value < 0 || value > 2) return fail(MB_EINVAL, "blocks kernel must be 0, 1 or 2");
    if (value == 1 && tl->nxi > 12) return fail(MB_EUNSUPPORTED, "no matrix-core blocks for 18 quark indices");
    tl->blocks_kernel = value;
    return MB_OK;
  }
  if (step != -1 && (step < 1 || step >= tl->nstages)) return fail(MB_EINVAL, "step out of range");
  for (int s = 1; s < tl->nstages; s++) {
    if (step != -1 && s != step) continue;
    Stage &S = tl->st[s];
    const int npass = S.npass();
    if (what == MB_TUNE_PASS_GROUP) {
      if (value < 0 || value > 6 || value == 4 || value == 5 || (value > 0 && npass % value != 0)) {
        if (step != -1) return fail(MB_EINVAL, "passthrough group must divide the passthrough count");
        continue;
      }
      S.tune_pg = value;
    } else if (what == MB_TUNE_LANE_TILE) {
      if (value != 16 && value != 64) return fail(MB_EINVAL, "lane tile must be 16 or 64");
      S.tune_tile = value;
    } else if (what == MB_TUNE_GROUP) {
      if (value != 1 && value != 2 && value != 4) return fail(MB_EINVAL, "group must be 1, 2 or 4");
      S.tune_group = value;
    } else if (what == MB_TUNE_UNROLL) {
      if (value < 0 || value > 2) return fail(MB_EINVAL, "unroll must be 0, 1 or 2");
      S.tune_unroll = value;
    } else if (what == MB_TUNE_TWO_PHASE) {
      if (value != 0 && value != 1) return fail(MB_EINVAL, "two-phase must be 0 or 1");
      S.tune_two_phase = value;
    } else if (what == MB_TUNE_PAIRED) {
      if (value != 0 && value != 1) return fail(MB_EINVAL, "paired must be 0 or 1");
      S.tune_paired = value;
    } else if (what == MB_TUNE_KERNEL) {
      if (value != 0 && value != 1) return fail(MB_EINVAL, "kernel must be 0 or 1");
      S.tune_kernel = value;
    } else if (what == MB_TUNE_LDS_BYTES) {
      if (value < 0 || value > 65536) return fail(MB_EINVAL, "LDS bytes out of range");
      S.tune_lds = value;
    } else {
      return fail(MB_EINVAL, "unknown tuning item");
    }
  }
  return MB_OK;
}

int mb_workspace_query(const mb_term_list *tl, const mb_problem *p, size_t *blocks_bytes,
                       size_t *blocks_ws_bytes, size_t *contract_ws_bytes) {
  int rc = check_problem(tl, p);
  if (rc) return rc;
  if (blocks_bytes) *blocks_bytes = blocks_bytes_of(tl, p);
  if (blocks_ws_bytes) *blocks_ws_bytes = blocks_ws_of(tl, p);
  if (contract_ws_bytes) {
    size_t e, o;
    stage_buffer_sizes(tl, p, &e, &o);
    *contract_ws_bytes = e + o + proj_bytes_of(tl, p) + h_bytes_of(tl, p);
  }
  return MB_OK;
}

int mb_make_blocks(const mb_term_list *tl, const mb_problem *p, void *blocks, size_t blocks_bytes,
                   void *ws, size_t ws_bytes, void *stream) {
  return mb::make_blocks_with(tl, p, blocks, blocks_bytes, ws, ws_bytes, stream);
}

static int contract_steps(const mb_term_list *tl, const mb_problem *p, const void *blocks,
                          size_t blocks_bytes, double *corr_out, int32_t *exp_out, double *err_out, void *ws,
                          size_t ws_bytes, void *stream, int first_step, int last_step) {
  int rc = check_problem(tl, p);
  if (rc) return rc;
  if (!tl->dev) return fail(MB_EINVAL, "term list not uploaded");
  if (!blocks || !ws) return fail(MB_EINVAL, "null device buffer");
  if (last_step == tl->nstages && !corr_out) return fail(MB_EINVAL, "null correlator buffer");
  for (const mb::Side &sd : tl->sides)
    if (sd.stage >= first_step && sd.stage <= last_step && !corr_out)
      return fail(MB_EINVAL, "null correlator buffer (side nucleus output)");
  if (blocks_bytes < blocks_bytes_of(tl, p)) return fail(MB_ENOWORKSPACE, "blocks buffer too small");
  size_t ev, od;
  stage_buffer_sizes(tl, p, &ev, &od);
  const size_t main_ws = ev + od + proj_bytes_of(tl, p) + h_bytes_of(tl, p);
  if (ws_bytes < main_ws) return fail(MB_ENOWORKSPACE, "contraction workspace too small");
  const bool mixed = p->precision != MB_FP64;
  // steps read float copies of the blocks (stage 0 and the error estimate
  // read the double entries)
  const bool fb32 = p->precision == MB_MIXED_F32B;
  // error estimates of the float stages (mixed path only; the FP64 path
  // reports 0): two error stages and the projected partials after the stages
  const bool err_stages = err_out && mixed;
  if (err_out && (first_step != 0 || last_step != tl->nstages))
    return fail(MB_EINVAL, "error estimates need the whole contraction");
  if (err_stages && ws_bytes < main_ws + err_bytes_of(tl, p))
    return fail(MB_ENOWORKSPACE, "contraction workspace too small for the error estimates");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t Bp = lanes_padded(p->batch);
  const int nxi = tl->nxi;
  const int nyq = nxi * (nxi - 1) / 2 * nxi;
  const char *blk = static_cast<const char *>(blocks);
  // proton, neutron, Lambda
  const void *fblk[3] = {blk, blk + size_t(tl->npsi) * nyq * Bp * 16, blk + size_t(tl->npsi) * 2 * nyq * Bp * 16};
  const char *blk32 = blk + blocks_f32_offset(tl, p);
  const void *fblk32[3] = {blk32, blk32 + f32_species_bytes(tl, p, PROTON),
                           blk32 + f32_species_bytes(tl, p, PROTON) + f32_species_bytes(tl, p, NEUTRON)};
  char *buf[2] = {static_cast<char *>(ws), static_cast<char *>(ws) + ev};
  char *hbuf = static_cast<char *>(ws) + ev + od + proj_bytes_of(tl, p);   // two-phase partials
  size_t eev = 0, eod = 0;
  err_stage_sizes(tl, p, &eev, &eod);
  char *ebuf[2] = {static_cast<char *>(ws) + main_ws, static_cast<char *>(ws) + main_ws + eev};
  double *eproj = reinterpret_cast<double *>(static_cast<char *>(ws) + main_ws + eev + eod);
  const char *img = static_cast<const char *>(tl->dev);
  const int32_t *lane_exp = reinterpret_cast<const int32_t *>(blk + blocks_entry_bytes(tl, p));

  // Float stage j is stored in the paired layout (neighbouring spin parts of
  // a lane together, one 16-byte load) when every thread of the step that
  // reads it takes both parts of each pair: 1, the direct kernel of a proton
  // step with 64-lane tiles, an even passthrough count and group (pairs of
  // passthrough parts); 2, the direct kernel with 64-lane tiles or the
  // grouped kernel, with an even number of input sets that are neighbours in
  // the stage order (a neutron step, or one passthrough part).  Stages read
  // by a side nucleus or by the final sum stay plain.  Returns the mode.
  auto paired = [&](int j) {
    if (!mixed || j + 1 >= tl->nstages) return 0;
    for (const mb::Side &sd : tl->sides)
      if (sd.stage == j) return 0;
    const Stage &C = tl->st[j + 1];
    if (C.tune_kernel != 0 || !C.tune_paired) return 0;
    const bool AP = C.type == PROTON;
    const int npass = C.npass();
    const int M = __builtin_popcount(base_of(tl, C.type));
    // steps with more than four sink indices per species run one
    // passthrough part per thread in the direct kernel
    const int pg = M > 4 ? 1 : C.tune_pg ? C.tune_pg : npass % 3 == 0 ? 3 : npass % 2 == 0 ? 2 : 1;
    const bool grouped = M <= 4 && (C.tune_group == 2 || C.tune_group == 4) && pg <= 3;
    const bool direct64 = !grouped && C.tune_tile == 64;
    const int nin = binom(M, AP ? tl->st[j].kP : C.type == NEUTRON ? tl->st[j].kN : tl->st[j].kL);
    if (direct64 && AP && npass % 2 == 0 && pg % 2 == 0) return 1;
    if ((direct64 || grouped) && nin % 2 == 0 && (!AP || npass == 1)) return 2;
    return 0;
  };
  // a launcher's refusal in the validation pass: no kernel for this shape
  auto launch_rc = [&](hipError_t e, const char *what) {
    if (e == hipSuccess) return MB_OK;
    if (e == hipErrorInvalidValue || e == hipErrorInvalidConfiguration)
      return fail(MB_EUNSUPPORTED, std::string(what) + ": no kernel for this step's shape and launch settings");
    return fail(MB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  auto final_args = [&](const void *F, size_t o_row, size_t o_col, size_t o_val, double *out, int n_delta,
                        int n_alpha, int A, double inv_fact) {
    FinalArgs a{};
    a.F = F;
    a.crow = reinterpret_cast<const int64_t *>(img + o_row);
    a.ccol = reinterpret_cast<const int32_t *>(img + o_col);
    a.cval = reinterpret_cast<const double *>(img + o_val);
    a.corr = out;
    a.scale_exp = p->scale_exp;
    a.B = p->batch;
    a.Bp = Bp;
    a.n_delta = n_delta;
    a.n_alpha = n_alpha;
    a.A = A;
    a.lane_exp = lane_exp;
    a.inv_fact = inv_fact;
    return a;
  };
  auto err_final = [&](const FinalArgs &f, const void *E, double *out, int diag) {
    ErrFinalArgs a{};
    a.E = E;
    a.crow = f.crow;
    a.ccol = f.ccol;
    a.cval = f.cval;
    a.err = out;
    a.lane_exp = lane_exp;
    a.B = f.B;
    a.Bp = Bp;
    a.n_delta = f.n_delta;
    a.n_alpha = f.n_alpha;
    a.A = f.A;
    a.inv_fact = f.inv_fact;
    a.diag = diag;
    return launch_err_final(a, s);
  };

  // Pass 0 validates every launch (nothing runs); pass 1 launches.
  for (int pass = 0; pass < 2; pass++) {
    const bool dry = pass == 0;
    for (int step = first_step; step <= last_step; step++) {
      if (step == 0) {
        // the first baryon's block restricted to the required components
        const Stage &S0 = tl->st[0];
        Stage0Args a{};
        a.fblk = fblk[S0.type];
        a.Fout = buf[0];
        a.first = reinterpret_cast<const uint32_t *>(img + tl->off_first);
        a.nq = int64_t(S0.quark.size());
        a.Bp = Bp;
        a.nyq = nyq;
        a.ns = int(S0.nspin());
        a.npsi = tl->npsi;
        psi_positions(base_of(tl, S0.type), a.psi_of_pos);
        a.paired_out = paired(0) != 0;
        if (!dry && a.nq * a.ns > 0) {
          HIP_CHECK(launch_stage0(a, mixed, s));
          if (err_stages) {
            ErrStageArgs e{};
            e.Eout = ebuf[0];
            e.F = buf[0];
            e.nq_out = a.nq;
            e.Bp = Bp;
            e.ns_out = a.ns;
            e.paired_F = a.paired_out;
            HIP_CHECK(launch_err_stage0(e, s));
          }
        }
      } else if (step < tl->nstages) {
        const Stage &S = tl->st[step], &Pv = tl->st[step - 1];
        StageArgs a{};
        a.Fin = buf[(step - 1) % 2];
        a.Fout = buf[step % 2];
        a.fblk = fb32 ? fblk32[S.type] : fblk[S.type];
        a.fb32 = fb32;
        a.qsplit = reinterpret_cast<const uint32_t *>(img + tl->off_qsplit[step]);
        a.nq_out = int64_t(S.quark.size());
        a.Bp = Bp;
        a.Sq = S.Sq;
        a.nyq = nyq;
        // the active species' spin index is the major one for a proton
        // step, the minor one for a neutron or Lambda step
        a.act_is_P = S.type == PROTON;
        a.M = __builtin_popcount(base_of(tl, S.type));
        a.K = S.type == PROTON ? Pv.kP : S.type == NEUTRON ? Pv.kN : Pv.kL;
        a.npass = S.npass();
        a.pg = S.tune_pg;
        a.lds_bytes = S.tune_lds;
        a.tile = S.tune_tile;
        a.unroll = S.tune_unroll;
        a.group = S.tune_group;
        a.paired_in = paired(step - 1);
        a.paired_out = paired(step) != 0;
        a.npsi = tl->npsi;
        a.dry = dry;
        // the LDS-staged kernel and the two-phase step follow the pair and
        // single-index structure of nucleon splits
        if (S.type == LAMBDA && (S.tune_kernel == 1 || S.tune_two_phase))
          return fail(MB_EUNSUPPORTED, "a Lambda step runs the direct or grouped kernel in one phase");
        const bool two_phase = S.tune_two_phase && S.tune_kernel == 0;
        if (two_phase) {
          a.two_phase = 1;
          a.items = reinterpret_cast<const uint32_t *>(img + tl->off_items[step]);
          a.nsingle = S.nsingle();
          a.n_items = a.nq_out * a.nsingle;
          a.pp = S.Sq / a.nsingle;
          a.H = hbuf;
          a.hstride = S.nreq() * Bp;
        }
        psi_positions(base_of(tl, S.type), a.psi_of_pos);
        if (a.M > 6) return fail(MB_EUNSUPPORTED, "more than 6 sink indices per species");
        if (a.nq_out > 0 && fb32 && S.tune_kernel == 1)
          return fail(MB_EUNSUPPORTED, "float block copies: the direct or grouped step kernel");
        if (a.nq_out > 0 && S.tune_kernel == 1) {
          // the LDS-staged kernel holds one range of at most 36 pair rows:
          // n_xi <= 12 (one source relativistic, up to two nonrelativistic)
          if (nxi > 12) return fail(MB_EUNSUPPORTED, "LDS-staged step kernel: more than 12 quark indices");
          StageLdsArgs b{};
          b.Fin = a.Fin;
          b.Fout = a.Fout;
          b.fblk = a.fblk;
          b.qsplit = a.qsplit;
          b.masks = reinterpret_cast<const uint32_t *>(img + tl->off_masks[step]);
          b.nq_out = a.nq_out;
          b.Bp = Bp;
          b.Sq = S.Sq;
          b.pp = S.Sq / (S.type == PROTON ? S.kd : S.ku);
          b.npass = a.npass;
          b.pg = (S.tune_pg >= 1 && S.tune_pg <= 3) ? S.tune_pg : (a.npass % 3 == 0 ? 3 : a.npass % 2 == 0 ? 2 : 1);
          b.npg = a.npass / b.pg;
          b.act_is_P = a.act_is_P;
          b.M = a.M;
          b.K = a.K;
          b.nxi = nxi;
          b.npair = nxi * (nxi - 1) / 2;
          b.npsi = tl->npsi;
          b.bsplit = nxi > 9 ? 9 : nxi;
          b.div_magic = uint32_t(((uint64_t(1) << 32) + uint64_t(nxi) - 1) / uint64_t(nxi));
          for (int i = 0; i < 8; i++) b.psi_of_pos[i] = a.psi_of_pos[i];
          b.paired_out = a.paired_out;
          b.dry = dry;
          if ((rc = launch_rc(launch_stage_lds(b, mixed, s), "recursion step (LDS-staged kernel)"))) return rc;
        } else if (a.nq_out > 0) {
          if ((rc = launch_rc(launch_stage(a, mixed, s), "recursion step"))) return rc;
          if (two_phase && !dry) {
            StageSumArgs b{};
            b.H = hbuf;
            b.Fout = a.Fout;
            b.nq = a.nq_out;
            b.Bp = Bp;
            b.hstride = a.hstride;
            b.ns = int(S.nspin());
            b.nsingle = a.nsingle;
            b.paired_out = a.paired_out;
            HIP_CHECK(launch_stage_sum(b, mixed, s));
          }
        }
        if (err_stages && a.nq_out > 0) {
          if (dry) {
            if (!grid_x_fits(a.nq_out * a.npass, 64))
              return fail(MB_EUNSUPPORTED, "error estimate: grid too large for this step");
          } else {
            ErrStageArgs e{};
            e.Ein = ebuf[(step - 1) % 2];
            e.Eout = ebuf[step % 2];
            e.F = a.Fout;
            e.fblk = fblk[S.type];
            if (fb32) {
              e.fb32 = 1;
              e.Fprev = a.Fin;
              e.paired_prev = a.paired_in != 0;
            }
            e.qsplit = a.qsplit;
            e.nq_out = a.nq_out;
            e.Bp = Bp;
            e.Sq = a.Sq;
            e.npass = a.npass;
            e.ns_out = int(S.nspin());
            e.act_is_P = a.act_is_P;
            e.M = a.M;
            e.K = a.K;
            e.npsi = tl->npsi;
            for (int i = 0; i < 8; i++) e.psi_of_pos[i] = a.psi_of_pos[i];
            e.paired_F = a.paired_out;
            if (two_phase) {
              e.H = hbuf;
              e.nh = a.nsingle;
              e.hstride = a.hstride;
            }
            HIP_CHECK(launch_err_stage(e, s));
          }
        }
      } else if (!dry) {
        const Stage &SN = tl->st[tl->nstages - 1];
        const int last = tl->nstages - 1;
        FinalArgs a = final_args(buf[last % 2], tl->off_crow, tl->off_ccol, tl->off_cval, corr_out,
                                 int(SN.nspin()), int(tl->alphas.size()), tl->A,
                                 1.0 / (double(factorial(tl->nuc.n_P)) * double(factorial(tl->nuc.n_N))));
        a.exp_out = exp_out;
        if (tl->projected) {
          // row delta of the list pairs with sink set delta only; the sums per
          // delta go to the workspace and are then added in delta order
          a.diag = 1;
          a.corr = reinterpret_cast<double *>(buf[1] + od);
          HIP_CHECK(launch_final(a, mixed, s));
          HIP_CHECK(launch_project(a.corr, corr_out, p->batch, a.n_delta, s));
          if (err_stages) {
            HIP_CHECK(err_final(a, ebuf[last % 2], eproj, 1));
            HIP_CHECK(launch_err_project(eproj, err_out, p->batch, a.n_delta, s));
          }
        } else {
          HIP_CHECK(launch_final(a, mixed, s));
          if (err_stages) HIP_CHECK(err_final(a, ebuf[last % 2], err_out, 0));
        }
        if (err_out && !err_stages) HIP_CHECK(launch_zero(err_out, 2 * p->batch * tl->main_outputs(), s));
      }
      // side nuclei read from the stage just formed (before a later step
      // overwrites its buffer): C_i = sum_z F(delta; z) c_i(alpha; z) / (k_P! k_N!)
      for (size_t i = 0; !dry && step < tl->nstages && i < tl->sides.size(); i++) {
        const mb::Side &sd = tl->sides[i];
        if (sd.stage != step) continue;
        const Stage &S = tl->st[step];
        FinalArgs a = final_args(buf[step % 2], sd.off_crow, sd.off_ccol, sd.off_cval,
                                 corr_out + 2 * p->batch * tl->side_offset(i), int(S.nspin()),
                                 int(sd.alphas.size()), step + 1,
                                 1.0 / (double(factorial(S.kP)) * double(factorial(S.kN))));
        HIP_CHECK(launch_final(a, mixed, s));
        if (err_out) {
          double *eo = err_out + 2 * p->batch * tl->side_offset(i);
          if (err_stages) HIP_CHECK(err_final(a, ebuf[step % 2], eo, 0));
          else HIP_CHECK(launch_zero(eo, 2 * p->batch * int64_t(S.nspin()) * int64_t(sd.alphas.size()), s));
        }
      }
    }
  }
  return MB_OK;
}

int mb_workspace_query_err(const mb_term_list *tl, const mb_problem *p, size_t *err_ws_bytes) {
  int rc = check_problem(tl, p);
  if (rc) return rc;
  if (!err_ws_bytes) return fail(MB_EINVAL, "null argument");
  *err_ws_bytes = p->precision != MB_FP64 ? err_bytes_of(tl, p) : 0;
  return MB_OK;
}

int mb_contract_correlator(const mb_term_list *tl, const mb_problem *p, const void *blocks,
                           size_t blocks_bytes, double *corr_out, int32_t *exp_out, double *err_out, void *ws,
                           size_t ws_bytes, void *stream) {
  if (!tl) return fail(MB_EINVAL, "null argument");
  return contract_steps(tl, p, blocks, blocks_bytes, corr_out, exp_out, err_out, ws, ws_bytes, stream, 0,
                        tl->nstages);
}

int mb_contract_step(const mb_term_list *tl, const mb_problem *p, const void *blocks,
                     size_t blocks_bytes, int step, double *corr_out, int32_t *exp_out, void *ws,
                     size_t ws_bytes, void *stream) {
  if (!tl) return fail(MB_EINVAL, "null argument");
  if (step < 0 || step > tl->nstages) return fail(MB_EINVAL, "step out of range");
  return contract_steps(tl, p, blocks, blocks_bytes, corr_out, exp_out, nullptr, ws, ws_bytes, stream, step,
                        step);
}

}  // extern "C"
