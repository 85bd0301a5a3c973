// Batched runs of uneven work: a list of (term list, problem) items recorded
// once into a HIP graph with several concurrent branches, then launched as a
// whole.  Each item runs exactly the launches of mb_make_blocks followed by
// mb_contract_correlator on its branch's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "internal.h"

using namespace mb;

struct mb_batch {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t kernels = 0;
};

namespace {

// Algorithmic flops of one item: the blocks as a dense contraction over
// sites (rows psi x xi1, columns the diquark index pairs, 3 colour terms per
// site; with a Lambda also its block) and 8 flops per complex multiply-add
// of the recursion.
double item_cost(const mb_term_list *tl, const mb_problem *p) {
  const double rows = double(tl->npsi) * tl->nxi;
  const bool sym = p->prop_u == p->prop_d;
  const double pairs = sym ? tl->nxi * (tl->nxi + 1) / 2.0 : double(tl->nxi) * tl->nxi;
  double blocks = 8.0 * 3.0 * rows * pairs * double(p->V) * (sym ? 1 : 2);
  // the Lambda's block runs over the same (u, d) pairs (every ordered pair
  // when u != d)
  if (tl->nLam) blocks += 8.0 * 3.0 * rows * pairs * double(p->V);
  int64_t nl = 0;
  for (const auto &s : tl->st) nl += s.n_lambda;
  return double(p->batch) * (blocks + 8.0 * double(nl));
}

struct Range {
  uintptr_t lo, hi;
  int branch;
};

struct Capture {
  hipStream_t origin = nullptr;
  std::vector<hipStream_t> br;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  ~Capture() {
    for (auto e : join)
      if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (auto s : br)
      if (s) (void)hipStreamDestroy(s);
    if (origin) (void)hipStreamDestroy(origin);
  }
};

}  // namespace

extern "C" {

int mb_batch_plan(const mb_term_list *const *tls, const mb_problem *probs, int n_items,
                  int n_branches, int *branch_out, double *cost_out) {
  if (n_items < 0 || n_branches < 1 || (n_items > 0 && (!tls || !probs || !branch_out)))
    return fail(MB_EINVAL, "bad batch plan arguments");
  std::vector<double> cost(n_items);
  for (int i = 0; i < n_items; i++) {
    if (!tls[i]) return fail(MB_EINVAL, "null term list in batch");
    if (probs[i].batch < 1 || probs[i].V < 1) return fail(MB_EINVAL, "batch and V must be positive");
    cost[i] = item_cost(tls[i], &probs[i]);
    if (cost_out) cost_out[i] = cost[i];
  }
  std::vector<int> order(n_items);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(n_branches, 0.0);
  for (int i : order) {
    const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
    branch_out[i] = k;
    load[k] += cost[i];
  }
  return MB_OK;
}

int mb_batch_create(const mb_batch_item *items, int n_items, int n_branches, mb_batch **out) {
  if (!out || n_items < 1 || !items || n_branches < 1 || n_branches > 64)
    return fail(MB_EINVAL, "bad batch arguments");
  *out = nullptr;
  // validation before anything is recorded
  std::vector<Range> ranges;
  for (int i = 0; i < n_items; i++) {
    const mb_batch_item &it = items[i];
    if (it.branch < 0 || it.branch >= n_branches) return fail(MB_EINVAL, "item branch out of range");
    if (!it.tl || !it.tl->dev) return fail(MB_EINVAL, "batch item without an uploaded term list");
    if (it.tl->projected || !it.tl->sides.empty())
      return fail(MB_EUNSUPPORTED, "projected term lists and side nuclei are not batched");
    size_t bb, bw, cw;
    int rc = mb_workspace_query(it.tl, &it.prob, &bb, &bw, &cw);
    if (rc) return rc;
    if (!it.blocks || !it.blocks_ws || !it.contract_ws || !it.corr_out)
      return fail(MB_EINVAL, "null device buffer in batch item");
    if (it.tl->nLam && !it.prob.prop_s) return fail(MB_EINVAL, "batch item with a Lambda and no strange propagator");
    if (it.blocks_bytes < bb || it.blocks_ws_bytes < bw || it.contract_ws_bytes < cw)
      return fail(MB_ENOWORKSPACE, "batch item buffer too small");
    const size_t corr_bytes = size_t(it.prob.batch) * size_t(it.tl->st.back().nspin()) *
                              it.tl->alphas.size() * 16;
    auto add = [&](const void *p, size_t n) {
      if (n) ranges.push_back({uintptr_t(p), uintptr_t(p) + n, it.branch});
    };
    add(it.blocks, bb);
    add(it.blocks_ws, bw);
    add(it.contract_ws, cw);
    add(it.corr_out, corr_bytes);
    if (it.exp_out) add(it.exp_out, size_t(it.prob.batch) * 4);
  }
  std::sort(ranges.begin(), ranges.end(), [](const Range &a, const Range &b) { return a.lo < b.lo; });
  for (size_t i = 0; i < ranges.size(); i++)
    for (size_t j = i + 1; j < ranges.size() && ranges[j].lo < ranges[i].hi; j++)
      if (ranges[j].branch != ranges[i].branch)
        return fail(MB_EINVAL, "items on different branches share a device buffer");

  Capture c;
#define CAP_CHECK(expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(MB_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)
  CAP_CHECK(hipStreamCreateWithFlags(&c.origin, hipStreamNonBlocking));
  c.br.assign(n_branches, nullptr);
  c.join.assign(n_branches, nullptr);
  for (int k = 0; k < n_branches; k++) {
    CAP_CHECK(hipStreamCreateWithFlags(&c.br[k], hipStreamNonBlocking));
    CAP_CHECK(hipEventCreateWithFlags(&c.join[k], hipEventDisableTiming));
  }
  CAP_CHECK(hipEventCreateWithFlags(&c.fork, hipEventDisableTiming));

  CAP_CHECK(hipStreamBeginCapture(c.origin, hipStreamCaptureModeThreadLocal));
  int rc = MB_OK;
  hipError_t he = hipEventRecord(c.fork, c.origin);
  for (int k = 0; k < n_branches && he == hipSuccess; k++) he = hipStreamWaitEvent(c.br[k], c.fork, 0);
  if (he != hipSuccess) rc = fail(MB_EHIP, std::string("batch fork: ") + hipGetErrorString(he));
  for (int i = 0; i < n_items && rc == MB_OK; i++) {
    const mb_batch_item &it = items[i];
    hipStream_t s = c.br[it.branch];
    rc = mb_make_blocks(it.tl, &it.prob, it.blocks, it.blocks_bytes, it.blocks_ws, it.blocks_ws_bytes, s);
    if (rc == MB_OK)
      rc = mb_contract_correlator(it.tl, &it.prob, it.blocks, it.blocks_bytes, it.corr_out, it.exp_out,
                                  nullptr, it.contract_ws, it.contract_ws_bytes, s);
  }
  for (int k = 0; k < n_branches && rc == MB_OK; k++) {
    he = hipEventRecord(c.join[k], c.br[k]);
    if (he == hipSuccess) he = hipStreamWaitEvent(c.origin, c.join[k], 0);
    if (he != hipSuccess) rc = fail(MB_EHIP, std::string("batch join: ") + hipGetErrorString(he));
  }
  hipGraph_t graph = nullptr;
  he = hipStreamEndCapture(c.origin, &graph);
  if (rc != MB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (he != hipSuccess || !graph)
    return fail(MB_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
  hipGraphExec_t exec = nullptr;
  he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (he != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(MB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
  }
  size_t nn = 0;
  int64_t nk = 0;
  if (hipGraphGetNodes(graph, nullptr, &nn) == hipSuccess && nn) {
    std::vector<hipGraphNode_t> nodes(nn);
    if (hipGraphGetNodes(graph, nodes.data(), &nn) == hipSuccess)
      for (size_t i = 0; i < nn; i++) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(nodes[i], &t) == hipSuccess && t == hipGraphNodeTypeKernel) nk++;
      }
  }
  mb_batch *b = new (std::nothrow) mb_batch;
  if (!b) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return fail(MB_ENOMEM, "out of host memory");
  }
  b->graph = graph;
  b->exec = exec;
  b->kernels = nk;
  *out = b;
  return MB_OK;
#undef CAP_CHECK
}

int mb_batch_launch(mb_batch *b, void *stream) {
  if (!b || !b->exec) return fail(MB_EINVAL, "null batch");
  const hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(MB_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return MB_OK;
}

int mb_batch_kernel_count(const mb_batch *b, int64_t *out) {
  if (!b || !out) return fail(MB_EINVAL, "null argument");
  *out = b->kernels;
  return MB_OK;
}

void mb_batch_free(mb_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
}

}  // extern "C"
