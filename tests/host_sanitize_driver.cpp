// Host-only exercise of the term-list C ABI, built with AddressSanitizer and
// UBSan by tests/test_host_sanitizers.py: builds term lists (nucleons, three
// sources, a Lambda, spin states, projections, side nuclei, explicit and
// searched orders), reads their counts and every export of every stage,
// saves and loads them, and feeds invalid input.  Argument: a scratch
// directory.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include "mbcontract.h"

static void exercise(const mb_term_list *tl, const char *name) {
  mb_counts c;
  if (mb_term_list_counts(tl, &c) != MB_OK) { printf("%s: counts failed: %s\n", name, mb_last_error()); return; }
  size_t total = 0;
  for (int what = 1; what <= 13; what++)
    for (int st = 0; st < c.n_stages; st++) {
      size_t bytes = 0;
      if (mb_term_list_export(tl, what, st, nullptr, &bytes) != MB_OK) continue;
      std::vector<char> buf(bytes + 1);
      size_t b2 = bytes;
      if (mb_term_list_export(tl, what, st, buf.data(), &b2) == MB_OK) total += b2;
    }
  printf("%-40s stages %d ops %lld exported %zu bytes\n", name, c.n_stages, (long long)c.n_lambda, total);
}

static mb_term_list *build(int nP, int nN, int rel, int nsrc, int nL, int path, unsigned order, bool all,
                           unsigned sP, unsigned sN, std::vector<unsigned> alphas, unsigned sL = 0,
                           std::vector<unsigned> alphaL = {}, const double *proj = nullptr) {
  mb_nucleus nuc{nP, nN, rel, nsrc, path, order, nL};
  mb_spin_request r{};
  r.all_components = all;
  r.sink_P = sP; r.sink_N = sN;
  r.n_alpha = int(alphas.size() / 2);
  r.alpha = alphas.empty() ? nullptr : alphas.data();
  r.proj = proj;
  r.sink_L = sL;
  r.alpha_L = alphaL.empty() ? nullptr : alphaL.data();
  mb_term_list *tl = nullptr;
  int rc = mb_build_term_list(&nuc, &r, &tl);
  if (rc != MB_OK) { printf("build (%d,%d,rel %d,src %d,L %d) rc %d: %s\n", nP, nN, rel, nsrc, nL, rc, mb_last_error()); return nullptr; }
  return tl;
}

int main(int argc, char **argv) {
  const std::string dir = argc > 1 ? argv[1] : "/tmp";
  const std::string saved = dir + "/tl.bin", junk = dir + "/junk.bin", missing = dir + "/missing.bin";
  struct Case { const char *name; int nP, nN, rel, nsrc, nL, path; unsigned order; };
  const Case all[] = {
    {"p+n NR", 1, 1, 0, 1, 0, MB_PATH_AUTO, 0}, {"3He NR", 2, 1, 0, 1, 0, MB_PATH_AUTO, 0},
    {"4He NR 2src", 2, 2, 0, 2, 0, MB_PATH_AUTO, 0}, {"3n NR 3src", 0, 3, 0, 3, 0, MB_PATH_AUTO, 0},
    {"Lambda + n", 0, 1, 0, 1, 1, MB_PATH_AUTO, 0}, {"Lambda + p + n NR", 1, 1, 0, 1, 1, MB_PATH_AUTO, 0},
    {"Lambda + n 2src", 0, 1, 0, 2, 1, MB_PATH_AUTO, 0}, {"pnpn explicit", 2, 2, 0, 1, 0, MB_PATH_EXPLICIT, 0x5},
    {"3H best", 1, 2, 0, 1, 0, MB_PATH_BEST, 0}, {"Lambda alone", 0, 0, 0, 1, 1, MB_PATH_AUTO, 0},
  };
  for (const Case &k : all) {
    mb_term_list *tl = build(k.nP, k.nN, k.rel, k.nsrc, k.nL, k.path, k.order, true, 0, 0, {});
    if (!tl) continue;
    exercise(tl, k.name);
    if (!k.nL && mb_term_list_save(tl, saved.c_str()) == MB_OK) {
      mb_term_list *t2 = nullptr;
      if (mb_term_list_load(saved.c_str(), &t2) == MB_OK) { exercise(t2, "  (loaded)"); mb_term_list_free(t2); }
    }
    mb_term_list_free(tl);
  }
  // spin states, with a Lambda, three sources, five neutrons
  if (mb_term_list *tl = build(1, 1, 0, 1, 1, MB_PATH_AUTO, 0, false, 0x1, 0x2, {0x1, 0x2}, 0x1, {0x1})) {
    exercise(tl, "Lambda + p + n spin state"); mb_term_list_free(tl); }
  if (mb_term_list *tl = build(0, 3, 0, 3, 0, MB_PATH_AUTO, 0, false, 0, 0x7, {0, 0x7})) {
    exercise(tl, "3n NR 3src spin state"); mb_term_list_free(tl); }
  // projection weights on p+n (all sink sets x all source sets of the full request)
  {
    mb_term_list *full = build(1, 1, 0, 1, 0, MB_PATH_AUTO, 0, true, 0, 0, {});
    mb_counts c; mb_term_list_counts(full, &c);
    std::vector<double> w(size_t(c.n_delta) * c.n_alpha, 0.0);
    for (size_t i = 0; i < w.size(); i += 3) w[i] = 1.0 + double(i % 7);
    mb_term_list_free(full);
    mb_nucleus nuc{1, 1, 0, 1, MB_PATH_AUTO, 0, 0};
    mb_spin_request r{}; r.all_components = 1; r.proj = w.data();
    mb_term_list *tl = nullptr;
    if (mb_build_term_list(&nuc, &r, &tl) == MB_OK) { exercise(tl, "p+n projected"); mb_term_list_free(tl); }
    else printf("projected: %s\n", mb_last_error());
  }
  // side nuclei on the path
  {
    mb_nucleus nuc{2, 2, 0, 1, MB_PATH_AUTO, 0, 0};
    mb_spin_request r{}; r.all_components = 1;
    mb_side_request sides[2] = {{0, 1, 0, nullptr}, {1, 1, 0, nullptr}};
    mb_term_list *tl = nullptr;
    if (mb_build_term_list_path(&nuc, &r, 2, sides, &tl) == MB_OK) { exercise(tl, "4He NR with sides"); mb_term_list_free(tl); }
    else printf("sides: %s\n", mb_last_error());
  }
  // invalid inputs must fail cleanly
  build(-1, 1, 0, 1, 0, MB_PATH_AUTO, 0, true, 0, 0, {});
  build(1, 1, 0, 4, 0, MB_PATH_AUTO, 0, true, 0, 0, {});
  build(1, 1, 1, 3, 0, MB_PATH_AUTO, 0, true, 0, 0, {});
  build(1, 1, 0, 1, 2, MB_PATH_AUTO, 0, true, 0, 0, {});
  build(5, 5, 0, 1, 0, MB_PATH_AUTO, 0, true, 0, 0, {});
  build(1, 1, 0, 1, 0, MB_PATH_EXPLICIT, 0x3, true, 0, 0, {});
  mb_term_list *bad = nullptr;
  printf("load missing: %d\n", mb_term_list_load(missing.c_str(), &bad));
  FILE *f = fopen(junk.c_str(), "wb"); fputs("junk junk junk", f); fclose(f);
  printf("load junk: %d\n", mb_term_list_load(junk.c_str(), &bad));
  printf("done\n");
  return 0;
}
