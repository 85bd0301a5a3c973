// Baryon blocks on gfx950 (Sec. 2, Sec. 6).
//
//   f_{q1}(psi; xi1, xi2, xi3) = sum_x w_{s'}(x) sum_a A_a(x)[psi][xi1] D_a(x)[xi2][xi3]
//   A_a[psi][xi1]  = S_q1[(alpha(psi), a), xi1]            (Gamma_1 = 1 on active spins)
//   D_a[xi2][xi3]  = sum_{b,c} eps_abc sum_{gamma,delta} (C g5)_{gamma delta}
//                    S_u[(gamma,b), xi2] S_d[(delta,c), xi3]   (the diquark)
// Proton: q1 = u; neutron: q1 = d (slots (d,u,d)); both share the diquark.
// With S_u = S_d the diquark is symmetric in (xi2, xi3) ((C g5)^T = -C g5 and
// eps is antisymmetric), so only xi2 <= xi3 is formed and one block serves
// both species; the Lambda (q1 = s) then also needs only xi2 <= xi3.
//
// A workgroup owns one lane and one chunk of sites and sums its sites on the
// matrix cores (below); a second kernel adds the chunk sums in double in a
// fixed order, antisymmetrises and writes the block layout, and a third
// scales every lane by its exponent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"

namespace mb {

// A propagator entry times scale (a power of two, so exact), in double.
__device__ inline double2 scaled(float2 v, double scale) { return make_double2(double(v.x) * scale, double(v.y) * scale); }
__device__ inline double2 scaled(double2 v, double scale) { return make_double2(v.x * scale, v.y * scale); }

// ---------------------------------------------------------------------------
// The site sums as one complex GEMM per lane on the matrix cores:
//   f[m = (psi, xi1)][n = pair] += sum_k A[m][k] B[k][n],  k = (site, colour a)
//   A[m][k] = w_{s'(psi)}(x) S_q1[(alpha(psi), a), xi1],  B[k][n] = D_a(x)[pair]
// with v_mfma_f64_16x16x4f64 (double products and sums).  Operand layout:
// A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k.  A complex product
// is three real MFMAs (below).
//
// The workgroup's waves take two roles.  Four builder waves stage the
// propagators of a group of sites in LDS and build the operands of that
// group there (the diquark on the vector units); NMW waves (four, or two for
// the two or three output tiles of nonrelativistic operators with one
// source) multiply the previous group on the matrix cores, each owning an
// equal share of the 16x16 output tiles.  Operands and staged propagators
// are double-buffered, so one barrier per group separates the roles, and a
// SIMD holds waves of both roles: its vector and matrix units work at the
// same time.
typedef double mb_d4 __attribute__((ext_vector_type(4)));

// NMW: multiplying waves (the builders are always four waves, 256 threads);
// fewer than four when there are fewer output tiles than four.  SYM: S_u =
// S_d (pairs xi2 <= xi3); SQ1 (with SYM): slot 1 holds a third propagator
// (the Lambda's S_s), staged beside S_u.
template <typename TIN, int NXI, int NPSI, int NROW, bool SYM, int NMW, bool SQ1 = false>
__global__ __launch_bounds__(64 * (NMW + 4)) void blocks_mfma_kernel(BlocksArgs a) {
  constexpr int NPAIR = SYM ? NXI * (NXI + 1) / 2 : NXI * NXI;
  constexpr int M = NPSI * NXI;
  constexpr int MT = (M + 15) / 16, NT = (NPAIR + 15) / 16;
  constexpr int MP = MT * 16, NP = NT * 16;
  constexpr int NS = 4;                // sites per group
  constexpr int KG = 3 * NS;           // k = 3 * site + colour, multiple of 4
  constexpr int NTILE = MT * NT;
  constexpr int TPW = (NTILE + NMW - 1) / NMW;  // tiles per multiplying wave
  constexpr int NT_ALL = 64 * (NMW + 4);        // threads of the workgroup
  constexpr int D = NROW / 3;
  constexpr int NB = SYM ? 1 : 2;      // buffers of the d slot
  constexpr bool Q1B = !SYM || SQ1;    // slot 1 has buffers of its own

  // Propagators are staged in double: the vector and matrix units share the
  // double-precision pipeline, so every entry is widened once, when it is
  // staged, rather than at each of its uses in the diquark.
  __shared__ double2 su[2][NS][NROW][NXI];
  // q1 when it differs from u: as read (complex float inputs stay float, half
  // the bytes; widened and scaled, exactly, when the A operand is built), so
  // that the Lambda's kernel with S_u = S_d fits two workgroups per CU
  using S1T = typename std::conditional<std::is_same<TIN, float2>::value, float2, double2>::type;
  __shared__ S1T s1[Q1B ? 2 : 1][Q1B ? NS : 1][Q1B ? NROW : 1][Q1B ? NXI : 1];
  __shared__ double2 sd[NB][SYM ? 1 : NS][SYM ? 1 : NROW][SYM ? 1 : NXI];
  __shared__ double2 Ac[2][KG][MP];   // (re, im) of the A operand
  __shared__ double2 Bc[2][KG][NP];   // (re, im) of the B operand
  __shared__ double2 wsh[2][NS][2];
  __shared__ unsigned char px2[NP], px3[NP];  // pair index -> (xi2, xi3)

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const bool builder = wave >= NMW;
  const int bt = (tid - 64 * NMW) & 255;   // thread index within its role (builders: 0..255)
  for (int p = tid; p < NP; p += NT_ALL) {
    int x2 = 0, x3 = 0;
    if (p < NPAIR) {
      if (SYM) {
        while ((x3 + 1) * (x3 + 2) / 2 <= p) x3++;
        x2 = p - x3 * (x3 + 1) / 2;
      } else {
        x2 = p / NXI;
        x3 = p % NXI;
      }
    }
    px2[p] = (unsigned char)x2;
    px3[p] = (unsigned char)x3;
  }
  __syncthreads();   // the pair tables are read below
  const int64_t ln = blockIdx.y;
  const int chunk = blockIdx.x;
  const int nsrc = a.nsrc;
  const int64_t x0 = int64_t(chunk) * a.sites_per_chunk;
  const int64_t x1 = min(a.V, x0 + a.sites_per_chunk);
  const int ngroups = x1 > x0 ? int((x1 - x0 + NS - 1) / NS) : 0;
  const double scale = a.scale_exp ? ldexp(1.0, a.scale_exp[ln]) : 1.0;
  const bool same1 = a.prop_q1 == a.prop_u;
  auto group_sites = [&](int g) { return int(min<int64_t>(NS, x1 - (x0 + int64_t(g) * NS))); };

  // ---- builders: operand sources, resolved once ----
  constexpr int AJ = (KG * MP + 255) / 256, BJ = (KG * NP + 255) / 256;
  int a_src[AJ], a_w[AJ], a_n[AJ];   // LDS index of S_q1 (-1: zero entry), sink weight, site
#pragma unroll
  for (int j = 0; j < AJ; j++) {
    const int i = bt + 256 * j;
    const int k = i / MP, m = i % MP, n = k / 3, ac = k % 3;
    a_src[j] = -1;
    a_w[j] = 0;
    a_n[j] = n;
    if (i < KG * MP && m < M) {
      const int psi = m / NXI, xi1 = m % NXI, alpha = psi / nsrc, sk = psi % nsrc;
      a_src[j] = (n * NROW + 3 * alpha + ac) * NXI + xi1;
      a_w[j] = n * 2 + sk;
    }
  }
  // diquark entry (site n, colour a, pair (x2, x3)): the eps terms are
  // (b, c) = (a+1, a+2) with + and (a+2, a+1) with -; a term reads rows
  // 3 g + b (at x2) and 3 (g^1) + c (at x3)
  int b_l0[BJ], b_r0[BJ], b_sw[BJ], b_n[BJ];   // b_sw: row offset from (b, c) to (c, b)
#pragma unroll
  for (int j = 0; j < BJ; j++) {
    const int i = bt + 256 * j;
    const int k = i / NP, pp = i % NP, n = k / 3, ac = k % 3;
    b_n[j] = (i < KG * NP && pp < NPAIR) ? n : NS;   // NS: zero entry
    const int x2 = pp < NPAIR ? px2[pp] : 0, x3 = pp < NPAIR ? px3[pp] : 0;
    const int bb = (ac + 1) % 3, cc = (ac + 2) % 3;
    b_l0[j] = (n * NROW + bb) * NXI + x2;
    b_r0[j] = (n * NROW + cc) * NXI + x3;
    b_sw[j] = (cc - bb) * NXI;
  }
  auto rd = [](const double2 *p, int i) { return p[i]; };

  // The propagator entries of the group after next are loaded into
  // registers while a group is built.
  constexpr int PFJ = (NS * NROW * NXI + 255) / 256;
  TIN pu[PFJ], pd[PFJ], p1[PFJ];
  double2 pw = make_double2(1.0, 0.0);
  auto fetch = [&](int g) {
    const int64_t xg = x0 + int64_t(g) * NS;
    const int ns = group_sites(g);
#pragma unroll
    for (int j = 0; j < PFJ; j++) {
      const int i = bt + 256 * j;
      if (i < ns * NROW * NXI) {
        const int n = i / (NROW * NXI), r = (i / NXI) % NROW, xi = i % NXI;
        const int s = xi % nsrc, kap = xi / nsrc;
        const int64_t off = (((ln * a.V + xg + n) * nsrc + s) * 12 + r) * 12 + kap;
        pu[j] = static_cast<const TIN *>(a.prop_u)[off];
        if constexpr (!SYM) pd[j] = static_cast<const TIN *>(a.prop_d)[off];
        if constexpr (Q1B) {
          if (!same1) p1[j] = static_cast<const TIN *>(a.prop_q1)[off];
        }
      }
    }
    if (bt < ns * nsrc && a.sink_w) {
      const int n = bt / nsrc, s = bt % nsrc;
      pw = reinterpret_cast<const double2 *>(a.sink_w)[int64_t(s) * a.V + xg + n];
    }
  };
  auto stage = [&](int g) {
    const int buf = g & 1, ns = group_sites(g);
#pragma unroll
    for (int j = 0; j < PFJ; j++) {
      const int i = bt + 256 * j;
      if (i < ns * NROW * NXI) {
        const int n = i / (NROW * NXI), r = (i / NXI) % NROW, xi = i % NXI;
        su[buf][n][r][xi] = scaled(pu[j], scale);
        if constexpr (!SYM) sd[buf][n][r][xi] = scaled(pd[j], scale);
        if constexpr (Q1B) {
          if (!same1) s1[buf][n][r][xi] = p1[j];
        }
      }
    }
    if (bt < ns * nsrc) {
      const int n = bt / nsrc, s = bt % nsrc;
      wsh[buf][n][s] = pw;
    }
  };
  auto build = [&](int g) {
    const int buf = g & 1, ns = group_sites(g);
    const double2 *su_f = &su[buf][0][0][0];
    const double2 *sd_f = SYM ? su_f : &sd[SYM ? 0 : buf][0][0][0];
    const bool q1_is_u = !Q1B || same1;
    const S1T *s1_f = &s1[Q1B ? buf : 0][0][0][0];
    // A operand: w S_q1[(alpha, a), xi1]
#pragma unroll
    for (int j = 0; j < AJ; j++) {
      const int i = bt + 256 * j;
      if (i < KG * MP) {
        double re = 0.0, im = 0.0;
        if (a_src[j] >= 0 && a_n[j] < ns) {
          const double2 w = (&wsh[buf][0][0])[a_w[j]];
          const double2 v = q1_is_u ? rd(su_f, a_src[j]) : scaled(s1_f[a_src[j]], scale);
          re = w.x * v.x - w.y * v.y;
          im = w.x * v.y + w.y * v.x;
        }
        (&Ac[buf][0][0])[i] = make_double2(re, im);
      }
    }
    // B operand: the diquark D_a[pair] = sum eps_abc (C g5)_{gd} S_u[(g,b)] S_d[(d,c)]
    // ((C g5): (0,1) -1, (1,0) +1, (2,3) -1, (3,2) +1)
#pragma unroll
    for (int j = 0; j < BJ; j++) {
      const int i = bt + 256 * j;
      if (i < KG * NP) {
        double re = 0.0, im = 0.0;
        if (b_n[j] < ns) {
#pragma unroll
          for (int gs = 0; gs < D; gs++) {
            const double sg = (gs & 1) ? 1.0 : -1.0;
            const int go = 3 * gs * NXI, gd = 3 * (gs ^ 1) * NXI;
            const double2 l0 = rd(su_f, b_l0[j] + go), r0 = rd(sd_f, b_r0[j] + gd);
            const double2 l1 = rd(su_f, b_l0[j] + b_sw[j] + go), r1 = rd(sd_f, b_r0[j] - b_sw[j] + gd);
            re += sg * ((l0.x * r0.x - l0.y * r0.y) - (l1.x * r1.x - l1.y * r1.y));
            im += sg * ((l0.x * r0.y + l0.y * r0.x) - (l1.x * r1.y + l1.y * r1.x));
          }
        }
        (&Bc[buf][0][0])[i] = make_double2(re, im);
      }
    }
  };

  // Pipeline: in round r the builders build group r (staged in round r - 1)
  // and stage group r + 1 (loaded in round r - 1), then load group r + 2;
  // the multipliers multiply group r - 1.  The two roles run separate loops
  // (the role is the same for the whole wave) with one barrier per round
  // each, so that their registers are not live at the same time.
  if (builder) {
    if (ngroups > 0) {
      fetch(0);
      stage(0);
      if (ngroups > 1) fetch(1);
    }
    __syncthreads();
    for (int r = 0; r <= ngroups; r++) {
      if (r < ngroups) {
        build(r);
        if (r + 1 < ngroups) {
          stage(r + 1);
          if (r + 2 < ngroups) fetch(r + 2);
        }
      }
      __syncthreads();
    }
    return;
  }

  // ---- multipliers: Gauss's three-product form of the complex product:
  // m1 = Ar Br, m2 = Ai Bi, m3 = (Ar + Ai)(Br + Bi); re = m1 - m2,
  // im = m3 - m1 - m2.  A wave with fewer tiles repeats its last tile into
  // an accumulator never stored.
  mb_d4 m1[TPW], m2[TPW], m3[TPW];
#pragma unroll
  for (int j = 0; j < TPW; j++) {
    m1[j] = mb_d4{0.0, 0.0, 0.0, 0.0};
    m2[j] = mb_d4{0.0, 0.0, 0.0, 0.0};
    m3[j] = mb_d4{0.0, 0.0, 0.0, 0.0};
  }
  __syncthreads();
  for (int r = 0; r <= ngroups; r++) {
    if (r >= 1) {
      const int buf = (r - 1) & 1;
#pragma unroll
      for (int ks = 0; ks < KG / 4; ks++) {
        const int k = 4 * ks + (lane >> 4);
        double oa[TPW][3], ob[TPW][3];
#pragma unroll
        for (int j = 0; j < TPW; j++) {
          const int t = min(wave + NMW * j, NTILE - 1);
          const int mt = t / NT, nt = t % NT;
          const int am = mt * 16 + (lane & 15), bn = nt * 16 + (lane & 15);
          const double2 av = Ac[buf][k][am], bv = Bc[buf][k][bn];
          oa[j][0] = av.x;
          oa[j][1] = av.y;
          oa[j][2] = av.x + av.y;
          ob[j][0] = bv.x;
          ob[j][1] = bv.y;
          ob[j][2] = bv.x + bv.y;
        }
#pragma unroll
        for (int j = 0; j < TPW; j++) {
          m1[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(oa[j][0], ob[j][0], m1[j], 0, 0, 0);
          m2[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(oa[j][1], ob[j][1], m2[j], 0, 0, 0);
          m3[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(oa[j][2], ob[j][2], m3[j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  double2 *out = reinterpret_cast<double2 *>(a.partial) + ((ln * a.nchunk + chunk) * NPSI) * int64_t(NXI) * NPAIR;
#pragma unroll
  for (int j = 0; j < TPW; j++) {
    const int t = wave + NMW * j;
    if (t < NTILE) {
      const int mt = t / NT, nt = t % NT;
      const int n = nt * 16 + (lane & 15);
#pragma unroll
      for (int rr = 0; rr < 4; rr++) {
        // v_mfma_f64_16x16x4f64 output: D[i][j] in lane j + 16 (i % 4), register i / 4
        const int m = mt * 16 + (lane >> 4) + 4 * rr;
        if (m < M && n < NPAIR)
          out[int64_t(m) * NPAIR + n] = make_double2(m1[j][rr] - m2[j][rr], m3[j][rr] - m1[j][rr] - m2[j][rr]);
      }
    }
  }
}

// Symmetric pairs with a third flavour in slot 1 (the Lambda with S_u = S_d)
// run the SQ1 variant; otherwise slot 1 is u, or (without symmetry) staged
// by the plain kernel.
template <typename TIN, int NXI, int NPSI, int NROW, bool SYM, int NMW = 4>
static hipError_t launch_bm(const BlocksArgs &a, hipStream_t s) {
  dim3 grid(a.nchunk, unsigned(a.B));
  if (SYM && a.prop_q1 != a.prop_u)
    hipLaunchKernelGGL((blocks_mfma_kernel<TIN, NXI, NPSI, NROW, SYM, NMW, true>), grid, dim3(64 * (NMW + 4)), 0, s,
                       a);
  else
    hipLaunchKernelGGL((blocks_mfma_kernel<TIN, NXI, NPSI, NROW, SYM, NMW>), grid, dim3(64 * (NMW + 4)), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The same site sums on the vector units, register-tiled.  Per lane and
// site chunk the blocks are f[r][p] += sum_{x, a} A_x[a][r] B_x[a][p] with
// r = (psi, xi1) (R rows), p the (xi2, xi3) pairs (P columns, ordered as in
// the matrix-core kernel), A_x = w S_q1 and B_x the diquark.  A thread owns
// a tile of TR rows x TP pairs in registers; when the tiles of one lane are
// fewer than the threads, G groups of threads take G different sites per
// round and their tiles are added (in group order) at the end.  Per round
// the workgroup stages the propagator rows of its sites in LDS (in double),
// forms A and B there, and every thread adds the 3 x TR x TP complex
// products of its tile: 3 (TR + TP) LDS operands for 3 TR TP fused
// products.  Shapes: any D and N_s with 3 D N_s <= 18; the matrix-core
// kernel is the default where it has an instantiation.
constexpr int VT_THREADS = 256, VT_TR = 4, VT_TP = 4;

struct VtShape {
  int nrow, nxi, npsi, nsrc, R, P, Rp, Pp, ntile, tpw, nz, G, spg, nflav, lds_main, lds_red;
};

static VtShape vt_shape(const BlocksArgs &a, bool sym) {
  VtShape v{};
  v.nrow = 3 * a.D;
  v.nsrc = a.nsrc;
  v.nxi = 3 * a.D * a.nsrc;
  v.npsi = a.D * a.nsrc;
  v.R = v.npsi * v.nxi;
  v.P = sym ? v.nxi * (v.nxi + 1) / 2 : v.nxi * v.nxi;
  const int nRT = (v.R + VT_TR - 1) / VT_TR, nPT = (v.P + VT_TP - 1) / VT_TP;
  v.Rp = nRT * VT_TR;
  v.Pp = nPT * VT_TP;
  v.ntile = nRT * nPT;
  v.tpw = v.ntile < VT_THREADS ? v.ntile : VT_THREADS;
  v.nz = (v.ntile + v.tpw - 1) / v.tpw;
  v.G = VT_THREADS / v.tpw;
  v.spg = v.G == 1 ? 2 : 1;   // sites per group and round (as VtC)
  v.nflav = sym ? 1 : 3;      // u (= d = q1), or u, d and q1 (q1 staged even when it is u)
  // per site of a round: propagator rows, sink weights, A, B (double2)
  v.lds_main = v.G * v.spg * (v.nflav * v.nrow * v.nxi + v.nsrc + 3 * v.Rp + 3 * v.Pp) * 16 + 2 * v.Pp;
  v.lds_red = v.G > 1 ? v.G * v.tpw * 4 * 16 : 0;
  return v;
}

// The shape (D, N_s) is a template parameter, so that every index
// division below is by a constant.
template <int D, int NSRC, bool SYM>
struct VtC {
  static constexpr int nrow = 3 * D, nxi = 3 * D * NSRC, npsi = D * NSRC, R = npsi * nxi;
  static constexpr int P = SYM ? nxi * (nxi + 1) / 2 : nxi * nxi;
  static constexpr int nRT = (R + VT_TR - 1) / VT_TR, nPT = (P + VT_TP - 1) / VT_TP;
  static constexpr int Rp = nRT * VT_TR, Pp = nPT * VT_TP, ntile = nRT * nPT;
  static constexpr int tpw = ntile < VT_THREADS ? ntile : VT_THREADS, G = VT_THREADS / tpw;
  static constexpr int spg = G == 1 ? 2 : 1;   // sites per group and round
  static constexpr int nflav = SYM ? 1 : 3, nrx = nrow * nxi, SR = G * spg, nsrc = NSRC;
};

template <typename TIN, bool SYM, int D, int NSRC>
__global__ __launch_bounds__(VT_THREADS) void blocks_vt_kernel(BlocksArgs a) {
  constexpr VtC<D, NSRC, SYM> v{};
  extern __shared__ double2 lds[];
  const int tid = threadIdx.x;
  const int g = tid / v.tpw, tl = tid % v.tpw;
  const int tile = int(blockIdx.z) * v.tpw + tl;
  const bool active = g < v.G && tile < v.ntile;
  const int nPT = v.Pp / VT_TP;
  const int r0 = (tile / nPT) * VT_TR, p0 = (tile % nPT) * VT_TP;
  const int64_t ln = blockIdx.y;
  const int chunk = blockIdx.x;
  const int64_t x0 = int64_t(chunk) * a.sites_per_chunk;
  const int64_t x1 = min(a.V, x0 + a.sites_per_chunk);
  const double scale = a.scale_exp ? ldexp(1.0, a.scale_exp[ln]) : 1.0;
  const int nrx = v.nrow * v.nxi;
  const int SR = v.G * v.spg;                                 // sites per round
  // LDS areas (per site i of the round)
  double2 *sprop = lds;                                       // [SR][nflav][nrow][nxi]
  double2 *sw = sprop + SR * v.nflav * nrx;                   // [SR][nsrc]
  double2 *sA = sw + SR * v.nsrc;                             // [SR][3][Rp]
  double2 *sB = sA + SR * 3 * v.Rp;                           // [SR][3][Pp]
  const void *src[3] = {a.prop_u, a.prop_d, a.prop_q1};       // staged flavours: u, d, q1
  const int fq1 = SYM ? 0 : 2, fu = 0, fd = SYM ? 0 : 1;

  // (x2, x3) of every pair, once per workgroup
  unsigned char *px = reinterpret_cast<unsigned char *>(sB + SR * 3 * v.Pp);   // [2][Pp]
  for (int p = tid; p < v.P; p += VT_THREADS) {
    int x2, x3;
    if (SYM) {
      x3 = 0;
      while ((x3 + 1) * (x3 + 2) / 2 <= p) x3++;
      x2 = p - x3 * (x3 + 1) / 2;
    } else {
      x2 = p / v.nxi;
      x3 = p % v.nxi;
    }
    px[p] = (unsigned char)x2;
    px[v.Pp + p] = (unsigned char)x3;
  }

  double2 acc[VT_TR][VT_TP];
#pragma unroll
  for (int i = 0; i < VT_TR; i++)
#pragma unroll
    for (int j = 0; j < VT_TP; j++) acc[i][j] = make_double2(0.0, 0.0);

  for (int64_t xb = x0; xb < x1; xb += SR) {
    const int ns = int(min<int64_t>(SR, x1 - xb));   // sites of this round
    __syncthreads();   // the previous round's operands are no longer read
    for (int e = tid; e < ns * v.nflav * nrx; e += VT_THREADS) {
      const int i = e / (v.nflav * nrx), f = (e / nrx) % v.nflav, rx = e % nrx;
      const int r = rx / v.nxi, xi = rx % v.nxi;
      const int s = xi % v.nsrc, kap = xi / v.nsrc;
      const TIN val = static_cast<const TIN *>(src[f])[(((ln * a.V + xb + i) * v.nsrc + s) * 12 + r) * 12 + kap];
      sprop[e] = make_double2(double(val.x) * scale, double(val.y) * scale);
    }
    if (tid < ns * v.nsrc)
      sw[tid] = a.sink_w ? reinterpret_cast<const double2 *>(a.sink_w)[int64_t(tid % v.nsrc) * a.V + xb + tid / v.nsrc]
                         : make_double2(1.0, 0.0);
    __syncthreads();
    // A[i][c][r] = w_{s'(psi)} S_q1[(alpha(psi), c), xi1]
    for (int e = tid; e < ns * 3 * v.Rp; e += VT_THREADS) {
      const int i = e / (3 * v.Rp), c = (e / v.Rp) % 3, r = e % v.Rp;
      double2 out = make_double2(0.0, 0.0);
      if (r < v.R) {
        const int psi = r / v.nxi, xi1 = r % v.nxi;
        const double2 w = sw[i * v.nsrc + psi % v.nsrc];
        const double2 q = sprop[(i * v.nflav + fq1) * nrx + (3 * (psi / v.nsrc) + c) * v.nxi + xi1];
        out = make_double2(w.x * q.x - w.y * q.y, w.x * q.y + w.y * q.x);
      }
      sA[e] = out;
    }
    // B[i][c][p]: the diquark sum eps_cbd (C g5)_{gamma delta} S_u[(gamma, b), x2]
    // S_d[(delta, d), x3]  ((C g5): (0,1) -1, (1,0) +1, (2,3) -1, (3,2) +1)
    for (int e = tid; e < ns * 3 * v.Pp; e += VT_THREADS) {
      const int i = e / (3 * v.Pp), c = (e / v.Pp) % 3, p = e % v.Pp;
      double re = 0.0, im = 0.0;
      if (p < v.P) {
        const int x2 = px[p], x3 = px[v.Pp + p];
        const int bb = (c + 1) % 3, cc = (c + 2) % 3;
        const double2 *su = sprop + (i * v.nflav + fu) * nrx, *sd = sprop + (i * v.nflav + fd) * nrx;
        for (int gs = 0; gs < D; gs++) {
          const double sg = (gs & 1) ? 1.0 : -1.0;
          const int gd = gs ^ 1;
          const double2 l0 = su[(3 * gs + bb) * v.nxi + x2], r0 = sd[(3 * gd + cc) * v.nxi + x3];
          const double2 l1 = su[(3 * gs + cc) * v.nxi + x2], r1 = sd[(3 * gd + bb) * v.nxi + x3];
          re += sg * ((l0.x * r0.x - l0.y * r0.y) - (l1.x * r1.x - l1.y * r1.y));
          im += sg * ((l0.x * r0.y + l0.y * r0.x) - (l1.x * r1.y + l1.y * r1.x));
        }
      }
      sB[e] = make_double2(re, im);
    }
    __syncthreads();
    if (active) {
      for (int ii = 0; ii < v.spg; ii++) {
        const int i = g * v.spg + ii;   // this group's sites of the round
        if (i >= ns) break;
#pragma unroll
        for (int c = 0; c < 3; c++) {
          double2 av[VT_TR], bv[VT_TP];
#pragma unroll
          for (int t = 0; t < VT_TR; t++) av[t] = sA[(i * 3 + c) * v.Rp + r0 + t];
#pragma unroll
          for (int t = 0; t < VT_TP; t++) bv[t] = sB[(i * 3 + c) * v.Pp + p0 + t];
#pragma unroll
          for (int t = 0; t < VT_TR; t++)
#pragma unroll
            for (int u = 0; u < VT_TP; u++) {
              acc[t][u].x = fma(av[t].x, bv[u].x, fma(-av[t].y, bv[u].y, acc[t][u].x));
              acc[t][u].y = fma(av[t].x, bv[u].y, fma(av[t].y, bv[u].x, acc[t][u].y));
            }
        }
      }
    }
  }
  const int64_t nent = int64_t(v.R) * v.P;
  double2 *out = reinterpret_cast<double2 *>(a.partial) + (ln * a.nchunk + chunk) * nent;
  auto store = [&](int i, int j, double2 val) {
    const int r = r0 + i, p = p0 + j;
    if (r < v.R && p < v.P) out[int64_t(r) * v.P + p] = val;
  };
  if (v.G == 1) {
    if (active) {
#pragma unroll
      for (int i = 0; i < VT_TR; i++)
#pragma unroll
        for (int j = 0; j < VT_TP; j++) store(i, j, acc[i][j]);
    }
    return;
  }
  // add the groups' tiles in group order, four accumulators at a time
  double2 *red = lds;   // [G][tpw][4]
#pragma unroll
  for (int q = 0; q < VT_TR * VT_TP / 4; q++) {
    __syncthreads();
    if (active) {
#pragma unroll
      for (int k = 0; k < 4; k++) red[(g * v.tpw + tl) * 4 + k] = acc[(4 * q + k) / VT_TP][(4 * q + k) % VT_TP];
    }
    __syncthreads();
    if (active && g == 0) {
#pragma unroll
      for (int k = 0; k < 4; k++) {
        double2 t = red[tl * 4 + k];
        for (int h = 1; h < v.G; h++) {
          const double2 u = red[(h * v.tpw + tl) * 4 + k];
          t.x += u.x;
          t.y += u.y;
        }
        store((4 * q + k) / VT_TP, (4 * q + k) % VT_TP, t);
      }
    }
  }
}

template <typename TIN, bool SYM, int D, int NSRC>
static hipError_t launch_vt_shape(const BlocksArgs &a, hipStream_t s) {
  const VtShape v = vt_shape(a, SYM);
  const int lds = v.lds_main > v.lds_red ? v.lds_main : v.lds_red;
  // one sink weight per thread and round
  if (lds > 65536 || v.G * v.spg * v.nsrc > VT_THREADS || v.G != VtC<D, NSRC, SYM>::G) return hipErrorInvalidValue;
  hipLaunchKernelGGL((blocks_vt_kernel<TIN, SYM, D, NSRC>), dim3(a.nchunk, unsigned(a.B), unsigned(v.nz)),
                     dim3(VT_THREADS), lds, s, a);
  return hipGetLastError();
}

template <typename TIN, bool SYM>
static hipError_t launch_vt(const BlocksArgs &a, hipStream_t s) {
  if (a.D == 2 && a.nsrc == 1) return launch_vt_shape<TIN, SYM, 2, 1>(a, s);
  if (a.D == 4 && a.nsrc == 1) return launch_vt_shape<TIN, SYM, 4, 1>(a, s);
  if (a.D == 2 && a.nsrc == 2) return launch_vt_shape<TIN, SYM, 2, 2>(a, s);
  if (a.D == 2 && a.nsrc == 3) return launch_vt_shape<TIN, SYM, 2, 3>(a, s);
  return hipErrorInvalidValue;
}

template <typename TIN>
static hipError_t dispatch_bm(const BlocksArgs &a, bool sym, hipStream_t s) {
  if (a.kernel == 2 || (a.D == 2 && a.nsrc == 3))
    return sym ? launch_vt<TIN, true>(a, s) : launch_vt<TIN, false>(a, s);
  if (a.D == 4 && a.nsrc == 1)
    return sym ? launch_bm<TIN, 12, 4, 12, true>(a, s) : launch_bm<TIN, 12, 4, 12, false>(a, s);
  // NR, one source: two output tiles (symmetric pairs) or three, so two
  // multiplying waves; the smaller workgroups fit more of them per CU
  if (a.D == 2 && a.nsrc == 1)
    return sym ? launch_bm<TIN, 6, 2, 6, true, 2>(a, s) : launch_bm<TIN, 6, 2, 6, false, 2>(a, s);
  if (a.D == 2 && a.nsrc == 2)
    return sym ? launch_bm<TIN, 12, 4, 6, true>(a, s) : launch_bm<TIN, 12, 4, 6, false>(a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_blocks_partial(const BlocksArgs &a, bool mixed, bool sym, hipStream_t s) {
  // Both precision modes form the site sums in double on the matrix cores
  // (FP64 MFMA) and store the blocks in double.
  (void)mixed;
  return a.in_c128 ? dispatch_bm<double2>(a, sym, s) : dispatch_bm<float2>(a, sym, s);
}

// ---------------------------------------------------------------------------
// Finish: chunk sum (double, fixed order), antisymmetrisation, block layout.
// One workgroup row per lane: the threads of a lane walk its components, so
// that the chunk sums they read lie in the lane's own contiguous partial rows.
template <typename TO>
__global__ __launch_bounds__(256) void blocks_finish_kernel(FinishArgs a, int nxi, int npsi) {
  const int64_t b = blockIdx.x;
  const int npair2 = nxi * (nxi - 1) / 2;
  const int nyq = npair2 * nxi;
  const int64_t comp = blockIdx.y * int64_t(blockDim.x) + threadIdx.x;  // over 2 * npsi * nyq
  if (comp >= 2 * int64_t(npsi) * nyq) return;
  const int species = int(comp / (int64_t(npsi) * nyq));
  const int rem = int(comp % (int64_t(npsi) * nyq));
  const int psi = rem / nyq, yq = rem % nyq;
  const int npair = a.sym ? nxi * (nxi + 1) / 2 : nxi * nxi;
  auto pidx = [&](int x2, int x3) {
    if (a.sym) {
      int lo = min(x2, x3), hi = max(x2, x3);
      return hi * (hi + 1) / 2 + lo;
    }
    return x2 * nxi + x3;
  };
  double2 v = make_double2(0.0, 0.0);
  if (b < a.B) {
    const double2 *part = reinterpret_cast<const double2 *>(species == 0 ? a.partP : a.partN);
    // f(psi; i, j, k) = part[b][chunk][psi][i][pair(j, k)]
    int i1, j1, k1, i2, j2, k2;
    if (species == 0) {  // proton: u pair (p<q) = yq / nxi, d = yq % nxi
      int pr = yq / nxi, c = yq % nxi;
      int q = 1;
      while (q * (q + 1) / 2 <= pr) q++;
      int p = pr - q * (q - 1) / 2;
      i1 = p; j1 = q; k1 = c;   // f(p, q, c)
      i2 = q; j2 = p; k2 = c;   // f(q, p, c)
    } else {             // neutron: u = yq / npair2, d pair (p<q)
      int c = yq / npair2, pr = yq % npair2;
      int q = 1;
      while (q * (q + 1) / 2 <= pr) q++;
      int p = pr - q * (q - 1) / 2;
      i1 = p; j1 = c; k1 = q;   // f(p, c, q)
      i2 = q; j2 = c; k2 = p;   // f(q, c, p)
    }
    const int64_t o1 = (int64_t(psi) * nxi + i1) * npair + pidx(j1, k1);
    const int64_t o2 = (int64_t(psi) * nxi + i2) * npair + pidx(j2, k2);
    const int64_t stride = int64_t(npsi) * nxi * npair;
    for (int ch = 0; ch < a.nchunk; ch++) {
      const double2 *pc = part + (b * a.nchunk + ch) * stride;
      double2 x = pc[o1], y = pc[o2];
      v.x += x.x - y.x;
      v.y += x.y - y.y;
    }
  }
  TO *out = static_cast<TO *>(a.blocks);
  TO o;
  o.x = decltype(o.x)(v.x);
  o.y = decltype(o.y)(v.y);
  out[(int64_t(species) * nyq + yq) * npsi * a.Bp + lane_off(b, npsi) + psi * 16] = o;
}

// The Lambda block: f_L(psi; e, c, f) with (s, u, d) indices (e, c, f) is
// the partial entry (psi, xi1 = e, pair (c, f)) summed over the site chunks:
// pair c*n_xi + f (all ordered pairs; then the block quark index
// (e*n_xi + c)*n_xi + f is the partial's offset inside the psi row, so that
// a thread's chunk sums are one strided walk), or with a.sym (S_u = S_d) the
// symmetric pair max(c,f)(max(c,f)+1)/2 + min(c,f).  Stored in double from
// block row row0 on.
__global__ __launch_bounds__(256) void blocks_finish_lambda_kernel(FinishArgs a, int nxi, int npsi, int64_t row0) {
  const int64_t b = blockIdx.x;
  const int64_t nyl = int64_t(nxi) * nxi * nxi;
  const int64_t comp = blockIdx.y * int64_t(blockDim.x) + threadIdx.x;   // over npsi * nyl
  if (comp >= npsi * nyl) return;
  const int psi = int(comp / nyl);
  const int64_t y = comp % nyl;
  const int npair = a.sym ? nxi * (nxi + 1) / 2 : nxi * nxi;
  const int e = int(y / (nxi * nxi)), c = int(y / nxi % nxi), f = int(y % nxi);
  const int hi = max(c, f), lo = min(c, f);
  const int64_t off = (int64_t(psi) * nxi + e) * npair + (a.sym ? hi * (hi + 1) / 2 + lo : c * nxi + f);
  double2 v = make_double2(0.0, 0.0);
  if (b < a.B) {
    const double2 *part = reinterpret_cast<const double2 *>(a.partP);
    const int64_t stride = int64_t(npsi) * nxi * npair;
    for (int ch = 0; ch < a.nchunk; ch++) {
      const double2 x = part[(b * a.nchunk + ch) * stride + off];
      v.x += x.x;
      v.y += x.y;
    }
  }
  static_cast<double2 *>(a.blocks)[(row0 + y) * npsi * a.Bp + lane_off(b, npsi) + psi * 16] = v;
}

hipError_t launch_blocks_finish_lambda(const FinishArgs &a, int nxi, int npsi, int64_t row0, hipStream_t s) {
  const int64_t n = int64_t(npsi) * nxi * nxi * nxi;
  hipLaunchKernelGGL(blocks_finish_lambda_kernel, dim3(unsigned(a.Bp), unsigned((n + 255) / 256)), dim3(256), 0, s,
                     a, nxi, npsi, row0);
  return hipGetLastError();
}

// Per-lane exponent: e_b with 2^(e_b - 1) <= max |Re|, |Im| over the lane's
// block entries (every species) < 2^e_b, and the entries multiplied by
// 2^-e_b (exact), so that products of many blocks stay near 1 whatever the
// size of the propagators.  Two passes over a grid of (lane tile of 16,
// chunk of entries): the first writes every chunk's exponent per lane, the
// second reduces them per lane (chunk 0 stores e_b) and scales its chunk.
// In a workgroup the 16 thread groups stride over the chunk's entries of
// their lane.
struct ScaleGrid {
  int64_t Bp, nent, per;   // padded lanes, entries per lane, entries per chunk
  int npsi, nchunk;
  __device__ int64_t addr(int64_t tile, int64_t e, int l) const {
    return (e / npsi) * npsi * Bp + tile * npsi * 16 + (e % npsi) * 16 + l;
  }
};

__global__ __launch_bounds__(256) void blocks_lane_max_kernel(const double2 *blk, int32_t *part, ScaleGrid g) {
  __shared__ int emax[16][16];
  const int l = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int64_t tile = blockIdx.x, c = blockIdx.y;
  const int64_t e1 = min(g.nent, (c + 1) * g.per);
  int em = -100000;
  for (int64_t e = c * g.per + grp; e < e1; e += 16) {
    const double2 v = blk[g.addr(tile, e, l)];
    const double m = fmax(fabs(v.x), fabs(v.y));
    if (m > 0.0) em = max(em, ilogb(m) + 1);
  }
  emax[grp][l] = em;
  __syncthreads();
  if (grp == 0) {
    for (int i = 1; i < 16; i++) em = max(em, emax[i][l]);
    part[(tile * g.nchunk + c) * 16 + l] = em;
  }
}

__global__ __launch_bounds__(256) void blocks_scale_kernel(double2 *blk, int32_t *lane_exp, const int32_t *part,
                                                           ScaleGrid g) {
  __shared__ int esh[16];
  const int l = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int64_t tile = blockIdx.x, c = blockIdx.y;
  if (grp == 0) {
    int e = -100000;
    for (int i = 0; i < g.nchunk; i++) e = max(e, part[(tile * g.nchunk + i) * 16 + l]);
    e = e == -100000 ? 0 : e;   // an all-zero lane keeps its scale
    esh[l] = e;
    if (c == 0) lane_exp[tile * 16 + l] = e;
  }
  __syncthreads();
  const int sh = -esh[l];
  const int64_t e1 = min(g.nent, (c + 1) * g.per);
  for (int64_t e = c * g.per + grp; e < e1; e += 16) {
    double2 v = blk[g.addr(tile, e, l)];
    v.x = ldexp(v.x, sh);
    v.y = ldexp(v.y, sh);
    blk[g.addr(tile, e, l)] = v;
  }
}

// Float copies of one species' block for the recursion steps (float
// stages, MB_MIXED_F32B): only the positions of the species' sink base set,
// two neighbouring positions per lane side by side, so that one 16-byte load
// of a lane fetches two block entries.  Entry (y, psi_of_pos[2j + h]) of lane
// b goes to complex float h of float4 ((y * Bp/16 + b/16) * P + j) * 16 + b%16,
// P = ceil(M / 2) position pairs (the odd tail padded with zeros).  One
// thread per output float4.
__global__ __launch_bounds__(256) void blocks_to_f32_kernel(const double2 *in, float4 *out, int64_t n, int64_t Bp,
                                                            int npsi, int M, PsiPos pos) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int P = (M + 1) / 2;
  const int l = int(i % 16);
  const int j = int((i / 16) % P);
  const int64_t yt = i / (16 * int64_t(P));   // y * Bp/16 + tile
  const int64_t y = yt / (Bp / 16), t = yt % (Bp / 16);
  const double2 *row = in + y * npsi * Bp + t * npsi * 16 + l;
  const double2 a = row[pos.p[2 * j] * 16];
  const double2 c = 2 * j + 1 < M ? row[pos.p[2 * j + 1] * 16] : make_double2(0.0, 0.0);
  out[i] = make_float4(float(a.x), float(a.y), float(c.x), float(c.y));
}

hipError_t launch_blocks_to_f32(const void *blocks, void *out, int64_t rows, int64_t Bp, int npsi, int M,
                                const int *psi_of_pos, hipStream_t s) {
  if (M <= 0 || rows <= 0) return hipSuccess;
  if (M > 8) return hipErrorInvalidValue;
  PsiPos pos{};
  for (int d = 0; d < M; d++) pos.p[d] = psi_of_pos[d];
  const int64_t n = rows * (Bp / 16) * ((M + 1) / 2) * 16;
  hipLaunchKernelGGL(blocks_to_f32_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s,
                     static_cast<const double2 *>(blocks), static_cast<float4 *>(out), n, Bp, npsi, M, pos);
  return hipGetLastError();
}

static int blocks_scale_chunks(int64_t Bp, int npsi, int nyq2, size_t scratch_bytes) {
  const int64_t tiles = Bp / 16, nent = int64_t(nyq2) * npsi;
  // about 2048 workgroups, at least 64 entries per chunk, within the scratch
  int64_t c = (2048 + tiles - 1) / tiles;
  c = std::min<int64_t>(c, std::max<int64_t>(1, nent / 64));
  c = std::min<int64_t>(c, std::max<int64_t>(1, int64_t(scratch_bytes / (size_t(tiles) * 16 * 4))));
  return int(std::max<int64_t>(1, c));
}

hipError_t launch_blocks_scale(void *blocks, int32_t *lane_exp, int64_t Bp, int npsi, int nyq2, void *scratch,
                               size_t scratch_bytes, hipStream_t s) {
  ScaleGrid g;
  g.Bp = Bp;
  g.npsi = npsi;
  g.nent = int64_t(nyq2) * npsi;
  g.nchunk = blocks_scale_chunks(Bp, npsi, nyq2, scratch_bytes);
  g.per = (g.nent + g.nchunk - 1) / g.nchunk;
  if (size_t(Bp / 16) * g.nchunk * 16 * 4 > scratch_bytes) return hipErrorInvalidValue;
  int32_t *part = static_cast<int32_t *>(scratch);
  dim3 grid(unsigned(Bp / 16), unsigned(g.nchunk));
  hipLaunchKernelGGL(blocks_lane_max_kernel, grid, dim3(256), 0, s, static_cast<const double2 *>(blocks), part, g);
  hipLaunchKernelGGL(blocks_scale_kernel, grid, dim3(256), 0, s, static_cast<double2 *>(blocks), lane_exp,
                     static_cast<const int32_t *>(part), g);
  return hipGetLastError();
}

hipError_t launch_blocks_finish(const FinishArgs &a, bool mixed, hipStream_t s) {
  const int npsi = a.D * a.nsrc, nxi = 3 * a.D * a.nsrc;
  const int nyq = nxi * (nxi - 1) / 2 * nxi;
  dim3 grid(unsigned(a.Bp), unsigned((2 * npsi * nyq + 255) / 256));
  (void)mixed;  // blocks are stored in double in both modes
  hipLaunchKernelGGL(blocks_finish_kernel<double2>, grid, dim3(256), 0, s, a, nxi, npsi);
  return hipGetLastError();
}

}  // namespace mb
