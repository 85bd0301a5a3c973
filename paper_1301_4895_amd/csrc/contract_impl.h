// Recursion F_-^(s) = F_-^(s-1) . f_T (eq. recr_F) and final contraction with L
// (eq. C_final) on gfx950.
//
// Layout: every stage holds F[q][tile][sigma][16] -- quark part q, spin part
// sigma = (proton rank) * (#neutron sets) + (neutron rank), lanes (problem,
// timeslice) in tiles of 16 (padded to 64 in all), so that 16 lanes of one
// component are one contiguous row and the rows of one component's spin
// parts are adjacent.
//
// A step adds one baryon of species T.  Its operation list factorises
// (Sec. 3 with eq. antis_product_2): an output (sigma, q) is a sum over the
// quark splits of q (table entries: previous quark part, block quark index,
// sign) times the splits of the T spin set of sigma (one element moves to the
// new baryon; sign = parity of moving it behind the rest).  The spins of the
// other species pass through.  A thread owns one lane, one output quark part
// and a group of passthrough spin parts; for every quark split it loads the C(M,K)
// previous components and the M block entries once and forms the C(M,K+1) x
// (K+1) products of the spin wedge in registers (M = size of the T sink base
// set, K = T baryons already present), with the spin tables resolved at
// compile time.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"

namespace mb {

template <typename T> struct c2;
template <> struct c2<float> { using type = float2; };
template <> struct c2<double> { using type = double2; };

__host__ __device__ constexpr int popc(int m) { return m ? (m & 1) + popc(m >> 1) : 0; }
__host__ __device__ constexpr int binom_c(int n, int k) {
  return (k < 0 || k > n) ? 0 : (k == 0 || k == n) ? 1 : binom_c(n - 1, k - 1) + binom_c(n - 1, k);
}
// rank of `mask` among the masks with its popcount, ordered by value
__host__ __device__ constexpr int rank_c(int mask) {
  int r = 0;
  for (int m = 0; m < mask; m++)
    if (popc(m) == popc(mask)) r++;
  return r;
}

// Load at a base pointer plus a 32-bit byte offset.
template <typename T>
__device__ __forceinline__ T ld(const T *base, uint32_t byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// A split-table entry read with scalar loads: the same for every lane.
__device__ __forceinline__ uint2 uniform(uint2 v) {
  return make_uint2(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y));
}

// The spin wedge of one quark split:
//   out-set (K+1 elements of the M-element base set) +=
//       sum over its elements d of sgn(d) x fin[out minus d] x fy[d],
// sgn(d) = parity of moving d behind the other elements (eq. antis_product_2
// restricted to one species), times -1 when NEG.  Resolved at compile time;
// every real product is one fused multiply-add into the accumulator.
template <int M, int K, bool NEG = false>
__device__ __forceinline__ void wedge_accumulate(const double2 *fin, const double2 *fy, double2 *acc) {
#pragma unroll
  for (int out = 0; out < (1 << M); out++) {
    if (popc(out) != K + 1) continue;
    const int ro = rank_c(out);
#pragma unroll
    for (int d = 0; d < M; d++) {
      if (!((out >> d) & 1)) continue;
      const int in = out & ~(1 << d);
      const int ri = rank_c(in);
      const bool neg = bool(popc(in >> (d + 1)) & 1) != NEG;
      const double2 x = fin[ri], y = fy[d];
      const double s = neg ? -1.0 : 1.0;   // folds into the operand's sign
      acc[ro].x = fma(s * x.x, y.x, acc[ro].x);
      acc[ro].x = fma(-s * x.y, y.y, acc[ro].x);
      acc[ro].y = fma(s * x.x, y.y, acc[ro].y);
      acc[ro].y = fma(s * x.y, y.x, acc[ro].y);
    }
  }
}

// The same wedge ordered by input element: each previous component is
// widened to double (and, when SX, multiplied by the split sign sx) just
// before its M - K products, so that one widened value is live at a time.
template <int M, int K, bool SX, typename CS>
__device__ __forceinline__ void wedge_accumulate_x(const CS *xin, const double2 *fy, double sx, double2 *acc) {
#pragma unroll
  for (int in = 0; in < (1 << M); in++) {
    if (popc(in) != K) continue;
    const int ri = rank_c(in);
    double2 x = make_double2(double(xin[ri].x), double(xin[ri].y));
    if constexpr (SX) x = make_double2(sx * x.x, sx * x.y);
#pragma unroll
    for (int d = 0; d < M; d++) {
      if ((in >> d) & 1) continue;
      const int ro = rank_c(in | (1 << d));
      const bool neg = bool(popc(in >> (d + 1)) & 1);
      const double2 y = fy[d];
      const double s = neg ? -1.0 : 1.0;   // folds into the operand's sign
      acc[ro].x = fma(s * x.x, y.x, acc[ro].x);
      acc[ro].x = fma(-s * x.y, y.y, acc[ro].x);
      acc[ro].y = fma(s * x.x, y.y, acc[ro].y);
      acc[ro].y = fma(s * x.y, y.x, acc[ro].y);
    }
  }
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Workgroup -> (lane tile, position o in the output order of the step; o runs
// over the n8 padded outputs of each passthrough group in turn).  Workgroups
// are dispatched round-robin over the 8 XCDs (linear id mod 8).  The work
// (lane tile major, then o) is cut into 8 contiguous ranges, one per XCD:
// an XCD walks whole lane tiles, or a segment of one or two, so that its L2
// holds only its own lanes' rows, and it walks its outputs in order
// (neighbouring outputs share operands).  The grid is (n8 x passthrough
// groups, lane tiles), so the work is a multiple of 8.
struct TileOut {
  int64_t tile, o;
};
__device__ __forceinline__ TileOut xcd_map() {
  const int64_t nout = gridDim.x;
  const int64_t L = blockIdx.x + nout * int64_t(blockIdx.y);
  const int64_t per = nout * int64_t(gridDim.y) / 8;   // workgroups per XCD
  const int64_t g = (L % 8) * per + L / 8;             // position in the tile-major work order
  return {g / nout, g % nout};
}

// PKI: input layout.  0 plain; 1 paired, the pairs along the passthrough
// parts (a proton step, even passthrough count and group); 2 paired, the
// pairs along the input spin sets of the added species (neighbours in the
// stage order: a neutron step, or a proton step with one passthrough part).
// PHA: part A of a two-phase step (work item = one output and one group of
// pair splits sharing a single index; partial sums to H).
template <typename TS, typename TY, int M, int K, int PG, int TILE, int U, bool AP, int PKI, bool PHA>
__device__ __forceinline__ void stage_body(const StageArgs &a) {
  using CS = typename c2<TS>::type;
  using CY = typename c2<TY>::type;
  constexpr int NIN = binom_c(M, K), NOUT = binom_c(M, K + 1);
  constexpr int SUB = 64 / TILE;   // sub-waves splitting the quark splits
  // Part A with 16-lane tiles: the four sub-waves take four consecutive work
  // items instead (no reduction at the end).  Neighbouring items mostly
  // share their output quark part and differ in the single index, so they
  // read the same previous-stage rows at every split position, and one load
  // instruction fetches those bytes once for all four sub-waves.
  constexpr bool SUBI = PHA && SUB > 1;
  const int quarter = SUB == 1 ? 0 : int(threadIdx.x) / TILE;
  const int64_t nwork = PHA ? (SUBI ? (a.n_items + SUB - 1) / SUB : a.n_items) : a.nq_out;
  const int64_t n8 = (nwork + 7) / 8 * 8;
  const TileOut to = xcd_map();
  const int64_t b = to.tile * TILE + (threadIdx.x & (TILE - 1));
  const int pass0 = int(to.o / n8) * PG;
  const int64_t w = to.o % n8;
  if (w >= nwork) return;
  int64_t q = w;
  int grp = 0;   // group of pair splits (part A), else the whole list
  bool item_ok = true;
  if constexpr (SUBI) {
    const int64_t k = w * SUB + quarter;
    item_ok = k < a.n_items;
    const uint32_t it = a.items[item_ok ? k : a.n_items - 1];
    q = it / uint32_t(a.nsingle);
    grp = int(it % uint32_t(a.nsingle));
  } else if constexpr (PHA) {
    const uint32_t it = __builtin_amdgcn_readfirstlane(a.items[w]);
    q = it / uint32_t(a.nsingle);
    grp = int(it % uint32_t(a.nsingle));
  }
  const int nspl = PHA ? a.pp : a.Sq;   // splits of this work item
  const int64_t Bp = a.Bp;
  const int ns_in = NIN * a.npass, ns_out = NOUT * a.npass;
  // spin index of active rank r with passthrough rank p
  auto sig_out = [&](int r, int p) { return AP ? r * a.npass + p : p * NOUT + r; };

  const char *Fin = static_cast<const char *>(a.Fin);
  const char *fb = static_cast<const char *>(a.fblk);
  const uint2 *qs = reinterpret_cast<const uint2 *>(a.qsplit) + q * a.Sq + grp * a.pp;

  // Byte offsets inside the rows of a split.  A spin row of a lane tile is
  // 16 values; previous component (r, g) of a thread sits at
  // roff[r] + g * GSTEP + lane offset, block entry d at yoff[d] + lane offset.
  // roff and yoff are the same for every lane; GSTEP is a constant, so the
  // passthrough parts of one r are loaded at immediate offsets.
  constexpr uint32_t ROW = 16 * sizeof(CS);
  constexpr uint32_t GSTEP = AP ? ROW : NIN * ROW;
  uint32_t roff[NIN], yoff[M];
#pragma unroll
  for (int rr = 0; rr < NIN; rr++) roff[rr] = AP ? uint32_t(rr * a.npass + pass0) * ROW : uint32_t(pass0 * NIN + rr) * ROW;
  // float block copies hold the base-set positions in pairs, 16 bytes per
  // lane and pair: one load fetches two entries (a 16-lane row segment of a
  // pair is 256 bytes, as one of a double entry)
  constexpr bool YF = std::is_same<TY, float>::value;
  constexpr int MP = (M + 1) / 2;
#pragma unroll
  for (int d = 0; d < M; d++) yoff[d] = (YF ? uint32_t(d / 2) : uint32_t(a.psi_of_pos[d])) * 256u;
  const uint32_t x_lane = uint32_t(lane_off(b, ns_in)) * uint32_t(sizeof(CS));
  // paired input: the pair (2j, 2j+1) of spin parts of this lane, 16 bytes
  const uint32_t x_lane_pk = uint32_t((b >> 4) * ns_in * 16 + (b & 15) * 2) * uint32_t(sizeof(CS));
  const uint32_t y_lane = uint32_t(lane_off(b, YF ? MP : a.npsi)) * 16u;
  const int64_t xstride = int64_t(ns_in) * Bp * int64_t(sizeof(CS));
  const int64_t ystride = int64_t(YF ? MP : a.npsi) * Bp * 16;

  double2 acc[PG][NOUT];
#pragma unroll
  for (int g = 0; g < PG; g++)
#pragma unroll
    for (int o = 0; o < NOUT; o++) acc[g][o] = make_double2(0.0, 0.0);

  // Split-table entry of sub-wave `quarter` at position s (past the end of
  // the list: the last split, loaded in bounds and dropped below).  One
  // sub-wave: wave-uniform, read with scalar loads.  Several: every lane
  // loads its sub-wave's entry, one round ahead of its use.
  auto entry = [&](int s) -> uint2 {
    if constexpr (SUBI) return qs[min(s, nspl - 1)];
    else if constexpr (SUB > 1) return qs[min(s + quarter, nspl - 1)];
    else return uniform(qs[min(s, nspl - 1)]);
  };
  constexpr int STEP = SUBI ? 1 : SUB;   // split positions between a sub-wave's rounds
  uint2 e[U];
#pragma unroll
  for (int u = 0; u < U; u++) e[u] = entry(u * STEP);

  // U splits per round (1 or 2): every operand load of the U splits is
  // issued before the first product, so that a wavefront keeps U splits of
  // loads in flight.
  constexpr bool SIGN_ON_X = NIN * PG < M;
  for (int s0 = 0; s0 < nspl; s0 += STEP * U) {
    CY fy[U][M];   // block entries as stored; widened to double at the products
    CS xin[U][PG][NIN];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const char *xrow = Fin + int64_t(e[u].x) * xstride;
      const char *yrow = fb + int64_t(e[u].y & 0x7fffffffu) * ystride;
      if constexpr (SUB == 1) {
        // wave-uniform row bases: scalar base plus a 32-bit lane offset
        if constexpr (YF) {
#pragma unroll
          for (int j = 0; j < MP; j++) {
            const float4 v = ld(reinterpret_cast<const float4 *>(yrow + yoff[2 * j]), y_lane);
            fy[u][2 * j] = make_float2(v.x, v.y);
            if (2 * j + 1 < M) fy[u][2 * j + 1] = make_float2(v.z, v.w);
          }
        } else {
#pragma unroll
          for (int d = 0; d < M; d++) fy[u][d] = ld(reinterpret_cast<const CY *>(yrow + yoff[d]), y_lane);
        }
#pragma unroll
        for (int rr = 0; rr < NIN; rr++) {
          if constexpr (PKI == 1) {
            // passthrough parts 2j and 2j+1 of row rr are neighbours: one load
#pragma unroll
            for (int j = 0; j < PG / 2; j++) {
              const float4 v = ld(reinterpret_cast<const float4 *>(xrow + roff[rr]), x_lane_pk + j * 2 * ROW);
              xin[u][2 * j][rr] = make_float2(v.x, v.y);
              xin[u][2 * j + 1][rr] = make_float2(v.z, v.w);
            }
          } else if constexpr (PKI == 2) {
            // input sets rr and rr + 1 of one passthrough part are neighbours
            if (rr % 2 == 0) {
#pragma unroll
              for (int g = 0; g < PG; g++) {
                const float4 v = ld(reinterpret_cast<const float4 *>(xrow + roff[rr]), x_lane_pk + g * GSTEP);
                xin[u][g][rr] = make_float2(v.x, v.y);
                xin[u][g][rr + 1] = make_float2(v.z, v.w);
              }
            }
          } else {
#pragma unroll
            for (int g = 0; g < PG; g++)
              xin[u][g][rr] = ld(reinterpret_cast<const CS *>(xrow + roff[rr]), x_lane + g * GSTEP);
          }
        }
      } else {
        // per-lane row bases: one 64-bit pointer per r (and per d), the
        // passthrough parts at immediate offsets from it
        const char *xl = xrow + x_lane, *yl = yrow + y_lane;
        if constexpr (YF) {
#pragma unroll
          for (int j = 0; j < MP; j++) {
            const float4 v = *reinterpret_cast<const float4 *>(yl + yoff[2 * j]);
            fy[u][2 * j] = make_float2(v.x, v.y);
            if (2 * j + 1 < M) fy[u][2 * j + 1] = make_float2(v.z, v.w);
          }
        } else {
#pragma unroll
          for (int d = 0; d < M; d++) fy[u][d] = *reinterpret_cast<const CY *>(yl + yoff[d]);
        }
#pragma unroll
        for (int rr = 0; rr < NIN; rr++) {
          const char *p = xl + roff[rr];
#pragma unroll
          for (int g = 0; g < PG; g++) xin[u][g][rr] = *reinterpret_cast<const CS *>(p + g * GSTEP);
        }
      }
    }
    bool valid[U];
    double sgn[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      valid[u] = SUBI ? s0 + u < nspl : s0 + u * SUB + quarter < nspl;
      sgn[u] = valid[u] ? ((e[u].y >> 31) ? -1.0 : 1.0) : 0.0;
    }
    if constexpr (SUB > 1) {
#pragma unroll
      for (int u = 0; u < U; u++) e[u] = entry(s0 + STEP * U + u * STEP);
    }
    // keep the instruction scheduler from sinking loads below products
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; u++) {
      // the split sign multiplies the smaller operand set; a dropped split
      // adds zeros (its operands are finite values of the last split)
      double2 fyd[M];
      if constexpr (SIGN_ON_X) {
#pragma unroll
        for (int d = 0; d < M; d++) fyd[d] = make_double2(double(fy[u][d].x), double(fy[u][d].y));
#pragma unroll
        for (int g = 0; g < PG; g++) wedge_accumulate_x<M, K, true>(xin[u][g], fyd, sgn[u], acc[g]);
      } else {
#pragma unroll
        for (int d = 0; d < M; d++) fyd[d] = make_double2(sgn[u] * double(fy[u][d].x), sgn[u] * double(fy[u][d].y));
#pragma unroll
        for (int g = 0; g < PG; g++) wedge_accumulate_x<M, K, false>(xin[u][g], fyd, 1.0, acc[g]);
      }
    }
    if constexpr (SUB == 1) {
#pragma unroll
      for (int u = 0; u < U; u++) e[u] = entry(s0 + U + u);
    }
  }
  // sum the sub-waves (every lane ends with the total), then let sub-wave j
  // write the outputs o = j, j+SUB, ...
  if constexpr (SUB > 1 && !SUBI) {
#pragma unroll
    for (int g = 0; g < PG; g++)
#pragma unroll
      for (int o = 0; o < NOUT; o++) {
        double x = acc[g][o].x, y = acc[g][o].y;
#pragma unroll
        for (int w = TILE; w < 64; w *= 2) {
          x += __shfl_xor(x, w);
          y += __shfl_xor(y, w);
        }
        acc[g][o] = make_double2(x, y);
      }
  }
  // part A writes its partial to H_grp in the plain layout
  CS *Fout = PHA ? static_cast<CS *>(a.H) + grp * a.hstride : static_cast<CS *>(a.Fout);
  const bool pk_out = PHA ? false : bool(a.paired_out);
  if (!item_ok) return;
#pragma unroll
  for (int g = 0; g < PG; g++)
#pragma unroll
    for (int o = 0; o < NOUT; o++) {
      if (!SUBI && o % SUB != quarter) continue;
      CS v;
      v.x = TS(acc[g][o].x);
      v.y = TS(acc[g][o].y);
      Fout[q * ns_out * Bp + spin_off(b, ns_out, sig_out(o, pass0 + g), pk_out)] = v;
    }
}

// TS: storage type of F (float for the mixed modes, double for MB_FP64); TY:
// storage type of the block entries the step reads (double, or float for
// MB_MIXED_F32B, whose float stages read float copies of the blocks).
// Products and sums run in double in every case: on CDNA4 double FMA issues
// at the rate of single FMA, so only the bandwidth-bound storage is narrowed.  PG passthrough parts share each thread so that the
// block entries of a split are loaded once for all of them.
//
// A wavefront owns TILE lanes (64 or 16) of one output quark part.  With
// TILE = 16 its four quarter-waves take every fourth quark split and their
// partial sums are added with two cross-lane exchanges at the end; every
// operand load is then a 16-lane row segment (one 128-byte line of a float
// stage), which keeps four times more previous-stage rows in L2.  Which tile
// is faster depends on the step; the autotuner decides.  The spin layout of
// the step (added species proton or neutron) selects one of two bodies.
template <typename TS, typename TY, int M, int K, int PG, int TILE, int U, int PKI, bool PHA>
__global__ __launch_bounds__(64) void stage_kernel(StageArgs a) {
  if constexpr (PKI == 1) {
    stage_body<TS, TY, M, K, PG, TILE, U, true, 1, PHA>(a);   // launched only for a proton step
  } else {
    if (a.act_is_P) stage_body<TS, TY, M, K, PG, TILE, U, true, PKI, PHA>(a);
    else stage_body<TS, TY, M, K, PG, TILE, U, false, PKI, PHA>(a);
  }
}

// ---------------------------------------------------------------------------
// Recursion step with the block of the added species staged in LDS.
//
// A workgroup owns 16 lanes (one lane tile) and NSLOT consecutive (output
// quark part, passthrough group) slots; thread = (slot, lane).  The block
// entries of a split are f_T[y][psi] with y = (pair of the same-flavour
// quarks, single quark): every split of an output with single index p reads
// rows y = (*, p) only.  So the workgroup walks the single indices its
// outputs contain ("phases"), each in two ranges of pair rows (pairs (a,b)
// with b < bsplit, then the rest) so that one range of M baryon indices x 16
// lanes stays within 36 KB of LDS, together with the split-table rows of
// the phase.  Every thread then runs the splits of its output that belong to
// the phase and range: previous-stage operands from global memory, block
// entries and table entries from LDS.  The rows of the next range are
// fetched into registers while the current one is computed.
constexpr int LDS_SLOTS = 32, LDS_THREADS = 16 * LDS_SLOTS, LDS_MAX_ROWS = 36;

// The y area holds LDS_MAX_ROWS rows (a range never has more for n_xi <= 12:
// 36 and 30 rows for n_xi = 12, 15 for n_xi = 6); the table rows follow.
inline int stage_lds_bytes(int nxi, int M, int pp) {
  (void)nxi;
  return LDS_MAX_ROWS * M * 16 * int(sizeof(double2)) + LDS_SLOTS * pp * int(sizeof(uint2));
}

template <typename TS, int M, int K, int PG>
__global__ __launch_bounds__(LDS_THREADS) void stage_lds_kernel(StageLdsArgs a) {
  using CS = typename c2<TS>::type;
  constexpr int NIN = binom_c(M, K), NOUT = binom_c(M, K + 1);
  constexpr int FPT = (LDS_MAX_ROWS * M * 16 + LDS_THREADS - 1) / LDS_THREADS;   // fill loads per thread
  extern __shared__ double2 smem[];
  double2 *ylds = smem;                                                        // [row][d][16 lanes]
  uint2 *tlds = reinterpret_cast<uint2 *>(smem + LDS_MAX_ROWS * M * 16);      // [slot][pp]
  __shared__ uint32_t s_single[LDS_SLOTS];
  __shared__ int64_t s_q[LDS_SLOTS];
  __shared__ uint32_t wg_single;
  const int l = threadIdx.x & 15, slot = threadIdx.x >> 4;
  const int64_t tile = blockIdx.y;
  const int64_t nwg = gridDim.x;      // a multiple of 8
  const int64_t wr = blockIdx.x;
  // workgroups are dispatched round-robin over the 8 XCDs: give every XCD a
  // contiguous range of outputs
  const int64_t w = (wr % 8) * (nwg / 8) + wr / 8;
  const int64_t gs = w * LDS_SLOTS + slot;
  const bool active = gs < a.nq_out * a.npg;
  const int64_t q = active ? gs / a.npg : 0;
  const int pass0 = active ? int(gs % a.npg) * PG : 0;
  const int64_t Bp = a.Bp;
  const int64_t b = tile * 16 + l;
  uint32_t pm = 0, sm = 0;   // masks of the pair flavour and of the single flavour
  if (active) {
    const uint32_t mu = a.masks[2 * q], md = a.masks[2 * q + 1];
    pm = a.act_is_P ? mu : md;
    sm = a.act_is_P ? md : mu;
  }
  if (threadIdx.x == 0) wg_single = 0;
  if (l == 0) {
    s_single[slot] = sm;
    s_q[slot] = q;
  }
  __syncthreads();
  if (active && l == 0) atomicOr(&wg_single, sm);
  __syncthreads();
  const uint32_t phases = wg_single;
  const int R1 = a.bsplit * (a.bsplit - 1) / 2;   // rows of the first range
  const int nrange = R1 < a.npair ? 2 : 1;
  const int c0 = [&] {                             // splits per phase in the first range
    const int n = __builtin_popcount(pm & ((1u << a.bsplit) - 1u));
    return n * (n - 1) / 2;
  }();
  const int ns_in = NIN * a.npass, ns_out = NOUT * a.npass;
  auto sig_in = [&](int r, int p) { return a.act_is_P ? r * a.npass + p : p * NIN + r; };
  auto sig_out = [&](int r, int p) { return a.act_is_P ? r * a.npass + p : p * NOUT + r; };
  const CS *Fin = static_cast<const CS *>(a.Fin);
  const double2 *fb = static_cast<const double2 *>(a.fblk);
  const uint32_t in_lane = uint32_t(lane_off(b, ns_in));
  const int64_t ftile = tile * a.npsi * 16;
  const int64_t xstride = int64_t(ns_in) * Bp;

  // the (phase, range) sequence of the workgroup, walked with a cursor
  auto next_step = [&](int p, int h, int &np, int &nh) {
    if (h + 1 < nrange) {
      np = p;
      nh = h + 1;
      return;
    }
    uint32_t rest = phases & ~((2u << p) - 1u);
    np = rest ? __builtin_ctz(rest) : -1;
    nh = 0;
  };
  auto range_rows = [&](int h, int &r0, int &r1) {
    r0 = h ? R1 : 0;
    r1 = (h || nrange == 1) ? a.npair : R1;
  };
  double2 pre[FPT];
  auto prefetch = [&](int p, int h) {
    int r0, r1;
    range_rows(h, r0, r1);
    const int nel = (r1 - r0) * M * 16;
#pragma unroll
    for (int i = 0; i < FPT; i++) {
      const int e = int(threadIdx.x) + i * LDS_THREADS;
      if (e < nel) {
        const int row = r0 + e / (M * 16), d = (e / 16) % M, ll = e & 15;
        const int64_t y = a.act_is_P ? int64_t(row) * a.nxi + p : int64_t(p) * a.npair + row;
        pre[i] = fb[y * a.npsi * Bp + ftile + a.psi_of_pos[d] * 16 + ll];
      }
    }
  };

  double2 acc[PG][NOUT];
#pragma unroll
  for (int g = 0; g < PG; g++)
#pragma unroll
    for (int r = 0; r < NOUT; r++) acc[g][r] = make_double2(0.0, 0.0);

  int p = phases ? __builtin_ctz(phases) : -1, h = 0;
  if (p >= 0) prefetch(p, h);
  while (p >= 0) {
    int r0, r1;
    range_rows(h, r0, r1);
    __syncthreads();   // the previous range is no longer read
#pragma unroll
    for (int i = 0; i < FPT; i++) {
      const int e = int(threadIdx.x) + i * LDS_THREADS;
      if (e < (r1 - r0) * M * 16) ylds[e] = pre[i];
    }
    if (h == 0) {
      // split-table rows of this phase: pp entries per slot whose output
      // contains the single index p
      for (int e = threadIdx.x; e < LDS_SLOTS * a.pp; e += LDS_THREADS) {
        const int sl = e / a.pp, t = e - sl * a.pp;
        const uint32_t ssm = s_single[sl];
        if ((ssm >> p) & 1u) {
          const int jj = __builtin_popcount(ssm & ((1u << p) - 1u));
          tlds[e] = reinterpret_cast<const uint2 *>(a.qsplit)[s_q[sl] * a.Sq + jj * a.pp + t];
        }
      }
    }
    __syncthreads();
    int np, nh;
    next_step(p, h, np, nh);
    if (np >= 0) prefetch(np, nh);   // in flight during the products below
    if (active && ((sm >> p) & 1u)) {
      const int t0 = h ? c0 : 0, t1 = (h || nrange == 1) ? a.pp : c0;
      const uint2 *trow = tlds + slot * a.pp;
      for (int t = t0; t < t1; t++) {
        const uint2 e = trow[t];
        const uint32_t y = e.y & 0x7fffffffu;
        const int row = a.act_is_P ? int(__umulhi(y - uint32_t(p), a.div_magic)) : int(y) - p * a.npair;
        const double sgn = (e.y >> 31) ? -1.0 : 1.0;
        const CS *xrow = Fin + int64_t(e.x) * xstride;
        CS xin[PG][NIN];
#pragma unroll
        for (int g = 0; g < PG; g++)
#pragma unroll
          for (int r = 0; r < NIN; r++)
            xin[g][r] = ld(xrow, (in_lane + uint32_t(sig_in(r, pass0 + g) * 16)) * uint32_t(sizeof(CS)));
        double2 fy[M];
#pragma unroll
        for (int d = 0; d < M; d++) {
          const double2 v = ylds[((row - r0) * M + d) * 16 + l];
          fy[d] = make_double2(sgn * v.x, sgn * v.y);
        }
#pragma unroll
        for (int g = 0; g < PG; g++) {
          double2 fin[NIN];
#pragma unroll
          for (int r = 0; r < NIN; r++) fin[r] = make_double2(double(xin[g][r].x), double(xin[g][r].y));
          wedge_accumulate<M, K>(fin, fy, acc[g]);
        }
      }
    }
    p = np;
    h = nh;
  }
  if (!active) return;
  CS *Fout = static_cast<CS *>(a.Fout);
#pragma unroll
  for (int g = 0; g < PG; g++)
#pragma unroll
    for (int r = 0; r < NOUT; r++) {
      CS o;
      o.x = TS(acc[g][r].x);
      o.y = TS(acc[g][r].y);
      Fout[q * ns_out * Bp + spin_off(b, ns_out, sig_out(r, pass0 + g), a.paired_out)] = o;
    }
}

template <typename T, int M, int K, int PG>
static hipError_t launch_stage_lds_mkp(const StageLdsArgs &a, hipStream_t s) {
  const int64_t nslot = a.nq_out * a.npg;
  const int64_t nwg = ((nslot + LDS_SLOTS - 1) / LDS_SLOTS + 7) / 8 * 8;
  if (!grid_x_fits(nwg, LDS_THREADS)) return hipErrorInvalidConfiguration;
  dim3 grid(unsigned(nwg), unsigned(a.Bp / 16));
  if (a.dry) return hipSuccess;   // validation pass: this launch exists and fits
  hipLaunchKernelGGL((stage_lds_kernel<T, M, K, PG>), grid, dim3(LDS_THREADS), stage_lds_bytes(a.nxi, M, a.pp), s,
                     a);
  return hipGetLastError();
}

template <typename T, int M, int K>
static hipError_t launch_stage_lds_mk(const StageLdsArgs &a, hipStream_t s) {
  if (a.pg == 3) return launch_stage_lds_mkp<T, M, K, 3>(a, s);
  if (a.pg == 2) return launch_stage_lds_mkp<T, M, K, 2>(a, s);
  return launch_stage_lds_mkp<T, M, K, 1>(a, s);
}

template <typename T>
hipError_t launch_stage_lds_t(const StageLdsArgs &a, hipStream_t s) {
#define MB_CASE(m, k) \
  if (a.M == m && a.K == k) return launch_stage_lds_mk<T, m, k>(a, s);
  MB_CASE(1, 0)
  MB_CASE(2, 0) MB_CASE(2, 1)
  MB_CASE(3, 0) MB_CASE(3, 1) MB_CASE(3, 2)
  MB_CASE(4, 0) MB_CASE(4, 1) MB_CASE(4, 2) MB_CASE(4, 3)
#undef MB_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Recursion step for G consecutive output quark parts per wavefront (64
// lanes).  Neighbouring outputs in the stage order often take the same block
// entries at the same split position (the quark parts differ in one index of
// the pair flavour, and every pair without it keeps its rank), so a
// wavefront reads the split entries of its G outputs (scalar loads), loads
// the block rows of the first output and of the first output whose row
// differs, and every other distinct row only when it occurs; each output
// still loads its own previous-stage operands.  Comparisons are on
// wave-uniform values, so every branch is uniform.
template <typename TS, typename TY, int M, int K, int PG, int G, bool PKI>
__global__ __launch_bounds__(64) void stage_group_kernel(StageArgs a) {
  using CS = typename c2<TS>::type;
  using CY = typename c2<TY>::type;
  constexpr int NIN = binom_c(M, K), NOUT = binom_c(M, K + 1);
  const int64_t ngrp = (a.nq_out + G - 1) / G;
  const int64_t n8 = (ngrp + 7) / 8 * 8;
  const TileOut to = xcd_map();
  const int64_t b = to.tile * 64 + threadIdx.x;
  const int pass0 = int(to.o / n8) * PG;
  const int64_t grp = to.o % n8;
  if (grp >= ngrp) return;
  const int64_t q0 = grp * G;
  const int64_t Bp = a.Bp;
  const int ns_in = NIN * a.npass, ns_out = NOUT * a.npass;
  auto sig_in = [&](int r, int p) { return a.act_is_P ? r * a.npass + p : p * NIN + r; };
  auto sig_out = [&](int r, int p) { return a.act_is_P ? r * a.npass + p : p * NOUT + r; };
  const CS *Fin = static_cast<const CS *>(a.Fin);
  const CY *fb = static_cast<const CY *>(a.fblk);
  // float block copies: base-set positions in pairs, one 16-byte load per
  // lane and pair
  constexpr bool YF = std::is_same<TY, float>::value;
  constexpr int MP = (M + 1) / 2;
  const float4 *fb4 = static_cast<const float4 *>(a.fblk);
  const uint32_t lane4 = uint32_t(lane_off(b, MP));
  const int64_t ystride4 = int64_t(MP) * a.Bp;
  const uint2 *qs[G];
#pragma unroll
  for (int g = 0; g < G; g++) qs[g] = reinterpret_cast<const uint2 *>(a.qsplit) + min(q0 + g, a.nq_out - 1) * a.Sq;
  uint32_t f_off[M];
#pragma unroll
  for (int d = 0; d < M; d++) f_off[d] = uint32_t(lane_off(b, a.npsi) + a.psi_of_pos[d] * 16);
  const uint32_t in_lane = uint32_t(lane_off(b, ns_in));
  // paired input (pairs along the input sets): element of the pair (2i, 2i+1)
  const uint32_t in_lane_pk = uint32_t((b >> 4) * ns_in * 16 + (b & 15) * 2);
  const int64_t xstride = int64_t(ns_in) * Bp, ystride = int64_t(a.npsi) * Bp;

  double2 acc[G][PG][NOUT];
#pragma unroll
  for (int g = 0; g < G; g++)
#pragma unroll
    for (int p = 0; p < PG; p++)
#pragma unroll
      for (int o = 0; o < NOUT; o++) acc[g][p][o] = make_double2(0.0, 0.0);

  auto load_y = [&](uint32_t yi, CY *y) {
    if constexpr (YF) {
      const float4 *yrow = fb4 + int64_t(yi) * ystride4;
#pragma unroll
      for (int j = 0; j < MP; j++) {
        const float4 v = ld(yrow, (lane4 + uint32_t(j) * 16u) * 16u);
        y[2 * j] = make_float2(v.x, v.y);
        if (2 * j + 1 < M) y[2 * j + 1] = make_float2(v.z, v.w);
      }
    } else {
      const CY *yrow = fb + int64_t(yi) * ystride;
#pragma unroll
      for (int d = 0; d < M; d++) y[d] = ld(yrow, f_off[d] * uint32_t(sizeof(CY)));
    }
  };
  // block entries as stored, widened to double for the products
  auto widen = [&](const CY *y, double2 *w) {
#pragma unroll
    for (int d = 0; d < M; d++) w[d] = make_double2(double(y[d].x), double(y[d].y));
  };
  for (int t = 0; t < a.Sq; t++) {
    uint2 e[G];
#pragma unroll
    for (int g = 0; g < G; g++) e[g] = uniform(qs[g][t]);
    const uint32_t ya = e[0].y & 0x7fffffffu;
    uint32_t yb = ya;
#pragma unroll
    for (int g = G - 1; g >= 1; g--)
      if ((e[g].y & 0x7fffffffu) != ya) yb = e[g].y & 0x7fffffffu;   // the first differing row
    // previous-stage rows: an output whose row at this position equals its
    // neighbour's reuses the neighbour's registers instead of loading again
    CS xin[G][PG][NIN];
#pragma unroll
    for (int g = 0; g < G; g++) {
      if (g > 0 && e[g].x == e[g - 1].x) {
#pragma unroll
        for (int p = 0; p < PG; p++)
#pragma unroll
          for (int rr = 0; rr < NIN; rr++) xin[g][p][rr] = xin[g - 1][p][rr];
        continue;
      }
      const CS *xrow = Fin + int64_t(e[g].x) * xstride;
#pragma unroll
      for (int p = 0; p < PG; p++)
#pragma unroll
        for (int rr = 0; rr < NIN; rr++) {
          if constexpr (PKI) {
            if (rr % 2 == 0) {
              const float4 v = ld(reinterpret_cast<const float4 *>(xrow),
                                  (in_lane_pk + uint32_t(sig_in(rr, pass0 + p) * 16)) * uint32_t(sizeof(CS)));
              xin[g][p][rr] = make_float2(v.x, v.y);
              xin[g][p][rr + 1] = make_float2(v.z, v.w);
            }
          } else {
            xin[g][p][rr] = ld(xrow, (in_lane + uint32_t(sig_in(rr, pass0 + p) * 16)) * uint32_t(sizeof(CS)));
          }
        }
    }
    CY ra[M], rb[M];
    load_y(ya, ra);
    if (yb != ya) load_y(yb, rb);
    __builtin_amdgcn_sched_barrier(0);
    double2 fya[M], fyb[M];
    widen(ra, fya);
    if (yb != ya) widen(rb, fyb);
#pragma unroll
    for (int g = 0; g < G; g++) {
      const uint32_t yg = e[g].y & 0x7fffffffu;
      const double sgn = (e[g].y >> 31) ? -1.0 : 1.0;
      if (yg == ya) {
#pragma unroll
        for (int p = 0; p < PG; p++) wedge_accumulate_x<M, K, true>(xin[g][p], fya, sgn, acc[g][p]);
      } else if (yg == yb) {
#pragma unroll
        for (int p = 0; p < PG; p++) wedge_accumulate_x<M, K, true>(xin[g][p], fyb, sgn, acc[g][p]);
      } else {
        CY rc[M];
        double2 fyc[M];
        load_y(yg, rc);
        widen(rc, fyc);
#pragma unroll
        for (int p = 0; p < PG; p++) wedge_accumulate_x<M, K, true>(xin[g][p], fyc, sgn, acc[g][p]);
      }
    }
  }
  CS *Fout = static_cast<CS *>(a.Fout);
#pragma unroll
  for (int g = 0; g < G; g++) {
    if (q0 + g >= a.nq_out) break;
#pragma unroll
    for (int p = 0; p < PG; p++)
#pragma unroll
      for (int o = 0; o < NOUT; o++) {
        CS v;
        v.x = TS(acc[g][p][o].x);
        v.y = TS(acc[g][p][o].y);
        Fout[(q0 + g) * ns_out * Bp + spin_off(b, ns_out, sig_out(o, pass0 + p), a.paired_out)] = v;
      }
  }
}

template <typename T, typename TY, int M, int K, int PG, int G>
static hipError_t launch_stage_group(const StageArgs &a, hipStream_t s) {
  const int64_t ngrp = (a.nq_out + G - 1) / G;
  const int64_t n8 = (ngrp + 7) / 8 * 8;
  if (!grid_x_fits(n8 * (a.npass / PG), 64)) return hipErrorInvalidConfiguration;
  dim3 grid(unsigned(n8 * (a.npass / PG)), unsigned(a.Bp / 64));
  if (a.paired_in == 2) {
    // pairs along the input sets (see launch_stage_mkptu)
    if constexpr (std::is_same<T, float>::value && binom_c(M, K) % 2 == 0) {
      if (a.act_is_P && a.npass != 1) return hipErrorInvalidValue;
      if (a.dry) return hipSuccess;   // validation pass: this launch exists and fits
      hipLaunchKernelGGL((stage_group_kernel<T, TY, M, K, PG, G, true>), grid, dim3(64), a.lds_bytes, s, a);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (a.paired_in) return hipErrorInvalidValue;
  if (a.dry) return hipSuccess;   // validation pass: this launch exists and fits
  hipLaunchKernelGGL((stage_group_kernel<T, TY, M, K, PG, G, false>), grid, dim3(64), a.lds_bytes, s, a);
  return hipGetLastError();
}

template <typename T, typename TY, int M, int K, int PG, int TILE, int U, bool PHA>
static hipError_t launch_stage_mkptuh(const StageArgs &a, hipStream_t s) {
  constexpr int SUB = 64 / TILE;
  const int64_t nwork = PHA ? (SUB > 1 ? (a.n_items + SUB - 1) / SUB : a.n_items) : a.nq_out;
  const int64_t n8 = (nwork + 7) / 8 * 8;
  if (!grid_x_fits(n8 * (a.npass / PG), 64)) return hipErrorInvalidConfiguration;
  dim3 grid(unsigned(n8 * (a.npass / PG)), unsigned(a.Bp / TILE));
  constexpr bool F32 = std::is_same<T, float>::value;
  if (a.paired_in == 1) {
    // pairs along the passthrough parts: float stages, 64-lane tiles, even
    // passthrough groups of a proton step with an even passthrough count
    if constexpr (F32 && TILE == 64 && PG % 2 == 0) {
      if (!a.act_is_P || a.npass % 2) return hipErrorInvalidValue;
      if (a.dry) return hipSuccess;   // validation pass: this launch exists and fits
      hipLaunchKernelGGL((stage_kernel<T, TY, M, K, PG, TILE, U, 1, PHA>), grid, dim3(64), a.lds_bytes, s, a);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (a.paired_in == 2) {
    // pairs along the input sets: an even number of them, neighbours in the
    // stage order (a neutron step, or one passthrough part)
    if constexpr (F32 && TILE == 64 && binom_c(M, K) % 2 == 0) {
      if (a.act_is_P && a.npass != 1) return hipErrorInvalidValue;
      if (a.dry) return hipSuccess;   // validation pass: this launch exists and fits
      hipLaunchKernelGGL((stage_kernel<T, TY, M, K, PG, TILE, U, 2, PHA>), grid, dim3(64), a.lds_bytes, s, a);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (a.dry) return hipSuccess;   // validation pass: this launch exists and fits
  hipLaunchKernelGGL((stage_kernel<T, TY, M, K, PG, TILE, U, 0, PHA>), grid, dim3(64), a.lds_bytes, s, a);
  return hipGetLastError();
}

// part A of a two-phase step, or the whole step
template <typename T, typename TY, int M, int K, int PG, int TILE, int U>
static hipError_t launch_stage_mkptu(const StageArgs &a, hipStream_t s) {
  return a.two_phase ? launch_stage_mkptuh<T, TY, M, K, PG, TILE, U, true>(a, s)
                     : launch_stage_mkptuh<T, TY, M, K, PG, TILE, U, false>(a, s);
}

// splits in flight per wavefront: as tuned, else 2 when the operands of two
// splits fit in 32 registers
template <typename T, typename TY, int M, int K, int PG, int TILE>
static hipError_t launch_stage_mkpt(const StageArgs &a, hipStream_t s) {
  constexpr int VG_SPLIT = (binom_c(M, K) * PG * int(sizeof(typename c2<T>::type)) + M * int(sizeof(typename c2<TY>::type))) / 4;
  const int u = a.unroll ? a.unroll : (VG_SPLIT <= 32 ? 2 : 1);
  return u == 2 ? launch_stage_mkptu<T, TY, M, K, PG, TILE, 2>(a, s) : launch_stage_mkptu<T, TY, M, K, PG, TILE, 1>(a, s);
}

// outputs per wavefront (grouped kernel, 64 lanes, passthrough groups up to
// 3), else lanes per wavefront
template <typename T, typename TY, int M, int K, int PG>
static hipError_t launch_stage_mkp(const StageArgs &a, hipStream_t s) {
  if constexpr (PG <= 3) {
    if (a.group == 2 || a.group == 4) {
      if (a.two_phase) return hipErrorInvalidValue;   // two-phase steps use the direct kernel
      return a.group == 2 ? launch_stage_group<T, TY, M, K, PG, 2>(a, s) : launch_stage_group<T, TY, M, K, PG, 4>(a, s);
    }
  }
  return a.tile == 16 ? launch_stage_mkpt<T, TY, M, K, PG, 16>(a, s) : launch_stage_mkpt<T, TY, M, K, PG, 64>(a, s);
}

// passthrough group: as tuned (1, 2, 3 or 6), else 3 if it divides the
// passthrough count, else 2, else 1
template <typename T, typename TY, int M, int K>
static hipError_t launch_stage_mk(const StageArgs &a, hipStream_t s) {
  if constexpr (M > 4) {
    // more than four sink indices per species (three sources): one
    // passthrough part per thread and the direct kernel (the wedge alone
    // holds up to C(6,3) = 20 outputs per thread)
    if (a.pg > 1 || a.group > 1) return hipErrorInvalidValue;
    return a.tile == 16 ? launch_stage_mkpt<T, TY, M, K, 1, 16>(a, s) : launch_stage_mkpt<T, TY, M, K, 1, 64>(a, s);
  } else {
    if (a.pg == 1) return launch_stage_mkp<T, TY, M, K, 1>(a, s);
    if (a.pg == 2) return launch_stage_mkp<T, TY, M, K, 2>(a, s);
    if (a.pg == 3) return launch_stage_mkp<T, TY, M, K, 3>(a, s);
    if (a.pg == 6) return launch_stage_mkp<T, TY, M, K, 6>(a, s);
    if (a.npass % 3 == 0) return launch_stage_mkp<T, TY, M, K, 3>(a, s);
    if (a.npass % 2 == 0) return launch_stage_mkp<T, TY, M, K, 2>(a, s);
    return launch_stage_mkp<T, TY, M, K, 1>(a, s);
  }
}

// Instantiates the step kernels of the base-set sizes lo <= M <= hi only
// (the translation units split the instantiations by M).
template <typename T, typename TY, int LO, int HI>
hipError_t launch_stage_t(const StageArgs &a, hipStream_t s) {
#define MB_CASE(m, k) \
  if constexpr (LO <= m && m <= HI) { \
    if (a.M == m && a.K == k) return launch_stage_mk<T, TY, m, k>(a, s); \
  }
  MB_CASE(1, 0)
  MB_CASE(2, 0) MB_CASE(2, 1)
  MB_CASE(3, 0) MB_CASE(3, 1) MB_CASE(3, 2)
  MB_CASE(4, 0) MB_CASE(4, 1) MB_CASE(4, 2) MB_CASE(4, 3)
  MB_CASE(5, 0) MB_CASE(5, 1) MB_CASE(5, 2) MB_CASE(5, 3) MB_CASE(5, 4)
  MB_CASE(6, 0) MB_CASE(6, 1) MB_CASE(6, 2) MB_CASE(6, 3) MB_CASE(6, 4) MB_CASE(6, 5)
#undef MB_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Part B of a two-phase step: every output component is the sum of its
// nsingle partials (in double, in partial order), stored in the stage layout.
template <typename TS>
__global__ __launch_bounds__(256) void stage_sum_kernel(StageSumArgs a) {
  using CS = typename c2<TS>::type;
  const int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t comp = blockIdx.y + int64_t(gridDim.y) * blockIdx.z;   // q * ns + sigma
  if (b >= a.Bp || comp >= a.nq * a.ns) return;
  const int64_t q = comp / a.ns;
  const int sig = int(comp % a.ns);
  const CS *H = static_cast<const CS *>(a.H);
  const int64_t off = q * a.ns * a.Bp + lane_off(b, a.ns) + sig * 16;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < a.nsingle; j++) {
    const CS v = H[j * a.hstride + off];
    re += double(v.x);
    im += double(v.y);
  }
  CS o;
  o.x = TS(re);
  o.y = TS(im);
  static_cast<CS *>(a.Fout)[q * a.ns * a.Bp + spin_off(b, a.ns, sig, a.paired_out)] = o;
}

template <typename TS>
hipError_t launch_stage_sum_t(const StageSumArgs &a, hipStream_t s) {
  const int64_t ncomp = a.nq * a.ns;
  const unsigned gy = unsigned(ncomp < 65535 ? ncomp : 65535);
  const unsigned gz = unsigned((ncomp + gy - 1) / gy);
  hipLaunchKernelGGL(stage_sum_kernel<TS>, dim3(unsigned((a.Bp + 255) / 256), gy, gz), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace mb
