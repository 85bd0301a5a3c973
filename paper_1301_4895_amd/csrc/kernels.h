// Kernel launchers of libmbcontract (implemented in blocks.hip, contract.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mb {

// Site-chunk partial sums of the full block f_{q1}(psi; xi1, (xi2, xi3)) for
// every lane.  partial layout: [lane][chunk][psi][xi1][pair] complex double,
// pair = xi3*(xi3+1)/2 + xi2 (xi2 <= xi3) when sym, else xi2*nxi + xi3.
struct BlocksArgs {
  const void *prop_q1;   // flavour in slot 1 (u for the proton, d for the neutron)
  const void *prop_u;    // slot 2
  const void *prop_d;    // slot 3
  const double *sink_w;  // [nsrc][V] complex or null
  const int32_t *scale_exp;  // [B] or null
  double *partial;
  int64_t B, V;
  int nsrc, D, nchunk, in_c128;
  int64_t sites_per_chunk;
  int kernel;            // 0 automatic (matrix cores where instantiated), 2 vector units
};
hipError_t launch_blocks_partial(const BlocksArgs &a, bool mixed, bool sym, hipStream_t s);

// Sums the chunks in double, antisymmetrises the same-flavour slots and
// writes the block arrays (lane-blocked layout below).  partN may equal
// partP (isospin limit).
struct FinishArgs {
  const double *partP, *partN;
  void *blocks;
  int64_t B, Bp;
  int nsrc, D, nchunk, sym;
};
hipError_t launch_blocks_finish(const FinishArgs &a, bool mixed, hipStream_t s);
// The Lambda block from the partials in a.partP (all ordered (u, d) pairs):
// chunk sum in double, stored from block row row0 on.
hipError_t launch_blocks_finish_lambda(const FinishArgs &a, int nxi, int npsi, int64_t row0, hipStream_t s);

// Per-lane block exponents (see blocks_scale_kernel): blocks scaled in place
// by 2^-lane_exp[b]; nyq2 = block quark indices of all species together.
// scratch: device memory for the per-chunk exponents (Bp/16 x chunks x 16
// int32, the chunk count fitted to scratch_bytes; the blocks workspace,
// free once the blocks are finished).
hipError_t launch_blocks_scale(void *blocks, int32_t *lane_exp, int64_t Bp, int npsi, int nyq2, void *scratch,
                               size_t scratch_bytes, hipStream_t s);
// Float copies of one species' block (rows block quark indices, npsi spin
// indices) for the steps of MB_MIXED_F32B: the M positions psi_of_pos of the
// species' sink base set, two per lane side by side (blocks_to_f32_kernel).
struct PsiPos {
  int p[8];
};
hipError_t launch_blocks_to_f32(const void *blocks, void *out, int64_t rows, int64_t Bp, int npsi, int M,
                                const int *psi_of_pos, hipStream_t s);

// Lane-blocked layouts (lanes grouped in tiles of 16, Bp = padded lanes):
//   stage   F[q][tile][sigma][16]     index q*ns*Bp + tile*ns*16 + sigma*16 + l
//   blocks  f[y][tile][psi][16]       index y*npsi*Bp + tile*npsi*16 + psi*16 + l
// (species blocks follow each other), so that the rows one thread needs for
// one operand (its spin parts, its baryon indices) are adjacent in memory.
__host__ __device__ inline int64_t lane_off(int64_t b, int n) { return (b >> 4) * n * 16 + (b & 15); }

// Element offset of spin part sigma of lane b inside one quark part of a
// stage with n spin parts.  Plain layout: [lane / 16][sigma][lane % 16].
// Paired layout (float stages whose next step reads neighbouring spin parts
// together): [lane / 16][sigma / 2][lane % 16][sigma % 2], so that a lane's
// spin parts 2j and 2j+1 are one 16-byte load.
__host__ __device__ inline int64_t spin_off(int64_t b, int n, int sigma, bool paired) {
  return paired ? (b >> 4) * n * 16 + (sigma >> 1) * 32 + (b & 15) * 2 + (sigma & 1)
                : (b >> 4) * n * 16 + sigma * 16 + (b & 15);
}

// A dispatch covers fewer than 2^32 work-items per dimension (the grid size
// of the dispatch packet is 32-bit); larger launches are refused, never
// truncated.
inline bool grid_x_fits(int64_t groups, int threads) { return groups * threads < (int64_t(1) << 32); }

// Stage 0: F0[q][sigma] = f_T0[psi(sigma)][first[q]].
struct Stage0Args {
  const void *fblk;
  void *Fout;
  const uint32_t *first;
  int64_t nq, Bp;
  int nyq, ns, npsi;
  int psi_of_pos[8];
  int paired_out;            // stage 0 stored in the paired layout
};
hipError_t launch_stage0(const Stage0Args &a, bool mixed, hipStream_t s);

// One recursion step F^(s) = F^(s-1) . f_T over the factorised operation list.
struct StageArgs {
  const void *Fin;
  void *Fout;
  const void *fblk;          // block of the added species, [npsi][nyq][Bp]
  const uint32_t *qsplit;    // [nq_out][Sq][2]
  int64_t nq_out, Bp;
  int Sq, nyq, npass;
  int act_is_P;              // 1: added species is the proton
  int M, K;                  // active base-set size, active input subset size
  int pg;                    // passthrough parts per thread (0 = automatic)
  int lds_bytes;             // LDS reserved per workgroup
  int tile;                  // lanes per wavefront: 64 or 16
  int unroll;                // splits in flight per wavefront: 1, 2 (0 = automatic)
  int group;                 // outputs per wavefront of the grouped kernel: 1 (off), 2, 4
  int npsi;                  // baryon indices of the block layout
  int psi_of_pos[8];
  int paired_in;             // input layout: 0 plain, 1 pairs along the passthrough parts,
                             // 2 pairs along the input sets (float stages, 64-lane waves)
  int paired_out;            // output stored in the paired layout (spin_off)
  int dry;                   // validate only: return what the launch would, launch nothing
  int fb32;                  // fblk holds the paired float copies of the block entries (MB_MIXED_F32B)
  // Two-phase step, part A (two_phase = 1, direct kernel): work item
  // items[i] = q * nsingle + j takes the j-th group of pp pair splits of
  // output q (those with the j-th single index of q) and writes its partial
  // sum to H + j * hstride in the plain layout; part B (launch_stage_sum)
  // adds the nsingle partials of every output.  Items are ordered by the
  // previous-stage parts they read, so that those stay in L2.
  int two_phase;
  const uint32_t *items;
  int64_t n_items;
  int pp, nsingle;
  void *H;
  int64_t hstride;           // elements (of the stage type) between partials
};
hipError_t launch_stage(const StageArgs &a, bool mixed, hipStream_t s);

// Part B of a two-phase step: F[q][sigma] = sum_j H_j[q][sigma] (in double,
// j ascending), written in the stage's layout.
struct StageSumArgs {
  const void *H;
  void *Fout;
  int64_t nq, Bp, hstride;
  int ns, nsingle, paired_out;
};
hipError_t launch_stage_sum(const StageSumArgs &a, bool mixed, hipStream_t s);

// The same step with the block of the added species staged in LDS.  Splits
// of an output are ordered by the single index of the added baryon, then by
// pair rank; the kernel walks the single indices in phases and, inside a
// phase, two ranges of pair rows (pairs (a,b) with b < bsplit, then the
// rest), holding only that part of the block in LDS.
struct StageLdsArgs {
  const void *Fin;
  void *Fout;
  const void *fblk;
  const uint32_t *qsplit;    // [nq_out][Sq][2]
  const uint32_t *masks;     // [nq_out][2]: (u mask, d mask) of every output
  int64_t nq_out, Bp;
  int Sq, pp;                // splits per output, per single index
  int npass, npg;            // passthrough parts, passthrough groups (npass / PG)
  int act_is_P;
  int M, K, pg;
  int nxi, npair, npsi, bsplit;
  uint32_t div_magic;        // ceil(2^32 / nxi): exact division of multiples of nxi
  int psi_of_pos[8];
  int paired_out;
  int dry;                   // validate only (as in StageArgs)
};
hipError_t launch_stage_lds(const StageLdsArgs &a, bool mixed, hipStream_t s);
// LDS bytes the staged kernel uses for a term list with nxi quark indices,
// base-set size M and pp splits per single index.
int stage_lds_bytes(int nxi, int M, int pp);

// Final signed sum C[b][delta][alpha] = 2^(A lane_exp[b]) / (n_P! n_N!) *
// sum_e c_e F[q_e][delta][b].
struct FinalArgs {
  const void *F;
  const int64_t *crow;
  const int32_t *ccol;
  const double *cval;
  double *corr;
  int32_t *exp_out;
  const int32_t *scale_exp;
  const int32_t *lane_exp;   // per-lane block exponents (undone here)
  int64_t B, Bp;
  int n_delta, n_alpha, A;
  double inv_fact;           // 1 / (n_P! n_N!)
  int diag;                  // projected list: row delta of the list with sink set delta only,
                             // corr[b][delta]
};
hipError_t launch_final(const FinalArgs &a, bool mixed, hipStream_t s);
// Projected correlator: out[b] = sum over delta (in order) of part[b][delta].
hipError_t launch_project(const double *part, double *out, int64_t B, int n_delta, hipStream_t s);

// Rounding-error estimate of the float stages (implemented in errest.hip):
// per stage component a float2 (E, S), E a first-order bound and S a
// standard deviation of the difference between the stored float value and
// the FP64 path's value, in the plain stage layout.
struct ErrStageArgs {
  const void *Ein;           // error stage s-1 (unused at stage 0)
  void *Eout;                // error stage s
  const void *F;             // float stage s as stored by step s
  const void *fblk;          // block of the added species
  const uint32_t *qsplit;    // [nq_out][Sq][2]
  int64_t nq_out, Bp;
  int Sq, npass, ns_out;
  int act_is_P, M, K, npsi;
  int psi_of_pos[8];
  int paired_F;              // stage s stored in the paired layout
  const void *H;             // two-phase step: its float partials (or null)
  int nh;                    // number of partials
  int64_t hstride;           // elements between partials
  // float block copies (MB_MIXED_F32B): the step multiplied the rounded
  // entries, so every split adds |F~_{s-1}(x)| u |f(y)|; Fprev is stage s-1
  // as stored (paired_prev: its layout)
  int fb32;
  const void *Fprev;
  int paired_prev;
};
hipError_t launch_err_stage0(const ErrStageArgs &a, hipStream_t s);
hipError_t launch_err_stage(const ErrStageArgs &a, hipStream_t s);

// err[b][delta][alpha] = (S_C, E_C) from the final error stage and |c|.
struct ErrFinalArgs {
  const void *E;
  const int64_t *crow;
  const int32_t *ccol;
  const double *cval;
  double *err;
  const int32_t *lane_exp;
  int64_t B, Bp;
  int n_delta, n_alpha, A;
  double inv_fact;
  int diag;
};
hipError_t launch_err_final(const ErrFinalArgs &a, hipStream_t s);
// Projected correlator: out[b] = (sqrt(sum S^2), sum E) over the sink sets.
hipError_t launch_err_project(const double *part, double *out, int64_t B, int n_delta, hipStream_t s);
// p[0..n) = 0 (a kernel, so that the call can be captured in a graph).
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);

}  // namespace mb
