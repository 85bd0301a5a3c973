// Recursion F_-^(s) = F_-^(s-1) . f_T (eq. recr_F) and final contraction with L
// (eq. C_final) on gfx950.
//
// Layout: every stage holds F[q][sigma][lane] -- quark part q (sorted (u, d)
// sets), spin part sigma = (proton rank) * (#neutron sets) + (neutron rank),
// lanes (problem, timeslice) innermost, padded to 64, so that one wavefront
// reads or writes 64 consecutive complex numbers of one component.
//
// A step adds one baryon of species T.  Its operation list factorises
// (Sec. 3 with eq. antis_product_2): an output (sigma, q) is a sum over the
// quark splits of q (table entries: previous quark part, block quark index,
// sign) times the splits of the T spin set of sigma (one element moves to the
// new baryon; sign = parity of moving it behind the rest).  The spins of the
// other species pass through.  A thread owns one lane, one output quark part
// and one passthrough spin part; for every quark split it loads the C(M,K)
// previous components and the M block entries once and forms the C(M,K+1) x
// (K+1) products of the spin wedge in registers (M = size of the T sink base
// set, K = T baryons already present), with the spin tables resolved at
// compile time.
#include <hip/hip_runtime.h>

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

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void stage0_kernel(Stage0Args a) {
  using C2 = typename c2<T>::type;
  const int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t comp = blockIdx.y + int64_t(gridDim.y) * blockIdx.z;  // q * ns + sigma
  if (b >= a.Bp || comp >= a.nq * a.ns) return;
  const int64_t q = comp / a.ns;
  const int sig = int(comp % a.ns);
  const C2 *f = static_cast<const C2 *>(a.fblk);
  C2 *F = static_cast<C2 *>(a.Fout);
  F[comp * a.Bp + b] = f[(int64_t(a.psi_of_pos[sig]) * a.nyq + a.first[q]) * a.Bp + b];
}

hipError_t launch_stage0(const Stage0Args &a, bool mixed, hipStream_t s) {
  const int64_t ncomp = a.nq * a.ns;
  const unsigned gy = unsigned(ncomp < 65535 ? ncomp : 65535);
  const unsigned gz = unsigned((ncomp + gy - 1) / gy);
  dim3 grid(unsigned((a.Bp + 255) / 256), gy, gz);
  if (mixed)
    hipLaunchKernelGGL(stage0_kernel<float>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(stage0_kernel<double>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <typename T, int M, int K>
__global__ __launch_bounds__(64) void stage_kernel(StageArgs a) {
  using C2 = typename c2<T>::type;
  constexpr int NIN = binom_c(M, K), NOUT = binom_c(M, K + 1);
  const int64_t b = blockIdx.y * 64 + threadIdx.x;
  const int64_t qp = blockIdx.x;               // output quark part * npass + pass
  const int64_t q = qp / a.npass;
  const int pass = int(qp % a.npass);
  const int64_t Bp = a.Bp;
  const int ns_in = NIN * a.npass, ns_out = NOUT * a.npass;
  // spin index of active rank r with the passthrough rank
  auto sig_in = [&](int r) { return a.act_is_P ? r * a.npass + pass : pass * NIN + r; };
  auto sig_out = [&](int r) { return a.act_is_P ? r * a.npass + pass : pass * NOUT + r; };

  const C2 *Fin = static_cast<const C2 *>(a.Fin);
  const C2 *fb = static_cast<const C2 *>(a.fblk);
  const uint2 *qs = reinterpret_cast<const uint2 *>(a.qsplit) + q * a.Sq;

  int64_t in_off[NIN];
#pragma unroll
  for (int r = 0; r < NIN; r++) in_off[r] = int64_t(sig_in(r)) * Bp + b;
  int64_t f_off[M];
#pragma unroll
  for (int d = 0; d < M; d++) f_off[d] = int64_t(a.psi_of_pos[d]) * a.nyq * Bp + b;

  C2 acc[NOUT];
#pragma unroll
  for (int r = 0; r < NOUT; r++) {
    acc[r].x = T(0);
    acc[r].y = T(0);
  }
  for (int s = 0; s < a.Sq; s++) {
    const uint2 e = qs[s];
    const int64_t xbase = int64_t(e.x) * ns_in * Bp;
    const int64_t ybase = int64_t(e.y & 0x7fffffffu) * Bp;
    const T sgn = (e.y >> 31) ? T(-1) : T(1);
    C2 fin[NIN], fy[M];
#pragma unroll
    for (int r = 0; r < NIN; r++) fin[r] = Fin[xbase + in_off[r]];
#pragma unroll
    for (int d = 0; d < M; d++) {
      C2 v = fb[ybase + f_off[d]];
      fy[d].x = sgn * v.x;
      fy[d].y = sgn * v.y;
    }
#pragma unroll
    for (int out = 0; out < (1 << M); out++) {
      if (popc(out) != K + 1) continue;
      const int ro = rank_c(out);
#pragma unroll
      for (int d = 0; d < M; d++) {
        if (!((out >> d) & 1)) continue;
        const int in = out & ~(1 << d);
        const int ri = rank_c(in);
        // moving element d behind the remaining elements of the set
        const bool neg = popc(in >> (d + 1)) & 1;
        const C2 x = fin[ri], y = fy[d];
        if (neg) {
          acc[ro].x -= x.x * y.x - x.y * y.y;
          acc[ro].y -= x.x * y.y + x.y * y.x;
        } else {
          acc[ro].x += x.x * y.x - x.y * y.y;
          acc[ro].y += x.x * y.y + x.y * y.x;
        }
      }
    }
  }
  C2 *Fout = static_cast<C2 *>(a.Fout);
#pragma unroll
  for (int r = 0; r < NOUT; r++) Fout[(q * ns_out + sig_out(r)) * Bp + b] = acc[r];
}

template <typename T, int M, int K>
static hipError_t launch_stage_mk(const StageArgs &a, hipStream_t s) {
  dim3 grid(unsigned(a.nq_out * a.npass), unsigned(a.Bp / 64));
  hipLaunchKernelGGL((stage_kernel<T, M, K>), grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_stage_t(const StageArgs &a, hipStream_t s) {
#define MB_CASE(m, k) \
  if (a.M == m && a.K == k) return launch_stage_mk<T, m, k>(a, s);
  MB_CASE(1, 0)
  MB_CASE(2, 0) MB_CASE(2, 1)
  MB_CASE(3, 0) MB_CASE(3, 1) MB_CASE(3, 2)
  MB_CASE(4, 0) MB_CASE(4, 1) MB_CASE(4, 2) MB_CASE(4, 3)
#undef MB_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_stage(const StageArgs &a, bool mixed, hipStream_t s) {
  return mixed ? launch_stage_t<float>(a, s) : launch_stage_t<double>(a, s);
}

// ---------------------------------------------------------------------------
// Final contraction, in double: C[b][delta][alpha] = norm * sum_e c_e F[q_e][delta][b]
constexpr int kDeltaChunk = 36;

template <typename T>
__global__ __launch_bounds__(64) void final_kernel(FinalArgs a) {
  using C2 = typename c2<T>::type;
  const int64_t b = blockIdx.y * 64 + threadIdx.x;
  const int alpha = blockIdx.x;
  const int d0 = blockIdx.z * kDeltaChunk;
  const int nd = min(kDeltaChunk, a.n_delta - d0);
  const C2 *F = static_cast<const C2 *>(a.F);
  double2 acc[kDeltaChunk];
#pragma unroll
  for (int d = 0; d < kDeltaChunk; d++) acc[d] = make_double2(0.0, 0.0);
  const int64_t e0 = a.crow[alpha], e1 = a.crow[alpha + 1];
  for (int64_t e = e0; e < e1; e++) {
    const int64_t base = (int64_t(a.ccol[e]) * a.n_delta + d0) * a.Bp + b;
    const double c = a.cval[e];
#pragma unroll
    for (int d = 0; d < kDeltaChunk; d++) {
      if (d < nd) {
        C2 v = F[base + int64_t(d) * a.Bp];
        acc[d].x += c * double(v.x);
        acc[d].y += c * double(v.y);
      }
    }
  }
  if (b < a.B) {
#pragma unroll
    for (int d = 0; d < kDeltaChunk; d++) {
      if (d < nd) {
        double2 v = make_double2(acc[d].x * a.norm, acc[d].y * a.norm);
        reinterpret_cast<double2 *>(a.corr)[(b * a.n_delta + d0 + d) * a.n_alpha + alpha] = v;
      }
    }
    if (a.exp_out && alpha == 0 && blockIdx.z == 0)
      a.exp_out[b] = a.scale_exp ? 3 * a.A * a.scale_exp[b] : 0;
  }
}

hipError_t launch_final(const FinalArgs &a, bool mixed, hipStream_t s) {
  dim3 grid(unsigned(a.n_alpha), unsigned(a.Bp / 64), unsigned((a.n_delta + kDeltaChunk - 1) / kDeltaChunk));
  if (mixed)
    hipLaunchKernelGGL(final_kernel<float>, grid, dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(final_kernel<double>, grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace mb
