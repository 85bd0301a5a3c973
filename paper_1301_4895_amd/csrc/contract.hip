// Recursion steps of eq. recr_F (first stage, final contraction with L of
// eq. C_final, and the dispatch of the step kernels by storage type); the
// step kernels themselves are in contract_impl.h, instantiated for float
// stages in contract_f32.hip (float blocks: contract_f32b.hip) and for double
// stages in contract_f64.hip.
#include <hip/hip_runtime.h>

#include "contract_impl.h"

namespace mb {

hipError_t launch_stage_f32(const StageArgs &a, hipStream_t s);
hipError_t launch_stage_f32b(const StageArgs &a, hipStream_t s);
hipError_t launch_stage_f64(const StageArgs &a, hipStream_t s);
hipError_t launch_stage_lds_f32(const StageLdsArgs &a, hipStream_t s);
hipError_t launch_stage_lds_f64(const StageLdsArgs &a, hipStream_t s);

hipError_t launch_stage(const StageArgs &a, bool mixed, hipStream_t s) {
  if (!mixed) return launch_stage_f64(a, s);
  return a.fb32 ? launch_stage_f32b(a, s) : launch_stage_f32(a, s);
}

hipError_t launch_stage_sum(const StageSumArgs &a, bool mixed, hipStream_t s) {
  return mixed ? launch_stage_sum_t<float>(a, s) : launch_stage_sum_t<double>(a, s);
}

hipError_t launch_stage_lds(const StageLdsArgs &a, bool mixed, hipStream_t s) {
  return mixed ? launch_stage_lds_f32(a, s) : launch_stage_lds_f64(a, s);
}

template <typename T>
__global__ __launch_bounds__(256) void stage0_kernel(Stage0Args a) {
  using C2 = typename c2<T>::type;  // storage of F; blocks are double
  const int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t comp = blockIdx.y + int64_t(gridDim.y) * blockIdx.z;  // q * ns + sigma
  if (b >= a.Bp || comp >= a.nq * a.ns) return;
  const int64_t q = comp / a.ns;
  const int sig = int(comp % a.ns);
  const double2 *f = static_cast<const double2 *>(a.fblk);
  C2 *F = static_cast<C2 *>(a.Fout);
  const double2 v = f[int64_t(a.first[q]) * a.npsi * a.Bp + lane_off(b, a.npsi) + a.psi_of_pos[sig] * 16];
  C2 o;
  o.x = T(v.x);
  o.y = T(v.y);
  F[q * a.ns * a.Bp + spin_off(b, a.ns, sig, a.paired_out)] = o;
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
// Final contraction, in double: C[b][delta][alpha] = norm * sum_e c_e F[q_e][delta][b].
// One thread per (alpha, delta, lane): the coefficient list of alpha is read
// with scalar loads, F with one coalesced load per entry, eight entries in
// flight (the sum keeps the order of the list).  A projected list (Sec. 5,
// eq. CM_final) has one row per sink set delta, used with that delta only
// (diag): then alpha = delta and the output is C[b][delta].
template <typename TS>
__global__ __launch_bounds__(64) void final_kernel(FinalArgs a) {
  using CS = typename c2<TS>::type;
  const int64_t b = blockIdx.z * 64 + threadIdx.x;
  const int delta = blockIdx.y;
  const int alpha = a.diag ? delta : int(blockIdx.x);
  const CS *F = static_cast<const CS *>(a.F);
  double ar = 0.0, ai = 0.0;
  const int64_t e0 = a.crow[alpha], e1 = a.crow[alpha + 1];
  const int64_t off = lane_off(b, a.n_delta) + delta * 16;
  const int64_t rowstride = int64_t(a.n_delta) * a.Bp;
  constexpr int EB = 8;
  int64_t e = e0;
  for (; e + EB <= e1; e += EB) {
    CS v[EB];
#pragma unroll
    for (int j = 0; j < EB; j++) v[j] = F[int64_t(a.ccol[e + j]) * rowstride + off];
#pragma unroll
    for (int j = 0; j < EB; j++) {
      const double c = a.cval[e + j];
      ar += c * double(v[j].x);
      ai += c * double(v[j].y);
    }
  }
  for (; e < e1; e++) {
    const CS v = F[int64_t(a.ccol[e]) * rowstride + off];
    const double c = a.cval[e];
    ar += c * double(v.x);
    ai += c * double(v.y);
  }
  if (b < a.B) {
    const int e = a.A * a.lane_exp[b];
    const int64_t oi = a.diag ? b * a.n_delta + delta : (b * a.n_delta + delta) * a.n_alpha + alpha;
    reinterpret_cast<double2 *>(a.corr)[oi] = make_double2(ldexp(ar * a.inv_fact, e), ldexp(ai * a.inv_fact, e));
    if (a.exp_out && alpha == 0 && delta == 0) a.exp_out[b] = a.scale_exp ? 3 * a.A * a.scale_exp[b] : 0;
  }
}

hipError_t launch_final(const FinalArgs &a, bool mixed, hipStream_t s) {
  dim3 grid(unsigned(a.diag ? 1 : a.n_alpha), unsigned(a.n_delta), unsigned(a.Bp / 64));
  if (mixed)
    hipLaunchKernelGGL(final_kernel<float>, grid, dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(final_kernel<double>, grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

// Sum of a projected correlator over the sink sets, in delta order (one
// thread per lane).
__global__ __launch_bounds__(256) void project_kernel(const double2 *part, double2 *out, int64_t B, int n_delta) {
  const int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (b >= B) return;
  double re = 0.0, im = 0.0;
  for (int d = 0; d < n_delta; d++) {
    const double2 v = part[b * n_delta + d];
    re += v.x;
    im += v.y;
  }
  out[b] = make_double2(re, im);
}

hipError_t launch_project(const double *part, double *out, int64_t B, int n_delta, hipStream_t s) {
  hipLaunchKernelGGL(project_kernel, dim3(unsigned((B + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(part), reinterpret_cast<double2 *>(out), B, n_delta);
  return hipGetLastError();
}

}  // namespace mb
