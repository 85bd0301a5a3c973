// Rounding-error estimate of the mixed-precision correlators (float stage
// storage) against the FP64 path, propagated through the recursion of
// eq. recr_F and the final sum of eq. C_final.
//
// The mixed path forms every product and sum in double and rounds each
// stage component to float when it is stored: F~ = F + D with
// |Re D| <= u |Re F~|, |Im D| <= u |Im F~|, u = 2^-24 (round to nearest).
// A step forms sum_splits +-F~_s(x) f(y) exactly enough (double), so to
// first order in u the deviation of a stored component from the FP64 path
// obeys
//   D_{s+1}(z) = sum_splits +-D_s(x) f(y) + (rounding of F~_{s+1}(z)).
// Two quantities are carried per component, as a float2 (E, S):
//   E  bound:    E_{s+1}(z) = sum_splits E_s(x) |f(y)| + u |F~_{s+1}(z)|
//   S  std-dev:  S_{s+1}(z)^2 = sum_splits S_s(x)^2 |f(y)|^2 + u^2 |F~_{s+1}(z)|^2 / 3
// (the rounding error of one real value is uniform on half an ulp each side,
// variance <= u^2 x^2 / 3; S treats the rounding errors as independent).
// With MB_MIXED_F32B a step multiplies float copies f~ = f + d of the block
// entries (|Re d| <= u |Re f|, |Im d| <= u |Im f|), which adds
// sum_splits +-F~_s(x) d(y) to D_{s+1}(z): E gains sum_splits u |F~_s(x)| |f(y)|
// and S^2 gains sum_splits u^2 |F~_s(x)|^2 |f(y)|^2 / 3 (a block entry enters
// many splits, so S, which takes these errors as independent too, is only an
// estimate; E stays a first-order bound).
// The final sum gives, per correlator, E_C = sum |c| E(z) and
// S_C^2 = sum c^2 S(z)^2, with the normalisation and the lane's block
// exponent of the correlator itself.  Error stages use the plain stage
// layout [q][lane / 16][sigma][lane % 16].
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace mb {

namespace {

constexpr double U_F32 = 5.9604644775390625e-08;   // 2^-24

__host__ __device__ constexpr int popc_e(int m) { return m ? (m & 1) + popc_e(m >> 1) : 0; }
__host__ __device__ constexpr int binom_e(int n, int k) {
  return (k < 0 || k > n) ? 0 : (k == 0 || k == n) ? 1 : binom_e(n - 1, k - 1) + binom_e(n - 1, k);
}
__host__ __device__ constexpr int rank_e(int mask) {
  int r = 0;
  for (int m = 0; m < mask; m++)
    if (popc_e(m) == popc_e(mask)) r++;
  return r;
}

__device__ inline double mag(float2 v) { return sqrt(double(v.x) * v.x + double(v.y) * v.y); }
__device__ inline double mag(double2 v) { return sqrt(v.x * v.x + v.y * v.y); }

}  // namespace

// Stage 0: the first block rounded to float.  One thread per (lane,
// component); the grid is (lane tiles of 256, components).
__global__ __launch_bounds__(256) void err_stage0_kernel(ErrStageArgs a) {
  const int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  const int64_t comp = blockIdx.y + int64_t(gridDim.y) * blockIdx.z;
  const int ns = a.ns_out;
  if (b >= a.Bp || comp >= a.nq_out * ns) return;
  const int64_t q = comp / ns;
  const int sig = int(comp % ns);
  const float2 v = static_cast<const float2 *>(a.F)[q * ns * a.Bp + spin_off(b, ns, sig, a.paired_F)];
  const double m = mag(v);
  static_cast<float2 *>(a.Eout)[q * ns * a.Bp + lane_off(b, ns) + sig * 16] =
      make_float2(float(U_F32 * m), float(U_F32 * m / 1.7320508075688772));
}

// Step s.  Thread = (lane, output quark part, passthrough part); it carries
// the C(M, K+1) outputs of the added species' wedge for its passthrough part.
template <int M, int K>
__global__ __launch_bounds__(64) void err_stage_kernel(ErrStageArgs a) {
  constexpr int NIN = binom_e(M, K), NOUT = binom_e(M, K + 1);
  const int64_t b = blockIdx.y * 64 + threadIdx.x;
  const int64_t item = blockIdx.x;              // q * npass + p
  const int64_t q = item / a.npass;
  const int p = int(item % a.npass);
  if (q >= a.nq_out) return;
  const int ns_in = NIN * a.npass, ns_out = a.ns_out;
  auto sig_in = [&](int r) { return a.act_is_P ? r * a.npass + p : p * NIN + r; };
  auto sig_out = [&](int r) { return a.act_is_P ? r * a.npass + p : p * NOUT + r; };
  const float2 *Ein = static_cast<const float2 *>(a.Ein);
  const double2 *fb = static_cast<const double2 *>(a.fblk);
  const uint2 *qs = reinterpret_cast<const uint2 *>(a.qsplit) + q * a.Sq;
  double e[NOUT], v[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; o++) e[o] = v[o] = 0.0;
  for (int t = 0; t < a.Sq; t++) {
    const uint2 en = qs[t];
    const uint32_t y = en.y & 0x7fffffffu;
    float2 ein[NIN];
#pragma unroll
    for (int r = 0; r < NIN; r++) ein[r] = Ein[int64_t(en.x) * ns_in * a.Bp + lane_off(b, ns_in) + sig_in(r) * 16];
    double fm[M];
#pragma unroll
    for (int d = 0; d < M; d++) fm[d] = mag(fb[int64_t(y) * a.npsi * a.Bp + lane_off(b, a.npsi) + a.psi_of_pos[d] * 16]);
    // float block copies: |F~_s(x)| of the stored previous stage
    double xm[NIN];
#pragma unroll
    for (int r = 0; r < NIN; r++) xm[r] = 0.0;
    if (a.fb32) {
      const float2 *Fp = static_cast<const float2 *>(a.Fprev);
#pragma unroll
      for (int r = 0; r < NIN; r++)
        xm[r] = mag(Fp[int64_t(en.x) * ns_in * a.Bp + spin_off(b, ns_in, sig_in(r), a.paired_prev)]);
    }
#pragma unroll
    for (int in = 0; in < (1 << M); in++) {
      if (popc_e(in) != K) continue;
      const int ri = rank_e(in);
#pragma unroll
      for (int d = 0; d < M; d++) {
        if ((in >> d) & 1) continue;
        const int ro = rank_e(in | (1 << d));
        e[ro] = fma(double(ein[ri].x), fm[d], e[ro]);
        const double s = double(ein[ri].y) * fm[d];
        v[ro] = fma(s, s, v[ro]);
        const double t = U_F32 * xm[ri] * fm[d];   // zero unless a.fb32
        e[ro] += t;
        v[ro] = fma(t, t / 3.0, v[ro]);
      }
    }
  }
  const float2 *F = static_cast<const float2 *>(a.F);
  const float2 *H = static_cast<const float2 *>(a.H);
  float2 *Eout = static_cast<float2 *>(a.Eout);
#pragma unroll
  for (int o = 0; o < NOUT; o++) {
    const double m = mag(F[q * ns_out * a.Bp + spin_off(b, ns_out, sig_out(o), a.paired_F)]);
    double ee = e[o] + U_F32 * m;
    double vv = v[o] + U_F32 * U_F32 * m * m / 3.0;
    // a two-phase step also rounded its partials to float before adding them
    for (int j = 0; j < a.nh; j++) {
      const double mh = mag(H[j * a.hstride + q * ns_out * a.Bp + lane_off(b, ns_out) + sig_out(o) * 16]);
      ee += U_F32 * mh;
      vv += U_F32 * U_F32 * mh * mh / 3.0;
    }
    Eout[q * ns_out * a.Bp + lane_off(b, ns_out) + sig_out(o) * 16] = make_float2(float(ee), float(sqrt(vv)));
  }
}

// Final sum: out[b][delta][alpha] = (S_C, E_C) (see the top of the file).
__global__ __launch_bounds__(64) void err_final_kernel(ErrFinalArgs a) {
  const int64_t b = blockIdx.z * 64 + threadIdx.x;
  const int delta = blockIdx.y;
  const int alpha = a.diag ? delta : int(blockIdx.x);
  const float2 *E = static_cast<const float2 *>(a.E);
  const int64_t off = lane_off(b, a.n_delta) + delta * 16;
  const int64_t rowstride = int64_t(a.n_delta) * a.Bp;
  double eb = 0.0, vv = 0.0;
  for (int64_t i = a.crow[alpha]; i < a.crow[alpha + 1]; i++) {
    const float2 x = E[int64_t(a.ccol[i]) * rowstride + off];
    const double c = fabs(a.cval[i]);
    eb = fma(c, double(x.x), eb);
    const double s = c * double(x.y);
    vv = fma(s, s, vv);
  }
  if (b < a.B) {
    const int e = a.A * a.lane_exp[b];
    const int64_t oi = a.diag ? b * a.n_delta + delta : (b * a.n_delta + delta) * a.n_alpha + alpha;
    reinterpret_cast<double2 *>(a.err)[oi] =
        make_double2(ldexp(sqrt(vv) * a.inv_fact, e), ldexp(eb * a.inv_fact, e));
  }
}

// Projected correlator: the bound adds, the variance adds over the sink sets.
__global__ __launch_bounds__(256) void err_project_kernel(const double2 *part, double2 *out, int64_t B, int n_delta) {
  const int64_t b = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (b >= B) return;
  double s2 = 0.0, e = 0.0;
  for (int d = 0; d < n_delta; d++) {
    const double2 v = part[b * n_delta + d];
    s2 = fma(v.x, v.x, s2);
    e += v.y;
  }
  out[b] = make_double2(sqrt(s2), e);
}

__global__ __launch_bounds__(256) void zero_kernel(double *p, int64_t n) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

hipError_t launch_err_stage0(const ErrStageArgs &a, hipStream_t s) {
  const int64_t ncomp = a.nq_out * a.ns_out;
  const unsigned gy = unsigned(ncomp < 65535 ? ncomp : 65535);
  const unsigned gz = unsigned((ncomp + gy - 1) / gy);
  hipLaunchKernelGGL(err_stage0_kernel, dim3(unsigned((a.Bp + 255) / 256), gy, gz), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int M, int K>
static hipError_t launch_err_mk(const ErrStageArgs &a, hipStream_t s) {
  const int64_t items = a.nq_out * a.npass;
  if (!grid_x_fits(items, 64)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((err_stage_kernel<M, K>), dim3(unsigned(items), unsigned(a.Bp / 64)), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_err_stage(const ErrStageArgs &a, hipStream_t s) {
#define MB_CASE(m, k) \
  if (a.M == m && a.K == k) return launch_err_mk<m, k>(a, s);
  MB_CASE(1, 0)
  MB_CASE(2, 0) MB_CASE(2, 1)
  MB_CASE(3, 0) MB_CASE(3, 1) MB_CASE(3, 2)
  MB_CASE(4, 0) MB_CASE(4, 1) MB_CASE(4, 2) MB_CASE(4, 3)
  MB_CASE(5, 0) MB_CASE(5, 1) MB_CASE(5, 2) MB_CASE(5, 3) MB_CASE(5, 4)
  MB_CASE(6, 0) MB_CASE(6, 1) MB_CASE(6, 2) MB_CASE(6, 3) MB_CASE(6, 4) MB_CASE(6, 5)
#undef MB_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_err_final(const ErrFinalArgs &a, hipStream_t s) {
  dim3 grid(unsigned(a.diag ? 1 : a.n_alpha), unsigned(a.n_delta), unsigned(a.Bp / 64));
  hipLaunchKernelGGL(err_final_kernel, grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_err_project(const double *part, double *out, int64_t B, int n_delta, hipStream_t s) {
  hipLaunchKernelGGL(err_project_kernel, dim3(unsigned((B + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const double2 *>(part), reinterpret_cast<double2 *>(out), B, n_delta);
  return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace mb
