// Device twin of synth/props.py: Philox4x32-10 counter-based propagators.
// Same definition, bit-identical values (see synth/props.py).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; r++) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ inline double gaussian_like(uint64_t seed, uint32_t stream, uint64_t n) {
  uint32_t c[4] = {uint32_t(n), uint32_t(n >> 32), stream, 0u};
  philox10(c, uint32_t(seed), uint32_t(seed >> 32));
  const double s = ((double(c[0]) + 0.5) * 0x1p-32 + (double(c[1]) + 0.5) * 0x1p-32) +
                   ((double(c[2]) + 0.5) * 0x1p-32) + ((double(c[3]) + 0.5) * 0x1p-32);
  return __dmul_rn(s - 2.0, 1.7320508075688772);
}

template <typename TO>
__global__ void props_kernel(TO *out, uint64_t seed, uint32_t stream, int64_t per_t, int T,
                             int64_t first_bt, int64_t nbt, const double *decay) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= nbt * per_t) return;
  const int64_t bt = first_bt + i / per_t;  // global (problem, t) index
  const int64_t e = bt * per_t + i % per_t;
  const double dec = decay[bt % T];
  const double re = __dmul_rn(gaussian_like(seed, stream, 2 * uint64_t(e)), dec);
  const double im = __dmul_rn(gaussian_like(seed, stream, 2 * uint64_t(e) + 1), dec);
  TO v;
  v.x = decltype(v.x)(re);
  v.y = decltype(v.y)(im);
  out[i] = v;
}

}  // namespace

extern "C" {

// Fills out[nbt][V][nsrc][12][12] with the propagators of the global
// (problem, timeslice) units first_bt .. first_bt+nbt-1 of a dataset with T
// timeslices (unit index = problem*T + t).  decay: device double [T].
// c128 != 0: complex double output, else complex float.  Returns a
// hipError_t value.
int mb_synth_props(void *out, int c128, uint64_t seed, uint32_t stream, int64_t V, int nsrc, int T,
                   int64_t first_bt, int64_t nbt, const double *decay, void *hip_stream) {
  const int64_t per_t = V * nsrc * 144;
  if (nbt <= 0 || per_t <= 0) return 0;
  // a launch covers at most 2^31 work-items (the dispatch grid size is 32-bit)
  const int64_t max_items = int64_t(1) << 31;
  if (per_t > max_items) return int(hipErrorInvalidValue);
  const int64_t units = max_items / per_t;   // whole units per launch
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  for (int64_t u0 = 0; u0 < nbt; u0 += units) {
    const int64_t nu = nbt - u0 < units ? nbt - u0 : units;
    dim3 grid(unsigned((nu * per_t + 255) / 256));
    if (c128)
      hipLaunchKernelGGL(props_kernel<double2>, grid, dim3(256), 0, s, static_cast<double2 *>(out) + u0 * per_t,
                         seed, stream, per_t, T, first_bt + u0, nu, decay);
    else
      hipLaunchKernelGGL(props_kernel<float2>, grid, dim3(256), 0, s, static_cast<float2 *>(out) + u0 * per_t,
                         seed, stream, per_t, T, first_bt + u0, nu, decay);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return int(e);
  }
  return 0;
}
}
