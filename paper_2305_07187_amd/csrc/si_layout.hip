// Staging kernels: validation of J, zero-padded packing of J and of the
// state into the device layout, and unpacking back to the caller's layout.
#include "si_internal.h"

namespace si {

__device__ __forceinline__ bool fp8_e4m3_exact(float v) {
  // e4m3 (no infinities): 1 sign, 4 exponent (bias 7), 3 mantissa bits;
  // normals 2^-6 .. 448, subnormals multiples of 2^-9.
  const float a = fabsf(v);
  if (a == 0.f) return true;
  if (!(a <= 448.f)) return false;
  if (a < 0.015625f) {  // subnormal range: a = m * 2^-9, m integer 1..7
    const float m = a * 512.f;
    return m == rintf(m);
  }
  int e;
  const float fr = frexpf(a, &e);  // a = fr * 2^e, fr in [0.5, 1)
  const float m = fr * 16.f;        // 4 significant bits
  return m == rintf(m);
}

__global__ void validate_kernel(const float *__restrict__ J, int n, int32_t *flags) {
  const int64_t total = (int64_t)n * n;
  int asym = 0, diag = 0, nonfin = 0, nonint = 0, nonfp8 = 0, nonbf16 = 0, maxabs = 0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), j = (int)(idx % n);
    const float v = J[idx];
    const float w = J[(int64_t)j * n + i];
    if (!(v == w)) asym = 1;
    if (i == j && v != 0.f) diag = 1;
    if (!isfinite(v)) {
      nonfin = 1;
      continue;
    }
    if (v != rintf(v) || fabsf(v) > 127.f)
      nonint = 1;
    else
      maxabs = max(maxabs, (int)fabsf(v));
    if (!fp8_e4m3_exact(v)) nonfp8 = 1;
    if ((__float_as_uint(v) & 0xFFFFu) != 0u) nonbf16 = 1;
  }
  if (asym) atomicOr(flags + 0, 1);
  if (diag) atomicOr(flags + 1, 1);
  if (nonfin) atomicOr(flags + 2, 1);
  if (nonint) atomicOr(flags + 3, 1);
  if (nonfp8) atomicOr(flags + 4, 1);
  if (nonbf16) atomicOr(flags + 5, 1);
  if (maxabs) atomicMax(flags + 6, maxabs);
}

__global__ void pack_matrix_kernel(const float *__restrict__ src, int n, float *__restrict__ dst,
                                   int8_t *__restrict__ dst8, int n_pad) {
  const int64_t total = (int64_t)n_pad * n_pad;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n_pad), j = (int)(idx % n_pad);
    const float v = (i < n && j < n) ? src[(int64_t)i * n + j] : 0.f;
    dst[idx] = v;
    if (dst8) dst8[idx] = (int8_t)(int)v;
  }
}

__global__ void pack_state_kernel(const float *__restrict__ src, int n, int r,
                                  float *__restrict__ dst, int n_pad, int64_t total) {
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int rr = (int)(idx / n_pad), i = (int)(idx % n_pad);
    dst[idx] = (src && rr < r && i < n) ? src[(int64_t)rr * n + i] : 0.f;
  }
}

__global__ void unpack_state_kernel(const float *__restrict__ src, int n, int r,
                                    float *__restrict__ dst, int n_pad) {
  const int64_t total = (int64_t)n * r;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int rr = (int)(idx / n), i = (int)(idx % n);
    dst[idx] = src[(int64_t)rr * n_pad + i];
  }
}

__global__ void unpack_spins_kernel(const int8_t *__restrict__ src, int n, int r,
                                    int8_t *__restrict__ dst, int n_pad) {
  const int64_t total = (int64_t)n * r;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int rr = (int)(idx / n), i = (int)(idx % n);
    dst[idx] = src[(int64_t)rr * n_pad + i];
  }
}

__global__ void pack_field_kernel(const float *__restrict__ h, int n, float *__restrict__ hf,
                                  int8_t *__restrict__ h8, int n_pad, int32_t *flags) {
  int nonint = 0, nonfin = 0, maxabs = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += gridDim.x * blockDim.x) {
    const float v = i < n ? h[i] : 0.f;
    hf[i] = v;
    if (!isfinite(v)) nonfin = 1;
    const bool integer = isfinite(v) && v == rintf(v) && fabsf(v) <= 127.f;
    if (!integer)
      nonint = 1;
    else
      maxabs = max(maxabs, (int)fabsf(v));
    h8[i] = integer ? (int8_t)(int)v : (int8_t)0;
  }
  if (nonfin) atomicOr(flags + 2, 1);
  if (nonint) atomicOr(flags + 3, 1);
  if (maxabs) atomicMax(flags + 6, maxabs);
}

static int grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  return b < 1 ? 1 : (int)b;
}

hipError_t launch_validate(const float *J, int32_t n, int32_t *flags, hipStream_t s) {
  validate_kernel<<<grid_for((int64_t)n * n), 256, 0, s>>>(J, n, flags);
  return hipGetLastError();
}

hipError_t launch_pack_matrix(const float *src, int32_t n, float *dst, int8_t *dst8,
                              int32_t n_pad, hipStream_t s) {
  pack_matrix_kernel<<<grid_for((int64_t)n_pad * n_pad), 256, 0, s>>>(src, n, dst, dst8, n_pad);
  return hipGetLastError();
}

hipError_t launch_pack_state(const float *src, int32_t n, int32_t r, float *dst, int32_t n_pad,
                             int32_t r_pad, hipStream_t s) {
  const int64_t total = (int64_t)n_pad * r_pad;
  pack_state_kernel<<<grid_for(total), 256, 0, s>>>(src, n, r, dst, n_pad, total);
  return hipGetLastError();
}

hipError_t launch_unpack_state(const float *src, int32_t n, int32_t r, float *dst,
                               int32_t n_pad, hipStream_t s) {
  unpack_state_kernel<<<grid_for((int64_t)n * r), 256, 0, s>>>(src, n, r, dst, n_pad);
  return hipGetLastError();
}

hipError_t launch_unpack_spins(const int8_t *src, int32_t n, int32_t r, int8_t *dst,
                               int32_t n_pad, hipStream_t s) {
  unpack_spins_kernel<<<grid_for((int64_t)n * r), 256, 0, s>>>(src, n, r, dst, n_pad);
  return hipGetLastError();
}

hipError_t launch_pack_field(const float *h, int32_t n, float *hf, int8_t *h8, int32_t n_pad,
                             int32_t *flags, hipStream_t s) {
  pack_field_kernel<<<grid_for(n_pad), 256, 0, s>>>(h, n, hf, h8, n_pad, flags);
  return hipGetLastError();
}

}  // namespace si
