// Exact Ising energy (Eq. 1) of caller-owned positions and couplings that
// allocates nothing: for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops).  Its only scratch memory is the
// file-scope array below, one copy per GPU, held until the process ends.
//
// Energy of s = sign(x) (+1 for x >= 0, also -0.0) for every replica r:
//   E_r = -1/2 sum_i s_i sum_j J_ij s_j     (= -sum_{i<j} J_ij s_i s_j for a
//                                            symmetric, zero-diagonal J)
// G = J.S runs on the int8 matrix cores (v_mfma_i32_16x16x64_i8) with int32
// accumulation, exact for integer |J_ij| <= 127; the couplings are converted
// to int8 while they are staged into LDS, so J is read in the caller's FP32
// layout (n x n, unpadded) and the positions in theirs (r x n, unpadded).
// Per-replica sums of s_i G_i go to 64-bit integer atomics, whose result
// does not depend on their order.
#include <atomic>

#include "si_internal.h"

namespace si {

typedef int intx4 __attribute__((ext_vector_type(4)));

namespace {
// scratch: [0, NOALLOC_R_MAX) per-replica 64-bit sums; [NOALLOC_R_MAX] the
// flag of couplings outside the exact int8 range.
constexpr int NOALLOC_R_MAX = 65536;
constexpr int NB = 64, NK = 64, NLDK = NK + 16;  // tile 64 x 64, slab 64 deep (bytes)
}  // namespace

static __device__ __align__(256) unsigned long long scratch[NOALLOC_R_MAX + 32];

// One element of the staged slabs: J_ij as int8 (flagging values that are
// not integers in [-127, 127]) and sign(x) as int8; zero outside the matrix.
__device__ __forceinline__ int8_t j_to_i8(float v, unsigned &bad) {
  const bool ok = v == rintf(v) && fabsf(v) <= 127.f;
  bad |= ok ? 0u : 1u;
  return ok ? (int8_t)(int)v : (int8_t)0;
}

__global__ __launch_bounds__(256) void noalloc_energy_kernel(const float *__restrict__ J,
                                                             const float *__restrict__ x, int n,
                                                             int r,
                                                             unsigned long long *__restrict__ sc) {
  __shared__ __attribute__((aligned(16))) int8_t As[NB * NLDK];
  __shared__ __attribute__((aligned(16))) int8_t Bs[NB * NLDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;  // 2 x 2 waves of 32 x 32
  const int m0 = blockIdx.x * NB, n0 = blockIdx.y * NB;
  const int lrow = lane & 15, lk = (lane >> 4) * 16;
  unsigned bad = 0;

  intx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = intx4{0, 0, 0, 0};

  // staging: element e of this thread is (row idx / 64, column idx % 64) with
  // idx = e * 256 + tid, so that each wave reads 64 consecutive floats of a row
  for (int k0 = 0; k0 < n; k0 += NK) {
#pragma unroll 4
    for (int e = 0; e < NB * NK / 256; ++e) {
      const int idx = e * 256 + tid, row = idx >> 6, kk = idx & 63;
      const int gk = k0 + kk;
      const int gi = m0 + row, gr = n0 + row;
      int8_t a = 0, b = 0;
      if (gi < n && gk < n) a = j_to_i8(J[(size_t)gi * n + gk], bad);
      if (gr < r && gk < n) b = x[(size_t)gr * n + gk] < 0.f ? (int8_t)-1 : (int8_t)1;
      As[row * NLDK + kk] = a;
      Bs[row * NLDK + kk] = b;
    }
    __syncthreads();
    intx4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const intx4 *>(&As[(wy * 32 + i * 16 + lrow) * NLDK + lk]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const intx4 *>(&Bs[(wx * 32 + j * 16 + lrow) * NLDK + lk]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  if (bad) atomicOr(sc + NOALLOC_R_MAX, 1ull);

  // sum_i s_i G_i over this tile's rows for each replica column
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = n0 + wx * 32 + j * 16 + (lane & 15);
    int c = 0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wy * 32 + i * 16 + (lane >> 4) * 4 + v;
        if (row < n && col < r) c += (x[(size_t)col * n + row] < 0.f ? -1 : 1) * acc[i][j][v];
      }
    c += __shfl_xor(c, 16);
    c += __shfl_xor(c, 32);
    if (lane < 16 && col < r) atomicAdd(sc + col, (unsigned long long)(long long)c);
  }
}

__global__ void noalloc_clear_kernel(unsigned long long *sc, int r) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < r; i += gridDim.x * blockDim.x)
    sc[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[NOALLOC_R_MAX] = 0ull;
}

// e_r = -(sum / 2); INT32_MIN when a coupling was outside the exact range or
// the energy does not fit in int32.
__global__ void noalloc_finalize_kernel(const unsigned long long *sc, int r, int32_t *e) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= r) return;
  const long long s = (long long)sc[col];
  const long long v = -(s / 2);
  const bool ok = sc[NOALLOC_R_MAX] == 0ull && v >= INT32_MIN + 1LL && v <= INT32_MAX;
  e[col] = ok ? (int32_t)v : INT32_MIN;
}

int32_t noalloc_r_max() { return NOALLOC_R_MAX; }

// Device address of this GPU's scratch array, looked up once per device.
hipError_t noalloc_scratch_ptr(int device, void **ptr) {
  static void *table[64] = {nullptr};
  static std::atomic<int> lock{0};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  while (lock.exchange(1, std::memory_order_acquire)) {
  }
  hipError_t e = hipSuccess;
  if (!table[device]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) table[device] = p;
  }
  *ptr = table[device];
  lock.store(0, std::memory_order_release);
  return e;
}

hipError_t launch_noalloc_energy(const float *J, const float *x, int32_t n, int32_t r,
                                 int32_t *e_int, void *sc_ptr, hipStream_t s) {
  if (n < 1 || r < 1 || r > NOALLOC_R_MAX || !sc_ptr) return hipErrorInvalidValue;
  auto *sc = static_cast<unsigned long long *>(sc_ptr);
  const int cb = (r + 255) / 256 < 256 ? (r + 255) / 256 : 256;
  noalloc_clear_kernel<<<cb, 256, 0, s>>>(sc, r);
  dim3 grid((n + NB - 1) / NB, (r + NB - 1) / NB);
  noalloc_energy_kernel<<<grid, 256, 0, s>>>(J, x, n, r, sc);
  noalloc_finalize_kernel<<<(r + 255) / 256, 256, 0, s>>>(sc, r, e_int);
  return hipGetLastError();
}

}  // namespace si
