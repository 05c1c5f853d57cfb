// FP32 coupling product fused with the Spring-Ising update (gfx950).
//
// One launch performs one iteration of Eq. (8): F = J.Q (the point
// convolution of Fig. 3, a dense N x N by N x R product) on the FP32 matrix
// cores, and the epilogue applies the update of q and p, the walls and the
// zeta_n / Delta_n weights while F is still in the accumulators.  F never
// reaches memory.
//
// Layout: J is [n_pad][n_pad] (symmetric, so row i of J is also column i),
// Q and P are [r_pad][n_pad] (replica-major).  Both GEMM operands are
// therefore contiguous along the contraction index: the tile loop stages a
// BM x 32 slab of J and a BN x 32 slab of Q through LDS per iteration and
// the waves read them with 128-bit LDS loads.
//
// MFMA used: v_mfma_f32_16x16x4_f32.  For one 16x16 block, lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; the result D[4*(l/16)+v][l%16] lands in
// accumulator element v.  Four consecutive MFMAs consume 16 contraction
// indices; lane group g = l/16 owns indices kk+4g .. kk+4g+3 (one 128-bit
// LDS read per operand), MFMA s using the s-th of them.  Every index is
// summed exactly once, so this is only a permutation of the contraction.
#include "si_internal.h"

namespace si {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int BM_, int BN_, int WM_, int WN_>
struct F32Cfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
  static constexpr int BK = 32;
  static constexpr int LDK = BK + 4;  // padded LDS row: conflict-free 128-bit reads
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / 16, TN = WTN / 16;
  static constexpr int NT = 256;
  static constexpr int A_F4 = BM * BK / 4 / NT;  // float4 loads per thread
  static constexpr int B_F4 = BN * BK / 4 / NT;
  static_assert(WM * WN == 4, "four waves per workgroup");
  static_assert(TM >= 1 && TN >= 1 && WTM % 16 == 0 && WTN % 16 == 0, "wave tile");
  static_assert(A_F4 >= 1 && B_F4 >= 1, "slab loads");
  static constexpr int LDS_FLOATS = 2 * (BM + BN) * LDK;
};

__device__ __forceinline__ float sign_pm1(float x) { return x < 0.f ? -1.f : 1.f; }

// Accumulate acc += J[m0:m0+BM, :] . X[n0:n0+BN, :]^T over k in [0, K).
// SIGN_B replaces each X element by sign(x) while staging (energy readout).
template <class C, bool SIGN_B>
__device__ __forceinline__ void f32_mainloop(const float *__restrict__ A,
                                             const float *__restrict__ B, int ld, int K,
                                             int m0, int n0, floatx4 (&acc)[C::TM][C::TN],
                                             float *smem) {
  float *As = smem;                          // [2][BM][LDK]
  float *Bs = smem + 2 * C::BM * C::LDK;     // [2][BN][LDK]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  const int lrow = lane & 15, lk = (lane >> 4) * 4;

#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  floatx4 ra[C::A_F4], rb[C::B_F4];
  const float *ga = A + (size_t)(m0 + (tid >> 3)) * ld + (tid & 7) * 4;
  const float *gb = B + (size_t)(n0 + (tid >> 3)) * ld + (tid & 7) * 4;
  constexpr int ROWS_PER_PASS = C::NT / 8;  // 32 rows of 32 floats per pass
  float *as_st = As + (tid >> 3) * C::LDK + (tid & 7) * 4;
  float *bs_st = Bs + (tid >> 3) * C::LDK + (tid & 7) * 4;
#define SI_GLOAD(k0)                                                                    \
  {                                                                                     \
    _Pragma("unroll") for (int f = 0; f < C::A_F4; ++f) ra[f] =                         \
        *reinterpret_cast<const floatx4 *>(ga + (size_t)f * ROWS_PER_PASS * ld + (k0)); \
    _Pragma("unroll") for (int f = 0; f < C::B_F4; ++f) {                               \
      floatx4 v = *reinterpret_cast<const floatx4 *>(gb + (size_t)f * ROWS_PER_PASS * ld + (k0)); \
      if (SIGN_B) {                                                                     \
        v[0] = sign_pm1(v[0]); v[1] = sign_pm1(v[1]); v[2] = sign_pm1(v[2]); v[3] = sign_pm1(v[3]); \
      }                                                                                 \
      rb[f] = v;                                                                        \
    }                                                                                   \
  }
#define SI_SSTORE(buf)                                                                  \
  {                                                                                     \
    _Pragma("unroll") for (int f = 0; f < C::A_F4; ++f) *reinterpret_cast<floatx4 *>(   \
        as_st + (buf) * C::BM * C::LDK + f * ROWS_PER_PASS * C::LDK) = ra[f];           \
    _Pragma("unroll") for (int f = 0; f < C::B_F4; ++f) *reinterpret_cast<floatx4 *>(   \
        bs_st + (buf) * C::BN * C::LDK + f * ROWS_PER_PASS * C::LDK) = rb[f];           \
  }

  const int nk = K / C::BK;
  SI_GLOAD(0);
  SI_SSTORE(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) SI_GLOAD((kt + 1) * C::BK);
    const float *as = As + buf * C::BM * C::LDK + (wy * C::WTM + lrow) * C::LDK + lk;
    const float *bs = Bs + buf * C::BN * C::LDK + (wx * C::WTN + lrow) * C::LDK + lk;
#pragma unroll
    for (int kk = 0; kk < C::BK; kk += 16) {
      floatx4 a[C::TM], b[C::TN];
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
        a[i] = *reinterpret_cast<const floatx4 *>(as + i * 16 * C::LDK + kk);
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
        b[j] = *reinterpret_cast<const floatx4 *>(bs + j * 16 * C::LDK + kk);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
          for (int j = 0; j < C::TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) SI_SSTORE(buf ^ 1);
    __syncthreads();
  }
#undef SI_GLOAD
#undef SI_SSTORE
}

// Eq. (8) + walls for one element.  f is sum_j J_ij q_j (+ h_i).
template <int ORDER, int WALL>
__device__ __forceinline__ void update(float q, float p, float f, float dt, float zeta,
                                       float k, float inv_m, float qmax, float pmax,
                                       float &qn, float &pn) {
  const float c = dt * inv_m;
  // force of Eq. (4) with q0 = 0, coupling weighted by zeta_n
  const float force = fmaf(zeta, f, -k * q);
  const float v = fmaf(dt, force, p);
  pn = fminf(fmaxf(v, -pmax), pmax);
  float u;
  if (ORDER == SI_ORDER_PAPER)
    u = fmaf(c, p, q);   // q(n+1) = q(n) + (Delta/m) p(n)
  else
    u = fmaf(c, pn, q);  // symplectic variant: moves with the new p
  qn = fminf(fmaxf(u, -qmax), qmax);
  if (WALL == SI_WALL_INELASTIC && fabsf(u) > qmax) pn = 0.f;
}

template <class C, int ORDER, int WALL>
__global__ __launch_bounds__(256) void step_f32_kernel(StepArgs a) {
  __shared__ __attribute__((aligned(16))) float smem[C::LDS_FLOATS];
  const int m0 = blockIdx.x * C::BM;
  const int n0 = blockIdx.y * C::BN;
  floatx4 acc[C::TM][C::TN];
  f32_mainloop<C, false>(a.J, a.q_in, a.ld, a.n_pad, m0, n0, acc, smem);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  const float dt = a.dt[a.t], zeta = a.zeta[a.t];
#pragma unroll
  for (int i = 0; i < C::TM; ++i) {
    const int row = m0 + wy * C::WTM + i * 16 + (lane >> 4) * 4;
    float4 h4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a.h) h4 = *reinterpret_cast<const float4 *>(a.h + row);
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int col = n0 + wx * C::WTN + j * 16 + (lane & 15);
      const size_t off = (size_t)col * a.ld + row;
      const float4 q4 = *reinterpret_cast<const float4 *>(a.q_in + off);
      const float4 p4 = *reinterpret_cast<const float4 *>(a.p_in + off);
      float4 qn, pn;
      update<ORDER, WALL>(q4.x, p4.x, acc[i][j][0] + h4.x, dt, zeta, a.k, a.inv_m, a.qmax, a.pmax, qn.x, pn.x);
      update<ORDER, WALL>(q4.y, p4.y, acc[i][j][1] + h4.y, dt, zeta, a.k, a.inv_m, a.qmax, a.pmax, qn.y, pn.y);
      update<ORDER, WALL>(q4.z, p4.z, acc[i][j][2] + h4.z, dt, zeta, a.k, a.inv_m, a.qmax, a.pmax, qn.z, pn.z);
      update<ORDER, WALL>(q4.w, p4.w, acc[i][j][3] + h4.w, dt, zeta, a.k, a.inv_m, a.qmax, a.pmax, qn.w, pn.w);
      *reinterpret_cast<float4 *>(a.q_out + off) = qn;
      *reinterpret_cast<float4 *>(a.p_out + off) = pn;
    }
  }
}

TileShape tile_shape(int32_t tile) {
  switch (tile) {
    case TILE_F32_64x128: return {64, 128, "step_f32_64x128"};
    case TILE_F32_64x64: return {64, 64, "step_f32_64x64"};
    case TILE_F32_32x32: return {32, 32, "step_f32_32x32"};
    case TILE_F32_128x64: return {128, 64, "step_f32_128x64"};
    case TILE_F32_128x128: return {128, 128, "step_f32_128x128"};
    case TILE_F32_32x64: return {32, 64, "step_f32_32x64"};
    default: return {0, 0, "invalid"};
  }
}

template <class C>
static hipError_t launch_cfg(const StepArgs &a, hipStream_t s) {
  if (a.n_pad % C::BM || a.r_pad % C::BN || a.n_pad % C::BK) return hipErrorInvalidValue;
  dim3 grid(a.n_pad / C::BM, a.r_pad / C::BN), block(C::NT);
  const int sel = a.order * 2 + a.wall;
  switch (sel) {
    case 0: step_f32_kernel<C, SI_ORDER_PAPER, SI_WALL_CLAMP><<<grid, block, 0, s>>>(a); break;
    case 1: step_f32_kernel<C, SI_ORDER_PAPER, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(a); break;
    case 2: step_f32_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_CLAMP><<<grid, block, 0, s>>>(a); break;
    case 3: step_f32_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step_f32(int32_t tile, const StepArgs &a, hipStream_t s) {
  switch (tile) {
    case TILE_F32_64x128: return launch_cfg<F32Cfg<64, 128, 2, 2>>(a, s);
    case TILE_F32_64x64: return launch_cfg<F32Cfg<64, 64, 2, 2>>(a, s);
    case TILE_F32_32x32: return launch_cfg<F32Cfg<32, 32, 2, 2>>(a, s);
    case TILE_F32_128x64: return launch_cfg<F32Cfg<128, 64, 2, 2>>(a, s);
    case TILE_F32_128x128: return launch_cfg<F32Cfg<128, 128, 2, 2>>(a, s);
    case TILE_F32_32x64: return launch_cfg<F32Cfg<32, 64, 2, 2>>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Real-valued energy: G = J.sign(Q) in FP32 (each product is +-J_ij, exact),
// then per replica the partial sum over this workgroup's 64 rows of
// s_i (G_i + 2 h_i).  E = -1/2 sum_i s_i (G_i + 2 h_i) = Eq. (1).
// ---------------------------------------------------------------------------
using ECfg = F32Cfg<64, 64, 2, 2>;

__global__ __launch_bounds__(256) void energy_f32_partial_kernel(const float *J, const float *q,
                                                                 const float *h, float *part,
                                                                 int ld, int r_pad) {
  __shared__ __attribute__((aligned(16))) float smem[ECfg::LDS_FLOATS];
  __shared__ float red[ECfg::WM][ECfg::BN];
  const int m0 = blockIdx.x * ECfg::BM;
  const int n0 = blockIdx.y * ECfg::BN;
  floatx4 acc[ECfg::TM][ECfg::TN];
  f32_mainloop<ECfg, true>(J, q, ld, ld, m0, n0, acc, smem);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wy = wave / ECfg::WN, wx = wave % ECfg::WN;
#pragma unroll
  for (int j = 0; j < ECfg::TN; ++j) {
    const int lcol = wx * ECfg::WTN + j * 16 + (lane & 15);
    float c = 0.f;
#pragma unroll
    for (int i = 0; i < ECfg::TM; ++i) {
      const int row = m0 + wy * ECfg::WTM + i * 16 + (lane >> 4) * 4;
      const float4 q4 = *reinterpret_cast<const float4 *>(q + (size_t)(n0 + lcol) * ld + row);
      float4 h4 = make_float4(0.f, 0.f, 0.f, 0.f);
      if (h) h4 = *reinterpret_cast<const float4 *>(h + row);
      c += sign_pm1(q4.x) * (acc[i][j][0] + 2.f * h4.x);
      c += sign_pm1(q4.y) * (acc[i][j][1] + 2.f * h4.y);
      c += sign_pm1(q4.z) * (acc[i][j][2] + 2.f * h4.z);
      c += sign_pm1(q4.w) * (acc[i][j][3] + 2.f * h4.w);
    }
    c += __shfl_xor(c, 16);
    c += __shfl_xor(c, 32);
    if (lane < 16) red[wy][lcol] = c;
  }
  __syncthreads();
  if (threadIdx.x < ECfg::BN) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < ECfg::WM; ++w) s += red[w][threadIdx.x];
    part[(size_t)blockIdx.x * r_pad + n0 + threadIdx.x] = s;
  }
}

__global__ void energy_f32_finalize_kernel(const float *part, int n_tiles, int r, int r_pad,
                                           double *e) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= r) return;
  // Neumaier-compensated FP32 sum over the row tiles, in fixed order.
  float s = 0.f, comp = 0.f;
  for (int t = 0; t < n_tiles; ++t) {
    const float x = part[(size_t)t * r_pad + col];
    const float y = s + x;
    if (fabsf(s) >= fabsf(x))
      comp += (s - y) + x;
    else
      comp += (x - y) + s;
    s = y;
  }
  e[col] = -0.5 * ((double)s + (double)comp);
}

hipError_t launch_energy_f32_partial(const float *J, const float *q, const float *h, float *part,
                                     int32_t n_pad, int32_t r_pad, hipStream_t s) {
  if (n_pad % ECfg::BM || r_pad % ECfg::BN) return hipErrorInvalidValue;
  dim3 grid(n_pad / ECfg::BM, r_pad / ECfg::BN);
  energy_f32_partial_kernel<<<grid, 256, 0, s>>>(J, q, h, part, n_pad, r_pad);
  return hipGetLastError();
}

hipError_t launch_energy_f32_finalize(const float *part, int32_t n_tiles, int32_t r,
                                      int32_t r_pad, double *e_real, hipStream_t s) {
  energy_f32_finalize_kernel<<<(r + 255) / 256, 256, 0, s>>>(part, n_tiles, r, r_pad, e_real);
  return hipGetLastError();
}

}  // namespace si
