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
// BM x BK slab of J and a BN x BK slab of Q through LDS per iteration and
// the waves read them with 128-bit LDS loads.
//
// Two MFMA shapes are used (MB = block edge):
//   MB = 16: v_mfma_f32_16x16x4_f32.  Lane l supplies A[l%16][l/16] and
//            B[l/16][l%16]; result D[4(l/16)+v][l%16] in accumulator v < 4.
//   MB = 32: v_mfma_f32_32x32x2_f32.  Lane l supplies A[l%32][l/32] and
//            B[l/32][l%32]; result D[8(v/4)+4(l/32)+v%4][l%32], v < 16.
// In both, lane group g = l/MB reads the four contraction indices
// kk+4g .. kk+4g+3 with one 128-bit LDS load per operand and MFMA s uses the
// s-th of them; each index is summed exactly once, in increasing kk order,
// so the permutation only changes which lane holds which index.
#include "si_internal.h"

namespace si {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int MB>
struct MfmaF32;
template <>
struct MfmaF32<16> {
  using acc_t = floatx4;
  static constexpr int NACC = 4;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaF32<32> {
  using acc_t = floatx16;
  static constexpr int NACC = 16;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};

template <int BM_, int BN_, int WM_, int WN_, int MB_, int BK_, int STAGES_ = 0, int KS_ = 1>
struct F32Cfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, MB = MB_, BK = BK_;
  // KS independent accumulators per output block, alternating over the
  // four MFMAs of each contraction step (shorter dependency chains) and
  // added at the end (direct-to-LDS pipeline only).
  static constexpr int KS = KS_;
  // STAGES = 0: slabs staged through registers into a padded double buffer.
  // STAGES >= 3: slabs copied straight into an LDS ring of STAGES slots by
  // direct-to-LDS loads, STAGES - 1 slabs in flight.
  static constexpr int STAGES = STAGES_;
  static constexpr int LDK = BK + 4;  // padded LDS row: conflict-free 128-bit reads
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / MB, TN = WTN / MB;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int KSTEP = 64 / MB * 4;  // contraction indices per LDS read step
  static constexpr int F4_PER_ROW = BK / 4;
  static constexpr int ROWS_PER_PASS = NT / F4_PER_ROW;
  static constexpr int A_F4 = BM * BK / 4 / NT;  // float4 loads per thread
  static constexpr int B_F4 = BN * BK / 4 / NT;
  using M = MfmaF32<MB>;
  using acc_t = typename M::acc_t;
  static_assert(TM >= 1 && TN >= 1 && WTM % MB == 0 && WTN % MB == 0, "wave tile");
  static_assert(A_F4 >= 1 && B_F4 >= 1 && BM * BK / 4 % NT == 0 && BN * BK / 4 % NT == 0,
                "slab loads");
  static_assert(BK % KSTEP == 0, "slab depth");
  static constexpr int LDS_FLOATS = STAGES ? STAGES * (BM + BN) * BK : 2 * (BM + BN) * LDK;
};

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

// Wait until at most N vector-memory operations of this wave are in flight,
// then synchronise the workgroup.  The memory clobber keeps every LDS access
// on its side of the barrier.
template <int N>
__device__ __forceinline__ void wait_vm_barrier() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

// Direct-to-LDS pipeline.  Each slab row of BK floats is stored unpadded;
// its 16-byte chunk c sits at position c ^ (row & 7), which spreads the
// 128-bit fragment reads of eight consecutive rows over distinct banks.  A
// direct-to-LDS load writes 16 bytes per lane at consecutive addresses, so
// lane L fetches the global chunk that belongs at its destination.
template <class C>
__device__ __forceinline__ void f32_mainloop_dma(const float *__restrict__ A,
                                                 const float *__restrict__ B, int ld, int K,
                                                 int m0, int n0,
                                                 typename C::acc_t (&acc)[C::TM][C::TN],
                                                 float *smem) {
  constexpr int S = C::STAGES;
  constexpr int NW = C::NT / 64;
  constexpr int CH = C::BK / 4;            // 16-byte chunks per row
  constexpr int RPD = 64 / CH;             // rows written by one wave-wide load
  constexpr int A_DMA = C::BM / RPD / NW;  // loads per wave per slab
  constexpr int B_DMA = C::BN / RPD / NW;
  constexpr int L = A_DMA + B_DMA;
  constexpr int SLAB = (C::BM + C::BN) * C::BK;  // floats per ring slot
  static_assert(A_DMA >= 1 && B_DMA >= 1 && C::BM % (RPD * NW) == 0 && C::BN % (RPD * NW) == 0,
                "direct-to-LDS slab split");
  static_assert((S - 2) * L <= 63, "vmcnt range");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  const int lrow = lane % C::MB, lk = (lane / C::MB) * 4;
  const int drow = lane / CH, dch = lane % CH;

  typename C::acc_t part[C::TM][C::TN][C::KS];
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j)
#pragma unroll
      for (int u = 0; u < C::KS; ++u)
#pragma unroll
        for (int v = 0; v < C::M::NACC; ++v) part[i][j][u][v] = 0.f;

  // global source of this lane for each of its loads (k offset added later)
  const float *srcA[A_DMA];
  const float *srcB[B_DMA];
#pragma unroll
  for (int d = 0; d < A_DMA; ++d) {
    const int row = (wave * A_DMA + d) * RPD + drow;
    srcA[d] = A + (size_t)(m0 + row) * ld + ((dch ^ (row & 7)) * 4);
  }
#pragma unroll
  for (int d = 0; d < B_DMA; ++d) {
    const int row = (wave * B_DMA + d) * RPD + drow;
    srcB[d] = B + (size_t)(n0 + row) * ld + ((dch ^ (row & 7)) * 4);
  }
  auto issue = [&](int kt, int slot) {
    float *st = smem + slot * SLAB;
#pragma unroll
    for (int d = 0; d < A_DMA; ++d)
      __builtin_amdgcn_global_load_lds((gbl_void_t *)(srcA[d] + kt * C::BK),
                                       (lds_void_t *)(st + (wave * A_DMA + d) * RPD * C::BK), 16,
                                       0, 0);
#pragma unroll
    for (int d = 0; d < B_DMA; ++d)
      __builtin_amdgcn_global_load_lds(
          (gbl_void_t *)(srcB[d] + kt * C::BK),
          (lds_void_t *)(st + (C::BM + (wave * B_DMA + d) * RPD) * C::BK), 16, 0, 0);
  };

  const int nk = K / C::BK;
#pragma unroll
  for (int s = 0; s < S - 1; ++s)
    if (s < nk) issue(s, s);
  const int ra = wy * C::WTM + lrow, rb = wx * C::WTN + lrow;  // fragment rows (i = j = 0)
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + S - 1 < nk) {
      wait_vm_barrier<(S - 2) * L>();
      issue(kt + S - 1, (kt + S - 1) % S);
    } else {
      wait_vm_barrier<0>();
    }
    const float *st = smem + (kt % S) * SLAB;
    // fragments of the next contraction step are read while the MFMAs of
    // the current one run
    floatx4 a[2][C::TM], b[2][C::TN];
    auto frag = [&](int kk, floatx4 (&fa)[C::TM], floatx4 (&fb)[C::TN]) {
      const int ch = (kk + lk) >> 2;
#pragma unroll
      for (int i = 0; i < C::TM; ++i) {
        const int r = ra + i * C::MB;
        fa[i] = *reinterpret_cast<const floatx4 *>(st + r * C::BK + ((ch ^ (r & 7)) << 2));
      }
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int r = rb + j * C::MB;
        fb[j] = *reinterpret_cast<const floatx4 *>(st + (C::BM + r) * C::BK + ((ch ^ (r & 7)) << 2));
      }
    };
    frag(0, a[0], b[0]);
#pragma unroll
    for (int kk = 0; kk < C::BK; kk += C::KSTEP) {
      const int cur = (kk / C::KSTEP) & 1;
      if (kk + C::KSTEP < C::BK) frag(kk + C::KSTEP, a[cur ^ 1], b[cur ^ 1]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
          for (int j = 0; j < C::TN; ++j)
            part[i][j][s % C::KS] =
                C::M::mma(a[cur][i][s], b[cur][j][s], part[i][j][s % C::KS]);
    }
  }
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      acc[i][j] = part[i][j][0];
#pragma unroll
      for (int u = 1; u < C::KS; ++u) acc[i][j] += part[i][j][u];
    }
  // all waves done reading the ring before the caller reuses LDS
  wait_vm_barrier<0>();
}

__device__ __forceinline__ float sign_pm1(float x) { return x < 0.f ? -1.f : 1.f; }

// Accumulate acc += J[m0:m0+BM, :] . X[n0:n0+BN, :]^T over k in [0, K).
// SIGN_B replaces each X element by sign(x) while staging (energy readout).
template <class C, bool SIGN_B>
__device__ __forceinline__ void f32_mainloop(const float *__restrict__ A,
                                             const float *__restrict__ B, int ld, int K,
                                             int m0, int n0,
                                             typename C::acc_t (&acc)[C::TM][C::TN],
                                             float *smem) {
  float *As = smem;                          // [2][BM][LDK]
  float *Bs = smem + 2 * C::BM * C::LDK;     // [2][BN][LDK]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  const int lrow = lane % C::MB, lk = (lane / C::MB) * 4;

#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j)
#pragma unroll
      for (int v = 0; v < C::M::NACC; ++v) acc[i][j][v] = 0.f;

  floatx4 ra[C::A_F4], rb[C::B_F4];
  const int srow = tid / C::F4_PER_ROW, sc4 = (tid % C::F4_PER_ROW) * 4;
  const float *ga = A + (size_t)(m0 + srow) * ld + sc4;
  const float *gb = B + (size_t)(n0 + srow) * ld + sc4;
  float *as_st = As + srow * C::LDK + sc4;
  float *bs_st = Bs + srow * C::LDK + sc4;
#define SI_GLOAD(k0)                                                                      \
  {                                                                                       \
    _Pragma("unroll") for (int f = 0; f < C::A_F4; ++f) ra[f] =                           \
        *reinterpret_cast<const floatx4 *>(ga + (size_t)f * C::ROWS_PER_PASS * ld + (k0));\
    _Pragma("unroll") for (int f = 0; f < C::B_F4; ++f) {                                 \
      floatx4 v = *reinterpret_cast<const floatx4 *>(gb + (size_t)f * C::ROWS_PER_PASS * ld + (k0)); \
      if (SIGN_B) {                                                                       \
        v[0] = sign_pm1(v[0]); v[1] = sign_pm1(v[1]); v[2] = sign_pm1(v[2]); v[3] = sign_pm1(v[3]); \
      }                                                                                   \
      rb[f] = v;                                                                          \
    }                                                                                     \
  }
#define SI_SSTORE(buf)                                                                    \
  {                                                                                       \
    _Pragma("unroll") for (int f = 0; f < C::A_F4; ++f) *reinterpret_cast<floatx4 *>(     \
        as_st + (buf) * C::BM * C::LDK + f * C::ROWS_PER_PASS * C::LDK) = ra[f];          \
    _Pragma("unroll") for (int f = 0; f < C::B_F4; ++f) *reinterpret_cast<floatx4 *>(     \
        bs_st + (buf) * C::BN * C::LDK + f * C::ROWS_PER_PASS * C::LDK) = rb[f];          \
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
    for (int kk = 0; kk < C::BK; kk += C::KSTEP) {
      floatx4 a[C::TM], b[C::TN];
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
        a[i] = *reinterpret_cast<const floatx4 *>(as + i * C::MB * C::LDK + kk);
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
        b[j] = *reinterpret_cast<const floatx4 *>(bs + j * C::MB * C::LDK + kk);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
#pragma unroll
          for (int j = 0; j < C::TN; ++j) acc[i][j] = C::M::mma(a[i][s], b[j][s], acc[i][j]);
    }
    if (kt + 1 < nk) SI_SSTORE(buf ^ 1);
    __syncthreads();
  }
#undef SI_GLOAD
#undef SI_SSTORE
}

// Row (within the MB x MB block) of accumulator element v for this lane.
template <int MB>
__device__ __forceinline__ int acc_row(int lane, int v) {
  return (v / 4) * 8 + (lane / MB) * 4 + (v % 4);
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
__global__ __launch_bounds__(C::NT) void step_f32_kernel(StepArgs a) {
  __shared__ __attribute__((aligned(16))) float smem[C::LDS_FLOATS];
  const int m0 = blockIdx.x * C::BM;
  const int n0 = blockIdx.y * C::BN;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  constexpr int G = C::M::NACC / 4;
  // The state this lane updates is loaded before the contraction so that
  // its latency overlaps the matrix work.
  floatx4 q4[C::TM][G][C::TN], p4[C::TM][G][C::TN], h4[C::TM][G];
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int row = m0 + wy * C::WTM + i * C::MB + g * 8 + (lane / C::MB) * 4;
      h4[i][g] = floatx4{0.f, 0.f, 0.f, 0.f};
      if (a.h) h4[i][g] = *reinterpret_cast<const floatx4 *>(a.h + row);
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int col = n0 + wx * C::WTN + j * C::MB + (lane % C::MB);
        const size_t off = (size_t)col * a.ld + row;
        q4[i][g][j] = *reinterpret_cast<const floatx4 *>(a.q_in + off);
        p4[i][g][j] = *reinterpret_cast<const floatx4 *>(a.p_in + off);
      }
    }

  typename C::acc_t acc[C::TM][C::TN];
  if constexpr (C::STAGES > 0)
    f32_mainloop_dma<C>(a.J, a.q_in, a.ld, a.n_pad, m0, n0, acc, smem);
  else
    f32_mainloop<C, false>(a.J, a.q_in, a.ld, a.n_pad, m0, n0, acc, smem);

  const float dt = a.dt[a.t], zeta = a.zeta[a.t];
#pragma unroll
  for (int i = 0; i < C::TM; ++i) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int row = m0 + wy * C::WTM + i * C::MB + g * 8 + (lane / C::MB) * 4;
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int col = n0 + wx * C::WTN + j * C::MB + (lane % C::MB);
        const size_t off = (size_t)col * a.ld + row;
        floatx4 qn, pn;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float qv, pv;
          update<ORDER, WALL>(q4[i][g][j][v], p4[i][g][j][v], acc[i][j][4 * g + v] + h4[i][g][v],
                              dt, zeta, a.k, a.inv_m, a.qmax, a.pmax, qv, pv);
          qn[v] = qv;
          pn[v] = pv;
        }
        *reinterpret_cast<floatx4 *>(a.q_out + off) = qn;
        *reinterpret_cast<floatx4 *>(a.p_out + off) = pn;
      }
    }
  }
}

// Tile table: id, BM, BN, waves (WM x WN), MFMA block edge, slab depth BK,
// LDS stages (0: register-staged double buffer; >= 3: direct-to-LDS ring).
#define SI_F32_TILES(X)                \
  X(1, 64, 128, 2, 2, 32, 32, 0, 1)    \
  X(2, 64, 64, 2, 2, 32, 32, 0, 1)        \
  X(3, 32, 32, 2, 2, 16, 32, 0, 1)        \
  X(4, 128, 64, 2, 2, 32, 32, 0, 1)       \
  X(5, 128, 128, 2, 2, 32, 32, 0, 1)      \
  X(6, 32, 64, 2, 2, 16, 32, 0, 1)        \
  X(7, 64, 128, 2, 2, 32, 64, 0, 1)       \
  X(8, 64, 128, 2, 4, 32, 32, 0, 1)       \
  X(9, 64, 64, 2, 2, 32, 64, 0, 1)        \
  X(10, 64, 128, 2, 2, 16, 32, 0, 1)      \
  X(11, 128, 128, 2, 4, 32, 32, 0, 1)     \
  X(12, 64, 64, 2, 2, 16, 32, 0, 1)       \
  X(13, 64, 64, 2, 2, 32, 32, 3, 1)       \
  X(14, 64, 64, 2, 2, 32, 32, 4, 1)       \
  X(15, 64, 64, 2, 2, 32, 64, 3, 1)       \
  X(16, 64, 128, 2, 2, 32, 32, 4, 1)      \
  X(17, 64, 64, 2, 2, 32, 32, 6, 1)       \
  X(18, 128, 64, 2, 2, 32, 32, 4, 1)      \
  X(19, 64, 64, 2, 2, 32, 32, 4, 2)    \
  X(20, 64, 64, 2, 2, 32, 32, 4, 4)    \
  X(21, 64, 64, 2, 1, 32, 32, 4, 1)    \
  X(22, 64, 64, 2, 1, 32, 32, 4, 2)    \
  X(23, 64, 64, 2, 2, 32, 64, 3, 2)    \
  X(24, 64, 128, 2, 2, 32, 32, 4, 2)

TileShape tile_shape(int32_t tile) {
  switch (tile) {
#define SI_SHAPE(id, bm, bn, wm, wn, mb, bk, st, ks) \
  case id:                                           \
    return {bm, bn,                                  \
            "step_f32_" #bm "x" #bn "_w" #wm "x" #wn "_mfma" #mb "_k" #bk "_s" #st "_a" #ks};
    SI_F32_TILES(SI_SHAPE)
#undef SI_SHAPE
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
#define SI_LAUNCH(id, bm, bn, wm, wn, mb, bk, st, ks) \
  case id:                                            \
    return launch_cfg<F32Cfg<bm, bn, wm, wn, mb, bk, st, ks>>(a, s);
    SI_F32_TILES(SI_LAUNCH)
#undef SI_LAUNCH
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Real-valued energy: G = J.sign(Q) in FP32 (each product is +-J_ij, exact),
// then per replica the partial sum over this workgroup's 64 rows of
// s_i (G_i + 2 h_i).  E = -1/2 sum_i s_i (G_i + 2 h_i) = Eq. (1).
// ---------------------------------------------------------------------------
using ECfg = F32Cfg<64, 64, 2, 2, 32, 32>;

__global__ __launch_bounds__(256) void energy_f32_partial_kernel(const float *J, const float *q,
                                                                 const float *h, float *part,
                                                                 int ld, int r_pad) {
  __shared__ __attribute__((aligned(16))) float smem[ECfg::LDS_FLOATS];
  __shared__ float red[ECfg::WM][ECfg::BN];
  const int m0 = blockIdx.x * ECfg::BM;
  const int n0 = blockIdx.y * ECfg::BN;
  ECfg::acc_t acc[ECfg::TM][ECfg::TN];
  f32_mainloop<ECfg, true>(J, q, ld, ld, m0, n0, acc, smem);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wy = wave / ECfg::WN, wx = wave % ECfg::WN;
#pragma unroll
  for (int j = 0; j < ECfg::TN; ++j) {
    const int lcol = wx * ECfg::WTN + j * ECfg::MB + (lane % ECfg::MB);
    float c = 0.f;
#pragma unroll
    for (int i = 0; i < ECfg::TM; ++i)
#pragma unroll
      for (int g = 0; g < ECfg::M::NACC / 4; ++g) {
        const int row = m0 + wy * ECfg::WTM + i * ECfg::MB + g * 8 + (lane / ECfg::MB) * 4;
        const floatx4 q4 = *reinterpret_cast<const floatx4 *>(q + (size_t)(n0 + lcol) * ld + row);
        floatx4 h4 = {0.f, 0.f, 0.f, 0.f};
        if (h) h4 = *reinterpret_cast<const floatx4 *>(h + row);
#pragma unroll
        for (int v = 0; v < 4; ++v) c += sign_pm1(q4[v]) * (acc[i][j][4 * g + v] + 2.f * h4[v]);
      }
    for (int off = ECfg::MB; off < 64; off <<= 1) c += __shfl_xor(c, off);
    if (lane < ECfg::MB) red[wy][lcol] = c;
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
