// FP32 matrix-core GEMM machinery shared by the step, energy and adjoint
// kernels: MFMA shape policies, tile configurations and the two main loops
// (register-staged double buffer, and the direct-to-LDS ring).
#pragma once

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
// its 16-byte chunk c sits at position c ^ lds_swz(row), which spreads the
// 128-bit fragment reads of consecutive rows over distinct banks.  A
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
    srcA[d] = A + (size_t)(m0 + row) * ld + ((dch ^ lds_swz<CH>(row)) * 4);
  }
#pragma unroll
  for (int d = 0; d < B_DMA; ++d) {
    const int row = (wave * B_DMA + d) * RPD + drow;
    srcB[d] = B + (size_t)(n0 + row) * ld + ((dch ^ lds_swz<CH>(row)) * 4);
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
  // ring slots read and written this iteration (kt % S and (kt + S - 1) % S,
  // kept as counters so that no division runs in the loop)
  int rd = 0, wr = S - 1;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + S - 1 < nk) {
      wait_vm_barrier<(S - 2) * L>();
      issue(kt + S - 1, wr);
    } else {
      wait_vm_barrier<0>();
    }
    wr = wr + 1 == S ? 0 : wr + 1;
    const float *st = smem + rd * SLAB;
    rd = rd + 1 == S ? 0 : rd + 1;
    // fragments of the next contraction step are read while the MFMAs of
    // the current one run
    floatx4 a[2][C::TM], b[2][C::TN];
    auto frag = [&](int kk, floatx4 (&fa)[C::TM], floatx4 (&fb)[C::TN]) {
      const int ch = (kk + lk) >> 2;
#pragma unroll
      for (int i = 0; i < C::TM; ++i) {
        const int r = ra + i * C::MB;
        fa[i] = *reinterpret_cast<const floatx4 *>(st + r * C::BK + ((ch ^ lds_swz<CH>(r)) << 2));
      }
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int r = rb + j * C::MB;
        fb[j] = *reinterpret_cast<const floatx4 *>(st + (C::BM + r) * C::BK + ((ch ^ lds_swz<CH>(r)) << 2));
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
enum BMode { B_PLAIN = 0, B_SIGN = 1, B_MASKED = 2 };

// BMODE = B_SIGN replaces each X element by sign(x) while staging (energy
// readout); B_MASKED multiplies it by bit 1 of the byte at the same position
// of bmask (the momentum-wall mask of the adjoint).
template <class C, int BMODE>
__device__ __forceinline__ void f32_mainloop(const float *__restrict__ A,
                                             const float *__restrict__ B, int ld, int K,
                                             int m0, int n0,
                                             typename C::acc_t (&acc)[C::TM][C::TN],
                                             float *smem, const uint8_t *__restrict__ bmask = nullptr) {
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
  const uint8_t *gm = BMODE == B_MASKED ? bmask + (size_t)(n0 + srow) * ld + sc4 : nullptr;
  float *as_st = As + srow * C::LDK + sc4;
  float *bs_st = Bs + srow * C::LDK + sc4;
#define SI_GLOAD(k0)                                                                      \
  {                                                                                       \
    _Pragma("unroll") for (int f = 0; f < C::A_F4; ++f) ra[f] =                           \
        *reinterpret_cast<const floatx4 *>(ga + (size_t)f * C::ROWS_PER_PASS * ld + (k0));\
    _Pragma("unroll") for (int f = 0; f < C::B_F4; ++f) {                                 \
      floatx4 v = *reinterpret_cast<const floatx4 *>(gb + (size_t)f * C::ROWS_PER_PASS * ld + (k0)); \
      if (BMODE == B_SIGN) {                                                              \
        v[0] = sign_pm1(v[0]); v[1] = sign_pm1(v[1]); v[2] = sign_pm1(v[2]); v[3] = sign_pm1(v[3]); \
      } else if (BMODE == B_MASKED) {                                                     \
        const uint32_t mk = *reinterpret_cast<const uint32_t *>(                          \
            gm + (size_t)f * C::ROWS_PER_PASS * ld + (k0));                               \
        v[0] = (mk & 0x2u) ? v[0] : 0.f;                                                  \
        v[1] = (mk & 0x200u) ? v[1] : 0.f;                                                \
        v[2] = (mk & 0x20000u) ? v[2] : 0.f;                                              \
        v[3] = (mk & 0x2000000u) ? v[3] : 0.f;                                            \
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
  X(24, 64, 128, 2, 2, 32, 32, 4, 2)   \
  X(25, 128, 64, 4, 2, 32, 32, 0, 1)   \
  X(26, 128, 64, 4, 2, 32, 32, 4, 1)   \
  X(27, 64, 128, 2, 4, 32, 32, 4, 1)   \
  X(28, 128, 64, 4, 2, 32, 64, 3, 1)   \
  X(29, 128, 128, 4, 4, 32, 32, 0, 1)  \
  X(30, 128, 64, 4, 2, 32, 32, 6, 1)   \
  X(31, 128, 64, 4, 2, 32, 32, 4, 2)   \
  X(32, 64, 128, 2, 4, 32, 32, 6, 1)   \
  X(33, 128, 64, 4, 2, 32, 32, 5, 1)   \
  X(34, 128, 64, 4, 2, 32, 32, 3, 1)

}  // namespace si
