// BF16 matrix-core forms of the coupling product fused with the update.
//
// Same iteration as the FP32 kernel (Eq. 8 with the walls and the zeta_n /
// Delta_n weights, master q and p in FP32), but the product F = J.Q runs on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  Operand formats:
//   J planes: one BF16 plane (J exact in BF16, e.g. +-1), one FP8 e4m3 plane
//     (J exact in FP8; expanded to BF16 while staged into LDS, so HBM and L2
//     carry one byte per coupling), or two BF16 planes hi = bf16(J) and
//     lo = bf16(J - hi) for real-valued J.
//   Q planes: one BF16 copy of the FP32 master positions, or three BF16
//     planes hi + mid + lo whose sum is the FP32 value exactly; with J exact
//     in BF16 every product is then exact and only the FP32 accumulation
//     rounds.
// The epilogue writes the new FP32 master state and the BF16 plane(s) of q
// that the next step consumes.
//
// MFMA layout (32x32x16, one block): lane l supplies 8 consecutive
// contraction slots of row l%32 of A and of column l%32 of B, slot group
// l/32; the result D[8(v/4)+4(l/32)+v%4][l%32] lands in accumulator v.
// Each lane fills its 8 slots with 8 contiguous contraction indices read by
// one 128-bit LDS load, identically for A and B, so the product sums every
// index exactly once.
#include "si_epilogue.h"
#include "si_trace.h"
#include "si_internal.h"

namespace si {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));
typedef unsigned int uintx2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 bits, round to nearest even (inputs are finite).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// FP8 e4m3 (bias 7, no infinities) -> BF16 bits; exact because every e4m3
// value has at most 4 significant bits.
__device__ __forceinline__ uint32_t fp8_to_bf16_bits(uint32_t b) {
  const uint32_t sign = (b & 0x80u) << 8;
  const uint32_t e = (b >> 3) & 0xFu, m = b & 7u;
  if (e == 0) {
    if (m == 0) return sign;
    // subnormal: m * 2^-9
    const float v = (float)m * 0.001953125f;
    return sign | (__float_as_uint(v) >> 16);
  }
  // normal: (1 + m/8) * 2^(e-7): bf16 exponent e - 7 + 127, mantissa m << 4
  return sign | ((e + 120u) << 7) | (m << 4);
}

template <int BM_, int BN_, int WM_, int WN_, int BK_, int JFMT_, int QP_>
struct Bf16Cfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, BK = BK_;
  static constexpr int JFMT = JFMT_;  // 0: bf16 J, 1: fp8 J, 2: hi/lo bf16 J
  static constexpr int QP = QP_;      // BF16 planes of Q: 1 or 3
  static constexpr int JP = JFMT == 2 ? 2 : 1;
  static constexpr int MB = 32, KSTEP = 16;
  static constexpr int LDK = BK + 8;  // bf16 elements per padded LDS row (144 B for BK=64)
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / MB, TN = WTN / MB;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int V8_PER_ROW = BK / 8;        // 16-byte vectors per row of a slab
  static constexpr int ROWS_PER_PASS = NT / V8_PER_ROW;
  static constexpr int A_V = BM * BK / 8 / NT;     // vectors per thread per plane
  static constexpr int B_V = BN * BK / 8 / NT;
  static_assert(TM >= 1 && TN >= 1 && WTM % MB == 0 && WTN % MB == 0, "wave tile");
  static_assert(A_V >= 1 && B_V >= 1 && (BM * BK / 8) % NT == 0 && (BN * BK / 8) % NT == 0,
                "slab loads");
  static constexpr int A_ELEMS = BM * LDK, B_ELEMS = BN * LDK;
  static constexpr int STAGE_ELEMS = JP * A_ELEMS + QP * B_ELEMS;
  static constexpr int LDS_ELEMS = 2 * STAGE_ELEMS;
};

template <class C>
__device__ __forceinline__ void bf16_mainloop(const BStepArgs &a, int m0, int n0,
                                              floatx16 (&acc)[C::TM][C::TN], uint16_t *smem) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  const int lrow = lane % 32, lk = (lane / 32) * 8;
  const int ld = a.ld;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  const int srow = tid / C::V8_PER_ROW, sc8 = (tid % C::V8_PER_ROW) * 8;
  uintx4 ra[C::JP][C::A_V], rb[C::QP][C::B_V];
  uintx2 ra8[C::A_V];

  auto gload = [&](int k0) {
    if (C::JFMT == 1) {
      const uint8_t *g = reinterpret_cast<const uint8_t *>(a.Ja) + (size_t)(m0 + srow) * ld + sc8 + k0;
#pragma unroll
      for (int f = 0; f < C::A_V; ++f)
        ra8[f] = *reinterpret_cast<const uintx2 *>(g + (size_t)f * C::ROWS_PER_PASS * ld);
    } else {
#pragma unroll
      for (int pl = 0; pl < C::JP; ++pl) {
        const uint16_t *g = (pl == 0 ? reinterpret_cast<const uint16_t *>(a.Ja)
                                     : reinterpret_cast<const uint16_t *>(a.Jb)) +
                            (size_t)(m0 + srow) * ld + sc8 + k0;
#pragma unroll
        for (int f = 0; f < C::A_V; ++f)
          ra[pl][f] = *reinterpret_cast<const uintx4 *>(g + (size_t)f * C::ROWS_PER_PASS * ld);
      }
    }
#pragma unroll
    for (int pl = 0; pl < C::QP; ++pl) {
      const uint16_t *g = a.qb_in + (size_t)pl * a.plane_stride + (size_t)(n0 + srow) * ld + sc8 + k0;
#pragma unroll
      for (int f = 0; f < C::B_V; ++f)
        rb[pl][f] = *reinterpret_cast<const uintx4 *>(g + (size_t)f * C::ROWS_PER_PASS * ld);
    }
  };
  auto sstore = [&](int buf) {
    uint16_t *st = smem + buf * C::STAGE_ELEMS;
#pragma unroll
    for (int f = 0; f < C::A_V; ++f) {
      const int off = (srow + f * C::ROWS_PER_PASS) * C::LDK + sc8;
      if (C::JFMT == 1) {
        uintx4 w;
        const uint32_t lo = ra8[f][0], hi = ra8[f][1];
        w[0] = fp8_to_bf16_bits(lo & 0xFF) | (fp8_to_bf16_bits((lo >> 8) & 0xFF) << 16);
        w[1] = fp8_to_bf16_bits((lo >> 16) & 0xFF) | (fp8_to_bf16_bits(lo >> 24) << 16);
        w[2] = fp8_to_bf16_bits(hi & 0xFF) | (fp8_to_bf16_bits((hi >> 8) & 0xFF) << 16);
        w[3] = fp8_to_bf16_bits((hi >> 16) & 0xFF) | (fp8_to_bf16_bits(hi >> 24) << 16);
        *reinterpret_cast<uintx4 *>(st + off) = w;
      } else {
#pragma unroll
        for (int pl = 0; pl < C::JP; ++pl)
          *reinterpret_cast<uintx4 *>(st + pl * C::A_ELEMS + off) = ra[pl][f];
      }
    }
#pragma unroll
    for (int pl = 0; pl < C::QP; ++pl)
#pragma unroll
      for (int f = 0; f < C::B_V; ++f)
        *reinterpret_cast<uintx4 *>(st + C::JP * C::A_ELEMS + pl * C::B_ELEMS +
                                    (srow + f * C::ROWS_PER_PASS) * C::LDK + sc8) = rb[pl][f];
  };

  const int nk = a.n_pad / C::BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * C::BK);
    const uint16_t *st = smem + buf * C::STAGE_ELEMS;
    const uint16_t *as = st + (wy * C::WTM + lrow) * C::LDK + lk;
    const uint16_t *bs = st + C::JP * C::A_ELEMS + (wx * C::WTN + lrow) * C::LDK + lk;
#pragma unroll
    for (int kk = 0; kk < C::BK; kk += C::KSTEP) {
      bf16x8 fa[C::JP][C::TM], fb[C::QP][C::TN];
#pragma unroll
      for (int pl = 0; pl < C::JP; ++pl)
#pragma unroll
        for (int i = 0; i < C::TM; ++i)
          fa[pl][i] = *reinterpret_cast<const bf16x8 *>(as + pl * C::A_ELEMS + i * 32 * C::LDK + kk);
#pragma unroll
      for (int pl = 0; pl < C::QP; ++pl)
#pragma unroll
        for (int j = 0; j < C::TN; ++j)
          fb[pl][j] = *reinterpret_cast<const bf16x8 *>(bs + pl * C::B_ELEMS + j * 32 * C::LDK + kk);
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
#pragma unroll
          for (int pa = 0; pa < C::JP; ++pa)
#pragma unroll
            for (int pb = 0; pb < C::QP; ++pb)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[pa][i], fb[pb][j], acc[i][j],
                                                                  0, 0, 0);
        }
    }
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Direct-to-LDS pipeline for the BF16 forms.  STAGES slots of LDS hold the
// J plane(s) and the q plane(s) of one slab each; STAGES - 1 slabs are in
// flight.  Rows are stored unpadded with the 16-byte chunk c of row r at
// position c ^ lds_swz(r) (rows of 128 or 256 bytes), which keeps the
// 128-bit fragment reads of 16 consecutive rows on distinct banks.  FP8 J
// stays one byte per coupling in LDS and is widened to BF16 by the hardware
// FP8 conversion when the fragment is read.
//
// Contraction slots: the MFMAs run in pairs over 32 indices; in MFMA s of a
// pair, lane half h = l/32 holds indices kk + 16h + 8s .. +7.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_b;
typedef __attribute__((address_space(1))) const void gbl_void_b;

template <int N>
__device__ __forceinline__ void wait_vm_barrier_b() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

// Pipelined ring: the counter wait goes through the builtin, which the
// compiler's wait insertion accounts for; the barrier stays in asm with a
// memory clobber.  The _lgkm form also waits for this wave's LDS reads (the
// slot they read may be refilled once every wave has passed the barrier).
template <int N>
__device__ __forceinline__ void wait_vm_barrier_pb() {
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
  asm volatile("s_barrier" ::: "memory");
}
template <int N>
__device__ __forceinline__ void wait_vm_lgkm_barrier_b() {
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
  asm volatile("s_barrier" ::: "memory");
}

template <int BM_, int BN_, int WM_, int WN_, int BK_, int JFMT_, int QP_, int STAGES_,
          int PIPE_ = 0, int SW_ = 0>
struct Bf16DmaCfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, BK = BK_;
  static constexpr int JFMT = JFMT_, QP = QP_, STAGES = STAGES_;
  // PIPE = 1: the barrier that hands over slab k + 1 comes before the last
  // 32-deep step of slab k, whose fragments are already in registers, so
  // that the first fragments of slab k + 1 are read while the last
  // matrix-core operations of slab k run.
  static constexpr int PIPE = PIPE_;
  // SW > 0 (pipelined ring only): SW state waves beside the NW matrix waves
  // own the tile's state (see bf16_dma_tile_sw).
  static constexpr int SW = SW_;
  static constexpr int JP = JFMT == 2 ? 2 : 1;
  static constexpr int EA = JFMT == 1 ? 1 : 2;  // bytes per J element in LDS
  static constexpr int MB = 32;
  static constexpr int WTM = BM / WM, WTN = BN / WN;
  static constexpr int TM = WTM / MB, TN = WTN / MB;
  static constexpr int NT = 64 * WM * WN, NW = NT / 64;
  static constexpr int NTT = NT + 64 * SW;  // threads of the workgroup
  static constexpr int ROWA = BK * EA, ROWB = BK * 2;  // bytes per row
  static constexpr int CHA = ROWA / 16, CHB = ROWB / 16;
  static constexpr int RPDA = 64 / CHA, RPDB = 64 / CHB;  // rows per wave-wide load
  static constexpr int A_DMA = BM / RPDA / NW, B_DMA = BN / RPDB / NW;
  static constexpr int L = JP * A_DMA + QP * B_DMA;  // loads per wave per slab
  static constexpr int A_BYTES = BM * ROWA, B_BYTES = BN * ROWB;
  static constexpr int SLOT = JP * A_BYTES + QP * B_BYTES;
  // the ring, or the update tile staged through the same LDS if larger
  static constexpr int EPI_BYTES = BN * (BM + 4) * 4;
  static constexpr int LDS_BYTES = STAGES * SLOT > EPI_BYTES ? STAGES * SLOT : EPI_BYTES;
  static_assert(CHA >= 8 && CHB >= 8, "rows of at least 128 bytes for the chunk swizzle");
  static_assert(A_DMA >= 1 && B_DMA >= 1 && BM % (RPDA * NW) == 0 && BN % (RPDB * NW) == 0,
                "direct-to-LDS slab split");
  static_assert(TM >= 1 && TN >= 1 && BK % 32 == 0, "tile");
  static_assert(STAGES >= 2 && (STAGES - 2) * L <= 63, "pipeline depth");
  static_assert(SW == 0 || PIPE, "state waves need the pipelined ring");
};

// 8 FP8 e4m3 values (two words) -> 8 BF16 (exact: e4m3 has 4 significant
// bits), two values per conversion instruction at unit scale.
__device__ __forceinline__ bf16x8 fp8x8_to_bf16x8(uint32_t w0, uint32_t w1) {
  uintx4 u;
  u[0] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, false));
  u[1] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, true));
  u[2] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, false));
  u[3] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, true));
  return __builtin_bit_cast(bf16x8, u);
}

template <class C>
__device__ __forceinline__ void bf16_mainloop_dma(const BStepArgs &a, int m0, int n0,
                                                  floatx16 (&acc)[C::TM][C::TN], uint8_t *smem) {
  constexpr int S = C::STAGES;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  const int lrow = lane % 32, h = lane / 32;
  const int ld = a.ld;

#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  // per-lane global sources (byte pointers), k offset added per slab
  const uint8_t *srcA[C::JP][C::A_DMA];
  const uint8_t *srcB[C::QP][C::B_DMA];
  {
    const int drow = lane / C::CHA, dch = lane % C::CHA;
#pragma unroll
    for (int pl = 0; pl < C::JP; ++pl) {
      const uint8_t *base = reinterpret_cast<const uint8_t *>(pl == 0 ? a.Ja : a.Jb);
#pragma unroll
      for (int d = 0; d < C::A_DMA; ++d) {
        const int row = (wave * C::A_DMA + d) * C::RPDA + drow;
        srcA[pl][d] = base + ((size_t)(m0 + row) * ld) * C::EA + (dch ^ lds_swz<C::CHA>(row)) * 16;
      }
    }
  }
  {
    const int drow = lane / C::CHB, dch = lane % C::CHB;
#pragma unroll
    for (int pl = 0; pl < C::QP; ++pl) {
      const uint8_t *base =
          reinterpret_cast<const uint8_t *>(a.qb_in + (size_t)pl * a.plane_stride);
#pragma unroll
      for (int d = 0; d < C::B_DMA; ++d) {
        const int row = (wave * C::B_DMA + d) * C::RPDB + drow;
        srcB[pl][d] = base + ((size_t)(n0 + row) * ld) * 2 + (dch ^ lds_swz<C::CHB>(row)) * 16;
      }
    }
  }
  auto issue = [&](int kt, int slot) {
    uint8_t *st = smem + slot * C::SLOT;
#pragma unroll
    for (int pl = 0; pl < C::JP; ++pl)
#pragma unroll
      for (int d = 0; d < C::A_DMA; ++d)
        __builtin_amdgcn_global_load_lds(
            (gbl_void_b *)(srcA[pl][d] + (size_t)kt * C::ROWA),
            (lds_void_b *)(st + pl * C::A_BYTES + (wave * C::A_DMA + d) * C::RPDA * C::ROWA), 16,
            0, 0);
#pragma unroll
    for (int pl = 0; pl < C::QP; ++pl)
#pragma unroll
      for (int d = 0; d < C::B_DMA; ++d)
        __builtin_amdgcn_global_load_lds(
            (gbl_void_b *)(srcB[pl][d] + (size_t)kt * C::ROWB),
            (lds_void_b *)(st + C::JP * C::A_BYTES + pl * C::B_BYTES +
                           (wave * C::B_DMA + d) * C::RPDB * C::ROWB),
            16, 0, 0);
  };

  const int nk = a.n_pad / C::BK;
  if constexpr (!C::PIPE) {
#pragma unroll
    for (int s = 0; s < S - 1; ++s)
      if (s < nk) issue(s, s);
  }
  // Raw fragments of one 32-deep step: FP8 J as one 16-byte chunk per row
  // block (both halves of the step), BF16 planes as two 16-byte chunks.
  constexpr int AC = C::JFMT == 1 ? 1 : 2;
  struct Frag {
    uintx4 fa[C::JP][C::TM][AC];
    uintx4 fb[C::QP][C::TN][2];
  };
  auto read_frag = [&](const uint8_t *st, int kk, Frag &f) {
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      const int r = wy * C::WTM + i * 32 + lrow;
      if (C::JFMT == 1) {
        const int ch = (kk + 16 * h) / 16;  // 16 fp8 per chunk
        f.fa[0][i][0] =
            *reinterpret_cast<const uintx4 *>(st + r * C::ROWA + ((ch ^ lds_swz<C::CHA>(r)) << 4));
      } else {
#pragma unroll
        for (int pl = 0; pl < C::JP; ++pl)
#pragma unroll
          for (int sidx = 0; sidx < 2; ++sidx) {
            const int ch = (kk + 16 * h + 8 * sidx) / 8;  // 8 bf16 per chunk
            f.fa[pl][i][sidx] = *reinterpret_cast<const uintx4 *>(
                st + pl * C::A_BYTES + r * C::ROWA + ((ch ^ lds_swz<C::CHA>(r)) << 4));
          }
      }
    }
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int r = wx * C::WTN + j * 32 + lrow;
#pragma unroll
      for (int pl = 0; pl < C::QP; ++pl)
#pragma unroll
        for (int sidx = 0; sidx < 2; ++sidx) {
          const int ch = (kk + 16 * h + 8 * sidx) / 8;
          f.fb[pl][j][sidx] = *reinterpret_cast<const uintx4 *>(
              st + C::JP * C::A_BYTES + pl * C::B_BYTES + r * C::ROWB + ((ch ^ lds_swz<C::CHB>(r)) << 4));
        }
    }
  };
  auto mma_frag = [&](const Frag &f) {
    bf16x8 fa[C::JP][C::TM][2];
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      if (C::JFMT == 1) {
        fa[0][i][0] = fp8x8_to_bf16x8(f.fa[0][i][0][0], f.fa[0][i][0][1]);
        fa[0][i][1] = fp8x8_to_bf16x8(f.fa[0][i][0][2], f.fa[0][i][0][3]);
      } else {
#pragma unroll
        for (int pl = 0; pl < C::JP; ++pl)
#pragma unroll
          for (int sidx = 0; sidx < 2; ++sidx)
            fa[pl][i][sidx] = __builtin_bit_cast(bf16x8, f.fa[pl][i][AC == 2 ? sidx : 0]);
      }
    }
#pragma unroll
    for (int sidx = 0; sidx < 2; ++sidx)
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j)
#pragma unroll
          for (int pa = 0; pa < C::JP; ++pa)
#pragma unroll
            for (int pb = 0; pb < C::QP; ++pb)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  fa[pa][i][sidx], __builtin_bit_cast(bf16x8, f.fb[pb][j][sidx]), acc[i][j], 0, 0,
                  0);
  };
  if constexpr (C::PIPE) {
    constexpr int NKS = C::BK / 32;
    Frag fr[2];
    int rd = 0, wr = S - 1;
    if (nk > 0) {
      // prologue: S - 1 slabs in flight, slab 0 awaited, slab S - 1 issued
      // (on the long path every slab is issued unconditionally, so that the
      // compiler's count of the loads issued before them is exact)
      if (S - 1 < nk) {
#pragma unroll
        for (int s = 0; s < S - 1; ++s) issue(s, s);
        wait_vm_barrier_pb<(S - 2) * C::L>();
        issue(S - 1, wr);
      } else {
#pragma unroll
        for (int s = 0; s < S - 1; ++s)
          if (s < nk) issue(s, s);
        wait_vm_barrier_pb<0>();
      }
      wr = wr + 1 == S ? 0 : wr + 1;
      read_frag(smem, 0, fr[0]);
    }
    for (int kt = 0; kt < nk; ++kt) {
      const uint8_t *st = smem + rd * C::SLOT;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const int cur = ks & 1;
        if (ks + 1 < NKS) {
          read_frag(st, (ks + 1) * 32, fr[cur ^ 1]);
        } else if (kt + 1 < nk) {
          // every wave holds its fragments of slab kt and slab kt + 1 has
          // landed: slot rd may be refilled with slab kt + S
          if (kt + S < nk) {
            wait_vm_lgkm_barrier_b<(S - 2) * C::L>();
            issue(kt + S, wr);
          } else {
            wait_vm_lgkm_barrier_b<0>();
          }
          wr = wr + 1 == S ? 0 : wr + 1;
          rd = rd + 1 == S ? 0 : rd + 1;
          read_frag(smem + rd * C::SLOT, 0, fr[cur ^ 1]);
        }
        mma_frag(fr[cur]);
      }
    }
  } else {
    // ring slots read and written this iteration, kept as counters
    int rd = 0, wr = S - 1;
    for (int kt = 0; kt < nk; ++kt) {
      if (kt + S - 1 < nk) {
        wait_vm_barrier_b<(S - 2) * C::L>();
        issue(kt + S - 1, wr);
      } else {
        wait_vm_barrier_b<0>();
      }
      wr = wr + 1 == S ? 0 : wr + 1;
      const uint8_t *st = smem + rd * C::SLOT;
      rd = rd + 1 == S ? 0 : rd + 1;
#pragma unroll
      for (int kk = 0; kk < C::BK; kk += 32) {
        Frag f;
        read_frag(st, kk, f);
        mma_frag(f);
      }
    }
  }
  wait_vm_barrier_b<0>();
}


// Update of one BF16-form tile: F through LDS into the state's layout,
// then the FP32 master state and the BF16 plane(s) of the new q.
template <class T, int QP, int ORDER, int WALL>
__device__ __forceinline__ void bf16_update(const BStepArgs &a, int m0, int n0, float *t,
                                            const floatx4 (&q4)[T::CPT],
                                            const floatx4 (&p4)[T::CPT]) {
  EpiArgs e;
  e.q_in = a.q_in;
  e.p_in = a.p_in;
  e.h = a.h;
  e.q_out = a.q_out;
  e.p_out = a.p_out;
  e.qb_out = a.qb_out;
  e.plane_stride = a.plane_stride;
  e.mask_out = nullptr;
  e.ld = a.ld;
  e.m0 = m0;
  e.n0 = n0;
  e.dt = a.dt[a.t];
  e.zeta = a.zeta[a.t];
  e.k = a.k;
  e.inv_m = a.inv_m;
  e.qmax = a.qmax;
  e.pmax = a.pmax;
  epi_apply<T, ORDER, WALL, QP>(t, e, q4, p4);
}

// The 32x32 accumulator blocks of this wave into the LDS tile (32x32x16
// layout: lane l holds rows 8(v/4) + 4(l/32) + v%4 of column l%32).
template <class C>
__device__ __forceinline__ void bf16_put(float *t, int ld, const floatx16 (&acc)[C::TM][C::TN]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
        epi_put(t, ld, wy * C::WTM + i * 32 + g * 8 + (lane / 32) * 4,
                wx * C::WTN + j * 32 + (lane % 32), acc[i][j][4 * g], acc[i][j][4 * g + 1],
                acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]);
}

template <class C, int ORDER, int WALL>
__global__ __launch_bounds__(C::NT) void step_bf16_kernel(BStepArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t smem[C::LDS_ELEMS];
  using T = EpiTile<C::BM, C::BN, C::NT>;
  static_assert(T::BYTES <= C::LDS_ELEMS * 2, "the update tile fits in the main loop's LDS");
  const int t = xcd_tile(blockIdx.x, gridDim.x), ncol = a.r_pad / C::BN;
  const int m0 = (t / ncol) * C::BM, n0 = (t % ncol) * C::BN;
  floatx16 acc[C::TM][C::TN];
  bf16_mainloop<C>(a, m0, n0, acc, smem);
  float *tile = reinterpret_cast<float *>(smem);
  bf16_put<C>(tile, T::LD, acc);
  floatx4 q4[T::CPT], p4[T::CPT];
  EpiArgs e;
  e.q_in = a.q_in;
  e.p_in = a.p_in;
  e.ld = a.ld;
  e.m0 = m0;
  e.n0 = n0;
  epi_load<T>(e, q4, p4);
  __syncthreads();
  bf16_update<T, C::QP, ORDER, WALL>(a, m0, n0, tile, q4, p4);
}

// One BM x BN output tile of one step on the direct-to-LDS pipeline: the
// product over the BF16 planes, then the update of the FP32 master state and
// the BF16 plane(s) of the new q.  Shared by the single-instance and the
// batched kernels.
template <class C, int ORDER, int WALL>
__device__ __forceinline__ void bf16_dma_tile(const BStepArgs &a, int m0, int n0, uint8_t *smem) {
  using T = EpiTile<C::BM, C::BN, C::NT>;
  static_assert(T::BYTES <= C::LDS_BYTES, "the update tile fits in the main loop's LDS");
  // State of this thread's chunks.  It is loaded before the contraction, so
  // that its latency overlaps the matrix work, when the registers allow: for
  // at most eight chunks per thread, or when a single four-wave group fills
  // the CU's LDS (one wave per SIMD owns the whole register file).
  // Otherwise it is loaded afterwards (eight registers per chunk would stay
  // live through the main loop).
  constexpr bool PREFETCH = T::CPT <= 8 || (C::NW == 4 && C::LDS_BYTES > 80 * 1024);
  floatx4 q4[T::CPT], p4[T::CPT];
  EpiArgs e;
  e.q_in = a.q_in;
  e.p_in = a.p_in;
  e.ld = a.ld;
  e.m0 = m0;
  e.n0 = n0;
  if constexpr (PREFETCH) epi_load<T>(e, q4, p4);
  floatx16 acc[C::TM][C::TN];
  bf16_mainloop_dma<C>(a, m0, n0, acc, smem);
  float *tile = reinterpret_cast<float *>(smem);
  bf16_put<C>(tile, T::LD, acc);
  if constexpr (!PREFETCH) epi_load<T>(e, q4, p4);
  __syncthreads();
  bf16_update<T, C::QP, ORDER, WALL>(a, m0, n0, tile, q4, p4);
}

// One tile with state waves (C::SW > 0).  The matrix waves run the ring and
// leave F in LDS; they never touch the state.  The state waves load the
// tile's q and p, and in the paper order (q' needs no coupling term) store
// q' and its BF16 plane(s) while the product runs, then apply p' from F.
// Their vector-memory counter holds only their own loads and stores, so the
// compiler's waits for them never drain the matrix waves' ring.  Both roles
// pass the same barriers: the ring's nk + 1 and the one before the update.
// The role is taken from readfirstlane, so the branch on it is a scalar
// branch that each wave takes whole.
__device__ __forceinline__ void bare_barrier() { asm volatile("s_barrier" ::: "memory"); }

template <class C, int ORDER, int WALL>
__device__ __forceinline__ void bf16_dma_tile_sw(const BStepArgs &a, int m0, int n0,
                                                 uint8_t *smem) {
  using TS = EpiTile<C::BM, C::BN, 64 * C::SW, C::NT>;
  static_assert(TS::BYTES <= C::LDS_BYTES, "the update tile fits in the main loop's LDS");
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  float *tile = reinterpret_cast<float *>(smem);
  if (wave < C::NW) {
    floatx16 acc[C::TM][C::TN];
    bf16_mainloop_dma<C>(a, m0, n0, acc, smem);  // nk + 1 barriers
    bf16_put<C>(tile, TS::LD, acc);
    __syncthreads();
    return;
  }
  EpiArgs e;
  e.q_in = a.q_in;
  e.p_in = a.p_in;
  e.h = a.h;
  e.q_out = a.q_out;
  e.p_out = a.p_out;
  e.qb_out = a.qb_out;
  e.plane_stride = a.plane_stride;
  e.mask_out = nullptr;
  e.ld = a.ld;
  e.m0 = m0;
  e.n0 = n0;
  e.dt = a.dt[a.t];
  e.zeta = a.zeta[a.t];
  e.k = a.k;
  e.inv_m = a.inv_m;
  e.qmax = a.qmax;
  e.pmax = a.pmax;
  floatx4 q4[TS::CPT], p4[TS::CPT];
  epi_load<TS>(e, q4, p4);
  const int nk = a.n_pad / C::BK;
  if (nk > 0) {
    bare_barrier();  // the ring's prologue barrier
    if constexpr (ORDER == SI_ORDER_PAPER) epi_apply_q<TS, C::QP>(e, q4, p4);
    for (int i = 1; i < nk; ++i) bare_barrier();  // the ring's slab hand-overs
  }
  bare_barrier();  // the ring's final barrier
  __syncthreads();
  if constexpr (ORDER == SI_ORDER_PAPER)
    epi_apply_p<TS, WALL>(tile, e, q4, p4);
  else
    epi_apply<TS, ORDER, WALL, C::QP>(tile, e, q4, p4);
}

template <class C, int ORDER, int WALL>
__global__ __launch_bounds__(C::NTT) void step_bf16_dma_kernel(BStepArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t smem[C::LDS_BYTES];
  const int t = xcd_tile(blockIdx.x, gridDim.x), ncol = a.r_pad / C::BN;
  if constexpr (C::SW > 0)
    bf16_dma_tile_sw<C, ORDER, WALL>(a, (t / ncol) * C::BM, (t % ncol) * C::BN, smem);
  else
    bf16_dma_tile<C, ORDER, WALL>(a, (t / ncol) * C::BM, (t % ncol) * C::BN, smem);
}

// Batched precision form: one launch advances every instance by one step.
// Work item (instance, row tile, column tile) as in the FP32 batch; each
// instance carries its own J format: FP8 e4m3 (J exact in FP8) with 128-deep
// slabs, hi + lo BF16 otherwise with 64-deep slabs.  Two tile heights, picked
// per batch: 128 rows (eight waves of 32x32) or 64 rows (four waves).  Both
// have the wave tile and slab depth of the 64x64 single-instance tiles of
// those formats, so every instance matches its standalone run on those tiles
// bit for bit.  The batch streams J from HBM once per step; the 128-row tile
// halves the re-reads of the BF16 q plane per byte of J against 64 rows
// (3.6 % less time per step on the 256-instance workload), the 64-row tile
// gives twice the work items to batches too small to fill the chip.
template <int BM>
struct BatchBf16Tiles {
  using Fp8 = Bf16DmaCfg<BM, BATCH_BN, BM / 32, 2, 128, 1, 1, 3>;
  using Hilo = Bf16DmaCfg<BM, BATCH_BN, BM / 32, 2, 64, 2, 1, 3>;
  static_assert(Fp8::NT == Hilo::NT, "one block shape for both formats");
  static constexpr int LDS = Fp8::LDS_BYTES > Hilo::LDS_BYTES ? Fp8::LDS_BYTES : Hilo::LDS_BYTES;
};

template <int BM, int ORDER, int WALL>
__global__ __launch_bounds__(BatchBf16Tiles<BM>::Fp8::NT) void step_batch_bf16_kernel(
    BStepArgs base, const BBatchDesc *__restrict__ descs, const int4 *__restrict__ items, int cur,
    unsigned long long *trace) {
  const unsigned long long start = wall_clock64();
  using T = BatchBf16Tiles<BM>;
  __shared__ __attribute__((aligned(16))) uint8_t smem[T::LDS];
  const int4 it = items[blockIdx.x];
  const BBatchDesc d = descs[it.x];
  BStepArgs a = base;
  a.Ja = d.Ja;
  a.Jb = d.Jb;
  // buffer parity by selection (a run-time index into the local copy of the
  // descriptor would place it in scratch memory)
  a.q_in = cur ? d.q[1] : d.q[0];
  a.p_in = cur ? d.p[1] : d.p[0];
  a.q_out = cur ? d.q[0] : d.q[1];
  a.p_out = cur ? d.p[0] : d.p[1];
  a.qb_in = cur ? d.qb[1] : d.qb[0];
  a.qb_out = cur ? d.qb[0] : d.qb[1];
  a.ld = d.n_pad;
  a.n_pad = d.n_pad;
  a.plane_stride = (int64_t)d.n_pad * base.r_pad;
  a.h = nullptr;
  if (d.fmt == 1)
    bf16_dma_tile<typename T::Fp8, ORDER, WALL>(a, it.y * BM, it.z * BATCH_BN, smem);
  else
    bf16_dma_tile<typename T::Hilo, ORDER, WALL>(a, it.y * BM, it.z * BATCH_BN, smem);
  if (trace) batch_trace_record(trace, start);
}

template <int BM>
static hipError_t launch_batch_bf16_bm(const BStepArgs &base, const BBatchDesc *descs,
                                       const int4 *items, int32_t n_items, int32_t cur,
                                       unsigned long long *trace, hipStream_t s) {
  dim3 grid(n_items), block(BatchBf16Tiles<BM>::Fp8::NT);
  switch (base.order * 2 + base.wall) {
    case 0: step_batch_bf16_kernel<BM, SI_ORDER_PAPER, SI_WALL_CLAMP><<<grid, block, 0, s>>>(base, descs, items, cur, trace); break;
    case 1: step_batch_bf16_kernel<BM, SI_ORDER_PAPER, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(base, descs, items, cur, trace); break;
    case 2: step_batch_bf16_kernel<BM, SI_ORDER_SYMPLECTIC, SI_WALL_CLAMP><<<grid, block, 0, s>>>(base, descs, items, cur, trace); break;
    case 3: step_batch_bf16_kernel<BM, SI_ORDER_SYMPLECTIC, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(base, descs, items, cur, trace); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step_batch_bf16(const BStepArgs &base, const BBatchDesc *descs,
                                  const int4 *items, int32_t n_items, int32_t cur, int32_t btile,
                                  unsigned long long *trace, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (btile) {
    case 1: return launch_batch_bf16_bm<BATCH_BF16_BM>(base, descs, items, n_items, cur, trace, s);
    case 2: return launch_batch_bf16_bm<64>(base, descs, items, n_items, cur, trace, s);
    default: return hipErrorInvalidValue;
  }
}

template <class C>
static hipError_t launch_bd(const BStepArgs &a, hipStream_t s) {
  if (a.n_pad % C::BM || a.r_pad % C::BN || a.n_pad % C::BK) return hipErrorInvalidValue;
  dim3 grid((a.n_pad / C::BM) * (a.r_pad / C::BN)), block(C::NTT);
  switch (a.order * 2 + a.wall) {
    case 0: step_bf16_dma_kernel<C, SI_ORDER_PAPER, SI_WALL_CLAMP><<<grid, block, 0, s>>>(a); break;
    case 1: step_bf16_dma_kernel<C, SI_ORDER_PAPER, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(a); break;
    case 2: step_bf16_dma_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_CLAMP><<<grid, block, 0, s>>>(a); break;
    case 3: step_bf16_dma_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// BF16 tile table: id, BM, BN, waves WM x WN, slab depth BK.
// Stages 0: register-staged double buffer; >= 2: direct-to-LDS ring of that
// many slabs (the FP8 J form needs BK = 128 there).  The two-slab rings
// (20, 21) give eight waves 64x64 output blocks, which halves the LDS
// fragment reads per matrix-core operation of the multi-plane forms (hi + lo
// J, three position planes); one slab loads while the other is consumed.
// Tile 22 is the two-slab ring that fits eight waves on a 128x128 block of
// the three-plane form (its three-slab ring would exceed the LDS); tile 23
// gives the single-plane forms eight waves on one 128x64 block per CU when
// the problem has that many blocks (N = 2000, R = 1024), and tile 24 the
// same for the three-plane form over 64-deep slabs.
#define SI_BF16_TILES(X)         \
  X(1, 64, 64, 2, 2, 64, 0, 0)      \
  X(2, 64, 128, 2, 2, 64, 0, 0)     \
  X(3, 128, 64, 2, 2, 64, 0, 0)     \
  X(4, 128, 128, 2, 2, 64, 0, 0)    \
  X(5, 128, 128, 2, 4, 64, 0, 0)    \
  X(6, 64, 64, 2, 2, 128, 0, 0)     \
  X(7, 64, 64, 2, 2, 64, 3, 0)      \
  X(8, 64, 64, 2, 2, 64, 4, 0)      \
  X(9, 64, 64, 2, 2, 128, 3, 0)     \
  X(10, 64, 128, 2, 2, 64, 3, 0)    \
  X(11, 128, 64, 2, 2, 64, 3, 0)    \
  X(12, 128, 128, 2, 2, 64, 3, 0)   \
  X(13, 64, 64, 2, 2, 128, 4, 0)    \
  X(14, 128, 128, 2, 2, 128, 3, 0)  \
  X(15, 128, 128, 2, 2, 64, 4, 0)   \
  X(16, 128, 256, 2, 4, 64, 3, 0)   \
  X(17, 256, 128, 4, 2, 64, 3, 0)   \
  X(18, 128, 128, 2, 4, 64, 3, 0)   \
  X(19, 128, 128, 4, 2, 128, 3, 0)  \
  X(20, 128, 256, 2, 4, 64, 2, 0)   \
  X(21, 256, 128, 4, 2, 64, 2, 0)   \
  X(22, 128, 128, 2, 4, 64, 2, 0)   \
  X(23, 128, 64, 4, 2, 128, 3, 0)   \
  X(24, 128, 64, 4, 2, 64, 3, 0)   \
  X(25, 128, 64, 4, 2, 128, 3, 1)  \
  X(26, 128, 64, 4, 2, 64, 3, 1)   \
  X(27, 128, 128, 4, 2, 128, 3, 1) \
  X(28, 128, 256, 2, 4, 64, 2, 1)  \
  X(29, 128, 256, 2, 4, 64, 3, 1)  \
  X(30, 256, 128, 4, 2, 64, 2, 1)  \
  X(31, 128, 128, 2, 4, 64, 2, 1)  \
  X(32, 128, 64, 4, 2, 128, 3, 2)  \
  X(33, 128, 64, 4, 2, 64, 3, 2)

TileShape tile_shape_bf16(int32_t tile) {
  switch (tile) {
#define SI_SHAPE(id, bm, bn, wm, wn, bk, st, pp) \
  case id:                                   \
    return {bm, bn,                          \
            pp == 2 ? "step_bf16_" #bm "x" #bn "_w" #wm "x" #wn "_k" #bk "_s" #st "_p2" \
            : pp    ? "step_bf16_" #bm "x" #bn "_w" #wm "x" #wn "_k" #bk "_s" #st "_p1" \
               : "step_bf16_" #bm "x" #bn "_w" #wm "x" #wn "_k" #bk "_s" #st,       \
            bk};
    SI_BF16_TILES(SI_SHAPE)
#undef SI_SHAPE
    default: return {0, 0, "invalid", 0};
  }
}

template <class C>
static hipError_t launch_b(const BStepArgs &a, hipStream_t s) {
  if (a.n_pad % C::BM || a.r_pad % C::BN || a.n_pad % C::BK) return hipErrorInvalidValue;
  dim3 grid((a.n_pad / C::BM) * (a.r_pad / C::BN)), block(C::NT);
  switch (a.order * 2 + a.wall) {
    case 0: step_bf16_kernel<C, SI_ORDER_PAPER, SI_WALL_CLAMP><<<grid, block, 0, s>>>(a); break;
    case 1: step_bf16_kernel<C, SI_ORDER_PAPER, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(a); break;
    case 2: step_bf16_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_CLAMP><<<grid, block, 0, s>>>(a); break;
    case 3: step_bf16_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, int BK, int ST, int JFMT, int QP, int PP>
static hipError_t launch_sel(const BStepArgs &a, hipStream_t s) {
  if constexpr (ST == 0) {
    return launch_b<Bf16Cfg<BM, BN, WM, WN, BK, JFMT, QP>>(a, s);
  } else if constexpr (JFMT == 1 && BK < 128) {
    return hipErrorInvalidValue;  // FP8 rows must be 128 bytes for the swizzle
  } else {
    using C = Bf16DmaCfg<BM, BN, WM, WN, BK, JFMT, QP, ST, PP ? 1 : 0, PP == 2 ? 4 : 0>;
    if constexpr (C::LDS_BYTES > 160 * 1024)
      return hipErrorInvalidValue;
    else
      return launch_bd<C>(a, s);
  }
}

template <int BM, int BN, int WM, int WN, int BK, int ST, int JFMT, int QP, int PP>
static constexpr bool sel_valid() {
  if constexpr (ST == 0)
    return true;
  else if constexpr (JFMT == 1 && BK < 128)
    return false;
  else
    return Bf16DmaCfg<BM, BN, WM, WN, BK, JFMT, QP, ST, PP ? 1 : 0, PP == 2 ? 4 : 0>::LDS_BYTES <=
           160 * 1024;
}

template <int JFMT, int QP>
static bool valid_fmt(int32_t tile) {
  switch (tile) {
#define SI_VALID(id, bm, bn, wm, wn, bk, st, pp) \
  case id:                                   \
    return sel_valid<bm, bn, wm, wn, bk, st, JFMT, QP, pp>();
    SI_BF16_TILES(SI_VALID)
#undef SI_VALID
    default: return false;
  }
}

bool tile_valid_bf16(int32_t tile, int32_t precision) {
  switch (precision) {
    case SI_PREC_BF16X_BF16J: return valid_fmt<0, 1>(tile);
    case SI_PREC_BF16X_FP8J: return valid_fmt<1, 1>(tile);
    case SI_PREC_BF16X_HILOJ: return valid_fmt<2, 1>(tile);
    case SI_PREC_BF16X3_EXACTJ: return valid_fmt<0, 3>(tile);
    default: return false;
  }
}

template <int JFMT, int QP>
static hipError_t launch_fmt(int32_t tile, const BStepArgs &a, hipStream_t s) {
  switch (tile) {
#define SI_LAUNCH(id, bm, bn, wm, wn, bk, st, pp) \
  case id:                                    \
    return launch_sel<bm, bn, wm, wn, bk, st, JFMT, QP, pp>(a, s);
    SI_BF16_TILES(SI_LAUNCH)
#undef SI_LAUNCH
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_bf16(int32_t tile, int32_t precision, const BStepArgs &a, hipStream_t s) {
  switch (precision) {
    case SI_PREC_BF16X_BF16J: return launch_fmt<0, 1>(tile, a, s);
    case SI_PREC_BF16X_FP8J: return launch_fmt<1, 1>(tile, a, s);
    case SI_PREC_BF16X_HILOJ: return launch_fmt<2, 1>(tile, a, s);
    case SI_PREC_BF16X3_EXACTJ: return launch_fmt<0, 3>(tile, a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Packing for the precision forms.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f32_to_fp8_exact(float v) {
  // v is known to be exact in e4m3 (validated); encode it.
  uint32_t sign = v < 0.f ? 0x80u : 0u;
  const float a = fabsf(v);
  if (a == 0.f) return sign;
  if (a < 0.015625f) return sign | (uint32_t)(a * 512.f);  // subnormal, exponent field 0
  int e;
  const float fr = frexpf(a, &e);  // a = fr * 2^e, fr in [0.5, 1)
  const uint32_t exp_field = (uint32_t)(e - 1 + 7);
  const uint32_t man = (uint32_t)(fr * 16.f) - 8u;
  return sign | (exp_field << 3) | man;
}

__global__ void pack_j_lowp_kernel(const float *__restrict__ J, int64_t total, int fmt,
                                   void *__restrict__ out_a, void *__restrict__ out_b) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = J[i];
    if (fmt == 1) {
      reinterpret_cast<uint8_t *>(out_a)[i] = (uint8_t)f32_to_fp8_exact(v);
    } else {
      const uint32_t hi = bf16_bits(v);
      reinterpret_cast<uint16_t *>(out_a)[i] = (uint16_t)hi;
      if (fmt == 2) reinterpret_cast<uint16_t *>(out_b)[i] = (uint16_t)bf16_bits(v - bf16_to_f32(hi));
    }
  }
}

__global__ void split_planes_kernel(const float *__restrict__ q, uint16_t *__restrict__ planes,
                                    int64_t total, int nplanes) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    float r = q[i];
    for (int pl = 0; pl < nplanes; ++pl) {
      const uint32_t b = bf16_bits(r);
      planes[(size_t)pl * total + i] = (uint16_t)b;
      r = r - bf16_to_f32(b);
    }
  }
}

static int grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > 8192) b = 8192;
  return b < 1 ? 1 : (int)b;
}

hipError_t launch_pack_j_lowp(const float *J, int64_t total, int32_t precision, void *out_a,
                              void *out_b, hipStream_t s) {
  int fmt = 0;
  if (precision == SI_PREC_BF16X_FP8J) fmt = 1;
  if (precision == SI_PREC_BF16X_HILOJ) fmt = 2;
  pack_j_lowp_kernel<<<grid_for(total), 256, 0, s>>>(J, total, fmt, out_a, out_b);
  return hipGetLastError();
}

hipError_t launch_split_planes(const float *q, uint16_t *planes, int64_t total, int32_t nplanes,
                               hipStream_t s) {
  split_planes_kernel<<<grid_for(total), 256, 0, s>>>(q, planes, total, nplanes);
  return hipGetLastError();
}

}  // namespace si
