// Fused update of one output tile of the coupling product, with the state
// traffic in the order of the state's memory layout.
//
// The matrix cores leave F = J.Q spread over the lanes in their own layout:
// a lane holds a few consecutive spins of one replica, and the 32 lanes of a
// row group hold 32 different replicas.  The state q, p is stored
// replica-major ([r_pad][n_pad], spins contiguous), so updating F in place
// would read and write 16-byte pieces of 32 different memory rows per
// instruction.  Instead the tile of F goes through LDS (the main loop's ring
// is free once the contraction has finished) in the memory layout, and every
// thread then updates whole 16-byte chunks of it, consecutive threads taking
// consecutive chunks of a replica's spins: each load and store instruction
// covers a few full cache lines.  The arithmetic per element is unchanged.
#pragma once

#include "si_internal.h"

namespace si {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int uintx2 __attribute__((ext_vector_type(2)));

// Eq. (8) and the walls for one element; f is sum_j J_ij q_j (+ h_i).
template <int ORDER, int WALL>
__device__ __forceinline__ void spring_update(float q, float p, float f, float dt, float zeta,
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

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t epi_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// The BM (spins) x BN (replicas) output tile in LDS, replica-major: element
// (row i, column j) at t[j * LD + i].  Rows are padded by four floats so that
// the 16-byte writes of 16 consecutive columns fall on distinct banks.  The
// NT threads from thread T0 on share the tile's chunks.
template <int BM, int BN, int NT, int T0 = 0>
struct EpiTile {
  static constexpr int LD = BM + 4;
  static constexpr int BYTES = BN * LD * 4;
  static constexpr int CHUNKS = BM * BN / 4;  // 16-byte chunks of the tile
  static constexpr int CPT = CHUNKS / NT;     // chunks per thread
  static_assert(BM % 4 == 0 && CHUNKS % NT == 0, "epilogue chunks");
  static __device__ __forceinline__ int tid() { return (int)threadIdx.x - T0; }
  // chunk c of this thread: tile-local column (replica) and first row (spin)
  static __device__ __forceinline__ int col(int c) { return (c * NT + tid()) / (BM / 4); }
  static __device__ __forceinline__ int row(int c) { return ((c * NT + tid()) % (BM / 4)) * 4; }
};

// What the update of one tile reads and writes.
struct EpiArgs {
  const float *q_in, *p_in, *h;  // h may be null
  float *q_out, *p_out;
  uint16_t *qb_out;              // BF16 plane(s) of the new q, or null
  int64_t plane_stride;
  uint8_t *mask_out;             // null, or the wall-mask bytes (adjoint recompute)
  int ld, m0, n0;
  float dt, zeta, k, inv_m, qmax, pmax;
};

// The state of this thread's chunks (issued early, so that the loads overlap
// the contraction when the registers allow).
template <class T>
__device__ __forceinline__ void epi_load(const EpiArgs &e, floatx4 (&q4)[T::CPT],
                                         floatx4 (&p4)[T::CPT]) {
#pragma unroll
  for (int c = 0; c < T::CPT; ++c) {
    const size_t off = (size_t)(e.n0 + T::col(c)) * e.ld + e.m0 + T::row(c);
    q4[c] = *reinterpret_cast<const floatx4 *>(e.q_in + off);
    p4[c] = *reinterpret_cast<const floatx4 *>(e.p_in + off);
  }
}

// Four accumulator values of rows row..row+3 (tile-local) of column col.
__device__ __forceinline__ void epi_put(float *t, int ld, int row, int col, float v0, float v1,
                                        float v2, float v3) {
  *reinterpret_cast<floatx4 *>(t + col * ld + row) = floatx4{v0, v1, v2, v3};
}

// Update every chunk of the tile held in LDS (the caller has synchronised
// the workgroup after the last epi_put).  QP: BF16 planes of q to write
// (0 for the FP32 form, 1, or 3 for the exact split).
template <class T, int ORDER, int WALL, int QP>
__device__ __forceinline__ void epi_apply(const float *t, const EpiArgs &e,
                                          const floatx4 (&q4)[T::CPT],
                                          const floatx4 (&p4)[T::CPT]) {
#pragma unroll
  for (int c = 0; c < T::CPT; ++c) {
    const int col = T::col(c), row = T::row(c);
    const size_t off = (size_t)(e.n0 + col) * e.ld + e.m0 + row;
    const floatx4 f = *reinterpret_cast<const floatx4 *>(t + col * T::LD + row);
    floatx4 h4 = {0.f, 0.f, 0.f, 0.f};
    if (e.h) h4 = *reinterpret_cast<const floatx4 *>(e.h + e.m0 + row);
    floatx4 qn, pn;
    uint32_t b0[4], b1[4], b2[4], mk = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float qv, pv;
      spring_update<ORDER, WALL>(q4[c][v], p4[c][v], f[v] + h4[v], e.dt, e.zeta, e.k, e.inv_m,
                                 e.qmax, e.pmax, qv, pv);
      qn[v] = qv;
      pn[v] = pv;
      if (QP >= 1) b0[v] = epi_bf16(qv);
      if (QP == 3) {
        const float r1 = qv - __uint_as_float(b0[v] << 16);  // exact
        b1[v] = epi_bf16(r1);
        const float r2 = r1 - __uint_as_float(b1[v] << 16);  // exact
        b2[v] = epi_bf16(r2);
      }
      if (QP == 0 && e.mask_out) {
        // the unclamped values, recomputed exactly as in spring_update()
        const float cc = e.dt * e.inv_m;
        const float force = fmaf(e.zeta, f[v] + h4[v], -e.k * q4[c][v]);
        const float vv = fmaf(e.dt, force, p4[c][v]);
        const float uu = fmaf(cc, p4[c][v], q4[c][v]);
        const uint32_t bits = (fabsf(uu) <= e.qmax ? 1u : 0u) | (fabsf(vv) <= e.pmax ? 2u : 0u);
        mk |= bits << (8 * v);
      }
    }
    *reinterpret_cast<floatx4 *>(e.q_out + off) = qn;
    *reinterpret_cast<floatx4 *>(e.p_out + off) = pn;
    if (QP >= 1)
      *reinterpret_cast<uintx2 *>(e.qb_out + off) =
          uintx2{b0[0] | (b0[1] << 16), b0[2] | (b0[3] << 16)};
    if (QP == 3) {
      *reinterpret_cast<uintx2 *>(e.qb_out + e.plane_stride + off) =
          uintx2{b1[0] | (b1[1] << 16), b1[2] | (b1[3] << 16)};
      *reinterpret_cast<uintx2 *>(e.qb_out + 2 * e.plane_stride + off) =
          uintx2{b2[0] | (b2[1] << 16), b2[2] | (b2[3] << 16)};
    }
    if (QP == 0 && e.mask_out) *reinterpret_cast<uint32_t *>(e.mask_out + off) = mk;
  }
}

// The paper-order update in two halves.  q' = clamp(q + (Delta/m) p) needs
// no coupling term, so epi_apply_q computes it, with its BF16 plane(s), and
// stores it while the product of the same tile still runs; epi_apply_p
// applies the coupling once F is in LDS.  Each value is computed with the
// same operations as spring_update (bit-identical results).
template <class T, int QP>
__device__ __forceinline__ void epi_apply_q(const EpiArgs &e, const floatx4 (&q4)[T::CPT],
                                            const floatx4 (&p4)[T::CPT]) {
  const float cdt = e.dt * e.inv_m;
#pragma unroll
  for (int c = 0; c < T::CPT; ++c) {
    const size_t off = (size_t)(e.n0 + T::col(c)) * e.ld + e.m0 + T::row(c);
    floatx4 qn;
    uint32_t b0[4], b1[4], b2[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float u = fmaf(cdt, p4[c][v], q4[c][v]);
      qn[v] = fminf(fmaxf(u, -e.qmax), e.qmax);
      if (QP >= 1) b0[v] = epi_bf16(qn[v]);
      if (QP == 3) {
        const float r1 = qn[v] - __uint_as_float(b0[v] << 16);  // exact
        b1[v] = epi_bf16(r1);
        const float r2 = r1 - __uint_as_float(b1[v] << 16);  // exact
        b2[v] = epi_bf16(r2);
      }
    }
    *reinterpret_cast<floatx4 *>(e.q_out + off) = qn;
    if (QP >= 1)
      *reinterpret_cast<uintx2 *>(e.qb_out + off) =
          uintx2{b0[0] | (b0[1] << 16), b0[2] | (b0[3] << 16)};
    if (QP == 3) {
      *reinterpret_cast<uintx2 *>(e.qb_out + e.plane_stride + off) =
          uintx2{b1[0] | (b1[1] << 16), b1[2] | (b1[3] << 16)};
      *reinterpret_cast<uintx2 *>(e.qb_out + 2 * e.plane_stride + off) =
          uintx2{b2[0] | (b2[1] << 16), b2[2] | (b2[3] << 16)};
    }
  }
}

template <class T, int WALL>
__device__ __forceinline__ void epi_apply_p(const float *t, const EpiArgs &e,
                                            const floatx4 (&q4)[T::CPT],
                                            const floatx4 (&p4)[T::CPT]) {
#pragma unroll
  for (int c = 0; c < T::CPT; ++c) {
    const int col = T::col(c), row = T::row(c);
    const size_t off = (size_t)(e.n0 + col) * e.ld + e.m0 + row;
    const floatx4 f = *reinterpret_cast<const floatx4 *>(t + col * T::LD + row);
    floatx4 h4 = {0.f, 0.f, 0.f, 0.f};
    if (e.h) h4 = *reinterpret_cast<const floatx4 *>(e.h + e.m0 + row);
    floatx4 pn;
    uint32_t mk = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float force = fmaf(e.zeta, f[v] + h4[v], -e.k * q4[c][v]);
      const float vv = fmaf(e.dt, force, p4[c][v]);
      pn[v] = fminf(fmaxf(vv, -e.pmax), e.pmax);
      if (WALL == SI_WALL_INELASTIC || e.mask_out) {
        const float uu = fmaf(e.dt * e.inv_m, p4[c][v], q4[c][v]);
        if (WALL == SI_WALL_INELASTIC && fabsf(uu) > e.qmax) pn[v] = 0.f;
        mk |= ((fabsf(uu) <= e.qmax ? 1u : 0u) | (fabsf(vv) <= e.pmax ? 2u : 0u)) << (8 * v);
      }
    }
    *reinterpret_cast<floatx4 *>(e.p_out + off) = pn;
    if (e.mask_out) *reinterpret_cast<uint32_t *>(e.mask_out + off) = mk;
  }
}

}  // namespace si
