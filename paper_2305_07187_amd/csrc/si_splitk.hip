// Split contraction for problems with fewer output tiles than CUs.
//
// With R = 64 replicas and N = 2000 spins the coupling product J.Q has
// only 2048 x 64 outputs: 128 tiles of 32 x 32 leave half the CUs idle and
// each tile runs through the whole contraction.  Here the contraction is cut
// into S ranges of k; launch 1 computes every (tile, range) product into a
// workspace W[s][r_pad][n_pad] (S times as many workgroups, each S times
// shorter), and launch 2 adds the S partial products in a fixed order
// (deterministic) and applies the update of Eq. (8) with the walls, or the
// adjoint's multiplier update, element by element in the state's layout.
#include "si_epilogue.h"
#include "si_f32_gemm.h"

namespace si {

// Partial products of one (tile, range) work item.  BMODE = B_MASKED
// multiplies the position operand by the momentum-wall bit of `mask` (the
// adjoint's J vb).
template <class C, int BMODE>
__global__ __launch_bounds__(C::NT) void coupling_partial_kernel(const float *__restrict__ J,
                                                                 const float *__restrict__ X,
                                                                 const uint8_t *__restrict__ mask,
                                                                 int ld, int r_pad, int K,
                                                                 int klen, float *__restrict__ W) {
  __shared__ __attribute__((aligned(16))) float smem[C::LDS_FLOATS];
  using T = EpiTile<C::BM, C::BN, C::NT>;
  static_assert(T::BYTES <= C::LDS_FLOATS * 4, "the partial tile fits in the main loop's LDS");
  const int ncol = r_pad / C::BN, tiles = (ld / C::BM) * ncol;
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int t = b % tiles, s = b / tiles;
  const int m0 = (t / ncol) * C::BM, n0 = (t % ncol) * C::BN;
  const int k0 = s * klen;
  const int kl = K - k0 < klen ? K - k0 : klen;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  constexpr int G = C::M::NACC / 4;
  typename C::acc_t acc[C::TM][C::TN];
  if (kl > 0) {
    if constexpr (C::STAGES > 0 && BMODE == B_PLAIN)
      f32_mainloop_dma<C>(J + k0, X + k0, ld, kl, m0, n0, acc, smem);
    else
      f32_mainloop<C, BMODE>(J + k0, X + k0, ld, kl, m0, n0, acc, smem,
                             BMODE == B_MASKED ? mask + k0 : nullptr);
  } else {
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
#pragma unroll
        for (int v = 0; v < C::M::NACC; ++v) acc[i][j][v] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int j = 0; j < C::TN; ++j)
        epi_put(smem, T::LD, wy * C::WTM + i * C::MB + g * 8 + (lane / C::MB) * 4,
                wx * C::WTN + j * C::MB + (lane % C::MB), acc[i][j][4 * g], acc[i][j][4 * g + 1],
                acc[i][j][4 * g + 2], acc[i][j][4 * g + 3]);
  __syncthreads();
  float *w = W + (size_t)s * r_pad * ld;
#pragma unroll
  for (int c = 0; c < T::CPT; ++c) {
    const int col = T::col(c), row = T::row(c);
    *reinterpret_cast<floatx4 *>(w + (size_t)(n0 + col) * ld + m0 + row) =
        *reinterpret_cast<const floatx4 *>(smem + col * T::LD + row);
  }
}

// Sum of the S partial products at element offset off (chunk of four).
__device__ __forceinline__ floatx4 split_sum(const float *__restrict__ W, int64_t plane, int S,
                                             int64_t off) {
  floatx4 f = *reinterpret_cast<const floatx4 *>(W + off);
  for (int s = 1; s < S; ++s) f += *reinterpret_cast<const floatx4 *>(W + s * plane + off);
  return f;
}

// Update of Eq. (8) with the walls for every element, F from the partials.
template <int ORDER, int WALL>
__global__ __launch_bounds__(256) void update_split_kernel(StepArgs a, const float *__restrict__ W,
                                                           int S) {
  const int64_t plane = (int64_t)a.r_pad * a.ld, chunks = plane / 4;
  const float dt = a.dt[a.t], zeta = a.zeta[a.t];
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < chunks;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t off = c * 4;
    const int row = (int)(off % a.ld);
    const floatx4 f = split_sum(W, plane, S, off);
    floatx4 h4 = {0.f, 0.f, 0.f, 0.f};
    if (a.h) h4 = *reinterpret_cast<const floatx4 *>(a.h + row);
    const floatx4 q4 = *reinterpret_cast<const floatx4 *>(a.q_in + off);
    const floatx4 p4 = *reinterpret_cast<const floatx4 *>(a.p_in + off);
    floatx4 qn, pn;
    uint32_t mk = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float qv, pv;
      spring_update<ORDER, WALL>(q4[v], p4[v], f[v] + h4[v], dt, zeta, a.k, a.inv_m, a.qmax,
                                 a.pmax, qv, pv);
      qn[v] = qv;
      pn[v] = pv;
      if (a.mask_out) {
        // the unclamped values, recomputed exactly as in spring_update()
        const float cc = dt * a.inv_m;
        const float force = fmaf(zeta, f[v] + h4[v], -a.k * q4[v]);
        const float vv = fmaf(dt, force, p4[v]);
        const float uu = fmaf(cc, p4[v], q4[v]);
        mk |= ((fabsf(uu) <= a.qmax ? 1u : 0u) | (fabsf(vv) <= a.pmax ? 2u : 0u)) << (8 * v);
      }
    }
    *reinterpret_cast<floatx4 *>(a.q_out + off) = qn;
    *reinterpret_cast<floatx4 *>(a.p_out + off) = pn;
    if (a.mask_out) *reinterpret_cast<uint32_t *>(a.mask_out + off) = mk;
  }
}

// Adjoint multiplier update with G = J vb from the partials; FP64 partial
// sums of <ub, p_n>, <vb, q_n>, <G, q_n> per workgroup (fixed order).
__global__ __launch_bounds__(256) void adj_update_split_kernel(
    const float *__restrict__ W, int S, const float *__restrict__ lamq_in,
    const float *__restrict__ lamp_in, const uint8_t *__restrict__ mask,
    const float *__restrict__ qn_, const float *__restrict__ pn_, float *__restrict__ lamq_out,
    float *__restrict__ lamp_out, double *__restrict__ part, const float *__restrict__ dts,
    const float *__restrict__ zetas, int n, float k, float inv_m, int ld, int r_pad) {
  __shared__ double red[3][4];
  const int64_t plane = (int64_t)r_pad * ld, chunks = plane / 4;
  const float dt = dts[n], zeta = zetas[n];
  const float c = dt * inv_m;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t ch = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ch < chunks;
       ch += (int64_t)gridDim.x * blockDim.x) {
    const int64_t off = ch * 4;
    const floatx4 G = split_sum(W, plane, S, off);
    const floatx4 lq = *reinterpret_cast<const floatx4 *>(lamq_in + off);
    const floatx4 lp = *reinterpret_cast<const floatx4 *>(lamp_in + off);
    const floatx4 q4 = *reinterpret_cast<const floatx4 *>(qn_ + off);
    const floatx4 p4 = *reinterpret_cast<const floatx4 *>(pn_ + off);
    const uint32_t mk = *reinterpret_cast<const uint32_t *>(mask + off);
    floatx4 oq, op;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t b = mk >> (8 * v);
      const float ub = (b & 1u) ? lq[v] : 0.f;
      const float vb = (b & 2u) ? lp[v] : 0.f;
      oq[v] = fmaf(dt * zeta, G[v], fmaf(-dt * k, vb, ub));
      op[v] = fmaf(c, ub, vb);
      s0 += (double)ub * (double)p4[v];
      s1 += (double)vb * (double)q4[v];
      s2 += (double)G[v] * (double)q4[v];
    }
    *reinterpret_cast<floatx4 *>(lamq_out + off) = oq;
    *reinterpret_cast<floatx4 *>(lamp_out + off) = op;
  }
  // workgroup sums: fixed shuffle and wave order
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s0 += __shfl_xor(s0, off);
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
    red[2][wave] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double *o = part + (size_t)blockIdx.x * 3;
#pragma unroll
    for (int q = 0; q < 3; ++q) o[q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  }
}

// Tiles of the step kernel with a split form: the automatic choices for
// problems with fewer tiles than CUs.
#define SI_HAS_SPLIT(id) \
  ((id) == 3 || (id) == 6 || (id) == 12 || (id) == 2 || (id) == 14 || (id) == 9 || (id) == 26 || \
   (id) == 27)

template <class C>
static hipError_t split_step(const StepArgs &a, hipStream_t s) {
  if (a.n_pad % C::BM || a.r_pad % C::BN || a.ld % C::BK || !a.fsplit || a.ksplit < 2)
    return hipErrorInvalidValue;
  const int K = (a.n + C::BK - 1) / C::BK * C::BK < a.ld ? (a.n + C::BK - 1) / C::BK * C::BK : a.ld;
  const int per = (K + a.ksplit - 1) / a.ksplit;
  const int klen = (per + C::BK - 1) / C::BK * C::BK;
  const int tiles = (a.n_pad / C::BM) * (a.r_pad / C::BN);
  coupling_partial_kernel<C, B_PLAIN><<<tiles * a.ksplit, C::NT, 0, s>>>(
      a.J, a.q_in, nullptr, a.ld, a.r_pad, K, klen, a.fsplit);
  const int64_t chunks = (int64_t)a.r_pad * a.ld / 4;
  int64_t blocks = (chunks + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  switch (a.order * 2 + a.wall) {
    case 0: update_split_kernel<SI_ORDER_PAPER, SI_WALL_CLAMP><<<(int)blocks, 256, 0, s>>>(a, a.fsplit, a.ksplit); break;
    case 1: update_split_kernel<SI_ORDER_PAPER, SI_WALL_INELASTIC><<<(int)blocks, 256, 0, s>>>(a, a.fsplit, a.ksplit); break;
    case 2: update_split_kernel<SI_ORDER_SYMPLECTIC, SI_WALL_CLAMP><<<(int)blocks, 256, 0, s>>>(a, a.fsplit, a.ksplit); break;
    case 3: update_split_kernel<SI_ORDER_SYMPLECTIC, SI_WALL_INELASTIC><<<(int)blocks, 256, 0, s>>>(a, a.fsplit, a.ksplit); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool tile_has_split(int32_t tile) {
  switch (tile) {
#define SI_HS(id, bm, bn, wm, wn, mb, bk, st, ks) \
  case id:                                       \
    return SI_HAS_SPLIT(id);
    SI_F32_TILES(SI_HS)
#undef SI_HS
    default: return false;
  }
}

hipError_t launch_step_f32_split(int32_t tile, const StepArgs &a, hipStream_t s) {
  switch (tile) {
#define SI_SL(id, bm, bn, wm, wn, mb, bk, st, ks)                              \
  case id:                                                                    \
    if constexpr (SI_HAS_SPLIT(id))                                           \
      return split_step<F32Cfg<bm, bn, wm, wn, mb, bk, st, ks>>(a, s);        \
    else                                                                      \
      return hipErrorInvalidValue;
    SI_F32_TILES(SI_SL)
#undef SI_SL
    default: return hipErrorInvalidValue;
  }
}

// Adjoint backward step with the split contraction (32 x 32 tiles of the
// 16x16x4 MFMA, register-staged, masked position operand).
using ASplitCfg = F32Cfg<ADJ_BM, ADJ_BN, 2, 2, 16, 32, 0, 1>;

int32_t adj_split_groups(int32_t n_pad, int32_t r_pad) {
  const int64_t chunks = (int64_t)n_pad * r_pad / 4;
  int64_t blocks = (chunks + 255) / 256;
  return (int32_t)(blocks > 1024 ? 1024 : blocks);
}

hipError_t launch_adj_step_split(const float *J, const float *lamq_in, const float *lamp_in,
                                 const uint8_t *mask, const float *q_n, const float *p_n,
                                 float *lamq_out, float *lamp_out, double *part, const float *dt,
                                 const float *zeta, int32_t n, float k, float inv_m, int32_t n_pad,
                                 int32_t n_spins, int32_t r_pad, int32_t ksplit, float *W,
                                 hipStream_t s) {
  using C = ASplitCfg;
  if (n_pad % C::BM || r_pad % C::BN || ksplit < 2 || !W) return hipErrorInvalidValue;
  const int K = (n_spins + C::BK - 1) / C::BK * C::BK < n_pad ? (n_spins + C::BK - 1) / C::BK * C::BK
                                                            : n_pad;
  const int per = (K + ksplit - 1) / ksplit;
  const int klen = (per + C::BK - 1) / C::BK * C::BK;
  const int tiles = (n_pad / C::BM) * (r_pad / C::BN);
  coupling_partial_kernel<C, B_MASKED><<<tiles * ksplit, C::NT, 0, s>>>(J, lamp_in, mask, n_pad,
                                                                         r_pad, K, klen, W);
  adj_update_split_kernel<<<adj_split_groups(n_pad, r_pad), 256, 0, s>>>(
      W, ksplit, lamq_in, lamp_in, mask, q_n, p_n, lamq_out, lamp_out, part, dt, zeta, n, k,
      inv_m, n_pad, r_pad);
  return hipGetLastError();
}

}  // namespace si
