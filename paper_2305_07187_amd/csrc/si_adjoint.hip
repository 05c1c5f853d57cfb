// Adjoint of the relaxed end-energy with respect to the step schedules.
//
// Forward map: the paper-order iteration, Eq. (8) (Eq. (5) with m), with the
// clamping walls of Eq. (6) and of the momentum box (Methods):
//   u_n = q_n + (D_n/m) p_n,           q_{n+1} = clamp(u_n, +-qmax)
//   v_n = p_n + D_n(-k q_n + z_n J q_n), p_{n+1} = clamp(v_n, +-pmax)
// Loss: L = (1/R) sum_r -1/2 q_S^T J q_S (mean over replicas of the
// continuous Ising energy of the final positions, field h = 0).
// Reverse sweep (J symmetric, clamp derivative 1 on the closed interval):
//   lq_S = -(1/R) J q_S, lp_S = 0
//   ub = lq_{n+1} [|u_n| <= qmax],  vb = lp_{n+1} [|v_n| <= pmax]
//   lq_n = ub - D_n k vb + D_n z_n J vb,   lp_n = (D_n/m) ub + vb
//   dL/dD_n = <ub, p_n>/m - k <vb, q_n> + z_n <J vb, q_n>
//   dL/dz_n = D_n <J vb, q_n>
// One backward step is one kernel: the product G = J vb on the FP32 matrix
// cores (vb formed while staging lp and the recorded wall mask), and an
// epilogue that updates the multipliers and forms this workgroup's FP64
// partial sums of <ub, p_n>, <vb, q_n> and <G, q_n>.  A one-block kernel then
// adds the partials in a fixed order (deterministic) and writes the two
// gradient entries of step n.  FP64 is used only for these reductions.
#include "si_f32_gemm.h"

namespace si {

using ACfg = F32Cfg<ADJ_BM, ADJ_BN, 2, 2, 16, 32, 0, 1>;

// Sum of a per-lane double over the workgroup (fixed shuffle/LDS order).
template <int NW>
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(ACfg::NT) void adj_seed_kernel(const float *__restrict__ J,
                                                            const float *__restrict__ q,
                                                            float *__restrict__ lamq,
                                                            float *__restrict__ lamp,
                                                            double *__restrict__ part, int ld,
                                                            float inv_r) {
  __shared__ __attribute__((aligned(16))) float smem[ACfg::LDS_FLOATS];
  __shared__ double red[ACfg::NT / 64];
  const int m0 = blockIdx.x * ACfg::BM, n0 = blockIdx.y * ACfg::BN;
  ACfg::acc_t acc[ACfg::TM][ACfg::TN];
  f32_mainloop<ACfg, B_PLAIN>(J, q, ld, ld, m0, n0, acc, smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wy = wave / ACfg::WN, wx = wave % ACfg::WN;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < ACfg::TM; ++i)
#pragma unroll
    for (int j = 0; j < ACfg::TN; ++j) {
      const int row = m0 + wy * ACfg::WTM + i * 16 + (lane / 16) * 4;
      const int col = n0 + wx * ACfg::WTN + j * 16 + (lane % 16);
      const size_t off = (size_t)col * ld + row;
      const floatx4 q4 = *reinterpret_cast<const floatx4 *>(q + off);
      floatx4 lq;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        lq[v] = -inv_r * acc[i][j][v];
        s += (double)q4[v] * (double)acc[i][j][v];
      }
      *reinterpret_cast<floatx4 *>(lamq + off) = lq;
      *reinterpret_cast<floatx4 *>(lamp + off) = floatx4{0.f, 0.f, 0.f, 0.f};
    }
  s = block_sum<ACfg::NT / 64>(s, red);
  if (threadIdx.x == 0) {
    double *o = part + (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * 3;
    o[0] = s;
    o[1] = 0.0;
    o[2] = 0.0;
  }
}

__global__ __launch_bounds__(ACfg::NT) void adj_step_kernel(
    const float *__restrict__ J, const float *__restrict__ lamq_in,
    const float *__restrict__ lamp_in, const uint8_t *__restrict__ mask,
    const float *__restrict__ qn_, const float *__restrict__ pn_, float *__restrict__ lamq_out,
    float *__restrict__ lamp_out, double *__restrict__ part, const float *__restrict__ dts,
    const float *__restrict__ zetas, int n, float k, float inv_m, int ld) {
  __shared__ __attribute__((aligned(16))) float smem[ACfg::LDS_FLOATS];
  __shared__ double red[ACfg::NT / 64];
  const int m0 = blockIdx.x * ACfg::BM, n0 = blockIdx.y * ACfg::BN;
  ACfg::acc_t acc[ACfg::TM][ACfg::TN];
  // G = J vb, vb = lamp_{n+1} masked by the momentum wall of step n
  f32_mainloop<ACfg, B_MASKED>(J, lamp_in, ld, ld, m0, n0, acc, smem, mask);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wy = wave / ACfg::WN, wx = wave % ACfg::WN;
  const float dt = dts[n], zeta = zetas[n];
  const float c = dt * inv_m;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int i = 0; i < ACfg::TM; ++i)
#pragma unroll
    for (int j = 0; j < ACfg::TN; ++j) {
      const int row = m0 + wy * ACfg::WTM + i * 16 + (lane / 16) * 4;
      const int col = n0 + wx * ACfg::WTN + j * 16 + (lane % 16);
      const size_t off = (size_t)col * ld + row;
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
        const float G = acc[i][j][v];
        oq[v] = fmaf(dt * zeta, G, fmaf(-dt * k, vb, ub));
        op[v] = fmaf(c, ub, vb);
        s0 += (double)ub * (double)p4[v];
        s1 += (double)vb * (double)q4[v];
        s2 += (double)G * (double)q4[v];
      }
      *reinterpret_cast<floatx4 *>(lamq_out + off) = oq;
      *reinterpret_cast<floatx4 *>(lamp_out + off) = op;
    }
  s0 = block_sum<ACfg::NT / 64>(s0, red);
  s1 = block_sum<ACfg::NT / 64>(s1, red);
  s2 = block_sum<ACfg::NT / 64>(s2, red);
  if (threadIdx.x == 0) {
    double *o = part + (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * 3;
    o[0] = s0;
    o[1] = s1;
    o[2] = s2;
  }
}

// One workgroup per step: workgroup b reduces the nwg partial triples of
// step n0 + b, stored at part + b * nwg * 3, in a fixed order.
__global__ __launch_bounds__(256) void adj_reduce_kernel(const double *__restrict__ part, int nwg,
                                                         int mode, double *loss, double *g_dt,
                                                         double *g_zeta, const float *dts,
                                                         const float *zetas, int n0, float k,
                                                         float inv_m, int r_count) {
  __shared__ double red[3][256];
  const int t = threadIdx.x;
  const int n = n0 + (int)blockIdx.x;
  part += (size_t)blockIdx.x * nwg * 3;
  double s[3] = {0.0, 0.0, 0.0};
  for (int w = t; w < nwg; w += 256)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] += part[(size_t)w * 3 + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) red[c][t] = s[c];
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int c = 0; c < 3; ++c) red[c][t] += red[c][t + h];
    __syncthreads();
  }
  if (t == 0) {
    if (mode == 0) {
      loss[0] = -0.5 * red[0][0] / (double)r_count;
    } else {
      const double dt = dts[n], zeta = zetas[n];
      g_dt[n] = red[0][0] * (double)inv_m - (double)k * red[1][0] + zeta * red[2][0];
      g_zeta[n] = dt * red[2][0];
    }
  }
}

__global__ void fill_f64_kernel(double *p, int64_t count, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_adj_seed(const float *J, const float *q, float *lamq, float *lamp, double *part,
                           int32_t n_pad, int32_t r_pad, float inv_r, hipStream_t s) {
  if (n_pad % ACfg::BM || r_pad % ACfg::BN) return hipErrorInvalidValue;
  dim3 grid(n_pad / ACfg::BM, r_pad / ACfg::BN);
  adj_seed_kernel<<<grid, ACfg::NT, 0, s>>>(J, q, lamq, lamp, part, n_pad, inv_r);
  return hipGetLastError();
}

hipError_t launch_adj_step(const float *J, const float *lamq_in, const float *lamp_in,
                           const uint8_t *mask, const float *q_n, const float *p_n,
                           float *lamq_out, float *lamp_out, double *part, const float *dt,
                           const float *zeta, int32_t n, float k, float inv_m, int32_t n_pad,
                           int32_t r_pad, hipStream_t s) {
  if (n_pad % ACfg::BM || r_pad % ACfg::BN) return hipErrorInvalidValue;
  dim3 grid(n_pad / ACfg::BM, r_pad / ACfg::BN);
  adj_step_kernel<<<grid, ACfg::NT, 0, s>>>(J, lamq_in, lamp_in, mask, q_n, p_n, lamq_out,
                                             lamp_out, part, dt, zeta, n, k, inv_m, n_pad);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const double *part, int32_t nwg, int32_t mode, double *loss,
                             double *g_dt, double *g_zeta, const float *dt, const float *zeta,
                             int32_t n, int32_t n_steps, float k, float inv_m, int32_t r_count,
                             hipStream_t s) {
  if (n_steps < 1 || (mode == 0 && n_steps != 1)) return hipErrorInvalidValue;
  adj_reduce_kernel<<<n_steps, 256, 0, s>>>(part, nwg, mode, loss, g_dt, g_zeta, dt, zeta, n, k,
                                            inv_m, r_count);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t b = (count + 255) / 256;
  if (b > 1024) b = 1024;
  fill_f64_kernel<<<(int)b, 256, 0, s>>>(p, count, v);
  return hipGetLastError();
}

}  // namespace si
