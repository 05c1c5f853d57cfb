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
#include "si_epilogue.h"
#include "si_trace.h"
#include "si_f32_gemm.h"

namespace si {

// Contraction length for n spins: n rounded up to the slab depth.  Columns
// of J beyond n are zero padding, so stopping there drops only exact zeros.
template <class C>
__device__ __forceinline__ int kdim(int n, int ld) {
  const int k = (n + C::BK - 1) / C::BK * C::BK;
  return k < ld ? k : ld;
}

// One BM x BN output tile of one step: contraction over k in [0, K) of the
// rows m0.. of J (leading dimension ld) with the replicas n0.. of q_in, then
// the update.  Shared by the single-instance and the batched kernels.
template <class C, int ORDER, int WALL>
__device__ __forceinline__ void step_tile(const StepArgs &a, const float *__restrict__ Jm,
                                          const float *__restrict__ q_in,
                                          const float *__restrict__ p_in, float *__restrict__ q_out,
                                          float *__restrict__ p_out, int ld, int K, int m0, int n0,
                                          float *smem) {
  using T = EpiTile<C::BM, C::BN, C::NT>;
  static_assert(T::BYTES <= C::LDS_FLOATS * 4, "the update tile fits in the main loop's LDS");
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  constexpr int G = C::M::NACC / 4;
  EpiArgs e;
  e.q_in = q_in;
  e.p_in = p_in;
  e.h = a.h;
  e.q_out = q_out;
  e.p_out = p_out;
  e.qb_out = nullptr;
  e.plane_stride = 0;
  e.mask_out = a.mask_out;
  e.ld = ld;
  e.m0 = m0;
  e.n0 = n0;
  // The state this thread updates is loaded before the contraction so that
  // its latency overlaps the matrix work.
  floatx4 q4[T::CPT], p4[T::CPT];
  epi_load<T>(e, q4, p4);

  typename C::acc_t acc[C::TM][C::TN];
  if constexpr (C::STAGES > 0)
    f32_mainloop_dma<C>(Jm, q_in, ld, K, m0, n0, acc, smem);
  else
    f32_mainloop<C, B_PLAIN>(Jm, q_in, ld, K, m0, n0, acc, smem);

  // F through LDS into the state's layout (the main loop has released it)
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
  e.dt = a.dt[a.t];
  e.zeta = a.zeta[a.t];
  e.k = a.k;
  e.inv_m = a.inv_m;
  e.qmax = a.qmax;
  e.pmax = a.pmax;
  epi_apply<T, ORDER, WALL, 0>(smem, e, q4, p4);
}

template <class C, int ORDER, int WALL>
__global__ __launch_bounds__(C::NT) void step_f32_kernel(StepArgs a) {
  __shared__ __attribute__((aligned(16))) float smem[C::LDS_FLOATS];
  const int t = xcd_tile(blockIdx.x, gridDim.x), ncol = a.r_pad / C::BN;
  step_tile<C, ORDER, WALL>(a, a.J, a.q_in, a.p_in, a.q_out, a.p_out, a.ld, kdim<C>(a.n, a.ld),
                            (t / ncol) * C::BM, (t % ncol) * C::BN, smem);
}

// Grid-wide barrier of a resident launch, without atomic read-modify-write:
// group g publishes the number of steps it has completed in flags[g] (a
// release store, which also writes this XCD's L2 back), and the first wave
// of every group polls all the flags, one per lane, with plain loads until
// each has reached `step`.  A single acquire fence per group then
// invalidates the stale lines before the next step reads q.  The wait is
// bounded (about 2 s of the 100 MHz real-time counter, and at most 2^26
// polls): a barrier that cannot complete sets *err and every group leaves
// instead of hanging.
__device__ __forceinline__ bool grid_barrier(uint32_t *flags, uint32_t step, int32_t *err) {
  __shared__ int32_t pass;
  const int groups = gridDim.x;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(flags + blockIdx.x, step, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const uint64_t start = __builtin_amdgcn_s_memrealtime();
    int32_t ok = 1;
    uint32_t polls = 0;
    for (;;) {
      bool ready = true;
      for (int g = lane; g < groups; g += 64)
        ready &= __hip_atomic_load(flags + g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= step;
      if (__all(ready)) break;
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (__builtin_amdgcn_s_memrealtime() - start > 200000000ull || ++polls > (1u << 26)) {
        if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (lane == 0) pass = ok;
  }
  __syncthreads();
  return pass != 0;
}

template <class C, int ORDER, int WALL>
__global__ __launch_bounds__(C::NT) void resident_f32_kernel(StepArgs a, ResidentArgs r) {
  __shared__ __attribute__((aligned(16))) float smem[C::LDS_FLOATS];
  const int groups = gridDim.x;
  const int t = xcd_tile(blockIdx.x, groups), ncol = a.r_pad / C::BN;
  const int m0 = (t / ncol) * C::BM, n0 = (t % ncol) * C::BN;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wy = wave / C::WN, wx = wave % C::WN;
  constexpr int G = C::M::NACC / 4;
  const int ld = a.ld, K = kdim<C>(a.n, a.ld);
  floatx4 q4[C::TM][G][C::TN], p4[C::TM][G][C::TN], h4[C::TM][G];
  int cur = r.cur;
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int row = m0 + wy * C::WTM + i * C::MB + g * 8 + (lane / C::MB) * 4;
      h4[i][g] = floatx4{0.f, 0.f, 0.f, 0.f};
      if (a.h) h4[i][g] = *reinterpret_cast<const floatx4 *>(a.h + row);
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const size_t off = (size_t)(n0 + wx * C::WTN + j * C::MB + (lane % C::MB)) * ld + row;
        q4[i][g][j] = *reinterpret_cast<const floatx4 *>(r.q[cur] + off);
        p4[i][g][j] = *reinterpret_cast<const floatx4 *>(r.p[cur] + off);
      }
    }
  for (int s = 0; s < r.n_steps; ++s) {
    typename C::acc_t acc[C::TM][C::TN];
    if constexpr (C::STAGES > 0)
      f32_mainloop_dma<C>(a.J, r.q[cur], ld, K, m0, n0, acc, smem);
    else
      f32_mainloop<C, B_PLAIN>(a.J, r.q[cur], ld, K, m0, n0, acc, smem);
    const float dt = a.dt[a.t + s], zeta = a.zeta[a.t + s];
    float *qd = r.q[cur ^ 1];
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int row = m0 + wy * C::WTM + i * C::MB + g * 8 + (lane / C::MB) * 4;
#pragma unroll
        for (int j = 0; j < C::TN; ++j) {
          const size_t off = (size_t)(n0 + wx * C::WTN + j * C::MB + (lane % C::MB)) * ld + row;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            float qv, pv;
            spring_update<ORDER, WALL>(q4[i][g][j][v], p4[i][g][j][v], acc[i][j][4 * g + v] + h4[i][g][v],
                                dt, zeta, a.k, a.inv_m, a.qmax, a.pmax, qv, pv);
            q4[i][g][j][v] = qv;
            p4[i][g][j][v] = pv;
          }
          *reinterpret_cast<floatx4 *>(qd + off) = q4[i][g][j];
        }
      }
    cur ^= 1;
    if (s + 1 < r.n_steps && !grid_barrier(r.count, (uint32_t)(s + 1), r.err)) return;
  }
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int row = m0 + wy * C::WTM + i * C::MB + g * 8 + (lane / C::MB) * 4;
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const size_t off = (size_t)(n0 + wx * C::WTN + j * C::MB + (lane % C::MB)) * ld + row;
        *reinterpret_cast<floatx4 *>(r.p[cur] + off) = p4[i][g][j];
      }
    }
}

// Batched form: one launch advances every instance of a batch by one step.
// Work item w = (instance, row tile, column tile); the host orders the list
// (whole instances per XCD, costliest items first on each).
template <class C, int ORDER, int WALL>
__global__ __launch_bounds__(C::NT) void step_batch_f32_kernel(StepArgs a,
                                                               const BatchDesc *__restrict__ descs,
                                                               const int4 *__restrict__ items,
                                                               int cur,
                                                               unsigned long long *trace) {
  const unsigned long long start = wall_clock64();
  __shared__ __attribute__((aligned(16))) float smem[C::LDS_FLOATS];
  const int4 it = items[blockIdx.x];
  const BatchDesc d = descs[it.x];
  step_tile<C, ORDER, WALL>(a, d.J, cur ? d.q1 : d.q0, cur ? d.p1 : d.p0, cur ? d.q0 : d.q1,
                            cur ? d.p0 : d.p1, d.n_pad, kdim<C>(d.n, d.n_pad), it.y * C::BM,
                            it.z * C::BN, smem);
  if (trace) batch_trace_record(trace, start);
}

TileShape tile_shape(int32_t tile) {
  switch (tile) {
#define SI_SHAPE(id, bm, bn, wm, wn, mb, bk, st, ks) \
  case id:                                           \
    return {bm, bn,                                  \
            "step_f32_" #bm "x" #bn "_w" #wm "x" #wn "_mfma" #mb "_k" #bk "_s" #st "_a" #ks, bk};
    SI_F32_TILES(SI_SHAPE)
#undef SI_SHAPE
    default: return {0, 0, "invalid", 0};
  }
}

template <class C>
static hipError_t launch_cfg(const StepArgs &a, hipStream_t s) {
  if (a.n_pad % C::BM || a.r_pad % C::BN || a.n_pad % C::BK) return hipErrorInvalidValue;
  dim3 grid((a.n_pad / C::BM) * (a.r_pad / C::BN)), block(C::NT);
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

template <class C>
static const void *resident_kernel(int order, int wall) {
  switch (order * 2 + wall) {
    case 0: return reinterpret_cast<const void *>(&resident_f32_kernel<C, SI_ORDER_PAPER, SI_WALL_CLAMP>);
    case 1: return reinterpret_cast<const void *>(&resident_f32_kernel<C, SI_ORDER_PAPER, SI_WALL_INELASTIC>);
    case 2: return reinterpret_cast<const void *>(&resident_f32_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_CLAMP>);
    case 3: return reinterpret_cast<const void *>(&resident_f32_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_INELASTIC>);
    default: return nullptr;
  }
}

template <class C>
static hipError_t resident_groups(int order, int wall, int *groups) {
  const void *k = resident_kernel<C>(order, wall);
  if (!k) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(groups, k, C::NT, 0);
}

template <class C>
static hipError_t resident_launch(const StepArgs &a, const ResidentArgs &r, hipStream_t s) {
  if (a.n_pad % C::BM || a.r_pad % C::BN || a.n_pad % C::BK) return hipErrorInvalidValue;
  const void *k = resident_kernel<C>(a.order, a.wall);
  if (!k) return hipErrorInvalidValue;
  StepArgs aa = a;
  ResidentArgs rr = r;
  void *args[] = {&aa, &rr};
  return hipLaunchCooperativeKernel(k, dim3((a.n_pad / C::BM) * (a.r_pad / C::BN)), dim3(C::NT),
                                    args, 0, s);
}

// Tiles with a resident form: the automatic choices of the FP32 path.
#define SI_HAS_RESIDENT(id) ((id) == 27 || (id) == 26 || (id) == 2 || (id) == 1 || (id) == 3)
hipError_t resident_f32_groups_per_cu(int32_t tile, int32_t order, int32_t wall, int *groups) {
  *groups = 0;
  switch (tile) {
#define SI_RES_Q(id, bm, bn, wm, wn, mb, bk, st, ks)                                  \
  case id:                                                                           \
    if constexpr (SI_HAS_RESIDENT(id))                                               \
      return resident_groups<F32Cfg<bm, bn, wm, wn, mb, bk, st, ks>>(order, wall, groups); \
    else                                                                             \
      return hipSuccess;
    SI_F32_TILES(SI_RES_Q)
#undef SI_RES_Q
    default: return hipSuccess;
  }
}

hipError_t launch_resident_f32(int32_t tile, const StepArgs &a, const ResidentArgs &r,
                               hipStream_t s) {
  switch (tile) {
#define SI_RES_L(id, bm, bn, wm, wn, mb, bk, st, ks)                    \
  case id:                                                             \
    if constexpr (SI_HAS_RESIDENT(id))                                 \
      return resident_launch<F32Cfg<bm, bn, wm, wn, mb, bk, st, ks>>(a, r, s); \
    else                                                               \
      return hipErrorInvalidValue;
    SI_F32_TILES(SI_RES_L)
#undef SI_RES_L
    default: return hipErrorInvalidValue;
  }
}

// Batched tiles, picked per batch (the autotuner times both): 128 x 64
// (eight waves of 32 x 32) or 64 x 64 (four waves; the configuration of
// single-instance tile 14), 32x32x2 MFMA over a 4-stage direct-to-LDS ring.
// Both have the contraction order of every single-instance direct-to-LDS tile
// with one accumulator chain, so the pick never changes a result.
using BatchCfg = F32Cfg<BATCH_BM, BATCH_BN, 4, 2, 32, 32, 4, 1>;
using BatchCfg64 = F32Cfg<64, BATCH_BN, 2, 2, 32, 32, 4, 1>;

template <class C>
static hipError_t launch_batch_cfg(const StepArgs &a, const BatchDesc *descs, const int4 *items,
                                   int32_t n_items, int32_t cur, unsigned long long *trace,
                                   hipStream_t s) {
  dim3 grid(n_items), block(C::NT);
  switch (a.order * 2 + a.wall) {
    case 0: step_batch_f32_kernel<C, SI_ORDER_PAPER, SI_WALL_CLAMP><<<grid, block, 0, s>>>(a, descs, items, cur, trace); break;
    case 1: step_batch_f32_kernel<C, SI_ORDER_PAPER, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(a, descs, items, cur, trace); break;
    case 2: step_batch_f32_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_CLAMP><<<grid, block, 0, s>>>(a, descs, items, cur, trace); break;
    case 3: step_batch_f32_kernel<C, SI_ORDER_SYMPLECTIC, SI_WALL_INELASTIC><<<grid, block, 0, s>>>(a, descs, items, cur, trace); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step_batch_f32(const StepArgs &a, const BatchDesc *descs, const int4 *items,
                                 int32_t n_items, int32_t cur, int32_t btile,
                                 unsigned long long *trace, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  static_assert(BatchCfg::BM == 128 && BatchCfg64::BM == 64, "batch tile rows");
  switch (btile) {
    case 1: return launch_batch_cfg<BatchCfg>(a, descs, items, n_items, cur, trace, s);
    case 2: return launch_batch_cfg<BatchCfg64>(a, descs, items, n_items, cur, trace, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_f32(int32_t tile, const StepArgs &a, hipStream_t s) {
  if (a.ksplit > 1) return launch_step_f32_split(tile, a, s);
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

// One 64 x 64 tile: the partial sums of this tile's rows for its 64
// replicas, written to part_row[n0 ..].
__device__ __forceinline__ void energy_f32_tile(const float *J, const float *q, const float *h,
                                                float *part_row, int ld, int m0, int n0) {
  __shared__ __attribute__((aligned(16))) float smem[ECfg::LDS_FLOATS];
  __shared__ float red[ECfg::WM][ECfg::BN];
  ECfg::acc_t acc[ECfg::TM][ECfg::TN];
  f32_mainloop<ECfg, B_SIGN>(J, q, ld, ld, m0, n0, acc, smem);
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
    part_row[n0 + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void energy_f32_partial_kernel(const float *J, const float *q,
                                                                 const float *h, float *part,
                                                                 int ld, int r_pad) {
  energy_f32_tile(J, q, h, part + (size_t)blockIdx.x * r_pad, ld, blockIdx.x * ECfg::BM,
                  blockIdx.y * ECfg::BN);
}

// Neumaier-compensated FP32 sum of one replica's row-tile partials (stride
// r_pad), in fixed order.
__device__ __forceinline__ double energy_f32_sum(const float *part, int n_tiles, int r_pad,
                                                 int col, float scale) {
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
  return (double)scale * ((double)s + (double)comp);
}

__global__ void energy_f32_finalize_kernel(const float *part, int n_tiles, int r, int r_pad,
                                           double *e, float scale) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= r) return;
  e[col] = energy_f32_sum(part, n_tiles, r_pad, col, scale);
}

// Batch: work item (instance, row tile, column tile) over the instances with
// real couplings; instance i's positions start at q + d.soff and its
// row-tile partials at part + d.part_row * r_pad.
__global__ __launch_bounds__(256) void energy_f32_batch_kernel(const EBatchDesc *__restrict__ descs,
                                                               const int4 *__restrict__ items,
                                                               const float *q, float *part,
                                                               int r_pad) {
  const int4 it = items[blockIdx.x];
  const EBatchDesc d = descs[it.x];
  energy_f32_tile(d.J, q + d.soff, nullptr, part + ((size_t)d.part_row + it.y) * r_pad, d.n_pad,
                  it.y * ECfg::BM, it.z * ECfg::BN);
}

__global__ void energy_f32_batch_finalize_kernel(const float *part,
                                                 const EBatchDesc *__restrict__ descs, int n_inst,
                                                 int r, int r_pad, double *e) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_inst * r) return;
  const int i = (int)(idx / r), col = (int)(idx % r);
  const EBatchDesc d = descs[i];
  if (d.J8) return;
  e[idx] = energy_f32_sum(part + (size_t)d.part_row * r_pad, d.n_pad / ECfg::BM, r_pad, col,
                          -0.5f);
}

// ---------------------------------------------------------------------------
// Hamiltonian of the spring system, Eq. (7), per replica (q0 = 0, qdot = p/m):
//   H = sum_i [ p_i^2 / (2m) + k q_i^2 / 2 ] + zeta_t H_Ising(q),
//   H_Ising(q) = -1/2 q^T J q - h.q  (the continuous Ising energy)
// = sum_i [ p_i^2/(2m) + k q_i^2/2 - zeta_t q_i (G_i + 2 h_i) / 2 ],  G = J q.
// Per row tile partial sums; the energy finaliser adds them (scale 1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void hamiltonian_partial_kernel(
    const float *J, const float *q, const float *p, const float *h, const float *zetas, int t,
    float k, float inv_m, float *part, int ld, int r_pad) {
  __shared__ __attribute__((aligned(16))) float smem[ECfg::LDS_FLOATS];
  __shared__ float red[ECfg::WM][ECfg::BN];
  const int m0 = blockIdx.x * ECfg::BM;
  const int n0 = blockIdx.y * ECfg::BN;
  ECfg::acc_t acc[ECfg::TM][ECfg::TN];
  f32_mainloop<ECfg, B_PLAIN>(J, q, ld, ld, m0, n0, acc, smem);
  const float zeta = zetas[t];
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
        const size_t off = (size_t)(n0 + lcol) * ld + row;
        const floatx4 q4 = *reinterpret_cast<const floatx4 *>(q + off);
        const floatx4 p4 = *reinterpret_cast<const floatx4 *>(p + off);
        floatx4 h4 = {0.f, 0.f, 0.f, 0.f};
        if (h) h4 = *reinterpret_cast<const floatx4 *>(h + row);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          c += 0.5f * p4[v] * p4[v] * inv_m + 0.5f * k * q4[v] * q4[v] -
               0.5f * zeta * q4[v] * (acc[i][j][4 * g + v] + 2.f * h4[v]);
      }
    for (int off = ECfg::MB; off < 64; off <<= 1) c += __shfl_xor(c, off);
    if (lane < ECfg::MB) red[wy][lcol] = c;
  }
  __syncthreads();
  if (threadIdx.x < ECfg::BN) {
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < ECfg::WM; ++w) sum += red[w][threadIdx.x];
    part[(size_t)blockIdx.x * r_pad + n0 + threadIdx.x] = sum;
  }
}

hipError_t launch_hamiltonian_partial(const float *J, const float *q, const float *p,
                                      const float *h, const float *zetas, int32_t t, float k,
                                      float inv_m, float *part, int32_t n_pad, int32_t r_pad,
                                      hipStream_t s) {
  if (n_pad % ECfg::BM || r_pad % ECfg::BN) return hipErrorInvalidValue;
  dim3 grid(n_pad / ECfg::BM, r_pad / ECfg::BN);
  hamiltonian_partial_kernel<<<grid, 256, 0, s>>>(J, q, p, h, zetas, t, k, inv_m, part, n_pad,
                                                  r_pad);
  return hipGetLastError();
}

// Keep, per replica, the lowest energy seen and the spins that had it.  A
// replica whose record is not valid (valid[r] == 0: nothing recorded since
// the last reset) takes the current energy unconditionally.  The reset is a
// device flag so that captured launch sequences replay correctly.
__device__ __forceinline__ void best_update_one(double en, double *best_e, int32_t *valid,
                                                const int8_t *src, int8_t *dst, int n_pad) {
  if (*valid && !(en < *best_e)) return;  // block-uniform decision
  for (int i = threadIdx.x * 4; i < n_pad; i += blockDim.x * 4)
    *reinterpret_cast<char4 *>(dst + i) = *reinterpret_cast<const char4 *>(src + i);
  __syncthreads();
  if (threadIdx.x == 0) {
    *best_e = en;
    *valid = 1;
  }
}

__global__ void best_update_kernel(const double *e, double *best_e, int32_t *valid,
                                   const int8_t *S8, int8_t *best_s, int n_pad) {
  const int r = blockIdx.x;
  best_update_one(e[r], best_e + r, valid + r, S8 + (size_t)r * n_pad,
                  best_s + (size_t)r * n_pad, n_pad);
}

// Batch: block i * r + col updates replica col of instance i (energies and
// records in the instances-by-replicas order of the batch outputs; spins in
// the batch's state layout).
__global__ void best_update_batch_kernel(const double *e, double *best_e, int32_t *valid,
                                         const int8_t *S8, int8_t *best_s,
                                         const EBatchDesc *__restrict__ descs, int r) {
  const int64_t idx = blockIdx.x;
  const int i = (int)(idx / r), col = (int)(idx % r);
  const EBatchDesc d = descs[i];
  const size_t off = (size_t)d.soff + (size_t)col * d.n_pad;
  best_update_one(e[idx], best_e + idx, valid + idx, S8 + off, best_s + off, d.n_pad);
}

hipError_t launch_best_update(const double *e, double *best_e, int32_t *valid, const int8_t *S8,
                              int8_t *best_s, int32_t r, int32_t n_pad, hipStream_t s) {
  best_update_kernel<<<r, 256, 0, s>>>(e, best_e, valid, S8, best_s, n_pad);
  return hipGetLastError();
}

hipError_t launch_best_update_batch(const double *e, double *best_e, int32_t *valid,
                                    const int8_t *S8, int8_t *best_s, const EBatchDesc *descs,
                                    int32_t n_inst, int32_t r, hipStream_t s) {
  best_update_batch_kernel<<<(unsigned)((int64_t)n_inst * r), 256, 0, s>>>(e, best_e, valid, S8,
                                                                         best_s, descs, r);
  return hipGetLastError();
}

hipError_t launch_energy_f32_partial(const float *J, const float *q, const float *h, float *part,
                                     int32_t n_pad, int32_t r_pad, hipStream_t s) {
  if (n_pad % ECfg::BM || r_pad % ECfg::BN) return hipErrorInvalidValue;
  dim3 grid(n_pad / ECfg::BM, r_pad / ECfg::BN);
  energy_f32_partial_kernel<<<grid, 256, 0, s>>>(J, q, h, part, n_pad, r_pad);
  return hipGetLastError();
}

hipError_t launch_energy_f32_batch(const EBatchDesc *descs, const int4 *items, int32_t n_items,
                                   const float *q, float *part, int32_t n_inst, int32_t r,
                                   int32_t r_pad, double *e_real, hipStream_t s) {
  if (n_items > 0)
    energy_f32_batch_kernel<<<n_items, 256, 0, s>>>(descs, items, q, part, r_pad);
  const int64_t total = (int64_t)n_inst * r;
  energy_f32_batch_finalize_kernel<<<(int)((total + 255) / 256), 256, 0, s>>>(
      part, descs, n_inst, r, r_pad, e_real);
  return hipGetLastError();
}

hipError_t launch_energy_f32_finalize(const float *part, int32_t n_tiles, int32_t r,
                                      int32_t r_pad, double *e_real, hipStream_t s, float scale) {
  energy_f32_finalize_kernel<<<(r + 255) / 256, 256, 0, s>>>(part, n_tiles, r, r_pad, e_real,
                                                             scale);
  return hipGetLastError();
}

}  // namespace si
