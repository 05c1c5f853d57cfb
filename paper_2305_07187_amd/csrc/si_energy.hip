// Readout and exact Ising energy (Eq. 1) on the int8 matrix cores.
//
// For integer couplings |J_ij| <= 127 the energy of s = sign(q) is exact:
// G = J.S is an int8 x int8 product with int32 accumulation
// (v_mfma_i32_32x32x32_i8 for a single instance, v_mfma_i32_16x16x32_i8 for
// the batch's 64 x 64 items), and sum_i s_i (G_i + 2 h_i) = 2 sum_{i<j} J_ij
// s_i s_j + 2 sum_i h_i s_i is even, so E = -(that sum)/2 is exact.
// Partial sums from all workgroups are combined with integer atomics, whose
// result does not depend on their order.
//
// Batch item layout (one 16x16 block, K = 32): lane l supplies the 8 bytes
// A[l%16][8(l/16) .. 8(l/16)+7] and B[8(l/16) .. +7][l%16]; D as for the FP32
// shape.  Each lane reads 16 contiguous bytes per operand and per 64-byte
// slab; MFMA s = 0, 1 uses bytes 8s .. 8s+7 of them (a permutation of the
// contraction index applied identically to both operands).
#include "si_internal.h"

namespace si {

typedef int intx4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int EBM = 64, EBN = 64, EBK = 64, ELDK = EBK + 16;  // bytes
constexpr int EWTM = 32, EWTN = 32;  // 2 x 2 waves
}  // namespace

// One 64 x 64 output tile (rows m0.., replicas n0..) of G = J.S, reduced
// against s (and h) into acc_out[col] by integer atomics.
__device__ __forceinline__ void energy_i8_tile(const int8_t *__restrict__ J8,
                                               const int8_t *__restrict__ S8,
                                               const int8_t *__restrict__ h8,
                                               int32_t *__restrict__ acc_out, int ld, int m0,
                                               int n0) {
  __shared__ __attribute__((aligned(16))) int8_t As[2][EBM * ELDK];
  __shared__ __attribute__((aligned(16))) int8_t Bs[2][EBN * ELDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int lrow = lane & 15, lk = (lane >> 4) * 16;
  // staging: each thread moves 16 bytes of A and 16 bytes of B per slab
  const int srow = tid >> 2, sc = (tid & 3) * 16;

  intx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = intx4{0, 0, 0, 0};

  const int nk = ld / EBK;
  int4 ra = *reinterpret_cast<const int4 *>(J8 + (size_t)(m0 + srow) * ld + sc);
  int4 rb = *reinterpret_cast<const int4 *>(S8 + (size_t)(n0 + srow) * ld + sc);
  *reinterpret_cast<int4 *>(&As[0][srow * ELDK + sc]) = ra;
  *reinterpret_cast<int4 *>(&Bs[0][srow * ELDK + sc]) = rb;
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) {
      ra = *reinterpret_cast<const int4 *>(J8 + (size_t)(m0 + srow) * ld + (kt + 1) * EBK + sc);
      rb = *reinterpret_cast<const int4 *>(S8 + (size_t)(n0 + srow) * ld + (kt + 1) * EBK + sc);
    }
    int4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const int4 *>(&As[buf][(wy * EWTM + i * 16 + lrow) * ELDK + lk]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const int4 *>(&Bs[buf][(wx * EWTN + j * 16 + lrow) * ELDK + lk]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        long a0 = ((long)(uint32_t)a[i].y << 32) | (uint32_t)a[i].x;
        long a1 = ((long)(uint32_t)a[i].w << 32) | (uint32_t)a[i].z;
        long b0 = ((long)(uint32_t)b[j].y << 32) | (uint32_t)b[j].x;
        long b1 = ((long)(uint32_t)b[j].w << 32) | (uint32_t)b[j].z;
        acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a0, b0, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a1, b1, acc[i][j], 0, 0, 0);
      }
    if (kt + 1 < nk) {
      *reinterpret_cast<int4 *>(&As[buf ^ 1][srow * ELDK + sc]) = ra;
      *reinterpret_cast<int4 *>(&Bs[buf ^ 1][srow * ELDK + sc]) = rb;
    }
    __syncthreads();
  }

#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = n0 + wx * EWTN + j * 16 + (lane & 15);
    int c = 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int row = m0 + wy * EWTM + i * 16 + (lane >> 4) * 4;
      const char4 s4 = *reinterpret_cast<const char4 *>(S8 + (size_t)col * ld + row);
      char4 h4 = make_char4(0, 0, 0, 0);
      if (h8) h4 = *reinterpret_cast<const char4 *>(h8 + row);
      c += (int)s4.x * (acc[i][j][0] + 2 * (int)h4.x);
      c += (int)s4.y * (acc[i][j][1] + 2 * (int)h4.y);
      c += (int)s4.z * (acc[i][j][2] + 2 * (int)h4.z);
      c += (int)s4.w * (acc[i][j][3] + 2 * (int)h4.w);
    }
    c += __shfl_xor(c, 16);
    c += __shfl_xor(c, 32);
    if (lane < 16) atomicAdd(acc_out + col, c);
  }
}

// ---------------------------------------------------------------------------
// Single-instance energy on gfx950's int8 shape v_mfma_i32_32x32x32_i8.
// Lane l supplies the 16 bytes A[l%32][16(l/32) .. +15] and
// B[16(l/32) .. +15][l%32] of each 32-deep contraction step (A and B use the
// same assignment of contraction bytes to lanes, so the product is a plain
// sum over them); the result D[8(v/4) + 4(l/32) + v%4][l%32] lands in
// accumulator v < 16.  One 128 x 64 output tile per workgroup, eight waves of
// 32 x 32, the J and S slabs (QBK contraction bytes deep) copied straight
// into a three-slot LDS ring with the chunk swizzle of their rows.  With
// ks > 1 the contraction is split over ks workgroups per tile, each adding
// its part of s^T (J s) to the replica's integer accumulator (the field term
// in part 0 only): integer sums, so the result does not depend on the order.
// ---------------------------------------------------------------------------
namespace {
constexpr int QBM = 128, QBN = 64, QBK = 128, QST = 3, QNT = 512, QNW = QNT / 64;
constexpr int QSLOT = (QBM + QBN) * QBK;  // bytes per ring slot
constexpr int QCH = QBK / 16;             // 16-byte chunks per slab row
constexpr int QRPD = 64 / QCH;            // rows written by one wave-wide load
constexpr int QAD = QBM / QRPD / QNW, QBD = QBN / QRPD / QNW;  // loads per wave per slab
constexpr int QL = QAD + QBD;
static_assert(QAD >= 1 && QBD >= 1 && (QST - 2) * QL <= 63, "energy ring");
}  // namespace

typedef int intx16 __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void_e;
typedef __attribute__((address_space(1))) const void gbl_void_e;

template <int N>
__device__ __forceinline__ void e_wait_barrier() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

__global__ __launch_bounds__(QNT) void energy_i8_kernel(const int8_t *__restrict__ J8,
                                                        const int8_t *__restrict__ S8,
                                                        const int8_t *__restrict__ h8,
                                                        int32_t *__restrict__ acc_out, int ld,
                                                        int r_pad, int ks) {
  __shared__ __attribute__((aligned(16))) int8_t smem[QST * QSLOT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;  // 4 x 2 waves of 32 x 32
  const int ncol = r_pad / QBN;
  const int u = xcd_tile(blockIdx.x, gridDim.x);
  const int t = u / ks, part = u % ks;
  const int m0 = (t / ncol) * QBM, n0 = (t % ncol) * QBN;
  const int nk = ld / QBK / ks, k0 = part * nk * QBK;  // this part's slabs
  // A wave-wide direct-to-LDS load writes 64 x 16 bytes: QRPD rows.  Lane
  // L fills position L % QCH of row L / QCH with the chunk that belongs
  // there (chunk c of row r is stored at position c ^ swz(r)).
  const int drow = lane / QCH, dch = lane % QCH;
  const int8_t *srcA[QAD];
  const int8_t *srcB[QBD];
#pragma unroll
  for (int d = 0; d < QAD; ++d) {
    const int row = (wave * QAD + d) * QRPD + drow;
    srcA[d] = J8 + (size_t)(m0 + row) * ld + k0 + ((dch ^ lds_swz<QCH>(row)) << 4);
  }
#pragma unroll
  for (int d = 0; d < QBD; ++d) {
    const int row = (wave * QBD + d) * QRPD + drow;
    srcB[d] = S8 + (size_t)(n0 + row) * ld + k0 + ((dch ^ lds_swz<QCH>(row)) << 4);
  }
  auto issue = [&](int kt, int slot) {
    int8_t *st = smem + slot * QSLOT;
#pragma unroll
    for (int d = 0; d < QAD; ++d)
      __builtin_amdgcn_global_load_lds((gbl_void_e *)(srcA[d] + (size_t)kt * QBK),
                                       (lds_void_e *)(st + (wave * QAD + d) * QRPD * QBK), 16, 0,
                                       0);
#pragma unroll
    for (int d = 0; d < QBD; ++d)
      __builtin_amdgcn_global_load_lds((gbl_void_e *)(srcB[d] + (size_t)kt * QBK),
                                       (lds_void_e *)(st + (QBM + (wave * QBD + d) * QRPD) * QBK),
                                       16, 0, 0);
  };
#pragma unroll
  for (int s = 0; s < QST - 1; ++s)
    if (s < nk) issue(s, s);
  intx16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0;
  const int ra = wy * 32 + (lane & 31), rb = wx * 32 + (lane & 31), h = lane >> 5;
  int rd = 0, wr = QST - 1;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + QST - 1 < nk) {
      e_wait_barrier<(QST - 2) * QL>();
      issue(kt + QST - 1, wr);
    } else {
      e_wait_barrier<0>();
    }
    wr = wr + 1 == QST ? 0 : wr + 1;
    const int8_t *st = smem + rd * QSLOT;
    rd = rd + 1 == QST ? 0 : rd + 1;
#pragma unroll
    for (int kk = 0; kk < QBK / 32; ++kk) {
      const int ch = kk * 2 + h;  // 16-byte chunk of this lane in the slab row
      const intx4 a =
          *reinterpret_cast<const intx4 *>(st + ra * QBK + ((ch ^ lds_swz<QCH>(ra)) << 4));
      const intx4 b = *reinterpret_cast<const intx4 *>(st + (QBM + rb) * QBK +
                                                       ((ch ^ lds_swz<QCH>(rb)) << 4));
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc, 0, 0, 0);
    }
  }
  // sum_i s_i (G_i + 2 h_i) over this wave's 32 rows for each of its columns
  const int col = n0 + wx * 32 + (lane & 31);
  int c = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int row = m0 + wy * 32 + g * 8 + h * 4;
    const char4 s4 = *reinterpret_cast<const char4 *>(S8 + (size_t)col * ld + row);
    char4 h4 = make_char4(0, 0, 0, 0);
    if (h8 && part == 0) h4 = *reinterpret_cast<const char4 *>(h8 + row);
    c += (int)s4.x * (acc[4 * g] + 2 * (int)h4.x);
    c += (int)s4.y * (acc[4 * g + 1] + 2 * (int)h4.y);
    c += (int)s4.z * (acc[4 * g + 2] + 2 * (int)h4.z);
    c += (int)s4.w * (acc[4 * g + 3] + 2 * (int)h4.w);
  }
  c += __shfl_xor(c, 32);
  if (h == 0) atomicAdd(acc_out + col, c);
}

// Batch: work item (instance, row tile, column tile) over the instances with
// integer couplings; instance i's spins start at S8 + d.soff and its
// accumulators at acc + i * r_pad.
__global__ __launch_bounds__(256) void energy_i8_batch_kernel(const EBatchDesc *__restrict__ descs,
                                                              const int4 *__restrict__ items,
                                                              const int8_t *__restrict__ S8,
                                                              int32_t *__restrict__ acc,
                                                              int r_pad) {
  const int4 it = items[blockIdx.x];
  const EBatchDesc d = descs[it.x];
  energy_i8_tile(d.J8, S8 + d.soff, nullptr, acc + (size_t)it.x * r_pad, d.n_pad, it.y * EBM,
                 it.z * EBN);
}

// Batch finalisation: entry i * r + col of the outputs for every instance
// with integer couplings (J8 set in its descriptor), accumulators reset.
__global__ void energy_i8_batch_finalize_kernel(int32_t *acc, const EBatchDesc *__restrict__ descs,
                                                int n_inst, int r, int r_pad, int32_t *e_int,
                                                double *e_real) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_inst * r) return;
  const int i = (int)(idx / r), col = (int)(idx % r);
  if (!descs[i].J8) return;
  int32_t *a = acc + (size_t)i * r_pad + col;
  const int32_t e = -(*a / 2);
  if (e_int) e_int[idx] = e;
  if (e_real) e_real[idx] = (double)e;
  *a = 0;
}

__global__ void sign_kernel(const float4 *__restrict__ q, char4 *__restrict__ s, int64_t n4) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = q[i];
    s[i] = make_char4(v.x < 0.f ? -1 : 1, v.y < 0.f ? -1 : 1, v.z < 0.f ? -1 : 1,
                      v.w < 0.f ? -1 : 1);
  }
}

__global__ void energy_i8_finalize_kernel(int32_t *acc, int r, int32_t *e_int, double *e_real) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= r) return;
  const int32_t e = -(acc[col] / 2);
  if (e_int) e_int[col] = e;
  if (e_real) e_real[col] = (double)e;
  acc[col] = 0;  // ready for the next evaluation
}

__global__ void zero_i32_kernel(int32_t *p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_sign(const float *q, int8_t *s8, int32_t n_pad, int32_t r_pad, hipStream_t s) {
  const int64_t n4 = (int64_t)n_pad * r_pad / 4;
  const int blocks = (int)((n4 + 255) / 256 < 4096 ? (n4 + 255) / 256 : 4096);
  sign_kernel<<<blocks, 256, 0, s>>>(reinterpret_cast<const float4 *>(q),
                                     reinterpret_cast<char4 *>(s8), n4);
  return hipGetLastError();
}

hipError_t launch_energy_i8(const int8_t *J8, const int8_t *S8, const int8_t *h8, int32_t *acc,
                            int32_t n_pad, int32_t r_pad, int32_t ks, hipStream_t s) {
  if (n_pad % QBM || n_pad % QBK || r_pad % QBN || ks < 1 || (n_pad / QBK) % ks)
    return hipErrorInvalidValue;
  energy_i8_kernel<<<(n_pad / QBM) * (r_pad / QBN) * ks, QNT, 0, s>>>(J8, S8, h8, acc, n_pad,
                                                                      r_pad, ks);
  return hipGetLastError();
}

int32_t energy_i8_ksplit(int32_t n_pad, int32_t r_pad, int num_cus) {
  const int64_t tiles = (int64_t)(n_pad / QBM) * (r_pad / QBN);
  const int32_t nk = n_pad / QBK;
  int32_t ks = 1;
  // two workgroups fit a CU (72 KB of LDS each): split while the grid has
  // fewer than that and every part keeps at least two slabs.  At N = 2000,
  // R = 1024 (256 tiles) the readout took 15.6 us per call with 2 parts,
  // 15.7 us unsplit, 20.1 and 30.7 us with 4 and 8 (more atomics per
  // accumulator); the kernel waits on its slab loads, not on the matrix cores.
  while (tiles * ks < 2 * (int64_t)num_cus && nk % (ks * 2) == 0 && nk / (ks * 2) >= 2) ks *= 2;
  return ks;
}

hipError_t launch_energy_i8_finalize(int32_t *acc, int32_t r, int32_t *e_int, double *e_real,
                                     hipStream_t s) {
  energy_i8_finalize_kernel<<<(r + 255) / 256, 256, 0, s>>>(acc, r, e_int, e_real);
  return hipGetLastError();
}

hipError_t launch_energy_i8_batch(const EBatchDesc *descs, const int4 *items, int32_t n_items,
                                  const int8_t *S8, int32_t *acc, int32_t n_inst, int32_t r,
                                  int32_t r_pad, int32_t *e_int, double *e_real, hipStream_t s) {
  if (n_items > 0)
    energy_i8_batch_kernel<<<n_items, 256, 0, s>>>(descs, items, S8, acc, r_pad);
  const int64_t total = (int64_t)n_inst * r;
  energy_i8_batch_finalize_kernel<<<(int)((total + 255) / 256), 256, 0, s>>>(
      acc, descs, n_inst, r, r_pad, e_int, e_real);
  return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t *p, int64_t count, hipStream_t s) {
  const int blocks = (int)((count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024);
  zero_i32_kernel<<<blocks > 0 ? blocks : 1, 256, 0, s>>>(p, count);
  return hipGetLastError();
}

}  // namespace si
