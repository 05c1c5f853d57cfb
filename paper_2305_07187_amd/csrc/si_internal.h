// Internal declarations shared by the host runtime and the kernel files of
// the Spring-Ising library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spring_ising.h"

namespace si {

// Tile ids of the FP32 step kernel (see the tile table in si_step_f32.hip);
// 0 selects automatically.
constexpr int32_t TILE_AUTO = 0;
constexpr int32_t TILE_F32_LAST = 34;

// Work-groups of a launch are dispatched to the eight XCDs in turn (group b
// runs on XCD b % 8), and each XCD has its own L2.  xcd_tile() renumbers the
// groups so that every XCD takes one contiguous range of the row-major tile
// order: the groups resident on an XCD at one time then share rows of J and
// sweep the same replica columns, so each slab of J reaches that L2 once for
// all column tiles instead of once per group.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int groups) {
  const int per = groups / NUM_XCD;
  if (b >= per * NUM_XCD) return b;
  return (b % NUM_XCD) * per + b / NUM_XCD;
}

// Chunk swizzle of the direct-to-LDS slabs: the 16-byte chunk c of slab row
// r (CH chunks per row) is stored at position c ^ lds_swz<CH>(r), so that
// the 128-bit fragment reads of 16 consecutive rows (the lanes the LDS
// serves together, over 64 banks) hit distinct banks.  Rows of 256 bytes or
// more start on the same bank, so 16 distinct positions suffice.  Rows of
// 128 bytes (CH = 8) pair up on the banks (rows r and r + 2 share them), so
// the second half of each 16-row group uses the order of the first with
// the lowest bit flipped; a plain eight-row order would meet itself there.
template <int CH>
__device__ __forceinline__ int lds_swz(int r) {
  static_assert(CH == 8 || CH >= 16, "rows of 8 or more chunks");
  if constexpr (CH == 8)
    return (r ^ (r >> 3)) & 7;
  else
    return r & 15;
}

struct TileShape {
  int32_t bm, bn;
  const char *name;
  int32_t bk;  // slab depth: the padded contraction length must be a multiple
};
TileShape tile_shape(int32_t tile);

// Scalars of one step, shared by every step launcher.
struct StepArgs {
  const float *J;     // [n_pad][n_pad], zero padded, symmetric
  const float *q_in;  // [r_pad][n_pad]
  const float *p_in;
  float *q_out;
  float *p_out;
  const float *dt;    // schedule arrays [S]
  const float *zeta;
  const float *h;     // field [n_pad] or nullptr
  int32_t t;          // schedule index of this step
  int32_t ld;         // n_pad
  int32_t n;          // spins; the contraction stops at n rounded up to the slab depth
  int32_t n_pad, r_pad;
  float k, inv_m, qmax, pmax;
  int32_t order;      // si_order
  int32_t wall;       // si_wall
  uint8_t *mask_out;  // nullable: per element bit 0 = |u| <= qmax, bit 1 = |v| <= pmax
  int32_t ksplit;     // >= 2: split contraction into ksplit ranges (workspace fsplit)
  float *fsplit;      // [ksplit][r_pad][n_pad] partial products, or null
};

hipError_t launch_step_f32(int32_t tile, const StepArgs &a, hipStream_t s);
// Split contraction (tiles listed in si_splitk.hip): partial products into
// a.fsplit, then the update from their fixed-order sum.
bool tile_has_split(int32_t tile);
hipError_t launch_step_f32_split(int32_t tile, const StepArgs &a, hipStream_t s);

// Resident form: one cooperative launch runs n_steps steps.  Every workgroup
// owns one output tile for the whole launch and keeps that tile's q and p in
// registers; only q, which every other tile's product needs, goes to memory
// (the two q buffers alternate), and a grid-wide barrier separates the
// steps.  p reaches p[cur at exit] after the last step.
struct ResidentArgs {
  float *q[2];
  float *p[2];
  int32_t cur;        // buffer index holding the state at entry
  int32_t n_steps;
  uint32_t *count;    // per-group count of completed steps [groups]; zero at launch
  int32_t *err;       // set to 1 when a barrier wait times out
};
// Workgroups of tile `tile` that fit on one CU at once (0: no resident form
// for this tile).
hipError_t resident_f32_groups_per_cu(int32_t tile, int32_t order, int32_t wall, int *groups);
hipError_t launch_resident_f32(int32_t tile, const StepArgs &a, const ResidentArgs &r,
                               hipStream_t s);

// Batched form: per-instance buffers and the work list of one grouped launch.
// Batch tiles (both precisions): 1 = 128 x 64 work items, 2 = 64 x 64.
constexpr int BATCH_BM = 128, BATCH_BN = 64;
constexpr int32_t BATCH_TILE_LAST = 2;
inline int32_t batch_tile_rows(int32_t btile) { return btile == 2 ? 64 : 128; }
struct BatchDesc {
  const float *J;         // [n_pad][n_pad]
  float *q0, *q1, *p0, *p1;  // [r_pad][n_pad] ping-pong state
  int32_t n_pad, n;
};
// trace: null, or n_items records of 4 words written by the launch (see
// batch_trace_record).
hipError_t launch_step_batch_f32(const StepArgs &a, const BatchDesc *descs, const int4 *items,
                                 int32_t n_items, int32_t cur, int32_t btile,
                                 unsigned long long *trace, hipStream_t s);

// Step on the BF16 matrix cores (precision forms).
constexpr int32_t TILE_BF16_LAST = 33;
TileShape tile_shape_bf16(int32_t tile);
struct BStepArgs {
  const void *Ja;         // J plane: bf16 or fp8 [n_pad][n_pad]
  const void *Jb;         // second J plane (lo of hi/lo) or nullptr
  const uint16_t *qb_in;  // BF16 plane(s) of q, plane stride plane_stride
  uint16_t *qb_out;
  int64_t plane_stride;   // n_pad * r_pad
  const float *q_in, *p_in;
  float *q_out, *p_out;
  const float *dt, *zeta, *h;
  int32_t t, ld, n_pad, r_pad;
  float k, inv_m, qmax, pmax;
  int32_t order, wall;
};
hipError_t launch_step_bf16(int32_t tile, int32_t precision, const BStepArgs &a, hipStream_t s);
// Batched precision form: per-instance J format (fmt 1: FP8 e4m3, 2: hi + lo
// BF16), BF16 plane of q per instance; instances padded to 128 (FP8 slabs
// are 128 deep), work items of the batch tile's rows.  `base` carries the
// schedules, constants and r_pad.
constexpr int BATCH_BF16_NPAD = 128, BATCH_BF16_BM = 128;
struct BBatchDesc {
  const void *Ja, *Jb;
  float *q[2], *p[2];
  uint16_t *qb[2];
  int32_t n_pad, fmt;
};
hipError_t launch_step_batch_bf16(const BStepArgs &base, const BBatchDesc *descs,
                                  const int4 *items, int32_t n_items, int32_t cur, int32_t btile,
                                  unsigned long long *trace, hipStream_t s);
bool tile_valid_bf16(int32_t tile, int32_t precision);
hipError_t launch_pack_j_lowp(const float *J, int64_t total, int32_t precision, void *out_a,
                              void *out_b, hipStream_t s);
hipError_t launch_split_planes(const float *q, uint16_t *planes, int64_t total, int32_t nplanes,
                               hipStream_t s);

// G = J.sign(Q) in FP32, per-row-tile partial sums of s_i (G_i + 2 h_i):
// part[row_tile][r].  BM is fixed at 64 rows.
// Batched energies: one descriptor per instance; work items (instance, row
// tile, column tile) over 64 x 64 tiles, one list per path.
struct EBatchDesc {
  const int8_t *J8;   // integer couplings (exact int32 energy), or null: real path
  const float *J;     // FP32 couplings
  int64_t soff;       // offset of the instance's state in the batch's state buffers
  int32_t n_pad;      // instance rows (multiple of 64)
  int32_t part_row;   // first row of its row-tile partials (real path)
};
hipError_t launch_energy_i8_batch(const EBatchDesc *descs, const int4 *items, int32_t n_items,
                                  const int8_t *S8, int32_t *acc, int32_t n_inst, int32_t r,
                                  int32_t r_pad, int32_t *e_int, double *e_real, hipStream_t s);
hipError_t launch_energy_f32_batch(const EBatchDesc *descs, const int4 *items, int32_t n_items,
                                   const float *q, float *part, int32_t n_inst, int32_t r,
                                   int32_t r_pad, double *e_real, hipStream_t s);
hipError_t launch_best_update_batch(const double *e, double *best_e, int32_t *valid,
                                    const int8_t *S8, int8_t *best_s, const EBatchDesc *descs,
                                    int32_t n_inst, int32_t r, hipStream_t s);
hipError_t launch_energy_f32_partial(const float *J, const float *q, const float *h,
                                     float *part, int32_t n_pad, int32_t r_pad,
                                     hipStream_t s);
hipError_t launch_energy_f32_finalize(const float *part, int32_t n_tiles, int32_t r,
                                      int32_t r_pad, double *e_real, hipStream_t s,
                                      float scale = -0.5f);
// Eq. (7) Hamiltonian per replica (partials per row tile, add with scale 1).
hipError_t launch_hamiltonian_partial(const float *J, const float *q, const float *p,
                                      const float *h, const float *zetas, int32_t t, float k,
                                      float inv_m, float *part, int32_t n_pad, int32_t r_pad,
                                      hipStream_t s);
hipError_t launch_best_update(const double *e, double *best_e, int32_t *valid, const int8_t *S8,
                              int8_t *best_s, int32_t r, int32_t n_pad, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t count, double v, hipStream_t s);

// Exact energy: s = sign(q) as int8 into S8, then G = J8.S8 on int8 MFMA,
// acc[r] += sum_i s_i (G_i + 2 h_i), then e[r] = -acc[r]/2.
hipError_t launch_sign(const float *q, int8_t *s8, int32_t n_pad, int32_t r_pad,
                       hipStream_t s);
hipError_t launch_energy_i8(const int8_t *J8, const int8_t *S8, const int8_t *h8,
                            int32_t *acc, int32_t n_pad, int32_t r_pad, int32_t ks,
                            hipStream_t s);
// Contraction split of launch_energy_i8 for this shape (a power of two).
int32_t energy_i8_ksplit(int32_t n_pad, int32_t r_pad, int num_cus);
hipError_t launch_energy_i8_finalize(int32_t *acc, int32_t r, int32_t *e_int,
                                     double *e_real, hipStream_t s);
hipError_t launch_zero_i32(int32_t *p, int64_t count, hipStream_t s);

// Adjoint of the relaxed end-energy (paper order, clamping walls, FP32).
constexpr int ADJ_BM = 32, ADJ_BN = 32;
hipError_t launch_adj_seed(const float *J, const float *q, float *lamq, float *lamp, double *part,
                           int32_t n_pad, int32_t r_pad, float inv_r, hipStream_t s);
hipError_t launch_adj_step(const float *J, const float *lamq_in, const float *lamp_in,
                           const uint8_t *mask, const float *q_n, const float *p_n,
                           float *lamq_out, float *lamp_out, double *part, const float *dt,
                           const float *zeta, int32_t n, float k, float inv_m, int32_t n_pad,
                           int32_t r_pad, hipStream_t s);
// Backward step with the split contraction; writes adj_split_groups()
// partial triples to part.
int32_t adj_split_groups(int32_t n_pad, int32_t r_pad);
hipError_t launch_adj_step_split(const float *J, const float *lamq_in, const float *lamp_in,
                                 const uint8_t *mask, const float *q_n, const float *p_n,
                                 float *lamq_out, float *lamp_out, double *part, const float *dt,
                                 const float *zeta, int32_t n, float k, float inv_m, int32_t n_pad,
                                 int32_t n_spins, int32_t r_pad, int32_t ksplit, float *W,
                                 hipStream_t s);
// mode 0 (n_steps = 1): loss[0] = -1/2 * sum(part[:,0]) / r_count;  mode 1:
// gradient entries g_dt[n + i], g_zeta[n + i] for i < n_steps from the nwg
// partial triples of step n + i at part + i * nwg * 3.
hipError_t launch_adj_reduce(const double *part, int32_t nwg, int32_t mode, double *loss,
                             double *g_dt, double *g_zeta, const float *dt, const float *zeta,
                             int32_t n, int32_t n_steps, float k, float inv_m, int32_t r_count,
                             hipStream_t s);

// Layout conversion and validation.
hipError_t launch_pack_matrix(const float *src, int32_t n, float *dst, int8_t *dst8,
                              int32_t n_pad, hipStream_t s);
hipError_t launch_pack_state(const float *src, int32_t n, int32_t r, float *dst,
                             int32_t n_pad, int32_t r_pad, hipStream_t s);
hipError_t launch_unpack_state(const float *src, int32_t n, int32_t r, float *dst,
                               int32_t n_pad, hipStream_t s);
hipError_t launch_unpack_spins(const int8_t *src, int32_t n, int32_t r, int8_t *dst,
                               int32_t n_pad, hipStream_t s);
hipError_t launch_pack_field(const float *h, int32_t n, float *hf, int8_t *h8,
                             int32_t n_pad, int32_t *flags, hipStream_t s);

// Allocation-free exact energy: scratch is a static device array per GPU
// (its device address looked up once per device), at most noalloc_r_max()
// replicas.
int32_t noalloc_r_max();
hipError_t noalloc_scratch_ptr(int device, void **ptr);
hipError_t launch_noalloc_energy(const float *J, const float *x, int32_t n, int32_t r,
                                 int32_t *e_int, void *scratch_ptr, hipStream_t s);

// flags[0]: asymmetric, [1]: nonzero diagonal, [2]: non-finite,
// [3]: non-integer or |J|>127, [4]: not FP8-e4m3 exact, [5]: not BF16 exact
hipError_t launch_validate(const float *J, int32_t n, int32_t *flags, hipStream_t s);

}  // namespace si
