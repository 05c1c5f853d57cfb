// Host runtime of the Spring-Ising library: the C ABI declared in
// include/spring_ising.h.  Owns the padded device buffers, builds the
// zeta/Delta schedules, validates J, picks the step kernel and launches it.
#include <errno.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <algorithm>
#include <vector>

#include "si_internal.h"

using namespace si;

namespace {

thread_local std::string g_last_error;

si_status fail(si_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  memset(&attr, 0, sizeof attr);
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Piecewise-constant linear zeta(t_step): K = ceil(S/L) stairs, stair s of
// step n is floor(n/L), zeta = zs + (ze - zs) * s / (K - 1) (zs alone when
// K = 1).  Formed in double, rounded once to float.  Contraction is off so
// the double expression rounds exactly as written.
#pragma clang fp contract(off)
void build_schedules(const si_params &p, std::vector<float> &dt, std::vector<float> &zeta) {
  const int32_t S = p.total_steps, L = p.stair_len;
  const int64_t K = (S + (int64_t)L - 1) / L;
  dt.assign(S, p.dt);
  zeta.resize(S);
  const double zs = p.zeta_start, ze = p.zeta_end;
  for (int32_t n = 0; n < S; ++n) {
    const int64_t s = n / L;
    double v;
    if (K == 1)
      v = zs;
    else
      v = zs + (ze - zs) * ((double)s / (double)(K - 1));
    zeta[n] = (float)v;
  }
}

}  // namespace

struct si_ctx {
  int32_t n = 0, r = 0, n_pad = 0, r_pad = 0;
  si_params prm{};
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cus = 0;
  int32_t tile = 0;
  float *J = nullptr;
  int8_t *J8 = nullptr;
  void *Ja = nullptr, *Jb = nullptr;        // low-precision J planes
  uint16_t *qb[2] = {nullptr, nullptr};     // BF16 plane(s) of q, ping-pong
  int32_t qplanes = 0;                      // 0 for the FP32 form
  float *q[2] = {nullptr, nullptr}, *p[2] = {nullptr, nullptr};
  int cur = 0;
  float *dt = nullptr, *zeta = nullptr;
  float *hf = nullptr;
  int8_t *h8 = nullptr;
  bool has_field = false, field_integer = false;
  int32_t field_maxabs = 0;
  int8_t *S8 = nullptr;
  int32_t *eacc = nullptr;
  float *epart = nullptr;
  int32_t *flags = nullptr;  // device validation flags [8]
  int32_t hflags[8] = {0};
  int32_t t = 0;
  bool poisoned = false;
  int32_t inject_countdown = 0;  // test hook: > 0 fails the n-th checked HIP call
  uint16_t *tune_qb = nullptr;    // autotune: saved BF16 planes of q
  float *tune_save = nullptr;     // autotune of a batch: saved q and p
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  int64_t bytes = 0;
  std::vector<void *> allocs;
  std::vector<float> host_dt, host_zeta;  // kept alive for the async upload
  // batched form (n_inst > 0): per-instance buffers inside shared allocations
  int32_t n_inst = 0;
  std::vector<int32_t> b_n, b_npad, b_jmax;
  std::vector<int64_t> b_xoff;            // offset of instance i in caller layouts (floats)
  std::vector<float *> b_J, b_q[2], b_p[2];
  std::vector<int8_t *> b_J8;             // nullptr for non-integer instances
  std::vector<BatchDesc> b_desc_host;
  std::vector<int4> b_items_host;
  BatchDesc *b_desc = nullptr;
  int4 *b_items = nullptr;
  int32_t b_max_npad = 0;
  int64_t b_total_n = 0;
  int64_t b_stot = 0;                     // elements of one state buffer (all instances)
  std::vector<int64_t> b_soff;            // offset of instance i in the state buffers
  // grouped energy: one descriptor per instance; work items of the integer
  // instances first (eb_n_i8 of them), then those of the real ones
  std::vector<EBatchDesc> eb_desc_host;
  std::vector<int4> eb_items_host;
  EBatchDesc *eb_desc = nullptr;
  int4 *eb_items = nullptr;
  int32_t eb_n_i8 = 0, eb_n_f32 = 0;
  // batched precision form: per-instance J format (1: FP8, 2: hi + lo BF16)
  bool b_lowp = false;
  std::vector<int32_t> b_fmt;
  std::vector<uint16_t *> b_qb[2];
  std::vector<BBatchDesc> bb_desc_host;
  BBatchDesc *bb_desc = nullptr;
  // captured HIP graphs of run(n) launch sequences, keyed by (t0, n, cur)
  struct GraphEntry {
    int32_t t0, n, cur;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  int32_t graph_min_steps = 0;  // 0: graphs off
  // resident launches of run(n): n >= resident_min_steps (0: off)
  int32_t resident_min_steps = 0;
  int32_t resident_tile = -1, resident_per_cu = 0;  // occupancy cache for `tile`
  // split contraction: 0 = automatic, >= 1 = forced number of k ranges
  int32_t ksplit_mode = 0;
  int32_t user_tile = 0;        // tile requested at init (0: automatic)
  int32_t table_tile = 0, table_split = 0;  // measured default for few replicas
  int32_t tile_source = SI_TILE_FROM_TABLE;
  int64_t b_items_cap = 0;      // int4 entries of the device work list
  unsigned long long *b_trace = nullptr;  // timeline records of traced steps
  int64_t b_trace_cap = 0;                // records
  float *fsplit = nullptr;      // partial products of the split contraction
  int64_t fsplit_cap = 0;       // floats
  int32_t *res_sync = nullptr;  // [0] time-out flag, [64 ..] per-group step counts
  int32_t res_sync_cap = 0;
  hipStream_t cap_stream = nullptr;
  // best state per replica (per instance and replica on a batch): lowest
  // energy seen since the last reset and its spins; best_valid[k] == 0 marks
  // a record that the next update overwrites (reset on the device, so that
  // captured launch sequences replay correctly)
  double *best_e = nullptr, *e_scratch = nullptr;
  int8_t *best_s = nullptr;
  int32_t *best_valid = nullptr;
  bool best_any = false;  // an update was issued since init or the last set_state
  // in-run energy checks: every e_every steps the energies of all replicas
  // go to row t / e_every - 1 of the trace [e_rows][out_rows()] and update
  // the best state
  int32_t e_every = 0, e_rows = 0;
  double *etrace = nullptr;
  int64_t out_rows() const { return n_inst ? (int64_t)n_inst * r : (int64_t)r; }
  // every call that changes the trajectory (schedule, field, state, steps,
  // kernel choice) bumps the epoch; the adjoint's forward half records it
  int64_t epoch = 0;
  struct {
    bool valid = false;
    int64_t epoch = 0;
    int32_t t0 = 0, ckpt = 0;
  } tape;
  // adjoint workspace
  float *adj_ckpt = nullptr, *adj_seg = nullptr, *adj_lam = nullptr;
  uint8_t *adj_mask = nullptr;
  double *adj_part = nullptr;
  int64_t adj_part_cap = 0;       // doubles
  int64_t adj_ckpt_cap = 0, adj_seg_cap = 0;

  template <class T>
  hipError_t alloc(T **ptr, int64_t count) {
    void *raw = nullptr;
    hipError_t e = hipMalloc(&raw, (size_t)count * sizeof(T));
    if (e != hipSuccess) return e;
    allocs.push_back(raw);
    bytes += count * (int64_t)sizeof(T);
    *ptr = static_cast<T *>(raw);
    return hipSuccess;
  }
  void drop_graphs() {
    for (auto &g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
  }
  ~si_ctx() {
    drop_graphs();
    for (hipEvent_t e : tune_ev)
      if (e) (void)hipEventDestroy(e);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void *a : allocs) (void)hipFree(a);
  }
};

// Every HIP call of a context goes through this check: a failure poisons
// the context.  A test hook (spring_ising_debug_inject_hip_error) can make
// the n-th checked call after it report a failure although the call itself
// succeeded, so that the poisoning path runs without any device fault.
#define SI_HIP(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if ((ctx) && (ctx)->inject_countdown > 0 && --(ctx)->inject_countdown == 0 &&      \
        _e == hipSuccess)                                                              \
      _e = hipErrorUnknown;                                                            \
    if (_e != hipSuccess) {                                                            \
      if (ctx) (ctx)->poisoned = true;                                                 \
      return fail(_e == hipErrorOutOfMemory ? SI_ERR_OOM : SI_ERR_HIP, "%s: %s (%s)",  \
                  __func__, hipGetErrorString(_e), #expr);                             \
    }                                                                                  \
  } while (0)

#define SI_USABLE(ctx)                                                                 \
  do {                                                                                 \
    if (!(ctx)) return fail(SI_ERR_INVALID, "%s: null context", __func__);             \
    if ((ctx)->poisoned)                                                               \
      return fail(SI_ERR_STATE, "%s: context poisoned by an earlier HIP failure",      \
                  __func__);                                                           \
  } while (0)

static si_status check_params(const si_params *p) {
  if (!p) return fail(SI_ERR_INVALID, "params: null");
  if (p->total_steps < 1) return fail(SI_ERR_INVALID, "params: total_steps must be >= 1");
  if (p->stair_len < 1) return fail(SI_ERR_INVALID, "params: stair_len must be >= 1");
  if (!(p->m > 0.f) || !isfinite(p->m)) return fail(SI_ERR_INVALID, "params: m must be > 0");
  if (!(p->dt > 0.f) || !isfinite(p->dt)) return fail(SI_ERR_INVALID, "params: dt must be > 0");
  if (!(p->qmax > 0.f) || !isfinite(p->qmax))
    return fail(SI_ERR_INVALID, "params: qmax must be > 0");
  if (!(p->pmax > 0.f) || !isfinite(p->pmax))
    return fail(SI_ERR_INVALID, "params: pmax must be > 0");
  if (!isfinite(p->k) || !isfinite(p->zeta_start) || !isfinite(p->zeta_end))
    return fail(SI_ERR_INVALID, "params: k and zeta must be finite");
  if (p->order != SI_ORDER_PAPER && p->order != SI_ORDER_SYMPLECTIC)
    return fail(SI_ERR_INVALID, "params: unknown order %d", p->order);
  if (p->wall != SI_WALL_CLAMP && p->wall != SI_WALL_INELASTIC)
    return fail(SI_ERR_INVALID, "params: unknown wall %d", p->wall);
  if (p->precision < SI_PREC_FP32 || p->precision > SI_PREC_BF16X_MIXEDJ)
    return fail(SI_ERR_INVALID, "params: unknown precision %d", p->precision);
  const int32_t last = p->precision == SI_PREC_FP32 ? TILE_F32_LAST : TILE_BF16_LAST;
  if (p->tile < 0 || p->tile > last)
    return fail(SI_ERR_INVALID, "params: unknown tile %d", p->tile);
  if (p->energy_every < 0) return fail(SI_ERR_INVALID, "params: energy_every must be >= 0");
  return SI_OK;
}

// Largest-work tile that still gives at least one workgroup per CU; with no
// such tile, the one with the most workgroups (small problems).
static TileShape shape_of(int32_t precision, int32_t tile) {
  return precision == SI_PREC_FP32 ? tile_shape(tile) : tile_shape_bf16(tile);
}

// Number of contraction ranges for a problem whose output has fewer
// workgroups (`tiles`) than there are CUs: enough to give every CU two (at
// most 8 ranges), each range at least four 32-deep slabs long.  (At N=2000,
// R=64 on MI355X: 32x32 tiles, 4 ranges, 12.4 us per step against 26.9 us
// unsplit and 17.8 us with 2 ranges.)
static int32_t auto_split(int64_t tiles, int32_t n, int num_cus) {
  if (tiles >= num_cus) return 1;
  int64_t s = (2 * (int64_t)num_cus + tiles - 1) / tiles;
  if (s > 8) s = 8;
  const int64_t smax = round_up(n, 32) / 128;
  if (s > smax) s = smax;
  return s < 1 ? 1 : (int32_t)s;
}

// Split of the FP32 step for tile `tile` in this context (1: none).
static int32_t split_for(const si_ctx *c, int32_t tile) {
  if (c->n_inst || c->qplanes || !tile_has_split(tile)) return 1;
  if (c->ksplit_mode >= 1) return c->ksplit_mode;
  if (c->user_tile != 0) return 1;
  if (c->table_split > 0 && tile == c->table_tile) return c->table_split;
  const TileShape ts = tile_shape(tile);
  return auto_split((int64_t)(c->n_pad / ts.bm) * (c->r_pad / ts.bn), c->n, c->num_cus);
}

// Split of the adjoint's backward product (32 x 32 tiles).
static int32_t adj_split(const si_ctx *c) {
  if (c->ksplit_mode >= 1) return c->ksplit_mode;
  return auto_split((int64_t)(c->n_pad / ADJ_BM) * (c->r_pad / ADJ_BN), c->n, c->num_cus);
}

// Workspace for the split contraction of the current tile and of the
// adjoint (allocated here, never while a launch sequence is captured).
static hipError_t ensure_split_ws(si_ctx *c, bool adjoint = false) {
  const int64_t NR = (int64_t)c->n_pad * c->r_pad;
  int64_t need = split_for(c, c->tile) > 1 ? split_for(c, c->tile) * NR : 0;
  if (adjoint && adj_split(c) > 1 && adj_split(c) * NR > need) need = adj_split(c) * NR;
  if (need <= c->fsplit_cap) return hipSuccess;
  hipError_t e = c->alloc(&c->fsplit, need);
  if (e == hipSuccess) c->fsplit_cap = need;
  return e;
}

static int32_t choose_tile_bf16(int32_t n, int32_t r, int num_cus, int32_t precision) {
  // Preference from tile sweeps on MI355X at N=2000 (R=1024 and 2048),
  // N=4000 and N=8000 (R=2048): the largest tiles (64x64 waves: 128x256,
  // 256x128 with a double-buffered ring for the multi-plane forms, whose
  // fragment reads load the LDS most) once the problem gives every CU a
  // workgroup of that size, then 128x128 (for the three-plane form the
  // two-slab ring of eight waves), eight-wave 128x64 (single-plane and
  // three-plane forms) and 64x64 direct-to-LDS rings, then register-staged
  // tiles as the fallback for small problems.  Tiles 26 and 28 are the
  // pipelined twins (bit-identical results) of the three-plane 128x64 tile
  // and the hi + lo 128x256 tile: 32.1 -> 30.5 us at N=2000, R=1024 and
  // 482 -> 470 us at N=8000, R=2048.  Tiles 32 and 33 add state waves to
  // the eight-wave 128x64 tiles (single-plane forms at N=2000, R=1024: FP8
  // J 18.2 -> 17.1 us, BF16 J 19.4 -> 18.4 us; hi + lo 26.3 -> 25.6 us
  // against the 64x64 tile).
  static const int32_t pref_bf16j[] = {16, 18, 32, 8, 7, 11, 10, 1, 2, 3};
  static const int32_t pref_fp8j[] = {19, 14, 32, 9, 13, 1, 6, 2, 3};
  static const int32_t pref_hilo[] = {28, 18, 33, 7, 10, 11, 1, 2, 3};
  static const int32_t pref_exact[] = {21, 22, 26, 11, 8, 7, 1, 2, 3};
#define SI_PREF(a) order = a, count = (int)(sizeof a / sizeof a[0])
  const int32_t *order;
  int count;
  SI_PREF(pref_bf16j);
  if (precision == SI_PREC_BF16X_FP8J) SI_PREF(pref_fp8j);
  if (precision == SI_PREC_BF16X_HILOJ) SI_PREF(pref_hilo);
  if (precision == SI_PREC_BF16X3_EXACTJ) SI_PREF(pref_exact);
#undef SI_PREF
  int32_t best = 1;
  int64_t best_tiles = -1;
  for (int c = 0; c < count; ++c) {
    const int32_t t = order[c];
    if (!tile_valid_bf16(t, precision)) continue;
    TileShape ts = tile_shape_bf16(t);
    const int64_t np = round_up(n, ts.bm > 64 ? ts.bm : 64);
    const int64_t rp = round_up(r, ts.bn > 64 ? ts.bn : 64);
    const int64_t tiles = (np / ts.bm) * (rp / ts.bn);
    if (tiles >= num_cus) return t;
    if (tiles > best_tiles) {
      best_tiles = tiles;
      best = t;
    }
  }
  return best;
}

// Measured FP32 defaults for few replicas: the fastest (tile, contraction
// split) of a sweep over every FP32 tile and split 1, 2, 4, 8 on MI355X at
// N = 1000, 2000, 4000, 8000 and R = 32 .. 512, keyed by the N-bucket b
// (2^(b-1) < N <= 2^b) and R rounded up to 64.  Against the size rule below
// they run N = 8000, R = 64 in 83 us instead of 157 (J is streamed once per
// step by 64-replica-wide tiles instead of twice, and the split fills the
// chip), N = 4000, R = 64 in 28 us instead of 54, N = 2000, R = 128 in 18 us
// instead of 28.
struct FewReplicaDefault {
  int32_t nb, r64, tile, split;
};
static const FewReplicaDefault k_few_replicas[] = {
    {10, 64, 3, 4},  {10, 128, 3, 4},  {10, 256, 3, 2},  {10, 512, 3, 1},
    {11, 64, 3, 4},  {11, 128, 14, 4}, {11, 256, 26, 4}, {11, 512, 23, 1},
    {12, 64, 26, 8}, {12, 128, 26, 4}, {12, 256, 14, 2}, {12, 512, 34, 1},
    {13, 64, 26, 4}, {13, 128, 26, 2}, {13, 256, 26, 1}, {13, 512, 1, 1},
};

static bool few_replica_default(int32_t n, int32_t r, int32_t *tile, int32_t *split) {
  int32_t nb = 0;
  while (nb < 31 && (1 << nb) < n) ++nb;
  const int32_t r64 = (int32_t)round_up(r, 64);
  for (const FewReplicaDefault &d : k_few_replicas)
    if (d.nb == nb && d.r64 == r64) {
      *tile = d.tile;
      // a split needs at least 128 contraction entries per range
      int32_t s = d.split;
      while (s > 1 && s > round_up(n, 32) / 128) s /= 2;
      *split = s;
      return true;
    }
  return false;
}

static int32_t choose_tile(int32_t n, int32_t r, int num_cus) {
  // Preference from tile sweeps on MI355X: at N=2000, R=1024 the 8-wave
  // direct-to-LDS tiles (64x128, then 128x64) lead; a problem with at least
  // two 64x128 tiles per CU and at least 128 replicas (N=2000 with R=2048,
  // N=4000 with R=1024, N=8000) runs best on the register-staged 64x128
  // tile, two of whose four-wave workgroups share a CU and keep its matrix
  // cores busy through each other's barriers.  Rows are counted as init
  // pads them (to a multiple of 128).
  {
    const TileShape big = tile_shape(1);
    if (r >= big.bn &&
        (round_up(n, 128) / big.bm) * (round_up(r, big.bn) / big.bn) >= 2 * (int64_t)num_cus)
      return 1;
  }
  const int32_t order[] = {27, 26, 2, 9, 12, 6, 3};
  int32_t best = 3;
  int64_t best_tiles = -1;
  for (int32_t t : order) {
    TileShape ts = tile_shape(t);
    const int64_t np = round_up(n, ts.bm > 64 ? ts.bm : 64);
    const int64_t rp = round_up(r, ts.bn > 64 ? ts.bn : 64);
    const int64_t tiles = (np / ts.bm) * (rp / ts.bn);
    if (tiles >= num_cus) return t;
    if (tiles > best_tiles) {
      best_tiles = tiles;
      best = t;
    }
  }
  return best;
}

// Buffers of the best-state record (allocated once, records invalid).
static hipError_t ensure_best_buffers(si_ctx *c) {
  if (c->best_e) return hipSuccess;
  const int64_t rows = c->n_inst ? (int64_t)c->n_inst * c->r : c->r_pad;
  const int64_t sbytes = c->n_inst ? c->b_stot : (int64_t)c->r_pad * c->n_pad;
  hipError_t e = c->alloc(&c->best_e, rows);
  if (e == hipSuccess) e = c->alloc(&c->e_scratch, rows);
  if (e == hipSuccess) e = c->alloc(&c->best_valid, rows);
  if (e == hipSuccess) e = c->alloc(&c->best_s, sbytes);
  if (e == hipSuccess) e = launch_zero_i32(c->best_valid, rows, c->stream);
  return e;
}

// In-run energy checks requested at init: the trace and the best record.
static hipError_t init_energy_checks(si_ctx *c) {
  c->e_every = c->prm.energy_every;
  if (c->e_every <= 0) return hipSuccess;
  c->e_rows = c->prm.total_steps / c->e_every;
  hipError_t e = c->alloc(&c->etrace, (c->e_rows > 0 ? c->e_rows : 1) * c->out_rows());
  if (e == hipSuccess) e = ensure_best_buffers(c);
  return e;
}

// Hash of the sources and build flags this library was compiled from, set
// by the build script; the marker prefix lets a loader read it from the
// file before loading it.
#ifndef SI_BUILD_ID
#define SI_BUILD_ID "unstamped"
#endif
static const char k_build_id[] = "SI_BUILD_ID:" SI_BUILD_ID;

// The process's tile cache: (kind, precision, N-bucket, largest-N bucket,
// R rounded to 64, CU count) -> (tile, us per step).  Kind 0: single
// instance (largest-N bucket 0), kind 1: batch.
namespace {
using TileKey = std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t>;
struct TileEntry {
  int32_t tile;
  float us;
};
std::mutex g_tile_mu;
std::map<TileKey, TileEntry> g_tile_cache;

int32_t n_bucket(int64_t x) {
  int32_t b = 0;
  while (b < 62 && ((int64_t)1 << b) < x) ++b;
  return b;
}

TileKey tile_key(const si_ctx *c) {
  if (c->n_inst) {
    int64_t rows = 0;
    for (int32_t np : c->b_npad) rows += np;
    return TileKey{1, c->prm.precision, n_bucket(rows), n_bucket(c->b_max_npad),
                   (int32_t)round_up(c->r, 64), c->num_cus};
  }
  return TileKey{0, c->prm.precision, n_bucket(c->n), 0, (int32_t)round_up(c->r, 64),
                 c->num_cus};
}

// Can `tile` serve contexts of this key at all (padding aside)?
bool tile_serves(int32_t kind, int32_t precision, int32_t tile) {
  if (kind == 1) return tile >= 1 && tile <= BATCH_TILE_LAST;
  if (precision == SI_PREC_FP32) return tile >= 1 && tile <= TILE_F32_LAST;
  return tile >= 1 && tile <= TILE_BF16_LAST && tile_valid_bf16(tile, precision);
}

bool tile_cache_get(const TileKey &k, int32_t *tile) {
  std::lock_guard<std::mutex> lock(g_tile_mu);
  auto it = g_tile_cache.find(k);
  if (it == g_tile_cache.end()) return false;
  *tile = it->second.tile;
  return true;
}

void tile_cache_put(const TileKey &k, int32_t tile, float us) {
  std::lock_guard<std::mutex> lock(g_tile_mu);
  g_tile_cache[k] = TileEntry{tile, us};
}

const char k_cache_magic[] = "# spring_ising tile cache 1";
}  // namespace

// Work list of a batch for its tile (instance, row tile, column tile).
// The hardware hands workgroup b to XCD b % 8, and each XCD has its own L2;
// all items of an instance read that instance's position plane.  So whole
// instances are dealt to the XCDs (costliest first, each to the XCD with the
// least work of its J format so far), the queues are evened out to the number of workgroups
// each XCD receives by moving their cheapest items, every queue runs its
// costliest items first, and queue x fills positions x, x + 8, ...  An
// item's cost is its contraction length, doubled for hi + lo J (two
// matrix-core planes).  On the 256-instance workload (N 64..4096, R = 64)
// the cost order took the mixed BF16 step from 0.915 to 0.895 ms against
// plain length order; dealing whole instances, instead of handing
// consecutive items to consecutive XCDs, cut the bytes fetched per step
// from 4.73 to 4.28 GB (BF16 form) and from 7.52 to 6.61 GB (FP32), within
// 2 % of the algorithmic bytes, at the same step time.
static hipError_t batch_items(si_ctx *c) {
  constexpr int NX = NUM_XCD;
  const int32_t rows = batch_tile_rows(c->tile), ncol = c->r_pad / BATCH_BN;
  auto cost = [&](int32_t x) { return (int64_t)c->b_npad[x] * (c->b_fmt[x] == 2 ? 2 : 1); };
  std::vector<int32_t> order(c->n_inst);
  for (int32_t i = 0; i < c->n_inst; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const int64_t cx = cost(x) * (c->b_npad[x] / rows), cy = cost(y) * (c->b_npad[y] / rows);
    return cx > cy;
  });
  std::vector<std::vector<int4>> q(NX);
  // work per XCD, kept for each J format apart, so that every XCD receives
  // the same share of each whatever their relative cost
  int64_t load[3][NX] = {{0}};
  int64_t n = 0;
  for (int32_t i : order) {
    const int f = c->b_fmt[i];
    int x = 0;
    for (int k = 1; k < NX; ++k)
      if (load[f][k] < load[f][x]) x = k;
    for (int32_t rt = 0; rt < c->b_npad[i] / rows; ++rt)
      for (int32_t ct = 0; ct < ncol; ++ct) q[x].push_back(int4{i, rt, ct, 0});
    const int64_t k_items = (int64_t)(c->b_npad[i] / rows) * ncol;
    load[f][x] += cost(i) * k_items;
    n += k_items;
  }
  auto by_cost = [&](const int4 &u, const int4 &v) { return cost(u.x) > cost(v.x); };
  for (auto &qq : q) std::stable_sort(qq.begin(), qq.end(), by_cost);
  // queue x must hold exactly the items of positions x, x + NX, ... < n
  auto want = [&](int x) { return x < n ? (n - x + NX - 1) / NX : 0; };
  for (;;) {
    int over = -1, under = -1;
    for (int x = 0; x < NX; ++x) {
      if (over < 0 && (int64_t)q[x].size() > want(x)) over = x;
      if (under < 0 && (int64_t)q[x].size() < want(x)) under = x;
    }
    if (over < 0 || under < 0) break;
    q[under].push_back(q[over].back());  // the cheapest item of the long queue
    q[over].pop_back();
  }
  for (auto &qq : q) std::stable_sort(qq.begin(), qq.end(), by_cost);
  c->b_items_host.assign((size_t)n, int4{0, 0, 0, 0});
  for (int x = 0; x < NX; ++x)
    for (size_t g = 0; g < q[x].size(); ++g) c->b_items_host[(size_t)g * NX + x] = q[x][g];
  if ((int64_t)c->b_items_host.size() > c->b_items_cap) {
    hipError_t e = c->alloc(&c->b_items, (int64_t)c->b_items_host.size());
    if (e != hipSuccess) return e;
    c->b_items_cap = (int64_t)c->b_items_host.size();
  }
  hipError_t e = hipMemcpyAsync(c->b_items, c->b_items_host.data(),
                                sizeof(int4) * c->b_items_host.size(), hipMemcpyHostToDevice,
                                c->stream);
  // the host list may change before an asynchronous copy from pageable
  // memory has read it
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e;
}

extern "C" {

const char *spring_ising_last_error(void) { return g_last_error.c_str(); }

const char *spring_ising_build_id(void) { return k_build_id + 12; }

si_status spring_ising_energy_noalloc(int32_t n, int32_t r, const float *J, const float *x,
                                      int32_t *e_int, void *hip_stream) {
  if (n < 1 || n > 65536)
    return fail(SI_ERR_INVALID, "energy_noalloc: n=%d outside 1..65536", n);
  if (r < 1 || r > noalloc_r_max())
    return fail(SI_ERR_INVALID, "energy_noalloc: r=%d outside 1..%d (the static scratch holds "
                "%d replicas)", r, noalloc_r_max(), noalloc_r_max());
  if (!is_device_ptr(J) || !is_device_ptr(x) || !is_device_ptr(e_int))
    return fail(SI_ERR_INVALID, "energy_noalloc: J, x and e_int must be device pointers");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  void *sc = nullptr;
  if (e == hipSuccess) e = noalloc_scratch_ptr(dev, &sc);
  if (e == hipSuccess)
    e = launch_noalloc_energy(J, x, n, r, e_int, sc, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(SI_ERR_HIP, "energy_noalloc: %s", hipGetErrorString(e));
  return SI_OK;
}

si_status spring_ising_debug_inject_hip_error(si_ctx *c, int32_t n) {
  SI_USABLE(c);
  if (n < 0) return fail(SI_ERR_INVALID, "debug_inject_hip_error: n=%d < 0", n);
  c->inject_countdown = n;
  return SI_OK;
}

si_status spring_ising_default_params(si_params *prm, int32_t total_steps) {
  if (!prm) return fail(SI_ERR_INVALID, "default_params: null");
  memset(prm, 0, sizeof *prm);
  prm->k = 0.5f;
  prm->m = 1.0f;
  prm->dt = 0.2f;
  prm->zeta_start = 0.04f;  // 0.8 * zeta0, zeta0 = 0.05
  prm->zeta_end = 0.5f;     // 10 * zeta0
  prm->total_steps = total_steps;
  prm->stair_len = 1;
  prm->qmax = sqrtf(2.0f);
  prm->pmax = 2.0f;
  prm->order = SI_ORDER_PAPER;
  prm->wall = SI_WALL_CLAMP;
  prm->precision = SI_PREC_FP32;
  prm->tile = 0;
  if (total_steps < 1) return fail(SI_ERR_INVALID, "default_params: total_steps must be >= 1");
  return SI_OK;
}

si_status spring_ising_init(si_ctx **out, int32_t n, int32_t r, const float *J, const float *x0,
                            const float *p0, const si_params *prm, void *hip_stream) {
  if (!out) return fail(SI_ERR_INVALID, "init: out is null");
  *out = nullptr;
  if (n < 1 || r < 1) return fail(SI_ERR_INVALID, "init: n=%d r=%d must be >= 1", n, r);
  if (n > 65536 || r > (1 << 24))
    return fail(SI_ERR_INVALID, "init: n=%d r=%d beyond the supported range", n, r);
  if (!J || !x0) return fail(SI_ERR_INVALID, "init: J and x0 are required");
  si_status st = check_params(prm);
  if (st != SI_OK) return st;
  if (!is_device_ptr(J) || !is_device_ptr(x0) || (p0 && !is_device_ptr(p0)))
    return fail(SI_ERR_INVALID, "init: J, x0 and p0 must be device pointers");

  si_ctx *c = new (std::nothrow) si_ctx();
  if (!c) return fail(SI_ERR_OOM, "init: host allocation failed");
  c->n = n;
  c->r = r;
  c->prm = *prm;
  c->stream = static_cast<hipStream_t>(hip_stream);
#define INIT_HIP(expr)                                                                  \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess) {                                                             \
      delete c;                                                                         \
      return fail(_e == hipErrorOutOfMemory ? SI_ERR_OOM : SI_ERR_HIP, "init: %s (%s)", \
                  hipGetErrorString(_e), #expr);                                        \
    }                                                                                   \
  } while (0)
  INIT_HIP(hipGetDevice(&c->device));
  INIT_HIP(hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device));
  {
    void *sc = nullptr;  // set-up of the allocation-free entry point on this device
    INIT_HIP(noalloc_scratch_ptr(c->device, &sc));
  }

  // validation of J: one host round trip
  INIT_HIP(c->alloc(&c->flags, 8));
  INIT_HIP(launch_zero_i32(c->flags, 8, c->stream));
  INIT_HIP(launch_validate(J, n, c->flags, c->stream));
  INIT_HIP(hipMemcpyAsync(c->hflags, c->flags, sizeof c->hflags, hipMemcpyDeviceToHost,
                          c->stream));
  INIT_HIP(hipStreamSynchronize(c->stream));
  if (c->hflags[0] || c->hflags[1] || c->hflags[2]) {
    const int a = c->hflags[0], d = c->hflags[1], f = c->hflags[2];
    delete c;
    return fail(SI_ERR_INVALID, "init: J must be finite, symmetric with a zero diagonal "
                "(asymmetric=%d nonzero_diagonal=%d nonfinite=%d)", a, d, f);
  }
  if (c->prm.precision == SI_PREC_BF16X_MIXEDJ)
    c->prm.precision = c->hflags[4] == 0 ? SI_PREC_BF16X_FP8J : SI_PREC_BF16X_HILOJ;
  prm = &c->prm;

  const bool lowp = prm->precision != SI_PREC_FP32;
  c->user_tile = prm->tile;
  c->n = n;
  c->r = r;
  int32_t cached = 0;
  if (prm->tile) {
    c->tile = prm->tile;
    c->tile_source = SI_TILE_FROM_CALLER;
  } else if (tile_cache_get(tile_key(c), &cached) &&
             tile_serves(0, prm->precision, cached)) {
    c->tile = cached;
    c->tile_source = SI_TILE_FROM_CACHE;
  } else if (!lowp && c->num_cus == 256 &&
             few_replica_default(n, r, &c->table_tile, &c->table_split)) {
    c->tile = c->table_tile;
  } else {
    c->tile = lowp ? choose_tile_bf16(n, r, c->num_cus, prm->precision)
                   : choose_tile(n, r, c->num_cus);
  }
  if (lowp && !tile_valid_bf16(c->tile, prm->precision)) {
    const int32_t bad = c->tile;
    delete c;
    return fail(SI_ERR_INVALID, "init: tile %d cannot run precision %d", bad, prm->precision);
  }
  const TileShape ts = shape_of(prm->precision, c->tile);
  c->n_pad = (int32_t)round_up(n, ts.bm > 128 ? ts.bm : 128);
  c->r_pad = (int32_t)round_up(r, ts.bn > 64 ? ts.bn : 64);
  const bool j_integer = c->hflags[3] == 0;
  const bool need_bf16 = prm->precision == SI_PREC_BF16X_BF16J ||
                         prm->precision == SI_PREC_BF16X3_EXACTJ;
  if ((need_bf16 && c->hflags[5]) || (prm->precision == SI_PREC_BF16X_FP8J && c->hflags[4])) {
    delete c;
    return fail(SI_ERR_UNSUPPORTED, "init: precision %d needs J exact in %s", prm->precision,
                need_bf16 ? "BF16" : "FP8 e4m3");
  }

  const int64_t nn = (int64_t)c->n_pad * c->n_pad;
  const int64_t nr = (int64_t)c->n_pad * c->r_pad;
  INIT_HIP(c->alloc(&c->J, nn));
  if (j_integer) INIT_HIP(c->alloc(&c->J8, nn));
  for (int b = 0; b < 2; ++b) {
    INIT_HIP(c->alloc(&c->q[b], nr));
    INIT_HIP(c->alloc(&c->p[b], nr));
  }
  INIT_HIP(c->alloc(&c->dt, prm->total_steps));
  INIT_HIP(c->alloc(&c->zeta, prm->total_steps));
  INIT_HIP(c->alloc(&c->S8, nr));
  INIT_HIP(c->alloc(&c->eacc, c->r_pad));
  INIT_HIP(c->alloc(&c->epart, (int64_t)(c->n_pad / 64) * c->r_pad));

  if (lowp) {
    c->qplanes = prm->precision == SI_PREC_BF16X3_EXACTJ ? 3 : 1;
    const int64_t jbytes = prm->precision == SI_PREC_BF16X_FP8J ? 1 : 2;
    INIT_HIP(c->alloc(reinterpret_cast<uint8_t **>(&c->Ja), nn * jbytes));
    if (prm->precision == SI_PREC_BF16X_HILOJ)
      INIT_HIP(c->alloc(reinterpret_cast<uint16_t **>(&c->Jb), nn));
    for (int b = 0; b < 2; ++b) INIT_HIP(c->alloc(&c->qb[b], nr * c->qplanes));
  }
  INIT_HIP(launch_pack_matrix(J, n, c->J, c->J8, c->n_pad, c->stream));
  if (lowp) INIT_HIP(launch_pack_j_lowp(c->J, nn, prm->precision, c->Ja, c->Jb, c->stream));
  INIT_HIP(launch_pack_state(x0, n, r, c->q[0], c->n_pad, c->r_pad, c->stream));
  INIT_HIP(launch_pack_state(p0, n, r, c->p[0], c->n_pad, c->r_pad, c->stream));
  if (lowp) INIT_HIP(launch_split_planes(c->q[0], c->qb[0], nr, c->qplanes, c->stream));
  INIT_HIP(launch_zero_i32(c->eacc, c->r_pad, c->stream));
  INIT_HIP(ensure_split_ws(c));
  build_schedules(*prm, c->host_dt, c->host_zeta);
  INIT_HIP(hipMemcpyAsync(c->dt, c->host_dt.data(), sizeof(float) * prm->total_steps,
                          hipMemcpyHostToDevice, c->stream));
  INIT_HIP(hipMemcpyAsync(c->zeta, c->host_zeta.data(), sizeof(float) * prm->total_steps,
                          hipMemcpyHostToDevice, c->stream));
  INIT_HIP(init_energy_checks(c));
#undef INIT_HIP
  c->cur = 0;
  c->t = 0;
  *out = c;
  return SI_OK;
}

si_status spring_ising_init_batch(si_ctx **out, int32_t n_inst, const int32_t *n, int32_t r,
                                  const float *const *J, const float *const *x0,
                                  const float *const *p0, const si_params *prm,
                                  void *hip_stream) {
  if (!out) return fail(SI_ERR_INVALID, "init_batch: out is null");
  *out = nullptr;
  if (n_inst < 1 || r < 1 || !n || !J || !x0)
    return fail(SI_ERR_INVALID, "init_batch: n_inst, r >= 1 and n, J, x0 arrays are required");
  if (r > (1 << 20)) return fail(SI_ERR_INVALID, "init_batch: r=%d too large", r);
  si_status st = check_params(prm);
  if (st != SI_OK) return st;
  if (prm->precision == SI_PREC_BF16X_BF16J || prm->precision == SI_PREC_BF16X3_EXACTJ)
    return fail(SI_ERR_UNSUPPORTED, "init_batch: precision %d has no batched form", prm->precision);
  if (prm->tile < 0 || prm->tile > BATCH_TILE_LAST)
    return fail(SI_ERR_INVALID, "init_batch: batch tile %d not in 0..%d", prm->tile,
                BATCH_TILE_LAST);
  const bool lowp = prm->precision != SI_PREC_FP32;
  for (int32_t i = 0; i < n_inst; ++i) {
    if (n[i] < 1 || n[i] > 65536) return fail(SI_ERR_INVALID, "init_batch: n[%d]=%d", i, n[i]);
    if (!is_device_ptr(J[i]) || !is_device_ptr(x0[i]) ||
        (p0 && p0[i] && !is_device_ptr(p0[i])))
      return fail(SI_ERR_INVALID, "init_batch: J[%d], x0[%d], p0[%d] must be device pointers", i,
                  i, i);
  }
  si_ctx *c = new (std::nothrow) si_ctx();
  if (!c) return fail(SI_ERR_OOM, "init_batch: host allocation failed");
  c->prm = *prm;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->n_inst = n_inst;
  c->r = r;
  c->r_pad = (int32_t)round_up(r, BATCH_BN);
  c->tile = 0;
  c->b_lowp = lowp;
#define BINIT_HIP(expr)                                                                  \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      delete c;                                                                          \
      return fail(_e == hipErrorOutOfMemory ? SI_ERR_OOM : SI_ERR_HIP, "init_batch: %s (%s)", \
                  hipGetErrorString(_e), #expr);                                         \
    }                                                                                    \
  } while (0)
  BINIT_HIP(hipGetDevice(&c->device));
  BINIT_HIP(hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device));
  // validation of every J: one host round trip for the whole batch
  int32_t *flags = nullptr;
  BINIT_HIP(c->alloc(&flags, (int64_t)8 * n_inst));
  BINIT_HIP(launch_zero_i32(flags, (int64_t)8 * n_inst, c->stream));
  for (int32_t i = 0; i < n_inst; ++i) BINIT_HIP(launch_validate(J[i], n[i], flags + 8 * i, c->stream));
  std::vector<int32_t> hfl((size_t)8 * n_inst);
  BINIT_HIP(hipMemcpyAsync(hfl.data(), flags, hfl.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                           c->stream));
  BINIT_HIP(hipStreamSynchronize(c->stream));
  int64_t jtot = 0, j8tot = 0, stot = 0, xoff = 0, latot = 0, lbtot = 0;
  c->b_n.resize(n_inst);
  c->b_npad.resize(n_inst);
  c->b_jmax.resize(n_inst);
  c->b_xoff.resize(n_inst);
  c->b_fmt.assign(n_inst, 0);
  for (int32_t i = 0; i < n_inst; ++i) {
    const int32_t *f = &hfl[(size_t)8 * i];
    if (f[0] || f[1] || f[2]) {
      delete c;
      return fail(SI_ERR_INVALID, "init_batch: J[%d] must be finite, symmetric, zero diagonal", i);
    }
    if (lowp) {
      const bool fp8 = f[4] == 0 && prm->precision != SI_PREC_BF16X_HILOJ;
      if (!fp8 && prm->precision == SI_PREC_BF16X_FP8J) {
        delete c;
        return fail(SI_ERR_UNSUPPORTED, "init_batch: J[%d] is not exact in FP8 e4m3", i);
      }
      c->b_fmt[i] = fp8 ? 1 : 2;
    }
    c->b_n[i] = n[i];
    c->b_npad[i] = (int32_t)round_up(n[i], lowp ? BATCH_BF16_NPAD : BATCH_BM);
    if (lowp) {
      const int64_t nn = (int64_t)c->b_npad[i] * c->b_npad[i];
      latot += c->b_fmt[i] == 1 ? nn : 2 * nn;  // bytes of the first J plane
      if (c->b_fmt[i] == 2) lbtot += nn;        // BF16 elements of the lo plane
    }
    c->b_jmax[i] = f[3] == 0 ? f[6] : -1;  // -1: not integer
    c->b_xoff[i] = xoff;
    xoff += (int64_t)r * n[i];
    jtot += (int64_t)c->b_npad[i] * c->b_npad[i];
    if (f[3] == 0) j8tot += (int64_t)c->b_npad[i] * c->b_npad[i];
    stot += (int64_t)c->r_pad * c->b_npad[i];
    c->b_max_npad = c->b_npad[i] > c->b_max_npad ? c->b_npad[i] : c->b_max_npad;
    c->b_total_n += n[i];
  }
  c->n = (int32_t)(c->b_total_n > 0x7fffffff ? 0x7fffffff : c->b_total_n);
  c->n_pad = c->b_max_npad;
  float *Jall = nullptr, *sbuf[4] = {nullptr, nullptr, nullptr, nullptr};
  int8_t *J8all = nullptr;
  BINIT_HIP(c->alloc(&Jall, jtot));
  if (j8tot) BINIT_HIP(c->alloc(&J8all, j8tot));
  for (int b = 0; b < 4; ++b) BINIT_HIP(c->alloc(&sbuf[b], stot));
  uint8_t *JAall = nullptr;
  uint16_t *JBall = nullptr, *qball[2] = {nullptr, nullptr};
  if (lowp) {
    BINIT_HIP(c->alloc(&JAall, latot));
    if (lbtot) BINIT_HIP(c->alloc(&JBall, lbtot));
    for (int b = 0; b < 2; ++b) BINIT_HIP(c->alloc(&qball[b], stot));
  }
  BINIT_HIP(c->alloc(&c->dt, prm->total_steps));
  BINIT_HIP(c->alloc(&c->zeta, prm->total_steps));
  c->b_stot = stot;
  BINIT_HIP(c->alloc(&c->S8, stot));  // sign(q) of every instance, in the state layout
  BINIT_HIP(c->alloc(&c->eacc, (int64_t)n_inst * c->r_pad));
  BINIT_HIP(launch_zero_i32(c->eacc, (int64_t)n_inst * c->r_pad, c->stream));
  int64_t jo = 0, j8o = 0, so = 0;
  c->b_J.resize(n_inst);
  c->b_J8.resize(n_inst);
  for (int b = 0; b < 2; ++b) {
    c->b_q[b].resize(n_inst);
    c->b_p[b].resize(n_inst);
  }
  c->b_desc_host.resize(n_inst);
  c->b_soff.resize(n_inst);
  if (lowp) {
    c->bb_desc_host.resize(n_inst);
    for (int b = 0; b < 2; ++b) c->b_qb[b].resize(n_inst);
  }
  int64_t lao = 0, lbo = 0;
  for (int32_t i = 0; i < n_inst; ++i) {
    const int64_t nn = (int64_t)c->b_npad[i] * c->b_npad[i];
    c->b_J[i] = Jall + jo;
    c->b_J8[i] = c->b_jmax[i] >= 0 ? J8all + j8o : nullptr;
    jo += nn;
    if (c->b_jmax[i] >= 0) j8o += nn;
    c->b_soff[i] = so;
    c->b_q[0][i] = sbuf[0] + so;
    c->b_q[1][i] = sbuf[1] + so;
    c->b_p[0][i] = sbuf[2] + so;
    c->b_p[1][i] = sbuf[3] + so;
    so += (int64_t)c->r_pad * c->b_npad[i];
    BINIT_HIP(launch_pack_matrix(J[i], n[i], c->b_J[i], c->b_J8[i], c->b_npad[i], c->stream));
    BINIT_HIP(launch_pack_state(x0[i], n[i], r, c->b_q[0][i], c->b_npad[i], c->r_pad, c->stream));
    BINIT_HIP(launch_pack_state(p0 ? p0[i] : nullptr, n[i], r, c->b_p[0][i], c->b_npad[i],
                                c->r_pad, c->stream));
    c->b_desc_host[i] = BatchDesc{c->b_J[i], c->b_q[0][i], c->b_q[1][i], c->b_p[0][i], c->b_p[1][i],
                                  c->b_npad[i], n[i]};
    if (lowp) {
      const int64_t nr = (int64_t)c->r_pad * c->b_npad[i];
      uint8_t *ja = JAall + lao;
      uint16_t *jb = c->b_fmt[i] == 2 ? JBall + lbo : nullptr;
      lao += c->b_fmt[i] == 1 ? nn : 2 * nn;
      if (jb) lbo += nn;
      c->b_qb[0][i] = qball[0] + (so - nr);
      c->b_qb[1][i] = qball[1] + (so - nr);
      BINIT_HIP(launch_pack_j_lowp(c->b_J[i], nn,
                                   c->b_fmt[i] == 1 ? SI_PREC_BF16X_FP8J : SI_PREC_BF16X_HILOJ,
                                   ja, jb, c->stream));
      BINIT_HIP(launch_split_planes(c->b_q[0][i], c->b_qb[0][i], nr, 1, c->stream));
      BBatchDesc d;
      d.Ja = ja;
      d.Jb = jb;
      d.q[0] = c->b_q[0][i];
      d.q[1] = c->b_q[1][i];
      d.p[0] = c->b_p[0][i];
      d.p[1] = c->b_p[1][i];
      d.qb[0] = c->b_qb[0][i];
      d.qb[1] = c->b_qb[1][i];
      d.n_pad = c->b_npad[i];
      d.fmt = c->b_fmt[i];
      c->bb_desc_host[i] = d;
    }
  }
  // batch tile: the caller's, else the tile cache's, else 128-row items
  int32_t cached = 0;
  if (prm->tile) {
    c->tile = prm->tile;
    c->tile_source = SI_TILE_FROM_CALLER;
  } else if (tile_cache_get(tile_key(c), &cached) && tile_serves(1, prm->precision, cached)) {
    c->tile = cached;
    c->tile_source = SI_TILE_FROM_CACHE;
  } else {
    c->tile = 1;
  }
  // the device work list holds the longest list (64-row items)
  int64_t items_max = 0;
  for (int32_t i = 0; i < n_inst; ++i) items_max += (int64_t)(c->b_npad[i] / 64) * (c->r_pad / BATCH_BN);
  BINIT_HIP(c->alloc(&c->b_items, items_max));
  c->b_items_cap = items_max;
  std::vector<int32_t> order(n_inst);
  for (int32_t i = 0; i < n_inst; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return c->b_npad[x] > c->b_npad[y]; });
  // grouped energy: exact int32 where the couplings are integer and the sum
  // cannot overflow, else the FP32 coupling sum; 64 x 64 tiles
  c->eb_desc_host.resize(n_inst);
  int32_t part_rows = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int32_t i : order) {
      const int64_t bound = (int64_t)n[i] * n[i] * (c->b_jmax[i] < 0 ? 0 : c->b_jmax[i]);
      const bool exact = c->b_J8[i] != nullptr && bound < (1LL << 31);
      if (exact != (pass == 0)) continue;
      c->eb_desc_host[i] = EBatchDesc{exact ? c->b_J8[i] : nullptr, c->b_J[i], c->b_soff[i],
                                      c->b_npad[i], exact ? 0 : part_rows};
      if (!exact) part_rows += c->b_npad[i] / 64;
      for (int32_t rt = 0; rt < c->b_npad[i] / 64; ++rt)
        for (int32_t ct = 0; ct < c->r_pad / 64; ++ct) c->eb_items_host.push_back(int4{i, rt, ct, 0});
      (pass == 0 ? c->eb_n_i8 : c->eb_n_f32) += (c->b_npad[i] / 64) * (c->r_pad / 64);
    }
  BINIT_HIP(c->alloc(&c->epart, (int64_t)(part_rows > 0 ? part_rows : 1) * c->r_pad));
  BINIT_HIP(c->alloc(&c->eb_desc, n_inst));
  BINIT_HIP(c->alloc(&c->eb_items, (int64_t)c->eb_items_host.size()));
  BINIT_HIP(hipMemcpyAsync(c->eb_desc, c->eb_desc_host.data(), sizeof(EBatchDesc) * n_inst,
                           hipMemcpyHostToDevice, c->stream));
  BINIT_HIP(hipMemcpyAsync(c->eb_items, c->eb_items_host.data(),
                           sizeof(int4) * c->eb_items_host.size(), hipMemcpyHostToDevice,
                           c->stream));
  BINIT_HIP(c->alloc(&c->b_desc, n_inst));
  BINIT_HIP(hipMemcpyAsync(c->b_desc, c->b_desc_host.data(), sizeof(BatchDesc) * n_inst,
                           hipMemcpyHostToDevice, c->stream));
  if (lowp) {
    BINIT_HIP(c->alloc(&c->bb_desc, n_inst));
    BINIT_HIP(hipMemcpyAsync(c->bb_desc, c->bb_desc_host.data(), sizeof(BBatchDesc) * n_inst,
                             hipMemcpyHostToDevice, c->stream));
  }
  BINIT_HIP(batch_items(c));
  build_schedules(*prm, c->host_dt, c->host_zeta);
  BINIT_HIP(hipMemcpyAsync(c->dt, c->host_dt.data(), sizeof(float) * prm->total_steps,
                           hipMemcpyHostToDevice, c->stream));
  BINIT_HIP(hipMemcpyAsync(c->zeta, c->host_zeta.data(), sizeof(float) * prm->total_steps,
                           hipMemcpyHostToDevice, c->stream));
  BINIT_HIP(init_energy_checks(c));
  BINIT_HIP(hipStreamSynchronize(c->stream));  // host tables may go out of scope
#undef BINIT_HIP
  c->cur = 0;
  c->t = 0;
  *out = c;
  return SI_OK;
}

si_status spring_ising_set_schedule(si_ctx *c, const float *dt, const float *zeta) {
  SI_USABLE(c);
  if (!is_device_ptr(dt) || !is_device_ptr(zeta))
    return fail(SI_ERR_INVALID, "set_schedule: dt and zeta must be device pointers");
  c->epoch++;
  const size_t bytes = sizeof(float) * c->prm.total_steps;
  SI_HIP(c, hipMemcpyAsync(c->dt, dt, bytes, hipMemcpyDeviceToDevice, c->stream));
  SI_HIP(c, hipMemcpyAsync(c->zeta, zeta, bytes, hipMemcpyDeviceToDevice, c->stream));
  return SI_OK;
}

si_status spring_ising_get_schedule(si_ctx *c, float *dt, float *zeta) {
  SI_USABLE(c);
  if ((dt && !is_device_ptr(dt)) || (zeta && !is_device_ptr(zeta)))
    return fail(SI_ERR_INVALID, "get_schedule: outputs must be device pointers");
  const size_t bytes = sizeof(float) * c->prm.total_steps;
  if (dt) SI_HIP(c, hipMemcpyAsync(dt, c->dt, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (zeta) SI_HIP(c, hipMemcpyAsync(zeta, c->zeta, bytes, hipMemcpyDeviceToDevice, c->stream));
  return SI_OK;
}

si_status spring_ising_set_field(si_ctx *c, const float *h) {
  SI_USABLE(c);
  c->epoch++;
  // captured launch sequences hold the field pointer (or its absence) in
  // their kernel arguments, so none of them may be replayed after a change
  c->drop_graphs();
  if (!h) {
    c->has_field = false;
    return SI_OK;
  }
  if (!is_device_ptr(h)) return fail(SI_ERR_INVALID, "set_field: h must be a device pointer");
  if (c->n_inst) return fail(SI_ERR_UNSUPPORTED, "set_field: not available for a batch");
  if (!c->hf) {
    SI_HIP(c, c->alloc(&c->hf, c->n_pad));
    SI_HIP(c, c->alloc(&c->h8, c->n_pad));
  }
  int32_t *fl = c->flags;
  SI_HIP(c, launch_zero_i32(fl, 8, c->stream));
  SI_HIP(c, launch_pack_field(h, c->n, c->hf, c->h8, c->n_pad, fl, c->stream));
  int32_t hfl[8];
  SI_HIP(c, hipMemcpyAsync(hfl, fl, sizeof hfl, hipMemcpyDeviceToHost, c->stream));
  SI_HIP(c, hipStreamSynchronize(c->stream));
  if (hfl[2]) return fail(SI_ERR_INVALID, "set_field: h must be finite");
  c->has_field = true;
  c->field_integer = hfl[3] == 0;
  c->field_maxabs = hfl[6];
  return SI_OK;
}

// In-run energy check after the step that brought the context to time t.
static si_status record_check(si_ctx *c);
#define SI_ENERGY_CHECK(c)                                   \
  do {                                                       \
    if ((c)->e_every > 0 && (c)->t % (c)->e_every == 0) {    \
      si_status _st = record_check(c);                       \
      if (_st != SI_OK) return _st;                          \
    }                                                        \
  } while (0)

static si_status do_steps_lowp(si_ctx *c, int32_t n_steps) {
  BStepArgs a;
  a.Ja = c->Ja;
  a.Jb = c->Jb;
  a.plane_stride = (int64_t)c->n_pad * c->r_pad;
  a.dt = c->dt;
  a.zeta = c->zeta;
  a.h = c->has_field ? c->hf : nullptr;
  a.ld = c->n_pad;
  a.n_pad = c->n_pad;
  a.r_pad = c->r_pad;
  a.k = c->prm.k;
  a.inv_m = 1.0f / c->prm.m;
  a.qmax = c->prm.qmax;
  a.pmax = c->prm.pmax;
  a.order = c->prm.order;
  a.wall = c->prm.wall;
  for (int32_t s = 0; s < n_steps; ++s) {
    a.q_in = c->q[c->cur];
    a.p_in = c->p[c->cur];
    a.q_out = c->q[c->cur ^ 1];
    a.p_out = c->p[c->cur ^ 1];
    a.qb_in = c->qb[c->cur];
    a.qb_out = c->qb[c->cur ^ 1];
    a.t = c->t;
    SI_HIP(c, launch_step_bf16(c->tile, c->prm.precision, a, c->stream));
    c->cur ^= 1;
    c->t += 1;
    SI_ENERGY_CHECK(c);
  }
  return SI_OK;
}

static StepArgs step_args(si_ctx *c) {
  StepArgs a;
  a.J = c->J;
  a.dt = c->dt;
  a.zeta = c->zeta;
  a.h = c->has_field ? c->hf : nullptr;
  a.ld = c->n_pad;
  a.n = c->n;
  a.n_pad = c->n_pad;
  a.r_pad = c->r_pad;
  a.k = c->prm.k;
  a.inv_m = 1.0f / c->prm.m;
  a.qmax = c->prm.qmax;
  a.pmax = c->prm.pmax;
  a.order = c->prm.order;
  a.wall = c->prm.wall;
  a.mask_out = nullptr;
  a.ksplit = split_for(c, c->tile);
  a.fsplit = c->fsplit;
  return a;
}


// trace: null, or n_steps * (work items) records of 4 words, step-major.
static si_status do_steps_batch(si_ctx *c, int32_t n_steps, unsigned long long *trace = nullptr) {
  const int64_t n_items = (int64_t)c->b_items_host.size();
  if (c->b_lowp) {
    BStepArgs b;
    memset(&b, 0, sizeof b);
    b.dt = c->dt;
    b.zeta = c->zeta;
    b.h = nullptr;
    b.r_pad = c->r_pad;
    b.k = c->prm.k;
    b.inv_m = 1.0f / c->prm.m;
    b.qmax = c->prm.qmax;
    b.pmax = c->prm.pmax;
    b.order = c->prm.order;
    b.wall = c->prm.wall;
    for (int32_t s = 0; s < n_steps; ++s) {
      b.t = c->t;
      SI_HIP(c, launch_step_batch_bf16(b, c->bb_desc, c->b_items, (int32_t)n_items, c->cur,
                                       c->tile, trace ? trace + 4 * n_items * s : nullptr,
                                       c->stream));
      c->cur ^= 1;
      c->t += 1;
      SI_ENERGY_CHECK(c);
    }
    return SI_OK;
  }
  StepArgs a = step_args(c);
  for (int32_t s = 0; s < n_steps; ++s) {
    a.t = c->t;
    SI_HIP(c, launch_step_batch_f32(a, c->b_desc, c->b_items, (int32_t)n_items, c->cur, c->tile,
                                    trace ? trace + 4 * n_items * s : nullptr, c->stream));
    c->cur ^= 1;
    c->t += 1;
    SI_ENERGY_CHECK(c);
  }
  return SI_OK;
}

static si_status do_steps(si_ctx *c, int32_t n_steps) {
  if (c->n_inst) return do_steps_batch(c, n_steps);
  if (c->qplanes) return do_steps_lowp(c, n_steps);
  StepArgs a;
  a.J = c->J;
  a.dt = c->dt;
  a.zeta = c->zeta;
  a.h = c->has_field ? c->hf : nullptr;
  a.ld = c->n_pad;
  a.n = c->n;
  a.n_pad = c->n_pad;
  a.r_pad = c->r_pad;
  a.k = c->prm.k;
  a.inv_m = 1.0f / c->prm.m;
  a.qmax = c->prm.qmax;
  a.pmax = c->prm.pmax;
  a.order = c->prm.order;
  a.wall = c->prm.wall;
  a.ksplit = split_for(c, c->tile);
  a.fsplit = c->fsplit;
  if (a.ksplit > 1 && (int64_t)a.ksplit * c->n_pad * c->r_pad > c->fsplit_cap)
    return fail(SI_ERR_STATE, "step: split-contraction workspace missing");
  for (int32_t s = 0; s < n_steps; ++s) {
    a.q_in = c->q[c->cur];
    a.p_in = c->p[c->cur];
    a.q_out = c->q[c->cur ^ 1];
    a.p_out = c->p[c->cur ^ 1];
    a.t = c->t;
    a.mask_out = nullptr;
    SI_HIP(c, launch_step_f32(c->tile, a, c->stream));
    c->cur ^= 1;
    c->t += 1;
    SI_ENERGY_CHECK(c);
  }
  return SI_OK;
}

// Adjoint, forward half: run from the current step t0 to the end of the
// schedule, keeping the state at the start of every segment of ckpt_every
// steps, then the seed lq_S = -(1/R) J q_S, lp_S = 0 and the loss.  Records
// the tape that the backward half reads.
static si_status adj_forward(si_ctx *c, int32_t C, double *loss) {
  if (c->prm.order != SI_ORDER_PAPER || c->prm.wall != SI_WALL_CLAMP ||
      c->prm.precision != SI_PREC_FP32 || c->has_field || c->n_inst)
    return fail(SI_ERR_UNSUPPORTED, "relaxed energy adjoint: needs paper order, clamping walls, "
                "FP32 precision and no field");
  c->tape.valid = false;
  const int32_t S = c->prm.total_steps, t0 = c->t;
  // a segment never holds more than the remaining steps (the workspace is
  // sized by the segment length)
  if (C > S - t0) C = S - t0 > 0 ? S - t0 : 1;
  const int32_t nseg = (S - t0 + C - 1) / C;
  const int64_t NR = (int64_t)c->n_pad * c->r_pad;
  const int32_t asplit = adj_split(c);
  const int32_t nwg_seed = (c->n_pad / ADJ_BM) * (c->r_pad / ADJ_BN);
  const int32_t nwg = asplit > 1 ? adj_split_groups(c->n_pad, c->r_pad) : nwg_seed;
  SI_HIP(c, ensure_split_ws(c, true));
  if ((int64_t)nseg * 2 * NR > c->adj_ckpt_cap) {
    SI_HIP(c, c->alloc(&c->adj_ckpt, (int64_t)(nseg > 0 ? nseg : 1) * 2 * NR));
    c->adj_ckpt_cap = (int64_t)(nseg > 0 ? nseg : 1) * 2 * NR;
  }
  if ((int64_t)(C + 1) * 2 * NR > c->adj_seg_cap) {
    SI_HIP(c, c->alloc(&c->adj_seg, (int64_t)(C + 1) * 2 * NR));
    SI_HIP(c, c->alloc(&c->adj_mask, (int64_t)C * NR));
    c->adj_seg_cap = (int64_t)(C + 1) * 2 * NR;
  }
  if (!c->adj_lam) SI_HIP(c, c->alloc(&c->adj_lam, 4 * NR));
  // partial triples of every step of the sweep, reduced in one launch at the
  // end (the seed's triples use the start of the same buffer first)
  const int64_t part_need = (int64_t)(S - t0 > 1 ? S - t0 : 1) * (nwg > nwg_seed ? nwg : nwg_seed) * 3;
  if (part_need > c->adj_part_cap) {
    SI_HIP(c, c->alloc(&c->adj_part, part_need));
    c->adj_part_cap = part_need;
  }
  const float inv_r = 1.0f / (float)c->r, inv_m = 1.0f / c->prm.m, k = c->prm.k;
  // forward with checkpoints at the start of every segment
  for (int32_t sg = 0; sg < nseg; ++sg) {
    float *ck = c->adj_ckpt + (int64_t)sg * 2 * NR;
    SI_HIP(c, hipMemcpyAsync(ck, c->q[c->cur], NR * sizeof(float), hipMemcpyDeviceToDevice,
                             c->stream));
    SI_HIP(c, hipMemcpyAsync(ck + NR, c->p[c->cur], NR * sizeof(float),
                             hipMemcpyDeviceToDevice, c->stream));
    const int32_t len = (S - c->t) < C ? (S - c->t) : C;
    si_status st = do_steps(c, len);
    if (st != SI_OK) return st;
  }
  // seed: lq_S = -(1/R) J q_S, lp_S = 0, and the loss
  SI_HIP(c, launch_adj_seed(c->J, c->q[c->cur], c->adj_lam, c->adj_lam + NR, c->adj_part,
                            c->n_pad, c->r_pad, inv_r, c->stream));
  SI_HIP(c, launch_adj_reduce(c->adj_part, nwg_seed, 0, loss, nullptr, nullptr, c->dt, c->zeta, 0,
                              1, k, inv_m, c->r, c->stream));
  c->tape.valid = true;
  c->tape.epoch = c->epoch;
  c->tape.t0 = t0;
  c->tape.ckpt = C;
  return SI_OK;
}

// Adjoint, backward half: the reverse sweep over the recorded tape, one
// segment at a time (forward recomputed from its checkpoint, recording the
// wall masks), and the gradient entries of every step in one launch.
static si_status adj_backward(si_ctx *c, double *g_dt, double *g_zeta) {
  if (!c->tape.valid || c->tape.epoch != c->epoch)
    return fail(SI_ERR_STATE, "relaxed energy backward: no forward half since the last change of "
                "the trajectory (schedule, field, state, steps or kernel)");
  const int32_t S = c->prm.total_steps, t0 = c->tape.t0, C = c->tape.ckpt;
  const int32_t nseg = (S - t0 + C - 1) / C;
  const int64_t NR = (int64_t)c->n_pad * c->r_pad;
  const int32_t asplit = adj_split(c);
  const int32_t nwg = asplit > 1 ? adj_split_groups(c->n_pad, c->r_pad)
                                 : (c->n_pad / ADJ_BM) * (c->r_pad / ADJ_BN);
  const float inv_m = 1.0f / c->prm.m, k = c->prm.k;
  SI_HIP(c, launch_fill_f64(g_dt, S, 0.0, c->stream));
  SI_HIP(c, launch_fill_f64(g_zeta, S, 0.0, c->stream));
  float *lam[2][2] = {{c->adj_lam, c->adj_lam + NR}, {c->adj_lam + 2 * NR, c->adj_lam + 3 * NR}};
  int lc = 0;
  // the multipliers are rewritten by the sweep: one backward per forward
  c->tape.valid = false;
  StepArgs a = step_args(c);
  for (int32_t sg = nseg - 1; sg >= 0; --sg) {
    const int32_t t_a = t0 + sg * C;
    const int32_t len = (S - t_a) < C ? (S - t_a) : C;
    const float *ck = c->adj_ckpt + (int64_t)sg * 2 * NR;
    float *sq = c->adj_seg;  // state j of the segment: q at sq + 2 j NR, p at + NR
    SI_HIP(c, hipMemcpyAsync(sq, ck, 2 * NR * sizeof(float), hipMemcpyDeviceToDevice,
                             c->stream));
    for (int32_t j = 0; j < len; ++j) {  // recompute, recording the wall masks
      a.q_in = sq + 2 * j * NR;
      a.p_in = sq + 2 * j * NR + NR;
      a.q_out = sq + 2 * (j + 1) * NR;
      a.p_out = sq + 2 * (j + 1) * NR + NR;
      a.mask_out = c->adj_mask + (int64_t)j * NR;
      a.t = t_a + j;
      SI_HIP(c, launch_step_f32(c->tile, a, c->stream));
    }
    for (int32_t j = len - 1; j >= 0; --j) {
      const int32_t n = t_a + j;
      double *part = c->adj_part + (int64_t)(n - t0) * nwg * 3;
      if (asplit > 1)
        SI_HIP(c, launch_adj_step_split(c->J, lam[lc][0], lam[lc][1], c->adj_mask + (int64_t)j * NR,
                                        sq + 2 * j * NR, sq + 2 * j * NR + NR, lam[lc ^ 1][0],
                                        lam[lc ^ 1][1], part, c->dt, c->zeta, n, k, inv_m,
                                        c->n_pad, c->n, c->r_pad, asplit, c->fsplit, c->stream));
      else
        SI_HIP(c, launch_adj_step(c->J, lam[lc][0], lam[lc][1], c->adj_mask + (int64_t)j * NR,
                                  sq + 2 * j * NR, sq + 2 * j * NR + NR, lam[lc ^ 1][0],
                                  lam[lc ^ 1][1], part, c->dt, c->zeta, n, k, inv_m,
                                  c->n_pad, c->r_pad, c->stream));
      lc ^= 1;
    }
  }
  // every step's gradient entries from its partial triples, in one launch
  if (S > t0)
    SI_HIP(c, launch_adj_reduce(c->adj_part, nwg, 1, nullptr, g_dt, g_zeta, c->dt, c->zeta, t0,
                                S - t0, k, inv_m, c->r, c->stream));
  return SI_OK;
}

si_status spring_ising_relaxed_energy_forward(si_ctx *c, int32_t ckpt_every, double *loss) {
  SI_USABLE(c);
  if (ckpt_every < 1) return fail(SI_ERR_INVALID, "relaxed_energy_forward: ckpt_every < 1");
  if (!is_device_ptr(loss))
    return fail(SI_ERR_INVALID, "relaxed_energy_forward: loss must be a device pointer");
  return adj_forward(c, ckpt_every, loss);
}

si_status spring_ising_relaxed_energy_backward(si_ctx *c, double *g_dt, double *g_zeta) {
  SI_USABLE(c);
  if (!is_device_ptr(g_dt) || !is_device_ptr(g_zeta))
    return fail(SI_ERR_INVALID, "relaxed_energy_backward: outputs must be device pointers");
  return adj_backward(c, g_dt, g_zeta);
}

si_status spring_ising_relaxed_energy_grad(si_ctx *c, int32_t ckpt_every, double *loss,
                                           double *g_dt, double *g_zeta) {
  SI_USABLE(c);
  if (ckpt_every < 1) return fail(SI_ERR_INVALID, "relaxed_energy_grad: ckpt_every < 1");
  if (!is_device_ptr(loss) || !is_device_ptr(g_dt) || !is_device_ptr(g_zeta))
    return fail(SI_ERR_INVALID, "relaxed_energy_grad: outputs must be device pointers");
  si_status st = adj_forward(c, ckpt_every, loss);
  if (st != SI_OK) return st;
  return adj_backward(c, g_dt, g_zeta);
}

si_status spring_ising_step(si_ctx *c) {
  SI_USABLE(c);
  if (c->t >= c->prm.total_steps)
    return fail(SI_ERR_RANGE, "step: t=%d reached total_steps=%d", c->t, c->prm.total_steps);
  c->epoch++;
  return do_steps(c, 1);
}

// Replay of a captured launch sequence: the graph holds exactly the launches
// do_steps would issue for (t0, n, cur), so the result is bit-identical.
static si_status run_graph(si_ctx *c, int32_t n_steps) {
  si_ctx::GraphEntry *hit = nullptr;
  for (auto &g : c->graphs)
    if (g.t0 == c->t && g.n == n_steps && g.cur == c->cur) hit = &g;
  if (!hit) {
    if (!c->cap_stream) SI_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (c->graphs.size() >= 4) {
      (void)hipGraphExecDestroy(c->graphs.front().exec);
      (void)hipGraphDestroy(c->graphs.front().graph);
      c->graphs.erase(c->graphs.begin());
    }
    si_ctx::GraphEntry e{c->t, n_steps, c->cur, nullptr, nullptr};
    const int32_t t_save = c->t, cur_save = c->cur;
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    SI_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    si_status st = do_steps(c, n_steps);
    hipError_t ce = hipStreamEndCapture(c->cap_stream, &e.graph);
    c->stream = user;
    c->t = t_save;
    c->cur = cur_save;
    if (st != SI_OK) return st;
    SI_HIP(c, ce);
    SI_HIP(c, hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
    c->graphs.push_back(e);
    hit = &c->graphs.back();
  }
  SI_HIP(c, hipGraphLaunch(hit->exec, c->stream));
  // the replayed sequence holds the in-run checks of the steps it covers
  if (c->e_every > 0 && (c->t + n_steps) / c->e_every > c->t / c->e_every) c->best_any = true;
  c->t += n_steps;
  c->cur ^= (n_steps & 1);
  return SI_OK;
}

// Workgroups of the resident launch for the current tile, or 0 when the
// context has no resident form or they do not all fit on the device.
static int32_t resident_groups(si_ctx *c) {
  if (c->n_inst || c->qplanes || split_for(c, c->tile) > 1) return 0;
  if (c->resident_tile != c->tile) {
    int per = 0;
    if (resident_f32_groups_per_cu(c->tile, c->prm.order, c->prm.wall, &per) != hipSuccess)
      per = 0;
    (void)hipGetLastError();
    c->resident_tile = c->tile;
    c->resident_per_cu = per;
  }
  const TileShape ts = tile_shape(c->tile);
  const int64_t groups = (int64_t)(c->n_pad / ts.bm) * (c->r_pad / ts.bn);
  if (c->resident_per_cu <= 0 || groups > (int64_t)c->resident_per_cu * c->num_cus) return 0;
  return (int32_t)groups;
}

static si_status run_resident(si_ctx *c, int32_t n_steps, int32_t groups) {
  // res_sync: [0] time-out flag, [64 ..] one completed-step count per group
  if (c->res_sync_cap < groups) {
    SI_HIP(c, c->alloc(&c->res_sync, 64 + (int64_t)groups));
    c->res_sync_cap = groups;
  }
  SI_HIP(c, launch_zero_i32(c->res_sync, 64 + (int64_t)groups, c->stream));
  StepArgs a = step_args(c);
  a.t = c->t;
  ResidentArgs r;
  r.q[0] = c->q[0];
  r.q[1] = c->q[1];
  r.p[0] = c->p[0];
  r.p[1] = c->p[1];
  r.cur = c->cur;
  r.n_steps = n_steps;
  r.count = reinterpret_cast<uint32_t *>(c->res_sync + 64);
  r.err = c->res_sync;
  SI_HIP(c, launch_resident_f32(c->tile, a, r, c->stream));
  c->t += n_steps;
  c->cur ^= (n_steps & 1);
  int32_t err = 0;
  SI_HIP(c, hipMemcpyAsync(&err, c->res_sync, sizeof err, hipMemcpyDeviceToHost, c->stream));
  SI_HIP(c, hipStreamSynchronize(c->stream));
  if (err) {
    c->poisoned = true;
    return fail(SI_ERR_HIP, "run: a grid barrier of the resident launch timed out");
  }
  return SI_OK;
}

si_status spring_ising_run(si_ctx *c, int32_t n_steps) {
  SI_USABLE(c);
  if (n_steps < 0) return fail(SI_ERR_INVALID, "run: n_steps=%d < 0", n_steps);
  if ((int64_t)c->t + n_steps > c->prm.total_steps)
    return fail(SI_ERR_RANGE, "run: t=%d + n_steps=%d exceeds total_steps=%d", c->t, n_steps,
                c->prm.total_steps);
  c->epoch++;
  if (c->resident_min_steps > 0 && n_steps >= c->resident_min_steps && n_steps > 1 &&
      c->e_every == 0) {
    const int32_t groups = resident_groups(c);
    if (groups > 0) return run_resident(c, n_steps, groups);
  }
  if (c->graph_min_steps > 0 && n_steps >= c->graph_min_steps) return run_graph(c, n_steps);
  return do_steps(c, n_steps);
}

si_status spring_ising_set_ksplit(si_ctx *c, int32_t ksplit) {
  SI_USABLE(c);
  if (ksplit < 0 || ksplit > 16) return fail(SI_ERR_INVALID, "set_ksplit: ksplit=%d not in 0..16", ksplit);
  if (ksplit >= 2 && (c->n_inst || c->qplanes || !tile_has_split(c->tile)))
    return fail(SI_ERR_UNSUPPORTED, "set_ksplit: the split contraction needs a single FP32 "
                "instance on a tile with a split form (tile %d)", c->tile);
  c->epoch++;
  c->ksplit_mode = ksplit;
  SI_HIP(c, ensure_split_ws(c));
  c->drop_graphs();
  return SI_OK;
}

si_status spring_ising_set_resident(si_ctx *c, int32_t min_steps) {
  SI_USABLE(c);
  if (min_steps < 0) return fail(SI_ERR_INVALID, "set_resident: min_steps < 0");
  c->resident_min_steps = min_steps;
  return SI_OK;
}

si_status spring_ising_set_graph(si_ctx *c, int32_t min_steps) {
  SI_USABLE(c);
  if (min_steps < 0) return fail(SI_ERR_INVALID, "set_graph: min_steps < 0");
  c->graph_min_steps = min_steps;
  if (min_steps == 0) c->drop_graphs();
  return SI_OK;
}

// Whether the step kernel of `tile` accepts this context's padded shape:
// the checks its launcher makes (tile divides the padded rows and replicas,
// slab depth divides the contraction, the ring fits the LDS), decided on the
// host so that no candidate is rejected by a launch.
static bool tile_launchable(const si_ctx *c, int32_t tile) {
  if (c->qplanes && !tile_valid_bf16(tile, c->prm.precision)) return false;
  const TileShape ts = shape_of(c->prm.precision, tile);
  if (ts.bm <= 0 || ts.bn <= 0 || ts.bk <= 0) return false;
  return c->n_pad % ts.bm == 0 && c->r_pad % ts.bn == 0 && c->n_pad % ts.bk == 0;
}

// Time every step kernel that can serve this context from its current state
// and keep the fastest.  The state and step index are restored after each
// candidate (one host synchronisation per candidate).  Candidates are
// filtered on the host before anything is launched; once a candidate has
// been launched, any HIP failure poisons the context like everywhere else.
// Autotune of a batch: both batch tiles, timed from the current state of
// every instance, which is restored after each.
static si_status autotune_batch(si_ctx *c, int32_t steps, int32_t *best_tile, float *best_us) {
  const int64_t S = c->b_stot;
  if (!c->tune_save) SI_HIP(c, c->alloc(&c->tune_save, 2 * S));
  if (c->b_lowp && !c->tune_qb) SI_HIP(c, c->alloc(&c->tune_qb, S));
  const int32_t t0 = c->t, cur0 = c->cur, tile0 = c->tile;
  float *q0 = c->b_q[cur0][0], *p0 = c->b_p[cur0][0];
  uint16_t *qb0 = c->b_lowp ? c->b_qb[cur0][0] : nullptr;
  SI_HIP(c, hipMemcpyAsync(c->tune_save, q0, S * 4, hipMemcpyDeviceToDevice, c->stream));
  SI_HIP(c, hipMemcpyAsync(c->tune_save + S, p0, S * 4, hipMemcpyDeviceToDevice, c->stream));
  if (qb0) SI_HIP(c, hipMemcpyAsync(c->tune_qb, qb0, S * 2, hipMemcpyDeviceToDevice, c->stream));
  if (!c->tune_ev[0]) {
    SI_HIP(c, hipEventCreate(&c->tune_ev[0]));
    SI_HIP(c, hipEventCreate(&c->tune_ev[1]));
  }
  hipEvent_t e0 = c->tune_ev[0], e1 = c->tune_ev[1];
  struct KeepEvery {
    si_ctx *c;
    int32_t v;
    ~KeepEvery() { c->e_every = v; }
  } keep{c, c->e_every};
  c->e_every = 0;
  const int32_t timed = steps - 1 > 0 ? steps - 1 : 1;
  int32_t best = tile0;
  float best_t = 1e30f;
  for (int round = 0; round < 2; ++round)  // as for single instances
  for (int32_t tile = 1; tile <= BATCH_TILE_LAST; ++tile) {
    c->tile = tile;
    SI_HIP(c, batch_items(c));
    si_status st = do_steps(c, 1);  // warm-up
    if (st != SI_OK) return st;
    SI_HIP(c, hipEventRecord(e0, c->stream));
    st = do_steps(c, timed);
    if (st != SI_OK) return st;
    SI_HIP(c, hipEventRecord(e1, c->stream));
    SI_HIP(c, hipMemcpyAsync(q0, c->tune_save, S * 4, hipMemcpyDeviceToDevice, c->stream));
    SI_HIP(c, hipMemcpyAsync(p0, c->tune_save + S, S * 4, hipMemcpyDeviceToDevice, c->stream));
    if (qb0) SI_HIP(c, hipMemcpyAsync(qb0, c->tune_qb, S * 2, hipMemcpyDeviceToDevice, c->stream));
    c->t = t0;
    c->cur = cur0;
    SI_HIP(c, hipEventSynchronize(e1));
    float ms = 0.f;
    SI_HIP(c, hipEventElapsedTime(&ms, e0, e1));
    const float us = 1000.f * ms / (float)timed;
    if (us < best_t) {
      best_t = us;
      best = tile;
    }
  }
  c->tile = best;
  SI_HIP(c, batch_items(c));
  c->tile_source = SI_TILE_FROM_AUTOTUNE;
  c->drop_graphs();
  tile_cache_put(tile_key(c), best, best_t);
  if (best_tile) *best_tile = best;
  if (best_us) *best_us = best_t;
  return SI_OK;
}

si_status spring_ising_autotune(si_ctx *c, int32_t steps, int32_t *best_tile, float *best_us) {
  SI_USABLE(c);
  if (steps < 1) return fail(SI_ERR_INVALID, "autotune: steps < 1");
  if ((int64_t)c->t + steps > c->prm.total_steps)
    return fail(SI_ERR_RANGE, "autotune: %d steps from t=%d exceed total_steps", steps, c->t);
  c->epoch++;
  if (c->n_inst) return autotune_batch(c, steps, best_tile, best_us);
  const int64_t NR = (int64_t)c->n_pad * c->r_pad;
  // saved state: q and p in the adjoint's segment buffer, the BF16 planes of
  // q in a buffer of their own; both kept for later calls
  if (!c->adj_seg || c->adj_seg_cap < 2 * NR) {
    SI_HIP(c, c->alloc(&c->adj_seg, 2 * NR));
    SI_HIP(c, c->alloc(&c->adj_mask, NR));
    c->adj_seg_cap = 2 * NR;
  }
  float *save = c->adj_seg;
  if (c->qplanes && !c->tune_qb) SI_HIP(c, c->alloc(&c->tune_qb, NR * c->qplanes));
  uint16_t *save_b = c->qplanes ? c->tune_qb : nullptr;
  const int32_t t0 = c->t, cur0 = c->cur, tile0 = c->tile;
  SI_HIP(c, hipMemcpyAsync(save, c->q[cur0], NR * 4, hipMemcpyDeviceToDevice, c->stream));
  SI_HIP(c, hipMemcpyAsync(save + NR, c->p[cur0], NR * 4, hipMemcpyDeviceToDevice, c->stream));
  if (save_b)
    SI_HIP(c, hipMemcpyAsync(save_b, c->qb[cur0], NR * 2 * c->qplanes, hipMemcpyDeviceToDevice,
                             c->stream));
  if (!c->tune_ev[0]) {
    SI_HIP(c, hipEventCreate(&c->tune_ev[0]));
    SI_HIP(c, hipEventCreate(&c->tune_ev[1]));
  }
  hipEvent_t e0 = c->tune_ev[0], e1 = c->tune_ev[1];
  const bool lowp = c->qplanes != 0;
  // candidates' steps record no energy checks (their states are discarded)
  struct KeepEvery {
    si_ctx *c;
    int32_t v;
    ~KeepEvery() { c->e_every = v; }
  } keep{c, c->e_every};
  c->e_every = 0;
  const int32_t last = lowp ? TILE_BF16_LAST : TILE_F32_LAST;
  const int32_t timed = steps - 1 > 0 ? steps - 1 : 1;
  int32_t best = tile0;
  float best_t = 1e30f;
  // two rounds over the candidates, each keeping its faster round: the first
  // candidates of a single round ran measurably slow (cold clocks and caches)
  for (int round = 0; round < 2; ++round)
  for (int32_t tile = 1; tile <= last; ++tile) {
    if (!tile_launchable(c, tile)) continue;
    c->tile = tile;
    // the split contraction's workspace (a candidate whose workspace cannot
    // be allocated is skipped: nothing has been launched for it)
    if (ensure_split_ws(c) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    si_status st = do_steps(c, 1);  // warm-up (also loads the code object)
    if (st != SI_OK) return st;
    SI_HIP(c, hipEventRecord(e0, c->stream));
    st = do_steps(c, timed);
    if (st != SI_OK) return st;
    SI_HIP(c, hipEventRecord(e1, c->stream));
    // restore the state for the next candidate
    SI_HIP(c, hipMemcpyAsync(c->q[cur0], save, NR * 4, hipMemcpyDeviceToDevice, c->stream));
    SI_HIP(c, hipMemcpyAsync(c->p[cur0], save + NR, NR * 4, hipMemcpyDeviceToDevice, c->stream));
    if (save_b)
      SI_HIP(c, hipMemcpyAsync(c->qb[cur0], save_b, NR * 2 * c->qplanes, hipMemcpyDeviceToDevice,
                               c->stream));
    c->t = t0;
    c->cur = cur0;
    SI_HIP(c, hipEventSynchronize(e1));
    float ms = 0.f;
    SI_HIP(c, hipEventElapsedTime(&ms, e0, e1));
    const float us = 1000.f * ms / (float)timed;
    if (us < best_t) {
      best_t = us;
      best = tile;
    }
  }
  c->tile = best;
  SI_HIP(c, ensure_split_ws(c));
  c->drop_graphs();
  c->tile_source = SI_TILE_FROM_AUTOTUNE;
  tile_cache_put(tile_key(c), best, best_t);
  if (best_tile) *best_tile = best;
  if (best_us) *best_us = best_t;
  return SI_OK;
}


// ---- batched-context variants (instances concatenated in caller layouts) ----
static si_status batch_spins(si_ctx *c, int8_t *s) {
  SI_HIP(c, launch_sign(c->b_q[c->cur][0], c->S8, (int32_t)(c->b_stot / c->r_pad), c->r_pad,
                        c->stream));
  for (int32_t i = 0; i < c->n_inst; ++i)
    SI_HIP(c, launch_unpack_spins(c->S8 + c->b_soff[i], c->b_n[i], c->r, s + c->b_xoff[i],
                                  c->b_npad[i], c->stream));
  return SI_OK;
}

// Every instance in at most two grouped launches (plus their finalisations):
// the int8 matrix-core energy for the integer instances, the FP32 coupling
// sum for the others.
static si_status batch_energy(si_ctx *c, int32_t *e_int, double *e_real) {
  for (int32_t i = 0; i < c->n_inst; ++i)
    if (e_int && !c->eb_desc_host[i].J8)
      return fail(SI_ERR_UNSUPPORTED, "energy: instance %d has non-integer couplings", i);
  const float *q = c->b_q[c->cur][0];  // state of instance 0 starts the buffer
  if (c->eb_n_i8) {
    SI_HIP(c, launch_sign(q, c->S8, (int32_t)(c->b_stot / c->r_pad), c->r_pad, c->stream));
    SI_HIP(c, launch_energy_i8_batch(c->eb_desc, c->eb_items, c->eb_n_i8, c->S8, c->eacc,
                                     c->n_inst, c->r, c->r_pad, e_int, e_real, c->stream));
  }
  if (c->eb_n_f32 && e_real)
    SI_HIP(c, launch_energy_f32_batch(c->eb_desc, c->eb_items + c->eb_n_i8, c->eb_n_f32, q,
                                      c->epart, c->n_inst, c->r, c->r_pad, e_real, c->stream));
  return SI_OK;
}

static si_status batch_get_state(si_ctx *c, float *x, float *p) {
  for (int32_t i = 0; i < c->n_inst; ++i) {
    if (x)
      SI_HIP(c, launch_unpack_state(c->b_q[c->cur][i], c->b_n[i], c->r, x + c->b_xoff[i],
                                    c->b_npad[i], c->stream));
    if (p)
      SI_HIP(c, launch_unpack_state(c->b_p[c->cur][i], c->b_n[i], c->r, p + c->b_xoff[i],
                                    c->b_npad[i], c->stream));
  }
  return SI_OK;
}

static si_status batch_set_state(si_ctx *c, const float *x, const float *p) {
  for (int32_t i = 0; i < c->n_inst; ++i) {
    SI_HIP(c, launch_pack_state(x + c->b_xoff[i], c->b_n[i], c->r, c->b_q[c->cur][i], c->b_npad[i],
                                c->r_pad, c->stream));
    SI_HIP(c, launch_pack_state(p ? p + c->b_xoff[i] : nullptr, c->b_n[i], c->r,
                                c->b_p[c->cur][i], c->b_npad[i], c->r_pad, c->stream));
    if (c->b_lowp)
      SI_HIP(c, launch_split_planes(c->b_q[c->cur][i], c->b_qb[c->cur][i],
                                    (int64_t)c->r_pad * c->b_npad[i], 1, c->stream));
  }
  return SI_OK;
}

si_status spring_ising_spins(si_ctx *c, int8_t *s) {
  SI_USABLE(c);
  if (!is_device_ptr(s)) return fail(SI_ERR_INVALID, "spins: s must be a device pointer");
  if (c->n_inst) return batch_spins(c, s);
  SI_HIP(c, launch_sign(c->q[c->cur], c->S8, c->n_pad, c->r_pad, c->stream));
  SI_HIP(c, launch_unpack_spins(c->S8, c->n, c->r, s, c->n_pad, c->stream));
  return SI_OK;
}

// Energies of the current spins into device outputs (no argument checks).
static si_status energy_into(si_ctx *c, int32_t *e_int, double *e_real) {
  if (!e_int && !e_real) return SI_OK;
  if (c->n_inst) return batch_energy(c, e_int, e_real);
  // exact int32 path: integer J (and field) with a sum that cannot overflow
  const int64_t jmax = c->hflags[6];
  const int64_t bound = (int64_t)c->n * c->n * jmax +
                        (c->has_field ? 2 * (int64_t)c->n * c->field_maxabs : 0);
  const bool exact = c->J8 && (!c->has_field || c->field_integer) && bound < (1LL << 31);
  if (e_int && !exact)
    return fail(SI_ERR_UNSUPPORTED,
                "energy: exact int32 energy needs integer |J_ij| <= 127 (and integer field)");
  const int8_t *h8 = c->has_field ? c->h8 : nullptr;
  if (exact) {
    SI_HIP(c, launch_sign(c->q[c->cur], c->S8, c->n_pad, c->r_pad, c->stream));
    SI_HIP(c, launch_energy_i8(c->J8, c->S8, h8, c->eacc, c->n_pad, c->r_pad,
                               energy_i8_ksplit(c->n_pad, c->r_pad, c->num_cus), c->stream));
    SI_HIP(c, launch_energy_i8_finalize(c->eacc, c->r, e_int, e_real, c->stream));
  } else {
    const float *hf = c->has_field ? c->hf : nullptr;
    SI_HIP(c, launch_energy_f32_partial(c->J, c->q[c->cur], hf, c->epart, c->n_pad, c->r_pad,
                                        c->stream));
    SI_HIP(c, launch_energy_f32_finalize(c->epart, c->n_pad / 64, c->r, c->r_pad, e_real,
                                         c->stream));
  }
  return SI_OK;
}

si_status spring_ising_energy(si_ctx *c, int32_t *e_int, double *e_real) {
  SI_USABLE(c);
  if ((e_int && !is_device_ptr(e_int)) || (e_real && !is_device_ptr(e_real)))
    return fail(SI_ERR_INVALID, "energy: outputs must be device pointers");
  return energy_into(c, e_int, e_real);
}

// Best-state update from the energies e of the current spins (out_rows()
// doubles on the device).
static si_status best_update_from(si_ctx *c, const double *e) {
  SI_HIP(c, ensure_best_buffers(c));
  if (c->n_inst) {
    SI_HIP(c, launch_sign(c->b_q[c->cur][0], c->S8, (int32_t)(c->b_stot / c->r_pad), c->r_pad,
                          c->stream));
    SI_HIP(c, launch_best_update_batch(e, c->best_e, c->best_valid, c->S8, c->best_s, c->eb_desc,
                                       c->n_inst, c->r, c->stream));
  } else {
    SI_HIP(c, launch_sign(c->q[c->cur], c->S8, c->n_pad, c->r_pad, c->stream));
    SI_HIP(c, launch_best_update(e, c->best_e, c->best_valid, c->S8, c->best_s, c->r, c->n_pad,
                                 c->stream));
  }
  c->best_any = true;
  return SI_OK;
}

static si_status record_check(si_ctx *c) {
  const int32_t row = c->t / c->e_every - 1;
  if (row < 0 || row >= c->e_rows) return SI_OK;
  double *e = c->etrace + (int64_t)row * c->out_rows();
  si_status st = energy_into(c, nullptr, e);
  if (st != SI_OK) return st;
  return best_update_from(c, e);
}

si_status spring_ising_update_best(si_ctx *c) {
  SI_USABLE(c);
  SI_HIP(c, ensure_best_buffers(c));
  si_status st = energy_into(c, nullptr, c->e_scratch);
  if (st != SI_OK) return st;
  return best_update_from(c, c->e_scratch);
}

si_status spring_ising_get_best(si_ctx *c, double *best_e, int8_t *best_s) {
  SI_USABLE(c);
  if (!c->best_e || !c->best_any)
    return fail(SI_ERR_STATE, "get_best: no best-state update since init or set_state");
  if ((best_e && !is_device_ptr(best_e)) || (best_s && !is_device_ptr(best_s)))
    return fail(SI_ERR_INVALID, "get_best: outputs must be device pointers");
  if (best_e)
    SI_HIP(c, hipMemcpyAsync(best_e, c->best_e, sizeof(double) * c->out_rows(),
                             hipMemcpyDeviceToDevice, c->stream));
  if (best_s) {
    if (c->n_inst) {
      for (int32_t i = 0; i < c->n_inst; ++i)
        SI_HIP(c, launch_unpack_spins(c->best_s + c->b_soff[i], c->b_n[i], c->r,
                                      best_s + c->b_xoff[i], c->b_npad[i], c->stream));
    } else {
      SI_HIP(c, launch_unpack_spins(c->best_s, c->n, c->r, best_s, c->n_pad, c->stream));
    }
  }
  return SI_OK;
}

si_status spring_ising_get_energy_trace(si_ctx *c, double *e, int32_t *n_checks) {
  SI_USABLE(c);
  if (c->e_every <= 0)
    return fail(SI_ERR_STATE, "get_energy_trace: the context was created with energy_every = 0");
  if (e && !is_device_ptr(e))
    return fail(SI_ERR_INVALID, "get_energy_trace: e must be a device pointer");
  int32_t rows = c->t / c->e_every;
  if (rows > c->e_rows) rows = c->e_rows;
  if (n_checks) *n_checks = rows;
  if (e && rows > 0)
    SI_HIP(c, hipMemcpyAsync(e, c->etrace, sizeof(double) * rows * c->out_rows(),
                             hipMemcpyDeviceToDevice, c->stream));
  return SI_OK;
}

si_status spring_ising_hamiltonian(si_ctx *c, double *H) {
  SI_USABLE(c);
  if (c->n_inst) return fail(SI_ERR_UNSUPPORTED, "hamiltonian: not available for a batch");
  if (!is_device_ptr(H)) return fail(SI_ERR_INVALID, "hamiltonian: H must be a device pointer");
  const int32_t t = c->t < c->prm.total_steps ? c->t : c->prm.total_steps - 1;
  SI_HIP(c, launch_hamiltonian_partial(c->J, c->q[c->cur], c->p[c->cur],
                                       c->has_field ? c->hf : nullptr, c->zeta, t, c->prm.k,
                                       1.0f / c->prm.m, c->epart, c->n_pad, c->r_pad, c->stream));
  SI_HIP(c, launch_energy_f32_finalize(c->epart, c->n_pad / 64, c->r, c->r_pad, H, c->stream,
                                       1.0f));
  return SI_OK;
}

si_status spring_ising_get_state(si_ctx *c, float *x, float *p, int32_t *t) {
  SI_USABLE(c);
  if ((x && !is_device_ptr(x)) || (p && !is_device_ptr(p)))
    return fail(SI_ERR_INVALID, "get_state: x and p must be device pointers");
  if (c->n_inst) {
    if (t) *t = c->t;
    return batch_get_state(c, x, p);
  }
  if (x) SI_HIP(c, launch_unpack_state(c->q[c->cur], c->n, c->r, x, c->n_pad, c->stream));
  if (p) SI_HIP(c, launch_unpack_state(c->p[c->cur], c->n, c->r, p, c->n_pad, c->stream));
  if (t) *t = c->t;
  return SI_OK;
}

si_status spring_ising_set_state(si_ctx *c, const float *x, const float *p, int32_t t) {
  SI_USABLE(c);
  if (!x) return fail(SI_ERR_INVALID, "set_state: x is required");
  if (!is_device_ptr(x) || (p && !is_device_ptr(p)))
    return fail(SI_ERR_INVALID, "set_state: x and p must be device pointers");
  if (t < 0 || t > c->prm.total_steps)
    return fail(SI_ERR_RANGE, "set_state: t=%d outside [0, %d]", t, c->prm.total_steps);
  c->epoch++;
  if (c->best_valid)
    SI_HIP(c, launch_zero_i32(c->best_valid, c->n_inst ? c->out_rows() : c->r_pad, c->stream));
  c->best_any = false;
  if (c->n_inst) {
    si_status st = batch_set_state(c, x, p);
    if (st == SI_OK) c->t = t;
    return st;
  }
  SI_HIP(c, launch_pack_state(x, c->n, c->r, c->q[c->cur], c->n_pad, c->r_pad, c->stream));
  SI_HIP(c, launch_pack_state(p, c->n, c->r, c->p[c->cur], c->n_pad, c->r_pad, c->stream));
  if (c->qplanes)
    SI_HIP(c, launch_split_planes(c->q[c->cur], c->qb[c->cur], (int64_t)c->n_pad * c->r_pad,
                                  c->qplanes, c->stream));
  c->t = t;
  return SI_OK;
}

si_status spring_ising_batch_timeline(si_ctx *c, int32_t n_steps, uint64_t *out, int64_t cap,
                                      int64_t *n_records, double *clock_mhz) {
  SI_USABLE(c);
  if (n_records) *n_records = 0;
  if (!c->n_inst) return fail(SI_ERR_UNSUPPORTED, "batch_timeline: not a batch");
  if (n_steps < 1 || n_steps > 16) return fail(SI_ERR_INVALID, "batch_timeline: n_steps=%d not in 1..16", n_steps);
  if ((int64_t)c->t + n_steps > c->prm.total_steps)
    return fail(SI_ERR_RANGE, "batch_timeline: t=%d + n_steps=%d exceeds total_steps=%d", c->t,
                n_steps, c->prm.total_steps);
  const int64_t need = (int64_t)n_steps * (int64_t)c->b_items_host.size();
  if (n_records) *n_records = need;
  if (!out || cap < need)
    return fail(SI_ERR_INVALID, "batch_timeline: out must hold %lld records", (long long)need);
  int khz = 0;
  SI_HIP(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
  if (clock_mhz) *clock_mhz = khz / 1000.0;
  if (need > c->b_trace_cap) {
    SI_HIP(c, c->alloc(&c->b_trace, 4 * need));
    c->b_trace_cap = need;
  }
  c->epoch++;
  si_status st = do_steps_batch(c, n_steps, c->b_trace);
  if (st != SI_OK) return st;
  SI_HIP(c, hipMemcpyAsync(out, c->b_trace, 4 * need * sizeof(uint64_t), hipMemcpyDeviceToHost,
                           c->stream));
  SI_HIP(c, hipStreamSynchronize(c->stream));
  // item index -> (step << 32) | item
  for (int64_t k = 0; k < need; ++k)
    out[4 * k + 3] |= (uint64_t)(k / (int64_t)c->b_items_host.size()) << 32;
  return SI_OK;
}

si_status spring_ising_tile_cache_save(const char *path) {
  if (!path) return fail(SI_ERR_INVALID, "tile_cache_save: path is null");
  std::map<TileKey, TileEntry> snap;
  {
    std::lock_guard<std::mutex> lock(g_tile_mu);
    snap = g_tile_cache;
  }
  FILE *f = fopen(path, "w");
  if (!f) return fail(SI_ERR_INVALID, "tile_cache_save: cannot write %s", path);
  fprintf(f, "%s\nbuild %s\n", k_cache_magic, spring_ising_build_id());
  for (const auto &kv : snap) {
    const TileKey &k = kv.first;
    fprintf(f, "%d %d %d %d %d %d %d %.9g\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
            std::get<3>(k), std::get<4>(k), std::get<5>(k), kv.second.tile, (double)kv.second.us);
  }
  const bool ok = !ferror(f);
  if (fclose(f) != 0 || !ok) return fail(SI_ERR_INVALID, "tile_cache_save: write to %s failed", path);
  return SI_OK;
}

si_status spring_ising_tile_cache_load(const char *path, int32_t *n_loaded) {
  if (n_loaded) *n_loaded = 0;
  if (!path) return fail(SI_ERR_INVALID, "tile_cache_load: path is null");
  FILE *f = fopen(path, "r");
  if (!f) return fail(SI_ERR_INVALID, "tile_cache_load: cannot read %s", path);
  char line[256];
  std::map<TileKey, TileEntry> got;
  si_status st = SI_OK;
  int lineno = 0;
  while (fgets(line, sizeof line, f)) {
    ++lineno;
    const size_t len = strlen(line);
    if (len == sizeof line - 1 && line[len - 1] != '\n' && !feof(f)) {
      st = fail(SI_ERR_INVALID, "tile_cache_load: %s line %d: longer than %d characters", path,
                lineno, (int)sizeof line - 2);
      break;
    }
    if (len && line[len - 1] == '\n') line[len - 1] = 0;
    if (lineno == 1) {
      if (strcmp(line, k_cache_magic) != 0) {
        st = fail(SI_ERR_INVALID, "tile_cache_load: %s is not a tile cache", path);
        break;
      }
      continue;
    }
    if (lineno == 2) {
      char id[64];
      if (sscanf(line, "build %63s", id) != 1) {
        st = fail(SI_ERR_INVALID, "tile_cache_load: %s line 2: no build id", path);
        break;
      }
      if (strcmp(id, spring_ising_build_id()) != 0) {
        st = fail(SI_ERR_STATE, "tile_cache_load: %s was written by build %s, this is %s", path,
                  id, spring_ising_build_id());
        break;
      }
      continue;
    }
    if (!line[0]) continue;
    // eight whitespace-separated fields: seven decimal integers in int32
    // range, then a finite non-negative time
    int v[7];
    double us = -1.0;
    int fields = 0;
    bool ok = true;
    char *cur = line;
    while (ok) {
      while (*cur == ' ' || *cur == '\t' || *cur == '\r') ++cur;
      if (!*cur) break;
      char *end = nullptr;
      if (fields < 7) {
        errno = 0;
        const long long x = strtoll(cur, &end, 10);
        ok = end != cur && errno == 0 && x >= INT32_MIN && x <= INT32_MAX;
        if (ok) v[fields] = (int)x;
      } else if (fields == 7) {
        us = strtod(cur, &end);
        ok = end != cur && isfinite(us) && us >= 0.0;
      } else {
        ok = false;
      }
      if (ok && *end && *end != ' ' && *end != '\t' && *end != '\r') ok = false;
      cur = end;
      ++fields;
    }
    if (!ok || fields != 8 || (v[0] != 0 && v[0] != 1) || v[1] < SI_PREC_FP32 ||
        v[1] > SI_PREC_BF16X_MIXEDJ || v[2] < 0 || v[3] < 0 || v[4] < 64 || v[4] % 64 ||
        v[5] < 1 || !tile_serves(v[0], v[1], v[6])) {
      st = fail(SI_ERR_INVALID, "tile_cache_load: %s line %d: bad entry", path, lineno);
      break;
    }
    got[TileKey{v[0], v[1], v[2], v[3], v[4], v[5]}] = TileEntry{v[6], (float)us};
  }
  if (st == SI_OK && lineno < 2) st = fail(SI_ERR_INVALID, "tile_cache_load: %s is incomplete", path);
  fclose(f);
  if (st != SI_OK) return st;
  {
    std::lock_guard<std::mutex> lock(g_tile_mu);
    for (const auto &kv : got) g_tile_cache[kv.first] = kv.second;
  }
  if (n_loaded) *n_loaded = (int32_t)got.size();
  return SI_OK;
}

si_status spring_ising_tile_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tile_mu);
  g_tile_cache.clear();
  return SI_OK;
}

si_status spring_ising_info(si_ctx *c, si_info *info) {
  if (!c || !info) return fail(SI_ERR_INVALID, "info: null argument");
  memset(info, 0, sizeof *info);
  info->n = c->n;
  info->r = c->r;
  info->n_pad = c->n_pad;
  info->r_pad = c->r_pad;
  info->t = c->t;
  info->total_steps = c->prm.total_steps;
  info->j_integer = c->J8 != nullptr;
  if (c->n_inst) {
    info->j_integer = 1;
    for (int32_t i = 0; i < c->n_inst; ++i)
      if (!c->b_J8[i]) info->j_integer = 0;
  }
  info->j_fp8_exact = c->hflags[4] == 0;
  info->j_bf16_exact = c->hflags[5] == 0;
  info->tile = c->tile;
  info->tile_source = c->tile_source;
  info->n_inst = c->n_inst;
  info->precision = c->prm.precision;
  info->graph_steps = c->graph_min_steps;
  info->device_bytes = c->bytes;
  info->resident_groups = c->poisoned ? 0 : resident_groups(c);
  info->resident_steps = info->resident_groups ? c->resident_min_steps : 0;
  if (c->n_inst)
    snprintf(info->kernel_name, sizeof info->kernel_name, "step_batch_%s_%dx%d_x%d",
             c->b_lowp ? "bf16" : "f32", batch_tile_rows(c->tile), BATCH_BN, c->n_inst);
  else if (split_for(c, c->tile) > 1)
    snprintf(info->kernel_name, sizeof info->kernel_name, "%s_ks%d",
             shape_of(c->prm.precision, c->tile).name, split_for(c, c->tile));
  else
    snprintf(info->kernel_name, sizeof info->kernel_name, "%s",
             shape_of(c->prm.precision, c->tile).name);
  return SI_OK;
}

si_status spring_ising_destroy(si_ctx *c) {
  if (!c) return SI_OK;
  hipError_t e = hipStreamSynchronize(c->stream);
  delete c;
  if (e != hipSuccess) return fail(SI_ERR_HIP, "destroy: %s", hipGetErrorString(e));
  return SI_OK;
}

}  // extern "C"
