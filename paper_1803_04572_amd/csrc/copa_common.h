// Internal declarations shared by the HIP sources of libcopa.so (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/copa.h"

namespace copa {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kLMax = 8;           // spline basis functions per subject (padded row width of C)
constexpr int kNMax = 8;           // largest Procrustes eigenproblem handled one subject per lane
constexpr int kHistCap = 1024;     // per-iteration scalars buffered on the device
constexpr int kStatBlocks = 256;   // blocks of the stationarity residual
constexpr int kGramSlots = 6;      // F_H, W^TW, Psi, V^TV partials; adjoint G and its second Gram

// Layout of one Gram slot (R x R FP64 blocks): [maxnb block partials | total].
__host__ __device__ constexpr int64_t gram_total_offset(int maxnb) { return (int64_t)maxnb; }
constexpr int kChunkRows = 512;    // visit rows per chunk of the feature-sorted pass-2 layout
constexpr int kMaxR = 64;
constexpr int kNumKernels = 14;    // kernels of one outer iteration (see kernel_names)
constexpr int kTimingChunk = 64;   // iterations between event harvests when timing

void set_error(const std::string &msg);

#define COPA_HIP(call)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      ::copa::set_error(std::string(#call) + ": " + hipGetErrorString(e_));                    \
      return COPA_EDEVICE;                                                                     \
    }                                                                                          \
  } while (0)

// One entry of the per-pass wave work list: a wave takes `count` subjects of `order` starting at
// `first`, G = 1 << lg lanes per subject (lanes of one subject are consecutive).
struct WaveEntry {
  int32_t first;
  int32_t lg_count;  // lg | (count << 8)
};

// Scalars of one ADMM mode for one outer iteration, written by the single-block prep kernels.
struct ModeParams {
  double rho;
  double Gi[kMaxR * kMaxR];  // (G + rho I)^{-1}, row-major
};

// Device-side scalars of the fit (one struct, zeroed per copa_fit call).
struct FitScalars {
  int32_t cur;             // index of the outer iteration being run (within the current chunk);
                           // -1 before the chunk's first pass 1
  int32_t iter;            // iterations completed in this call
  int32_t fail_iter;       // first failing iteration or INT_MAX
  int32_t rank_deficient;  // subjects with truncated Procrustes rank (last iteration)
  int32_t rank_def_slot[2];  // same, accumulating for iterations of parity 0 / 1
  double hist_fit[kHistCap];
  double hist_obj[kHistCap];
  double last_fit, last_obj, last_sparsity;
};

struct Tiles {
  int nt;  // number of column tiles of R
  int rt;  // tile width
  int cg;  // pass 1: tiles one block stages together, one lane group of 64 / cg lanes per tile
};

}  // namespace copa

struct copa_plan {
  int device;
  int64_t K, J, S, nnz;
  int l;           // basis functions (0 = no smoothing)
  int R;
  int slot_rows;   // smoothed: l rows per subject; unsmoothed: rows follow the visit rows
  int64_t rows_total;  // rows of the T/Q/M row spaces
  copa_options opt;
  copa::Tiles tiles;   // pass 1 (and the V update's padded image of V)
  copa::Tiles tiles2;  // pass 2 over the feature-sorted chunks: F_V and u-row column tiles
  int lds_limit;

  // packed tensor
  int32_t *subj = nullptr;   // [K+1]
  int32_t *row = nullptr;    // [S+1]
  int32_t *col = nullptr;    // [nnz]
  float *val = nullptr;      // [nnz]
  int32_t *rowsubj = nullptr;  // [S] subject of each visit row (unsmoothed only)
  bool compact = false;      // nonzeros also stored as xc (pass 1 reads those)
  uint32_t *xc = nullptr;    // [nnz] feature (low 16 bits) | value as bfloat16 (high 16 bits)
  float *C = nullptr;        // [S x 8] smoothing basis rows (l > 0)
  int32_t *rk = nullptr;     // [K] basis ranks (l > 0)
  float *Ew = nullptr;       // [64 x K] Procrustes eigenvectors of the last outer iteration (l > 0)
  int32_t *order = nullptr;  // [K] subjects by decreasing visit count
  int32_t *order1 = nullptr; // [K] pass-1 subject order (by pair count for projected plans)
  copa::WaveEntry *waves = nullptr;
  int32_t n_waves = 0;
  copa::WaveEntry *waves1 = nullptr;  // pass-1 wave list for lane groups of 64 / tiles.cg lanes
  int32_t n_waves1 = 0;
  int32_t n_big = 0;         // unsmoothed subjects whose eigenproblem exceeds kNMax
  int32_t *big_list = nullptr;
  double normX2 = 0.0;

  // iteration buffers
  float *T = nullptr;   // [rows_total x R]  X'_k V rows (Procrustes input)
  float *Q = nullptr;   // [rows_total x R]  Q_k rows
  float *M = nullptr;   // [rows_total x R]  Q_k H S_k rows
  float *FW = nullptr;  // [K x R]
  float *Vp = nullptr;  // [nt x J x RTP] V in padded column tiles (pass-1 LDS image)
  float *FV = nullptr;  // [J x R]
  // projected pairs (smoothed plans with at most 2 nonzeros per visit row on average): one record
  // of pw floats per (subject, feature) pair: the feature's column of C_k^T X_k and a key
  bool proj = false;
  int pw = 0;
  int64_t npairs = 0;
  int32_t *pp = nullptr;      // [K+1] pair offsets per subject
  float *pairs1 = nullptr;    // [npairs x pw] by subject; key = feature id
  float *pairs2 = nullptr;    // [npairs x pw] by pass-2 chunk and feature; key = feature << 16 | s
  int32_t *pj = nullptr;      // [npairs] feature of each pair          (plan-creation input)
  int32_t *pn = nullptr;      // [npairs+1] offsets into nzr / nzx      (plan-creation input)
  int32_t *nzr = nullptr;     // [nnz] visit row of each nonzero, by (subject, feature, row)
  float *nzx = nullptr;       // [nnz] its value
  int32_t *perm2 = nullptr;   // [npairs] pairs1 index of each pairs2 record
  int32_t *key2 = nullptr;    // [npairs] pairs2 keys
  // mixed precision: the same records as 16-byte bfloat16 records (pass 2: the feature ids apart)
  uint4 *pairs1h = nullptr;   // [npairs] by subject; tag = feature id
  uint4 *pairs2h = nullptr;   // [npairs] pass-2 order; tag = subject within the chunk
  uint16_t *feat2h = nullptr; // [npairs] feature id of each pass-2 record
  bool use_bf = false;        // the launches being issued stream the bfloat16 records
  int pnchunks = 0;
  int pchunks_cap = 0;
  int32_t *pcq = nullptr;     // [pnchunks+1] pair offsets of the chunks
  int32_t *pcinfo = nullptr;  // [pnchunks x 2] first subject and subject count
  int32_t *pwsplit = nullptr; // [pnchunks x 9] wave slices on feature boundaries
  // pass-2 layout: per chunk of kChunkRows visit rows, nonzeros sorted by feature
  bool p2c = false;
  int nchunks = 0;
  int32_t *cptr = nullptr;   // [nchunks+1] nonzero offsets of the chunks
  int32_t *crow = nullptr;   // [nchunks+1] first visit row of each chunk
  int32_t *cinfo = nullptr;  // [nchunks x 2] first subject and subject count of each chunk
  int32_t *wsplit = nullptr; // [nchunks x 9] per-wave slices of each chunk (feature boundaries)
  uint2 *pkv = nullptr;      // [nnz] (feature << 16 | row within chunk, value bits)
  int n_cu = 0;
  // Gram slots (gstride doubles each): F_H, W^TW, Psi, V^TV partials of the V update, and two
  // more for the adjoint; a slot holds gcap block partials and then their total. Row-Gram
  // launches use at most gmaxnb blocks, the V update n_vblocks.
  double *gpart = nullptr;
  int gmaxnb = 0;
  int gcap = 0;  // partials a slot holds (largest block count of any launch writing them)
  int64_t gstride = 0;
  int32_t *gcount = nullptr;  // [8] last-block counters of the row Grams
  double *vpart = nullptr;  // [blocks x 4] V-ADMM scalar partials
  int n_vblocks = 0;
  double *wpart = nullptr;  // [max(n_wblocks, wf_cap)] |W|_1 partials of the W update
  int n_wblocks = 0;        // W-update blocks: 4 wavefronts of 64 / R subjects
  int wf_blocks = 0;        // order W -> H -> V: blocks of the persistent W-first launch,
  int mr_blocks = 0;        // of the M-row launch (resident blocks per CU x CUs),
  int wf_cap = 0;           // at most wf_cap <= gcap
  double *small = nullptr;  // FH, HtH, WtW, VtV, Psi : 5 x R x R
  copa::ModeParams *modes = nullptr;  // [3]
  copa::FitScalars *scal = nullptr;
  double *dloss = nullptr;  // loss/grad scalars
  // optional per-kernel event timing of copa_fit
  // hipGraph of one outer iteration (captured on cap_stream, replayed on the caller's stream);
  // captured again when the state buffers change
  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  copa_state gstate{};
  hipGraphExec_t gexec_bf = nullptr;  // the same for the mixed-precision iteration
  copa_state gstate_bf{};
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kid;
  int ev_used = 0;
  double t_ms[copa::kNumKernels] = {};
  int64_t t_cnt[copa::kNumKernels] = {};
  // launch shapes (set by the autotuner at the first copa_fit, else the defaults below)
  int p1_per_cu = 4;         // pass-1 persistent blocks per compute unit (LDS permitting)
  int proc_variant = 2;      // smoothed R > 16 Procrustes: 0 lane-per-subject blocks, 1 four-wavefront
                             // blocks, 2 three launches (Gram, eigenproblems without LDS, Q)
  double *pgb = nullptr;     // [36 x K] per-subject Gram, then B, of the three-launch Procrustes
  int p2_blocks = 0;         // pass-2 grid width (<= p2_blocks_cap)
  bool vtv_reduce = false;   // the V blocks' V^T V partials are added by k_gram_reduce (many, large)
  int gram_blocks = 0;       // row-Gram blocks (<= gmaxnb)
  int tuned = 0;             // 0 not yet, 1 timed on this plan, 2 read from the cache file
  float tune_ms = 0.0f;      // time the tuner took
  bool adjoint = false;      // the workspace holds the adjoint's buffers
  float *gradbuf = nullptr; // [2 x S x R + J x R] U and D rows and F of the adjoint
  float *statbuf = nullptr; // dH, dV, dW and the stationarity partials
  float *qtbuf = nullptr;   // [S x R] Qtilde for the stationarity stop
  size_t statfloats = 0;
  double *lpart = nullptr;  // per-block loss partials of the adjoint
  // every device buffer above lives in one workspace (the caller's, or one the plan allocated)
  char *arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  bool arena_owned = false;
  double *tmp = nullptr;     // plan-creation scratch (checks, partial sums)
  int nchunks_cap = 0;       // bound on the pass-2 chunks the workspace holds
  int p2_blocks_cap = 0;     // bound on the pass-2 grid width
  float *fvpart = nullptr;   // deterministic pass 2: each block's F_V tile [p2_blocks_cap x J x R]
  // Procrustes warm start: the state (buffers and iteration count) the last copa_fit returned
  copa_state last_state{};
  bool warm_valid = false;
  bool reset_warm = true;    // set by copa_fit: start the warm start from the identity
};
namespace copa {
enum { kSlotFH = 0, kSlotWtW = 1, kSlotPsi = 2, kSlotVtV = 3, kSlotG = 4, kSlotG2 = 5 };
inline double *gram_slot(const copa_plan *p, int slot) { return p->gpart + (int64_t)slot * p->gstride; }
// The reduced R x R total of a slot after a k_rows_gram launch.
inline double *gram_total(const copa_plan *p, int slot) {
  return gram_slot(p, slot) + gram_total_offset(p->gcap) * p->R * p->R;
}
}  // namespace copa


namespace copa {

// ---------------------------------------------------------------- launchers (copa_iter.hip)
copa_status launch_iteration(copa_plan *p, const copa_state *st, hipStream_t s);
copa_status launch_fit(copa_plan *p, const copa_state *st, hipStream_t s);
copa_status launch_init_grams(copa_plan *p, const copa_state *st, hipStream_t s);
copa_status launch_qtilde(copa_plan *p, float *Qt, hipStream_t s);
copa_status launch_tune(copa_plan *p, const copa_state *st, hipStream_t s);
copa_status harvest_timing(copa_plan *p);
extern const char *const kernel_names[kNumKernels];
bool rank_supported(int R);
Tiles choose_tiles(int R, int64_t J, int lds_limit);
Tiles choose_tiles2(int R, int64_t J, int lds_limit);
bool pass2_width_supported(int rt);

// ---------------------------------------------------------------- (copa_grad.hip)
copa_status launch_stationarity(copa_plan *p, const float *H, const float *V, const float *W,
                                const float *Qt, double *res_host, hipStream_t s);
copa_status launch_loss_grad(copa_plan *p, const float *H, const float *V, const float *W,
                             const float *Qt, float *dH, float *dV, float *dW, float *dS,
                             hipStream_t s);

// ---------------------------------------------------------------- device helpers
// Proximity operators of the constraints (Section "Examples of useful constraints"), without
// branches (kind is uniform across the wave; thr = lam / rho precomputed): nonnegativity,
// signed soft threshold at lam / rho, hard threshold keeping x when x^2 > lam, and their
// nonnegative combination.
__device__ __forceinline__ double prox_sel(double x, int kind, double lam, double thr) {
  const double a1 = fabs(x) - thr, a2 = x - thr;
  double r = x;
  r = kind == COPA_PROX_NONNEG ? (x > 0.0 ? x : 0.0) : r;
  r = kind == COPA_PROX_L1 ? (a1 > 0.0 ? copysign(a1, x) : 0.0) : r;
  r = kind == COPA_PROX_L0 ? (x * x > lam ? x : 0.0) : r;
  r = kind == COPA_PROX_NONNEG_L1 ? (a2 > 0.0 ? a2 : 0.0) : r;
  return r;
}

__device__ __forceinline__ float shfl_xor_f(float v, int m) { return __shfl_xor(v, m, kWave); }

// Value of the DPP source lane (CTRL: row_shr:n = 0x110 + n, row_bcast:15 = 0x142, row_bcast:31 =
// 0x143, wave_shl:1 = 0x130, wave_shr:1 = 0x138), or `old` where the source lane is outside the
// row or wave, or the lane's row is not in ROWMASK.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ int dpp_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ float dpp_f(float old, float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}

// Row width of an LDS factor tile: RT floats rounded up to a multiple of 4, so that a row moves
// with 16-byte LDS accesses (three instead of five for RT = 10).
__host__ __device__ constexpr int row4(int rt) { return (rt + 3) & ~3; }

// v[0, RT) from a 16-byte aligned LDS row, reading no pad: 16-byte reads for whole groups of
// four, then 8 and 4 bytes for the rest (RT = 10: 40 bytes in three reads instead of 48)
template <int RT>
__device__ __forceinline__ void lds_row(const float *row, float (&v)[RT]) {
  constexpr int B = RT / 4 * 4;
  const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll
  for (int q = 0; q < RT / 4; ++q) {
    const float4 a = r4[q];
    v[4 * q] = a.x;
    v[4 * q + 1] = a.y;
    v[4 * q + 2] = a.z;
    v[4 * q + 3] = a.w;
  }
  if constexpr (RT - B >= 2) {
    const float2 a = *reinterpret_cast<const float2 *>(row + B);
    v[B] = a.x;
    v[B + 1] = a.y;
  }
  if constexpr ((RT - B) & 1) v[RT - 1] = row[RT - 1];
}

// row[0, RT) += v[0, RT) on a 16-byte aligned LDS row with the same access widths as lds_row
template <int RT>
__device__ __forceinline__ void lds_row_add(float *row, const float *v) {
  constexpr int B = RT / 4 * 4;
  float4 *r4 = reinterpret_cast<float4 *>(row);
#pragma unroll
  for (int q = 0; q < RT / 4; ++q) {
    float4 a = r4[q];
    a.x += v[4 * q];
    a.y += v[4 * q + 1];
    a.z += v[4 * q + 2];
    a.w += v[4 * q + 3];
    r4[q] = a;
  }
  if constexpr (RT - B >= 2) {
    float2 a = *reinterpret_cast<float2 *>(row + B);
    a.x += v[B];
    a.y += v[B + 1];
    *reinterpret_cast<float2 *>(row + B) = a;
  }
  if constexpr ((RT - B) & 1) row[RT - 1] += v[RT - 1];
}

// Recursive-halving reduce-scatter over groups of G = 2^g <= 64 lanes (G wave-uniform, sub =
// lane index within the group). v[0, E) holds each lane's partial values of E elements (E a
// multiple of G); on return v[m], m < E / G, holds the group total of element m G + sub. Step b
// (from the top bit down) pairs each lane with a partner that differs in bit b and agrees on
// every higher bit (b = 5: xor 32 by permute; b = 4: xor 16 by swizzle; b = 3, 2: row and
// half-row mirrors, b = 1, 0: quad permutes, all DPP): the lane keeps the half of its elements
// whose bit b matches its own, and adds the partner's copy of that half. The partner maps
// generate every lane of the group.
template <int E, int G, int B>
__device__ __forceinline__ void reduce_scatter_step(float (&v)[E], int sub) {
  constexpr int g = G == 1 ? 0 : G == 2 ? 1 : G == 4 ? 2 : G == 8 ? 3 : G == 16 ? 4 : G == 32 ? 5 : 6;
  constexpr int half = 1 << B;
  constexpr int n = E >> (g - 1 - B);  // values held before this step
  // bitwise selects (a select between two array elements would become a dynamic index and
  // move the array to scratch memory)
  const int upm = -((sub >> B) & 1);
#pragma unroll
  for (int i = 0; i < n / 2; ++i) {
    const int m = i / half, s = i - m * half;
    const int lo = m * 2 * half + s, hi = lo + half;
    const int xl = __float_as_int(v[lo]), xh = __float_as_int(v[hi]);
    const float keep = __int_as_float((xh & upm) | (xl & ~upm));
    const int send = (xl & upm) | (xh & ~upm);
    int recv;
    if constexpr (B == 5)
      recv = __shfl_xor(send, 32, kWave);
    else if constexpr (B == 4)
      recv = __builtin_amdgcn_ds_swizzle(send, 0x401F);  // xor 16 within 32 lanes
    else if constexpr (B == 3)
      recv = __builtin_amdgcn_mov_dpp(send, 0x140, 0xF, 0xF, false);  // row_mirror
    else if constexpr (B == 2)
      recv = __builtin_amdgcn_mov_dpp(send, 0x141, 0xF, 0xF, false);  // row_half_mirror
    else if constexpr (B == 1)
      recv = __builtin_amdgcn_mov_dpp(send, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    else
      recv = __builtin_amdgcn_mov_dpp(send, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    v[i] = keep + __int_as_float(recv);
  }
  if constexpr (B > 0) reduce_scatter_step<E, G, B - 1>(v, sub);
}

template <int E, int G>
__device__ __forceinline__ void reduce_scatter(float (&v)[E], int sub) {
  static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0 && E % G == 0, "group size");
  constexpr int g = G == 1 ? 0 : G == 2 ? 1 : G == 4 ? 2 : G == 8 ? 3 : G == 16 ? 4 : G == 32 ? 5 : 6;
  if constexpr (g > 0) reduce_scatter_step<E, G, g - 1>(v, sub);
}

}  // namespace copa
