// Plan creation for libcopa.so: argument and CSR validation, packing of the tensor into the plan's
// device memory, per-subject smoothing bases and the wave work list of the streaming passes.
#include <algorithm>
#include <climits>
#include <cstring>
#include <numeric>
#include <thread>
#include <type_traits>

#include "copa_common.h"

namespace copa {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

// ------------------------------------------------------------------------------------ checks
enum : int32_t {
  kBadSubjPtr = 1, kBadRowPtr = 2, kBadCol = 4, kUnsortedCol = 8, kBadVal = 16, kBadDays = 32,
  kBadBasis = 64
};

__global__ void k_check_offsets(const int64_t *subj_ptr, const int64_t *row_ptr, int64_t K,
                                int64_t S, int64_t nnz, int32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= K) {
    int64_t v = subj_ptr[i];
    bool bad = (i == 0 && v != 0) || (i == K && v != S) || (i < K && subj_ptr[i + 1] < v);
    if (bad) atomicOr(flags, kBadSubjPtr);
  }
  if (i <= S) {
    int64_t v = row_ptr[i];
    bool bad = (i == 0 && v != 0) || (i == S && v != nnz) || (i < S && row_ptr[i + 1] < v);
    if (bad) atomicOr(flags, kBadRowPtr);
  }
}

// Thread per visit row: columns in range and strictly increasing, values finite, days (or the
// caller's basis row) finite. Only launched once the offsets are known to be monotone and in range.
__global__ void k_check_rows(const int64_t *row_ptr, const int32_t *col, const float *val,
                             const double *days, const double *basis, int l, int64_t S, int64_t J,
                             int32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  int64_t a = row_ptr[i], b = row_ptr[i + 1];
  int32_t f = 0;
  int64_t prev = -1;
  for (int64_t e = a; e < b; ++e) {
    int64_t c = col[e];
    if (c < 0 || c >= J) f |= kBadCol;
    if (c <= prev) f |= kUnsortedCol;
    prev = c;
    if (!isfinite(val[e])) f |= kBadVal;
  }
  if (days && !isfinite(days[i])) f |= kBadDays;
  if (basis)
    for (int a = 0; a < l; ++a)
      if (!isfinite(basis[i * l + a])) f |= kBadBasis;
  if (f) atomicOr(flags, f);
}

__global__ void k_pack_offsets(const int64_t *src, int32_t *dst, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (int32_t)src[i];
}

__global__ void k_row_subject(const int32_t *subj, int32_t *rowsubj, int64_t K) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  for (int32_t i = subj[k]; i < subj[k + 1]; ++i) rowsubj[i] = (int32_t)k;
}

// sum of squares of the values, FP64, one partial per block then a single-block finish
// flag[0] = 1 if some value is not exactly a bfloat16 (its low 16 bits are not zero)
__global__ void k_check_bf16(const float *val, int64_t n, int *flag) {
  int bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    bad |= (__float_as_uint(val[e]) & 0xffffu) != 0u;
  if (bad) atomicOr(flag, 1);
}

// Compact nonzero: feature id in the low 16 bits, the value's bfloat16 bits (exact) in the high.
__global__ void k_pack_compact(const int32_t *col, const float *val, int64_t n, uint32_t *xc) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    xc[e] = ((uint32_t)col[e] & 0xffffu) | (__float_as_uint(val[e]) & 0xffff0000u);
}

__global__ void k_sumsq(const float *val, int64_t n, double *part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = val[e];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------------- smoothing basis
// Cubic (degree min(3, L-1)) spline basis on the clamped knot vector of [t1, tn] with L-d-1
// equally spaced interior knots, evaluated by the triangular recursion of the smoothness section
// (degree-0 pieces are 1 on [b_i, b_{i+1}), the last nonempty piece also holds tn; a ratio with a
// zero denominator counts as 0). Every index is a compile-time constant.
template <int L>
__device__ __forceinline__ void spline_row(double t, const double (&beta)[L + 4], double (&m)[L]) {
  constexpr int d = L - 1 < 3 ? L - 1 : 3;
  constexpr int NB = L + d;  // degree-0 pieces
  double N[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    bool in = beta[i] <= t && t < beta[i + 1];
    if (i == L - 1 && t == beta[L]) in = true;  // last nonempty piece is closed
    N[i] = in ? 1.0 : 0.0;
  }
#pragma unroll
  for (int p = 1; p <= d; ++p) {
#pragma unroll
    for (int i = 0; i < NB - p; ++i) {
      double den1 = beta[i + p] - beta[i];
      double den2 = beta[i + p + 1] - beta[i + 1];
      double a = den1 != 0.0 ? (t - beta[i]) / den1 * N[i] : 0.0;
      double b = den2 != 0.0 ? (beta[i + p + 1] - t) / den2 * N[i + 1] : 0.0;
      N[i] = a + b;
    }
  }
#pragma unroll
  for (int i = 0; i < L; ++i) m[i] = N[i];
}

// One subject per lane. Streams the basis rows through Givens rotations into an L x L upper
// triangle R (M_k = Q_M R), takes the SVD of R by one-sided Jacobi (columns orthogonalised), sorts
// the singular values, keeps sigma > rtol * sigma_1 and writes C_k = M_k V_r Sigma_r^{-1}, an
// orthonormal basis of span(M_k), as FP32 rows of width kLMax.
// With `pp` set it also forms the projected data X'_k = C_k^T X_k in FP64, one record of `pw`
// floats per (subject, feature) pair: the column (entries 0..L-1), zeros, and the feature id in
// the last float (the subject's nonzeros come grouped by feature in nzr / nzx, pair q owning
// [pn[q], pn[q+1])).
template <int L>
__global__ void __launch_bounds__(64) k_basis(const int32_t *subj, const double *days,
                                              const double *basis, float *C, int32_t *rk,
                                              int64_t K, double rtol, const int32_t *pp,
                                              const int32_t *pj, const int32_t *pn,
                                              const int32_t *nzr, const float *nzx,
                                              float *recs, int pw) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int r0 = subj[k], r1 = subj[k + 1];
  if (r1 == r0) {
    rk[k] = 0;
    return;
  }
  // row i of M_k: the caller's basis row, or the spline basis evaluated at the visit day
  double beta[L + 4];
  auto basis_row = [&](int i, double (&m)[L]) {
    if (basis) {
#pragma unroll
      for (int a = 0; a < L; ++a) m[a] = basis[(int64_t)i * L + a];
    } else {
      spline_row<L>(days[i], beta, m);
    }
  };
  if (!basis) {
  double t1 = days[r0], tn = days[r0];
  for (int i = r0 + 1; i < r1; ++i) {
    t1 = fmin(t1, days[i]);
    tn = fmax(tn, days[i]);
  }
  if (t1 == tn) {  // no time span: the basis is the constant function
    const double cd = 1.0 / sqrt((double)(r1 - r0));
    const float c0 = (float)cd;
    for (int i = r0; i < r1; ++i) {
#pragma unroll
      for (int a = 0; a < kLMax; ++a) C[(int64_t)i * kLMax + a] = a == 0 ? c0 : 0.0f;
    }
    rk[k] = 1;
    if (pp) {
      for (int q = pp[k]; q < pp[k + 1]; ++q) {
        double x = 0.0;
        for (int n = pn[q]; n < pn[q + 1]; ++n) x += cd * (double)nzx[n];
        float *rec = recs + (int64_t)q * pw;
        for (int a = 0; a < pw - 1; ++a) rec[a] = a == 0 ? (float)x : 0.0f;
        rec[pw - 1] = __int_as_float(pj[q]);
      }
    }
    return;
  }
  constexpr int d = L - 1 < 3 ? L - 1 : 3;
  constexpr int ninner = L - d - 1;
#pragma unroll
  for (int i = 0; i < L + 4; ++i) beta[i] = tn;
#pragma unroll
  for (int i = 0; i <= d; ++i) beta[i] = t1;
#pragma unroll
  for (int j = 1; j <= ninner; ++j) beta[d + j] = t1 + (tn - t1) * j / (ninner + 1);
  }

  double R[L][L];
#pragma unroll
  for (int a = 0; a < L; ++a)
#pragma unroll
    for (int b = 0; b < L; ++b) R[a][b] = 0.0;
  for (int i = r0; i < r1; ++i) {
    double m[L];
    basis_row(i, m);
#pragma unroll
    for (int j = 0; j < L; ++j) {
      if (m[j] != 0.0) {
        double h = hypot(R[j][j], m[j]);
        double c = R[j][j] / h, s = m[j] / h;
#pragma unroll
        for (int q = j; q < L; ++q) {
          double x = R[j][q], y = m[q];
          R[j][q] = c * x + s * y;
          m[q] = -s * x + c * y;
        }
      }
    }
  }
  double Vr[L][L];
#pragma unroll
  for (int a = 0; a < L; ++a)
#pragma unroll
    for (int b = 0; b < L; ++b) Vr[a][b] = a == b ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int p = 0; p < L - 1; ++p) {
#pragma unroll
      for (int q = p + 1; q < L; ++q) {
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int i = 0; i < L; ++i) {
          al += R[i][p] * R[i][p];
          be += R[i][q] * R[i][q];
          ga += R[i][p] * R[i][q];
        }
        if (fabs(ga) > 1e-15 * sqrt(al * be) && ga != 0.0) {
          rotated = true;
          double zeta = (be - al) / (2.0 * ga);
          double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
#pragma unroll
          for (int i = 0; i < L; ++i) {
            double x = R[i][p], y = R[i][q];
            R[i][p] = c * x - s * y;
            R[i][q] = s * x + c * y;
            double u = Vr[i][p], v = Vr[i][q];
            Vr[i][p] = c * u - s * v;
            Vr[i][q] = s * u + c * v;
          }
        }
      }
    }
    if (!rotated) break;
  }
  double sig[L];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) s2 += R[i][j] * R[i][j];
    sig[j] = sqrt(s2);
  }
  // sort columns by decreasing sigma (exchange network on compile-time indices)
#pragma unroll
  for (int a = 0; a < L; ++a) {
#pragma unroll
    for (int b = 0; b < L - 1 - a; ++b) {
      if (sig[b] < sig[b + 1]) {
        double t = sig[b];
        sig[b] = sig[b + 1];
        sig[b + 1] = t;
#pragma unroll
        for (int i = 0; i < L; ++i) {
          double u = Vr[i][b];
          Vr[i][b] = Vr[i][b + 1];
          Vr[i][b + 1] = u;
        }
      }
    }
  }
  int r = 0;
#pragma unroll
  for (int j = 0; j < L; ++j) r += (sig[0] > 0.0 && sig[j] > rtol * sig[0]) ? 1 : 0;
  // E = V_r Sigma_r^{-1}
#pragma unroll
  for (int j = 0; j < L; ++j) {
    double inv = j < r ? 1.0 / sig[j] : 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) Vr[i][j] *= inv;
  }
  for (int i = r0; i < r1; ++i) {
    double m[L];
    basis_row(i, m);
#pragma unroll
    for (int j = 0; j < kLMax; ++j) {
      double c = 0.0;
      if (j < L) {
#pragma unroll
        for (int a = 0; a < L; ++a) c += m[a] * Vr[a][j < L ? j : 0];
      }
      C[(int64_t)i * kLMax + j] = (float)c;
    }
  }
  rk[k] = r;
  if (pp) {
    for (int q = pp[k]; q < pp[k + 1]; ++q) {
      double x[L];
#pragma unroll
      for (int j = 0; j < L; ++j) x[j] = 0.0;
      for (int n = pn[q]; n < pn[q + 1]; ++n) {
        double m[L];
        basis_row(nzr[n], m);
        const double v = (double)nzx[n];
#pragma unroll
        for (int j = 0; j < L; ++j) {
          double c = 0.0;
#pragma unroll
          for (int a = 0; a < L; ++a) c += m[a] * Vr[a][j];
          x[j] += c * v;
        }
      }
      float *rec = recs + (int64_t)q * pw;
#pragma unroll
      for (int j = 0; j < L; ++j) rec[j] = (float)x[j];
      for (int a = L; a < pw - 1; ++a) rec[a] = 0.0f;
      rec[pw - 1] = __int_as_float(pj[q]);
    }
  }
}

// FP32 -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// 16-byte mixed-precision records of both pair orders (see load_rec_bf)
__global__ void k_pack_bf16_pairs(const float *__restrict__ recs1, const float *__restrict__ recs2,
                                  int64_t n, uint4 *__restrict__ h1, uint4 *__restrict__ h2,
                                  uint16_t *__restrict__ feat2) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    for (int which = 0; which < 2; ++which) {
      const float *r = (which ? recs2 : recs1) + q * 8;
      const uint32_t key = __float_as_uint(r[7]);
      const uint32_t tag = which ? (key & 0xffffu) : key;
      uint4 w;
      w.x = bf16_bits(r[0]) | bf16_bits(r[1]) << 16;
      w.y = bf16_bits(r[2]) | bf16_bits(r[3]) << 16;
      w.z = bf16_bits(r[4]) | bf16_bits(r[5]) << 16;
      w.w = bf16_bits(r[6]) | tag << 16;
      (which ? h2 : h1)[q] = w;
      if (which) feat2[q] = (uint16_t)(key >> 16);
    }
  }
}

// pairs2[q] = pairs1[perm[q]] with the key replaced by key2[q]
__global__ void k_permute_pairs(const float *__restrict__ recs1, const int32_t *__restrict__ perm,
                                const int32_t *__restrict__ key2, int64_t n, int pw,
                                float *__restrict__ recs2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * pw;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e / pw;
    const int a = (int)(e - q * pw);
    recs2[e] = a == pw - 1 ? __int_as_float(key2[q]) : recs1[(int64_t)perm[q] * pw + a];
  }
}

static copa_status launch_basis(int l, const int32_t *subj, const double *days,
                                const double *basis, float *C, int32_t *rk, int64_t K,
                                double rtol, const copa_plan *p, hipStream_t s) {
  const bool pr = p->proj;
  dim3 g((unsigned)((K + 63) / 64)), b(64);
  switch (l) {
#define CASE(Lv) \
  case Lv:                                                                                      \
    k_basis<Lv><<<g, b, 0, s>>>(subj, days, basis, C, rk, K, rtol, pr ? p->pp : nullptr,       \
                                pr ? p->pj : nullptr, pr ? p->pn : nullptr,                    \
                                pr ? p->nzr : nullptr, pr ? p->nzx : nullptr,                  \
                                pr ? p->pairs1 : nullptr, p->pw);                              \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: set_error("l outside 0..8"); return COPA_EUNSUPPORTED;
  }
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

#define COPA_TRY(x)                   \
  do {                                \
    copa_status st_ = (x);            \
    if (st_ != COPA_OK) return st_;   \
  } while (0)

// Every device buffer of a plan is carved, 256-byte aligned, from one workspace.
template <typename T>
static copa_status dalloc(copa_plan *p, T **ptr, size_t count) {
  if (count == 0) count = 1;
  const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
  if (p->arena_used + bytes > p->arena_bytes) {
    *ptr = nullptr;
    set_error("workspace layout exceeds its computed size (internal error)");
    return COPA_EDEVICE;
  }
  *ptr = reinterpret_cast<T *>(p->arena + p->arena_used);
  p->arena_used += bytes;
  return COPA_OK;
}

// Sizes of a plan that follow from the shapes and options alone (host only).
static copa_status plan_dims(const copa_tensor *X, const copa_options *opt, copa_plan *p) {
  p->K = X->K;
  p->J = X->J;
  p->S = X->S;
  p->nnz = X->nnz;
  p->l = X->l;
  p->R = opt->R;
  p->opt = *opt;
  if (p->opt.rank_rtol <= 0.0) p->opt.rank_rtol = 1e-6;
  if (p->opt.basis_rtol <= 0.0) p->opt.basis_rtol = 1e-10;
  p->adjoint = opt->adjoint != 0 || opt->stop_tol > 0.0;
  COPA_HIP(hipGetDevice(&p->device));
  int lds = 0;
  COPA_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
  p->lds_limit = lds;  // 160 KB per workgroup on gfx950
  COPA_HIP(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device));
  const int R = p->R;
  const int64_t K = p->K;
  p->tiles = choose_tiles(R, p->J, p->lds_limit);
  if ((int64_t)p->J * (row4(p->tiles.rt)) * 4 + 16 > p->lds_limit) {
    set_error("J too large for the LDS-staged factor tile of this build");
    return COPA_EUNSUPPORTED;
  }
  p->tiles2 = choose_tiles2(R, p->J, p->lds_limit);
  // smoothed data with at most two nonzeros per visit row on average are streamed as projected
  // (subject, feature) pairs: fewer bytes than the nonzeros plus a basis row per visit row
  p->proj = p->l > 0 && p->J <= 65536 && p->nnz > 0 && p->nnz <= 2 * p->S && p->tiles2.nt > 0;
  p->pw = p->l <= 7 ? 8 : 12;
  // row chunks: pass 2 of plans without projected pairs, and the adjoint's scatter
  p->p2c = p->J <= 65536 && p->nnz > 0 && p->tiles2.nt > 0 && (!p->proj || p->adjoint);
  if (p->opt.deterministic && p->nnz > 0 && !(p->p2c || p->proj)) {
    set_error("deterministic mode needs the chunked pass 2 (J <= 65536 and an F_V tile that "
              "fits LDS)");
    return COPA_EUNSUPPORTED;
  }
  p->slot_rows = p->l > 0 ? p->l : 0;
  p->rows_total = p->l > 0 ? K * p->l : p->S;
  p->gmaxnb = 2 * std::max(1, p->n_cu);
  {
    // V update: 4 wavefronts per block, 64 / R rows per wavefront (R lanes per row)
    const int64_t rb = 4 * (kWave / R);
    p->n_vblocks =
        (int)std::max<int64_t>(1, std::min<int64_t>((p->J + rb - 1) / rb, 4 * std::max(1, p->n_cu)));
  }
  // V^T V partials beyond 64k doubles in all: a multi-block reduction instead of the FIT block's
  p->vtv_reduce = (int64_t)p->n_vblocks * R * R > 65536;
  // order W -> H -> V: persistent W-first and M-row launches, at most 4 blocks per compute unit
  p->wf_cap = p->opt.order == COPA_ORDER_WHV ? 4 * std::max(1, p->n_cu) : 0;
  p->wf_blocks = 0;  // set from the kernels' occupancy at the first fit
  p->mr_blocks = 0;
  p->gcap = std::max(std::max(p->gmaxnb, p->n_vblocks), p->wf_cap);
  p->gstride = ((int64_t)p->gcap + 1) * R * R;
  {
    const int64_t per_block = 4 * (kWave / R);
    p->n_wblocks = (int)std::max<int64_t>(1, (K + per_block - 1) / per_block);
  }
  // pass-2 chunks: at most kChunkRows rows and kChunkRows / l subjects each
  const int64_t msub = p->l > 0 ? kChunkRows / p->l : INT64_MAX;
  p->nchunks_cap = (int)std::min<int64_t>(INT32_MAX - 1, (p->S + kChunkRows - 1) / kChunkRows +
                                                          (p->l > 0 ? K / msub : 0) + 1);
  p->p2_blocks_cap = 2 * std::max(1, p->n_cu);
  p->p2_blocks = p->p2_blocks_cap;
  p->gram_blocks = p->gmaxnb;
  p->pchunks_cap = p->proj ? (int)std::min<int64_t>(INT32_MAX - 1, K / msub + 2) : 0;
  return COPA_OK;
}

// Carves every buffer of the plan in a fixed order, with bounds for the counts that depend on
// the data (wave lists, chunks, large eigenproblems). Run on an empty arena of size 0 it only
// adds up the bytes (the arena pointer stays null and nothing is written).
static copa_status carve_all(copa_plan *p, bool dry) {
  const int64_t K = p->K, S = p->S, nnz = p->nnz, J = p->J;
  const int R = p->R;
  size_t total = 0;
  auto take = [&](auto **ptr, size_t count) -> copa_status {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(*ptr)>>;
    if (count == 0) count = 1;
    const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    total += bytes;
    if (dry) return COPA_OK;
    return dalloc(p, ptr, count);
  };
  COPA_TRY(take(&p->tmp, 1024));
  COPA_TRY(take(&p->subj, K + 1));
  COPA_TRY(take(&p->row, S + 1));
  COPA_TRY(take(&p->col, nnz));
  COPA_TRY(take(&p->val, nnz));
  COPA_TRY(take(&p->xc, p->J <= 65536 ? nnz : 0));
  COPA_TRY(take(&p->order, K));
  COPA_TRY(take(&p->order1, K));
  COPA_TRY(take(&p->waves, K));
  COPA_TRY(take(&p->waves1, K));
  COPA_TRY(take(&p->rowsubj, S));
  if (p->l > 0) {
    COPA_TRY(take(&p->C, S * kLMax));
    COPA_TRY(take(&p->rk, K));
    COPA_TRY(take(&p->Ew, (size_t)K * kNMax * kNMax));
    if (R > 16) COPA_TRY(take(&p->pgb, (size_t)K * 36));
  } else {
    COPA_TRY(take(&p->big_list, K));
  }
  // (kLMax rows of slack past the end: kernels may load a subject's kLMax row slots whole)
  COPA_TRY(take(&p->T, (p->rows_total + kLMax) * R));
  COPA_TRY(take(&p->Q, (p->rows_total + kLMax) * R));
  COPA_TRY(take(&p->M, (p->rows_total + kLMax) * R));
  COPA_TRY(take(&p->FW, K * R));
  COPA_TRY(take(&p->FV, J * R));
  COPA_TRY(take(&p->Vp, (size_t)p->tiles.nt * J * row4(p->tiles.rt)));
  COPA_TRY(take(&p->gpart, (size_t)kGramSlots * p->gstride));
  COPA_TRY(take(&p->gcount, 8));
  if (p->p2c) {
    const size_t nch = (size_t)p->nchunks_cap;
    COPA_TRY(take(&p->wsplit, nch * 9));
    COPA_TRY(take(&p->cptr, nch + 1));
    COPA_TRY(take(&p->crow, nch + 1));
    COPA_TRY(take(&p->cinfo, 2 * nch));
    COPA_TRY(take(&p->pkv, nnz));
  }
  if (p->proj) {
    const size_t pcap = (size_t)nnz;  // pairs never outnumber nonzeros
    COPA_TRY(take(&p->pp, K + 1));
    COPA_TRY(take(&p->pairs1, pcap * p->pw));
    COPA_TRY(take(&p->pairs2, pcap * p->pw));
    COPA_TRY(take(&p->pj, pcap));
    COPA_TRY(take(&p->pn, pcap + 1));
    COPA_TRY(take(&p->nzr, nnz));
    COPA_TRY(take(&p->nzx, nnz));
    COPA_TRY(take(&p->perm2, pcap));
    COPA_TRY(take(&p->key2, pcap));
    if (p->opt.precision == COPA_PREC_MIXED) {
      COPA_TRY(take(&p->pairs1h, pcap));
      COPA_TRY(take(&p->pairs2h, pcap));
      COPA_TRY(take(&p->feat2h, pcap));
    }
    const size_t nch = (size_t)p->pchunks_cap;
    COPA_TRY(take(&p->pcq, nch + 1));
    COPA_TRY(take(&p->pcinfo, 2 * nch));
    COPA_TRY(take(&p->pwsplit, nch * 9));
  }
  if ((p->p2c || p->proj) && p->opt.deterministic)
    COPA_TRY(take(&p->fvpart, (size_t)p->p2_blocks_cap * J * R));
  COPA_TRY(take(&p->vpart, (size_t)p->n_vblocks * 4));
  COPA_TRY(take(&p->wpart, (size_t)std::max(p->n_wblocks, p->wf_cap)));
  COPA_TRY(take(&p->small, 8 * R * R));
  COPA_TRY(take(&p->modes, 3));
  COPA_TRY(take(&p->scal, 1));
  COPA_TRY(take(&p->dloss, 64));
  if (p->adjoint) {
    COPA_TRY(take(&p->gradbuf, (size_t)2 * S * R + (size_t)J * R));
    COPA_TRY(take(&p->lpart, (size_t)2 * ((K + 3) / 4 + 1)));
    p->statfloats = ((size_t)R * R + (size_t)(J + K) * R + 1) & ~(size_t)1;
    COPA_TRY(take(&p->statbuf, p->statfloats + 2 * (6 * kStatBlocks + 3)));
    COPA_TRY(take(&p->qtbuf, (size_t)S * R));
  }
  if (dry) p->arena_bytes = total;
  return COPA_OK;
}

// Host-side build of the pass-2 layout: for every chunk of kChunkRows visit rows, the chunk's
// nonzeros ordered by (feature, row), keyed as feature << 16 | row within the chunk.
static copa_status build_sorted_chunks(const copa_tensor *X, copa_plan *p, hipStream_t s) {
  const int64_t S = p->S, nnz = p->nnz;
  std::vector<int64_t> rp(S + 1);
  std::vector<int32_t> cl(nnz);
  std::vector<float> vl(nnz);
  COPA_HIP(hipMemcpyAsync(rp.data(), X->row_ptr, (S + 1) * sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
  COPA_HIP(hipMemcpyAsync(cl.data(), X->col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  COPA_HIP(hipMemcpyAsync(vl.data(), X->val, nnz * sizeof(float), hipMemcpyDeviceToHost, s));
  COPA_HIP(hipStreamSynchronize(s));
  // chunks of at most kChunkRows rows and, smoothed, at most kChunkRows / l subjects (so that the
  // chunk's M rows fit the LDS space of its u rows)
  const int64_t K = p->K;
  std::vector<int64_t> sp(K + 1);
  COPA_HIP(hipMemcpyAsync(sp.data(), X->subj_ptr, (K + 1) * sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
  COPA_HIP(hipStreamSynchronize(s));
  const int64_t msub = p->l > 0 ? kChunkRows / p->l : K + 1;
  std::vector<int32_t> crow, cinf;
  {
    int64_t r = 0, k = 0;
    while (r < S) {
      while (sp[k + 1] <= r) ++k;  // subject of row r
      int64_t end = std::min<int64_t>(r + kChunkRows, S);
      if (k + msub < K) end = std::min<int64_t>(end, sp[k + msub]);
      int64_t klast = k;
      while (sp[klast + 1] < end) ++klast;  // subject of row end - 1
      crow.push_back((int32_t)r);
      cinf.push_back((int32_t)k);
      cinf.push_back((int32_t)(klast - k + 1));
      r = end;
    }
    crow.push_back((int32_t)S);
  }
  const int nch = (int)crow.size() - 1;
  std::vector<int32_t> cp(nch + 1);
  for (int c = 0; c <= nch; ++c) cp[c] = (int32_t)rp[crow[c]];
  std::vector<uint32_t> key(nnz);
  std::vector<float> sv(nnz);
  const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned w = 0; w < nthreads; ++w) {
    pool.emplace_back([&, w]() {
      std::vector<uint64_t> tmp;
      for (int c = (int)w; c < nch; c += (int)nthreads) {
        const int64_t r0 = crow[c], r1 = crow[c + 1];
        const int64_t e0 = rp[r0];
        tmp.clear();
        for (int64_t i = r0; i < r1; ++i)
          for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const uint64_t k = ((uint64_t)cl[e] << 16) | (uint64_t)(i - r0);
            tmp.push_back((k << 32) | (uint64_t)(e - e0));
          }
        std::sort(tmp.begin(), tmp.end());
        for (size_t q = 0; q < tmp.size(); ++q) {
          key[e0 + q] = (uint32_t)(tmp[q] >> 32);
          sv[e0 + q] = vl[e0 + (int64_t)(tmp[q] & 0xffffffffu)];
        }
      }
    });
  }
  for (auto &t : pool) t.join();
  // 8 wave slices per chunk, cut on feature boundaries near equal shares
  std::vector<int32_t> ws((size_t)nch * 9);
  for (int c = 0; c < nch; ++c) {
    const int32_t e0 = cp[c], e1 = cp[c + 1];
    ws[c * 9] = e0;
    int32_t pos = e0;
    for (int w = 1; w < 8; ++w) {
      int32_t target = e0 + (int32_t)(((int64_t)(e1 - e0) * w) / 8);
      if (target < pos) target = pos;
      while (target > e0 && target < e1 && (key[target] >> 16) == (key[target - 1] >> 16)) ++target;
      pos = target;
      ws[c * 9 + w] = pos;
    }
    ws[c * 9 + 8] = e1;
  }
  if (nch > p->nchunks_cap) {
    set_error("pass-2 chunk count above its bound (internal error)");
    return COPA_EDEVICE;
  }
  p->nchunks = nch;
  COPA_HIP(hipMemcpyAsync(p->wsplit, ws.data(), ws.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  COPA_HIP(hipMemcpyAsync(p->crow, crow.data(), (nch + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  COPA_HIP(hipMemcpyAsync(p->cinfo, cinf.data(), 2 * nch * sizeof(int32_t), hipMemcpyHostToDevice, s));
  COPA_HIP(hipMemcpyAsync(p->cptr, cp.data(), (nch + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  {
    std::vector<uint2> kv(nnz);
    for (int64_t e = 0; e < nnz; ++e) {
      uint32_t vb;
      std::memcpy(&vb, &sv[e], sizeof(vb));
      kv[e] = make_uint2(key[e], vb);
    }
    COPA_HIP(hipMemcpyAsync(p->pkv, kv.data(), nnz * sizeof(uint2), hipMemcpyHostToDevice, s));
    COPA_HIP(hipStreamSynchronize(s));
  }
  COPA_HIP(hipStreamSynchronize(s));
  return COPA_OK;
}

// Host-side lists of the projected pairs: per subject, its nonzeros grouped by feature (rows in
// order within a feature); pair q of the subject's feature pj[q] owns nonzeros [pn[q], pn[q+1])
// of nzr (visit row) / nzx (value). The device basis kernel then forms the records.
static copa_status build_pair_lists(const copa_tensor *X, copa_plan *p,
                                    const std::vector<int64_t> &hs, std::vector<int32_t> &hpp,
                                    std::vector<int32_t> &hpj, hipStream_t s) {
  const int64_t K = p->K, S = p->S, nnz = p->nnz;
  std::vector<int64_t> rp(S + 1);
  std::vector<int32_t> cl(nnz);
  std::vector<float> vl(nnz);
  COPA_HIP(hipMemcpyAsync(rp.data(), X->row_ptr, (S + 1) * sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
  COPA_HIP(hipMemcpyAsync(cl.data(), X->col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  COPA_HIP(hipMemcpyAsync(vl.data(), X->val, nnz * sizeof(float), hipMemcpyDeviceToHost, s));
  COPA_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> nzr(nnz), cnt(K + 1, 0);
  std::vector<float> nzx(nnz);
  std::vector<int32_t> feat(nnz);  // feature of each nonzero in the grouped order
  const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto run = [&](auto &&body) {
    std::vector<std::thread> pool;
    for (unsigned w = 0; w < nthreads; ++w)
      pool.emplace_back([&, w]() {
        const int64_t a = K * w / nthreads, b = K * (w + 1) / nthreads;
        body(a, b);
      });
    for (auto &t : pool) t.join();
  };
  run([&](int64_t ka, int64_t kb) {
    std::vector<uint64_t> tmp;
    for (int64_t k = ka; k < kb; ++k) {
      const int64_t e0 = rp[hs[k]], e1 = rp[hs[k + 1]];
      tmp.clear();
      for (int64_t i = hs[k]; i < hs[k + 1]; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
          tmp.push_back(((uint64_t)(uint32_t)cl[e] << 32) | (uint64_t)(e - e0));
      std::sort(tmp.begin(), tmp.end());  // by feature, then by position (row order)
      int32_t distinct = 0;
      for (size_t q = 0; q < tmp.size(); ++q) {
        const int64_t e = e0 + (int64_t)(tmp[q] & 0xffffffffu);
        const int32_t j = (int32_t)(tmp[q] >> 32);
        if (q == 0 || j != feat[e0 + q - 1]) ++distinct;
        feat[e0 + q] = j;
        nzx[e0 + q] = vl[e];
        // visit row of nonzero e: the last row of the subject starting at or before e
        int64_t lo = hs[k], hi = hs[k + 1] - 1;
        while (lo < hi) {
          const int64_t mid = (lo + hi + 1) / 2;
          if (rp[mid] <= e) lo = mid; else hi = mid - 1;
        }
        nzr[e0 + q] = (int32_t)lo;
      }
      (void)e1;
      cnt[k] = distinct;
    }
  });
  hpp.assign(K + 1, 0);
  for (int64_t k = 0; k < K; ++k) hpp[k + 1] = hpp[k] + cnt[k];
  const int64_t P = hpp[K];
  p->npairs = P;
  hpj.assign(P, 0);
  std::vector<int32_t> hpn(P + 1);
  run([&](int64_t ka, int64_t kb) {
    for (int64_t k = ka; k < kb; ++k) {
      const int64_t e0 = rp[hs[k]], e1 = rp[hs[k + 1]];
      int64_t q = hpp[k];
      for (int64_t e = e0; e < e1; ++e)
        if (e == e0 || feat[e] != feat[e - 1]) {
          hpj[q] = feat[e];
          hpn[q] = (int32_t)e;
          ++q;
        }
    }
  });
  hpn[P] = (int32_t)nnz;
  COPA_HIP(hipMemcpyAsync(p->pp, hpp.data(), (K + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (P > 0) {
    COPA_HIP(hipMemcpyAsync(p->pj, hpj.data(), P * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  COPA_HIP(hipMemcpyAsync(p->pn, hpn.data(), (P + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  COPA_HIP(hipMemcpyAsync(p->nzr, nzr.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
  COPA_HIP(hipMemcpyAsync(p->nzx, nzx.data(), nnz * sizeof(float), hipMemcpyHostToDevice, s));
  COPA_HIP(hipStreamSynchronize(s));
  return COPA_OK;
}

// Pass-2 chunks of the projected pairs: runs of at most kChunkRows / l consecutive subjects,
// each chunk's pairs ordered by (feature, subject) into pairs2 and cut into eight wave slices on
// feature boundaries.
static copa_status build_pair_chunks(copa_plan *p, const std::vector<int32_t> &hpp,
                                     const std::vector<int32_t> &hpj, hipStream_t s) {
  const int64_t K = p->K, P = p->npairs;
  const int64_t msub = kChunkRows / p->l;
  std::vector<int32_t> cq, cinf;
  for (int64_t k = 0; k < K; k += msub) {
    const int64_t n = std::min<int64_t>(msub, K - k);
    cq.push_back(hpp[k]);
    cinf.push_back((int32_t)k);
    cinf.push_back((int32_t)n);
  }
  cq.push_back((int32_t)P);
  const int nch = (int)cinf.size() / 2;
  if (nch > p->pchunks_cap) {
    set_error("pass-2 chunk count above its bound (internal error)");
    return COPA_EDEVICE;
  }
  std::vector<int32_t> perm(P), key(P), ws((size_t)nch * 9);
  const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned w = 0; w < nthreads; ++w) {
    pool.emplace_back([&, w]() {
      std::vector<uint64_t> tmp;
      for (int c = (int)w; c < nch; c += (int)nthreads) {
        const int64_t k0 = cinf[2 * c], n = cinf[2 * c + 1];
        tmp.clear();
        for (int64_t k = k0; k < k0 + n; ++k)
          for (int64_t q = hpp[k]; q < hpp[k + 1]; ++q)
            tmp.push_back(((uint64_t)(uint32_t)hpj[q] << 48) | ((uint64_t)(k - k0) << 32) |
                          (uint64_t)q);
        std::sort(tmp.begin(), tmp.end());
        const int64_t q0 = cq[c];
        for (size_t i = 0; i < tmp.size(); ++i) {
          perm[q0 + i] = (int32_t)(tmp[i] & 0xffffffffu);
          key[q0 + i] = (int32_t)((tmp[i] >> 48) << 16 | ((tmp[i] >> 32) & 0xffffu));
        }
        const int32_t e0 = cq[c], e1 = cq[c + 1];
        ws[c * 9] = e0;
        int32_t pos = e0;
        for (int wv = 1; wv < 8; ++wv) {
          int32_t target = e0 + (int32_t)(((int64_t)(e1 - e0) * wv) / 8);
          if (target < pos) target = pos;
          while (target > e0 && target < e1 && (key[target] >> 16) == (key[target - 1] >> 16))
            ++target;
          pos = target;
          ws[c * 9 + wv] = pos;
        }
        ws[c * 9 + 8] = e1;
      }
    });
  }
  for (auto &t : pool) t.join();
  p->pnchunks = nch;
  COPA_HIP(hipMemcpyAsync(p->pcq, cq.data(), (nch + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  COPA_HIP(hipMemcpyAsync(p->pcinfo, cinf.data(), 2 * nch * sizeof(int32_t), hipMemcpyHostToDevice, s));
  COPA_HIP(hipMemcpyAsync(p->pwsplit, ws.data(), ws.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (P > 0) {
    COPA_HIP(hipMemcpyAsync(p->perm2, perm.data(), P * sizeof(int32_t), hipMemcpyHostToDevice, s));
    COPA_HIP(hipMemcpyAsync(p->key2, key.data(), P * sizeof(int32_t), hipMemcpyHostToDevice, s));
    k_permute_pairs<<<2048, 256, 0, s>>>(p->pairs1, p->perm2, p->key2, P, p->pw, p->pairs2);
    COPA_HIP(hipGetLastError());
    if (p->opt.precision == COPA_PREC_MIXED) {
      k_pack_bf16_pairs<<<2048, 256, 0, s>>>(p->pairs1, p->pairs2, P, p->pairs1h, p->pairs2h,
                                             p->feat2h);
      COPA_HIP(hipGetLastError());
    }
  }
  COPA_HIP(hipStreamSynchronize(s));
  return COPA_OK;
}

static copa_status build_plan(const copa_tensor *X, const copa_options *opt, void *workspace,
                              size_t ws_bytes, hipStream_t s, copa_plan *p) {
  COPA_TRY(plan_dims(X, opt, p));
  COPA_TRY(carve_all(p, true));
  const size_t need = p->arena_bytes;
  if (workspace) {
    if (ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255) != 0) {
      set_error("workspace of " + std::to_string(ws_bytes) + " bytes at a " +
                (((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) ? "misaligned"
                                                                         : "256-byte aligned") +
                " address; the plan needs " + std::to_string(need) + " bytes, 256-byte aligned");
      return COPA_EINVAL;
    }
    p->arena = static_cast<char *>(workspace);
    p->arena_owned = false;
  } else {
    hipError_t e = hipMalloc((void **)&p->arena, need);
    if (e != hipSuccess) {
      p->arena = nullptr;
      set_error("hipMalloc of the " + std::to_string(need) + "-byte workspace: " +
                hipGetErrorString(e));
      return COPA_ENOMEM;
    }
    p->arena_owned = true;
  }
  p->arena_bytes = need;
  p->arena_used = 0;
  COPA_TRY(carve_all(p, false));

  const int64_t K = p->K, S = p->S, nnz = p->nnz;
  const int R = p->R;
  const bool caller_basis = p->l > 0 && X->basis != nullptr;
  // ---- content checks on the device
  int32_t *flags = reinterpret_cast<int32_t *>(p->tmp);
  COPA_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
  {
    int64_t n = std::max(K, S) + 1;
    k_check_offsets<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(X->subj_ptr, X->row_ptr, K, S,
                                                                 nnz, flags);
    COPA_HIP(hipGetLastError());
  }
  int32_t hflags = 0;
  COPA_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  COPA_HIP(hipStreamSynchronize(s));
  if (hflags == 0 && S > 0) {
    k_check_rows<<<(unsigned)((S + 255) / 256), 256, 0, s>>>(
        X->row_ptr, X->col, X->val, p->l > 0 && !caller_basis ? X->days : nullptr,
        caller_basis ? X->basis : nullptr, p->l, S, p->J, flags);
    COPA_HIP(hipGetLastError());
    COPA_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    COPA_HIP(hipStreamSynchronize(s));
  }
  if (hflags) {
    std::string m = "invalid tensor:";
    if (hflags & kBadSubjPtr) m += " subj_ptr not 0..S non-decreasing;";
    if (hflags & kBadRowPtr) m += " row_ptr not 0..nnz non-decreasing;";
    if (hflags & kBadCol) m += " column id outside [0,J);";
    if (hflags & kUnsortedCol) m += " columns not strictly increasing within a row;";
    if (hflags & kBadVal) m += " non-finite value;";
    if (hflags & kBadDays) m += " non-finite visit day;";
    if (hflags & kBadBasis) m += " non-finite basis value;";
    set_error(m);
    return COPA_EINVAL;
  }

  // ---- packing
  k_pack_offsets<<<(unsigned)((K + 1 + 255) / 256), 256, 0, s>>>(X->subj_ptr, p->subj, K + 1);
  k_pack_offsets<<<(unsigned)((S + 1 + 255) / 256), 256, 0, s>>>(X->row_ptr, p->row, S + 1);
  COPA_HIP(hipGetLastError());
  if (nnz > 0) {
    COPA_HIP(hipMemcpyAsync(p->col, X->col, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    COPA_HIP(hipMemcpyAsync(p->val, X->val, nnz * sizeof(float), hipMemcpyDeviceToDevice, s));
  } else {
    // kernels read entry 0 as the clamped target of masked loads: keep it a valid feature
    COPA_HIP(hipMemsetAsync(p->col, 0, sizeof(int32_t), s));
    COPA_HIP(hipMemsetAsync(p->val, 0, sizeof(float), s));
  }
  {
    constexpr int nb = 512;
    double *part = p->tmp + 8;
    k_sumsq<<<nb, 256, 0, s>>>(p->val, nnz, part);
    COPA_HIP(hipGetLastError());
    std::vector<double> h(nb);
    COPA_HIP(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    COPA_HIP(hipStreamSynchronize(s));
    p->normX2 = 0.0;
    for (double v : h) p->normX2 += v;
  }
  // ---- compact nonzeros for pass 1 when lossless: features below 2^16 and every value exactly
  // a bfloat16 (count data); half the bytes and one load per nonzero
  p->compact = false;
  if (nnz > 0 && p->J <= 65536) {
    int *flag = reinterpret_cast<int *>(p->tmp + 4);
    COPA_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_check_bf16<<<1024, 256, 0, s>>>(p->val, nnz, flag);
    COPA_HIP(hipGetLastError());
    int hf = 1;
    COPA_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    COPA_HIP(hipStreamSynchronize(s));
    if (hf == 0) {
      k_pack_compact<<<2048, 256, 0, s>>>(p->col, p->val, nnz, p->xc);
      COPA_HIP(hipGetLastError());
      p->compact = true;
    }
  }

  // ---- subject order and wave work lists (host): subjects by decreasing visit count; a wave
  // gives G = 2^lg lanes to each subject with G ~ I_max / 4 rows per lane
  std::vector<int64_t> hs(K + 1);
  COPA_HIP(hipMemcpyAsync(hs.data(), X->subj_ptr, (K + 1) * sizeof(int64_t),
                          hipMemcpyDeviceToHost, s));
  COPA_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> ord(K);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    return hs[a + 1] - hs[a] > hs[b + 1] - hs[b];
  });
  // wave list over subjects in the order `o`: G = 2^lg lanes per subject with about `per` units
  // of work (visit rows, or projected pairs) per lane
  auto wave_list = [&](int lanes, const std::vector<int32_t> &o, auto work, int64_t per) {
    std::vector<WaveEntry> w;
    for (int64_t i = 0; i < K;) {
      const int64_t ik = work(o[i]);
      int lg = 0;
      while ((1 << lg) < lanes && (int64_t)(1 << lg) * per < ik) ++lg;
      int cnt = (int)std::min<int64_t>(lanes >> lg, K - i);
      w.push_back(WaveEntry{(int32_t)i, lg | (cnt << 8)});
      i += cnt;
    }
    return w;
  };
  auto visits = [&](int32_t k) { return hs[k + 1] - hs[k]; };
  const std::vector<WaveEntry> waves = wave_list(kWave, ord, visits, 4);
  // pass 1: projected plans stream pairs, so their subjects are ordered and split by pair count
  std::vector<int32_t> hpp, hpj;
  std::vector<int32_t> ord1;
  std::vector<WaveEntry> waves1;
  if (p->proj) {
    COPA_TRY(build_pair_lists(X, p, hs, hpp, hpj, s));
    ord1.resize(K);
    std::iota(ord1.begin(), ord1.end(), 0);
    auto pairs = [&](int32_t k) { return (int64_t)(hpp[k + 1] - hpp[k]); };
    std::stable_sort(ord1.begin(), ord1.end(),
                     [&](int32_t a, int32_t b) { return pairs(a) > pairs(b); });
    waves1 = wave_list(kWave / p->tiles.cg, ord1, pairs, 8);
  } else {
    ord1 = ord;
    waves1 = wave_list(kWave / p->tiles.cg, ord, visits, 4);
  }
  p->n_waves = (int32_t)waves.size();
  p->n_waves1 = (int32_t)waves1.size();
  if (K > 0) {
    COPA_HIP(hipMemcpyAsync(p->order, ord.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
    COPA_HIP(hipMemcpyAsync(p->order1, ord1.data(), K * sizeof(int32_t), hipMemcpyHostToDevice, s));
    COPA_HIP(hipMemcpyAsync(p->waves, waves.data(), waves.size() * sizeof(WaveEntry),
                            hipMemcpyHostToDevice, s));
    COPA_HIP(hipMemcpyAsync(p->waves1, waves1.data(), waves1.size() * sizeof(WaveEntry),
                            hipMemcpyHostToDevice, s));
  }
  if (K > 0) {
    k_row_subject<<<(unsigned)((K + 255) / 256), 256, 0, s>>>(p->subj, p->rowsubj, K);
    COPA_HIP(hipGetLastError());
  }
  // ---- smoothing basis (and, for projected plans, the pairs' records)
  std::vector<int32_t> big;
  if (p->l > 0) {
    if (K > 0)
      COPA_TRY(launch_basis(p->l, p->subj, caller_basis ? nullptr : X->days,
                            caller_basis ? X->basis : nullptr, p->C, p->rk, K,
                            p->opt.basis_rtol, p, s));
  } else {
    // subjects whose eigenproblem min(I_k, R) is larger than a lane can hold
    for (int64_t k = 0; k < K; ++k)
      if (std::min<int64_t>(hs[k + 1] - hs[k], p->R) > kNMax) big.push_back((int32_t)k);
    p->n_big = (int32_t)big.size();
    if (!big.empty())
      COPA_HIP(hipMemcpyAsync(p->big_list, big.data(), big.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
  }
  {
    const int rtp = row4(p->tiles.rt);
    COPA_HIP(hipMemsetAsync(p->Vp, 0, (size_t)p->tiles.nt * p->J * rtp * sizeof(float), s));
  }
  COPA_HIP(hipMemsetAsync(p->gcount, 0, 8 * sizeof(int32_t), s));
  // ---- feature-sorted chunks for pass 2
  if (p->proj) COPA_TRY(build_pair_chunks(p, hpp, hpj, s));
  if (p->p2c) COPA_TRY(build_sorted_chunks(X, p, s));
  COPA_HIP(hipMemsetAsync(p->T, 0, p->rows_total * R * sizeof(float), s));
  COPA_HIP(hipMemsetAsync(p->Q, 0, p->rows_total * R * sizeof(float), s));
  COPA_HIP(hipMemsetAsync(p->M, 0, p->rows_total * R * sizeof(float), s));
  COPA_HIP(hipMemsetAsync(p->FW, 0, K * R * sizeof(float), s));
  COPA_HIP(hipMemsetAsync(p->FV, 0, p->J * R * sizeof(float), s));
  COPA_HIP(hipMemsetAsync(p->small, 0, 8 * R * R * sizeof(double), s));
  COPA_HIP(hipStreamSynchronize(s));
  return COPA_OK;
}

}  // namespace copa

using namespace copa;

static void free_plan(copa_plan *p) {
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->gexec_bf) (void)hipGraphExecDestroy(p->gexec_bf);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->arena_owned && p->arena) (void)hipFree(p->arena);
  delete p;
}

extern "C" {

const char *copa_last_error(void) { return g_last_error.c_str(); }

const char *copa_status_string(copa_status st) {
  switch (st) {
    case COPA_OK: return "COPA_OK";
    case COPA_EINVAL: return "COPA_EINVAL";
    case COPA_ENOMEM: return "COPA_ENOMEM";
    case COPA_EDEVICE: return "COPA_EDEVICE";
    case COPA_ENUMERIC: return "COPA_ENUMERIC";
    case COPA_EUNSUPPORTED: return "COPA_EUNSUPPORTED";
  }
  return "COPA_UNKNOWN";
}

int32_t copa_rank_supported(int32_t R) { return rank_supported(R) ? 1 : 0; }

// Host-side checks of the shapes and options shared by the size query and plan creation.
static copa_status check_args(const copa_tensor *X, const copa_options *opt, bool arrays) {
  if (!X || !opt) {
    set_error("tensor or options is NULL");
    return COPA_EINVAL;
  }
  if (X->K < 0 || X->J < 1 || X->S < 0 || X->nnz < 0 || X->S >= INT32_MAX ||
      X->nnz >= INT32_MAX || X->J >= INT32_MAX || X->K >= INT32_MAX) {
    set_error("sizes must satisfy K >= 0, J >= 1, S >= 0, nnz >= 0, all below 2^31");
    return COPA_EINVAL;
  }
  if (arrays && (!X->subj_ptr || !X->row_ptr || (X->nnz > 0 && (!X->col || !X->val)))) {
    set_error("tensor array is NULL");
    return COPA_EINVAL;
  }
  if (X->l < 0) {
    set_error("l must be >= 0");
    return COPA_EINVAL;
  }
  if (X->l > kLMax) {
    set_error("l > 8 spline basis functions is not supported by this build");
    return COPA_EUNSUPPORTED;
  }
  if (arrays && X->l > 0 && X->S > 0 && !X->days && !X->basis) {
    set_error("days and basis are NULL with l > 0");
    return COPA_EINVAL;
  }
  if (opt->R < 1 || opt->inner_iters < 1) {
    set_error("R and inner_iters must be >= 1");
    return COPA_EINVAL;
  }
  for (int32_t k : {opt->prox_H, opt->prox_W, opt->prox_V})
    if (k < COPA_PROX_NONE || k > COPA_PROX_NONNEG_L1) {
      set_error("unknown prox kind");
      return COPA_EINVAL;
    }
  if (!(opt->lambda_H >= 0.0 && opt->lambda_W >= 0.0 && opt->lambda_V >= 0.0)) {
    set_error("lambda must be finite and >= 0");
    return COPA_EINVAL;
  }
  if (!rank_supported(opt->R)) {
    set_error("rank R=" + std::to_string(opt->R) + " has no kernels in this build");
    return COPA_EUNSUPPORTED;
  }
  if (opt->precision != COPA_PREC_FP32 && opt->precision != COPA_PREC_MIXED) {
    set_error("unknown precision");
    return COPA_EINVAL;
  }
  if (opt->precision == COPA_PREC_MIXED && (X->l < 1 || X->l > 7 || X->J > 65536 ||
                                              X->nnz > 2 * X->S || X->nnz == 0)) {
    set_error("mixed precision streams bfloat16 records of the projected data C_k^T X_k: it needs "
              "smoothing with l <= 7, J <= 65536 and at most two nonzeros per visit row on "
              "average");
    return COPA_EUNSUPPORTED;
  }
  if (opt->mixed_refine < 0) {
    set_error("mixed_refine must be >= 0");
    return COPA_EINVAL;
  }
  if (opt->order != COPA_ORDER_HWV && opt->order != COPA_ORDER_WHV) {
    set_error("unknown block order");
    return COPA_EINVAL;
  }
  return COPA_OK;
}

copa_status copa_workspace_bytes(const copa_tensor *X, const copa_options *opt, size_t *bytes) {
  if (!bytes) {
    set_error("bytes is NULL");
    return COPA_EINVAL;
  }
  COPA_TRY(check_args(X, opt, false));
  copa_plan tmp;
  COPA_TRY(plan_dims(X, opt, &tmp));
  COPA_TRY(carve_all(&tmp, true));
  *bytes = tmp.arena_bytes;
  return COPA_OK;
}

copa_status copa_plan_create(const copa_tensor *X, const copa_options *opt, void *workspace,
                             size_t workspace_bytes, void *stream, copa_plan **out) {
  if (!out) {
    set_error("out is NULL");
    return COPA_EINVAL;
  }
  *out = nullptr;
  COPA_TRY(check_args(X, opt, true));
  copa_plan *p = new copa_plan();
  copa_status st = build_plan(X, opt, workspace, workspace_bytes, (hipStream_t)stream, p);
  if (st != COPA_OK) {
    (void)hipDeviceSynchronize();
    free_plan(p);
    return st;
  }
  *out = p;
  return COPA_OK;
}

copa_status copa_plan_basis(copa_plan *p, float *C, int32_t *rank, void *stream) {
  if (!p || p->l == 0) {
    set_error("plan is NULL or has no smoothing basis");
    return COPA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  if (C) {
    // the plan keeps rows of width 8; hand out rows of width l
    COPA_HIP(hipMemcpy2DAsync(C, p->l * sizeof(float), p->C, kLMax * sizeof(float),
                              p->l * sizeof(float), p->S, hipMemcpyDeviceToDevice, s));
  }
  if (rank && p->K > 0)
    COPA_HIP(hipMemcpyAsync(rank, p->rk, p->K * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  return COPA_OK;
}

void copa_plan_destroy(copa_plan *p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  free_plan(p);
}

}  // extern "C"
