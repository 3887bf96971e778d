// Kernels and launch sequence of one outer iteration of COPA (Algorithm 1); included by
// copa_iter.hip and by the per-rank translation units copa_iter_r*.hip.
#pragma once
//
// Row spaces. With smoothing every subject owns l "projected rows" (rows of C_k^T X_k, zero past
// its basis rank); without it the rows are the subject's visit rows. Per row the iteration keeps
//   T : X'_k V row        (Procrustes input, MTTKRP inputs)
//   Q : row of Q_k        (truncated polar factor of X'_k V S_k H^T)
//   M : row of Q_k H S_k  (with the updated H and W; feeds the mode-V MTTKRP and the FIT)
//
// Kernel sequence of one iteration (Algorithm 1; block order H -> W -> V):
//   pass1       stream X once: T rows = C_k^T (X_k V)           (sparse X times V, LDS-staged V)
//   procrustes  per subject: Gram of A_k = T_k S_k H^T on its small side, FP64 Jacobi, Q rows
//   gram(F_H)   F_H = sum_rows q^T (t * w_k)   = Y_(1)(W (.) V)
//   mode_H      G_H = W^TW * V^TV, rho, FP64 Cholesky, inner ADMM on H; then G_W and its Cholesky
//   w_admm      per subject: F_W(k,:) = diag(H^T Y_k V), inner ADMM on W(k,:), M rows
//   gram(W), gram(M)   W^T W and Psi = sum_k S_k H^T Q_k^T Q_k H S_k
//   pass2       stream X again: F_V += x_ij * (c_i M_k)            = Y_(2)(W (.) H)
//   mode_V_prep G_V = H^TH * W^TW, rho, FP64 Cholesky
//   v_admm      inner ADMM on V rows, FIT/penalty/sparsity partials
//   gram(V), finalize  V^T V, FIT = 1 - (|X|^2 - 2<F_V,V> + <Psi, V^T V>) / |X|^2
#include <climits>
#include <type_traits>

#include "copa_common.h"
#include "copa_kernels.h"

namespace copa {

#define COPA_R_LIST(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(15) X(16) X(20) X(24) X(32) X(40)



// small-buffer layout (FP64 R x R each)
enum { kFH = 0, kHtH = 1, kWtW = 2, kVtV = 3, kPsi = 4 };

// ======================================================================= streaming pass 1
// Persistent blocks of 4 waves; each block stages one column tile of V (kept padded to RTP
// columns per row by the V update) in LDS once, then its waves walk the wave list: each wave takes
// `cnt` subjects and G lanes per subject stride over the subject's visit rows.
template <int RT, bool SMOOTH, bool COMPACT>
__global__ void __launch_bounds__(256)
    k_pass1(const WaveEntry *__restrict__ waves, int n_waves, const int32_t *__restrict__ order,
            const int32_t *__restrict__ subj, const int32_t *__restrict__ row,
            const int32_t *__restrict__ col, const float *__restrict__ val,
            const uint32_t *__restrict__ xc,
            const float *__restrict__ C, const float *__restrict__ Vp, int64_t J, int R, int l,
            int cg, float *__restrict__ T, float *__restrict__ FV, FitScalars *sc) {
  constexpr int RTP = row4(RT);
  extern __shared__ float4 smem4[];
  // pass 1 opens an outer iteration: advance the device iteration index (no other launch of the
  // iteration reads it before pass 1 ends)
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) sc->cur += 1;
  // F_V is accumulated by pass 2 of this iteration: clear it here
  if (blockIdx.y == 0)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < J * R;
         e += (int64_t)gridDim.x * blockDim.x)
      FV[e] = 0.0f;
  {
    // stage the block's cg tiles with 8 loads in flight per thread
    const float4 *src = reinterpret_cast<const float4 *>(Vp + (int64_t)blockIdx.y * cg * J * RTP);
    const int64_t n4 = cg * J * RTP / 4;
    for (int64_t e0 = 0; e0 < n4; e0 += 8 * (int64_t)blockDim.x) {
      float4 tmp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = e0 + u * blockDim.x + threadIdx.x;
        tmp[u] = src[e < n4 ? e : 0];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        // out-of-range lanes write the spare slot after the tile (no branch, so that the 8 loads
        // above stay in flight together)
        const int64_t e = e0 + u * blockDim.x + threadIdx.x;
        smem4[e < n4 ? e : n4] = tmp[u];
      }
    }
  }
  __syncthreads();
  // lane group cgi of 64 / cg lanes works on tile blockIdx.y * cg + cgi
  const int lane = threadIdx.x & 63;
  const int lpg = 64 / cg, cgi = lane / lpg, lgl = lane - cgi * lpg;
  const float *sV = reinterpret_cast<const float *>(smem4) + (int64_t)cgi * J * RTP;
  const int c0 = (blockIdx.y * cg + cgi) * RT;
  for (int wv = blockIdx.x * 4 + (threadIdx.x >> 6); wv < n_waves; wv += gridDim.x * 4) {
    const WaveEntry we = waves[wv];
    const int lg = we.lg_count & 255, cnt = we.lg_count >> 8;
    const int G = 1 << lg, sidx = lgl >> lg, sub = lgl & (G - 1);
    const bool active = sidx < cnt;
    const int k = active ? order[we.first + sidx] : 0;
    const int r0 = active ? subj[k] : 0, r1 = active ? subj[k + 1] : 0;
    if constexpr (SMOOTH) {
      float acc[kLMax][RT];
#pragma unroll
      for (int a = 0; a < kLMax; ++a)
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[a][r] = 0.0f;
      // two-stage pipeline over this lane's rows: the next row's bounds and basis row are
      // requested while the current row's nonzeros are loaded and used
      int i = r0 + sub;
      int e0n = 0, e1n = 0;
      float4 can = make_float4(0.f, 0.f, 0.f, 0.f), cbn = can;
      if (i < r1) {
        e0n = row[i];
        e1n = row[i + 1];
        const float4 *c4 = reinterpret_cast<const float4 *>(C + (int64_t)i * kLMax);
        can = c4[0];
        cbn = c4[1];
      }
      for (; i < r1; i += G) {
        const int e0 = e0n, e1 = e1n;
        const float4 ca = can, cb = cbn;
        {
          const int in = i + G < r1 ? i + G : r1 - 1;  // always a valid row of this subject
          e0n = row[in];
          e1n = row[in + 1];
          const float4 *c4 = reinterpret_cast<const float4 *>(C + (int64_t)in * kLMax);
          can = c4[0];
          cbn = c4[1];
        }
        float t[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) t[r] = 0.0f;
        for (int eb = e0; eb < e1; eb += 8) {
          int cj[8];
          float xv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const bool ok = eb + u < e1;
            const unsigned ec = (unsigned)(ok ? eb + u : e0);
            if constexpr (COMPACT) {
              const uint32_t w = xc[ec];
              cj[u] = (int)(w & 0xffffu);
              xv[u] = ok ? __uint_as_float(w & 0xffff0000u) : 0.0f;
            } else {
              cj[u] = col[ec];
              const float x = val[ec];
              xv[u] = ok ? x : 0.0f;
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            // a slot that no lane of the wavefront uses is skipped (no LDS gathers)
            if (u == 0 || eb + u < e1) {
              const float x = xv[u];
              float v[RT];
              lds_row<RT>(sV + cj[u] * RTP, v);
#pragma unroll
              for (int r = 0; r < RT; ++r) t[r] += x * v[r];
            }
          }
        }
        const float c[kLMax] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
#pragma unroll
        for (int a = 0; a < kLMax; ++a)
#pragma unroll
          for (int r = 0; r < RT; ++r) acc[a][r] += c[a] * t[r];
      }
      // sum over the subject's G lanes (wave-uniform G) by a reduce-scatter: each lane ends
      // with the totals of the elements e = m G + sub of the l x RT block (e = a RT + r; the
      // element list is padded with zeros to a multiple of G), which it stores, so the
      // subject's G lanes write consecutive words
      constexpr int E = kLMax * RT;
      float *dst = T + (int64_t)k * l * R + c0;
      auto scatter_store = [&](auto gc) {
        constexpr int Gc = decltype(gc)::value;
        constexpr int Ep = (E + Gc - 1) / Gc * Gc;
        float v[Ep];
#pragma unroll
        for (int e = 0; e < Ep; ++e) v[e] = e < E ? acc[e / RT][e % RT] : 0.0f;
        reduce_scatter<Ep, Gc>(v, sub);
        if (active) {
#pragma unroll
          for (int m = 0; m < Ep / Gc; ++m) {
            const int e = m * Gc + sub, a = e / RT, r = e - a * RT;
            if (e < E && a < l && c0 + r < R) dst[a * R + r] = v[m];
          }
        }
      };
      switch (lg) {
        case 0: scatter_store(std::integral_constant<int, 1>{}); break;
        case 1: scatter_store(std::integral_constant<int, 2>{}); break;
        case 2: scatter_store(std::integral_constant<int, 4>{}); break;
        case 3: scatter_store(std::integral_constant<int, 8>{}); break;
        case 4: scatter_store(std::integral_constant<int, 16>{}); break;
        case 5: scatter_store(std::integral_constant<int, 32>{}); break;
        default: scatter_store(std::integral_constant<int, 64>{}); break;
      }
    } else if (active) {
      for (int i = r0 + sub; i < r1; i += G) {
        float t[RTP];
#pragma unroll
        for (int r = 0; r < RTP; ++r) t[r] = 0.0f;
        const int e0 = row[i], e1 = row[i + 1];
        for (int eb = e0; eb < e1; eb += 8) {
          int cj[8];
          float xv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const bool ok = eb + u < e1;
            const unsigned ec = (unsigned)(ok ? eb + u : e0);
            if constexpr (COMPACT) {
              const uint32_t w = xc[ec];
              cj[u] = (int)(w & 0xffffu);
              xv[u] = ok ? __uint_as_float(w & 0xffff0000u) : 0.0f;
            } else {
              cj[u] = col[ec];
              const float x = val[ec];
              xv[u] = ok ? x : 0.0f;
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (u == 0 || eb + u < e1) {  // slots no lane uses skip their gathers
              const float x = xv[u];
              float v[RT];
              lds_row<RT>(sV + (int64_t)cj[u] * RTP, v);
#pragma unroll
              for (int r = 0; r < RT; ++r) t[r] += x * v[r];
            }
          }
        }
        float *dst = T + (int64_t)i * R + c0;
#pragma unroll
        for (int r = 0; r < RT; ++r)
          if (c0 + r < R) dst[r] = t[r];
      }
    }
  }
}

// Pass 1 on the projected pairs (smoothed plans with few nonzeros per visit row): the T rows of
// subject k are sum over its pairs (j, x'_j) of x'_j V(j, :)^T, with x'_j the l entries of column j
// of C_k^T X_k. Same persistent blocks, LDS-staged tiles, lane groups and reduce-scatter as
// k_pass1; a lane streams every G-th pair of its subject, four records in flight, with no
// dependent loads (a pair carries its feature id).
template <int RT, int PW, bool BF, int LC = 0>
__global__ void __launch_bounds__(256)
    k_pass1p(const WaveEntry *__restrict__ waves, int n_waves, const int32_t *__restrict__ order,
             const int32_t *__restrict__ pp, const void *__restrict__ recs,
             const float *__restrict__ Vp, int64_t J, int R, int l_in, int cg,
             float *__restrict__ T, float *__restrict__ FV, FitScalars *sc) {
  constexpr int RTP = row4(RT);
  constexpr int LM = LC > 0 ? LC : kLMax;  // basis functions held (LC: l fixed at compile time)
  const int l = LC > 0 ? LC : l_in;
  extern __shared__ float4 smem4[];
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) sc->cur += 1;
  if (blockIdx.y == 0)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < J * R;
         e += (int64_t)gridDim.x * blockDim.x)
      FV[e] = 0.0f;
  {
    const float4 *src = reinterpret_cast<const float4 *>(Vp + (int64_t)blockIdx.y * cg * J * RTP);
    const int64_t n4 = cg * J * RTP / 4;
    for (int64_t e0 = 0; e0 < n4; e0 += 8 * (int64_t)blockDim.x) {
      float4 tmp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = e0 + u * blockDim.x + threadIdx.x;
        tmp[u] = src[e < n4 ? e : 0];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = e0 + u * blockDim.x + threadIdx.x;
        smem4[e < n4 ? e : n4] = tmp[u];
      }
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int lpg = 64 / cg, cgi = lane / lpg, lgl = lane - cgi * lpg;
  const float *sV = reinterpret_cast<const float *>(smem4) + (int64_t)cgi * J * RTP;
  const int c0 = (blockIdx.y * cg + cgi) * RT;
  for (int wv = blockIdx.x * 4 + (threadIdx.x >> 6); wv < n_waves; wv += gridDim.x * 4) {
    const WaveEntry we = waves[wv];
    const int lg = we.lg_count & 255, cnt = we.lg_count >> 8;
    const int G = 1 << lg, sidx = lgl >> lg, sub = lgl & (G - 1);
    const bool active = sidx < cnt;
    const int k = active ? order[we.first + sidx] : 0;
    const int p0 = active ? pp[k] : 0, p1 = active ? pp[k + 1] : 0;
    float acc[LM][RT];
#pragma unroll
    for (int a = 0; a < LM; ++a)
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[a][r] = 0.0f;
    auto take = [&](const float (&f)[PW]) {
      const int j = (int)__float_as_uint(f[PW - 1]);
      float v[RT];
      lds_row<RT>(sV + j * RTP, v);
#pragma unroll
      for (int a = 0; a < LM; ++a)
        if (a < l)
#pragma unroll
          for (int r = 0; r < RT; ++r) acc[a][r] += f[a] * v[r];
    };
    for (int q = p0 + sub; q < p1; q += 4 * G) {
      float f[4][PW];
#pragma unroll
      for (int u = 0; u < 4; ++u) fetch_rec<BF, PW>(recs, nullptr, q + u * G < p1 ? q + u * G : q, f[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q + u * G < p1) take(f[u]);
    }
    constexpr int E = LM * RT;
    float *dst = T + (int64_t)k * l * R + c0;
    auto scatter_store = [&](auto gc) {
      constexpr int Gc = decltype(gc)::value;
      constexpr int Ep = (E + Gc - 1) / Gc * Gc;
      float v[Ep];
#pragma unroll
      for (int e = 0; e < Ep; ++e) v[e] = e < E ? acc[e / RT][e % RT] : 0.0f;
      reduce_scatter<Ep, Gc>(v, sub);
      if (active) {
#pragma unroll
        for (int m = 0; m < Ep / Gc; ++m) {
          const int e = m * Gc + sub, a = e / RT, r = e - a * RT;
          if (e < E && a < l && c0 + r < R) dst[a * R + r] = v[m];
        }
      }
    };
    switch (lg) {
      case 0: scatter_store(std::integral_constant<int, 1>{}); break;
      case 1: scatter_store(std::integral_constant<int, 2>{}); break;
      case 2: scatter_store(std::integral_constant<int, 4>{}); break;
      case 3: scatter_store(std::integral_constant<int, 8>{}); break;
      case 4: scatter_store(std::integral_constant<int, 16>{}); break;
      case 5: scatter_store(std::integral_constant<int, 32>{}); break;
      default: scatter_store(std::integral_constant<int, 64>{}); break;
    }
  }
}

// V (J x R) -> padded column tiles Vp[tile][j][0..RTP) (padding stays zero)
template <int R>
__global__ void k_pad_V(const float *__restrict__ V, float *__restrict__ Vp, int64_t J, int rt,
                        int rtp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J * R) return;
  const int64_t j = e / R;
  const int c = (int)(e - j * R);
  Vp[((int64_t)(c / rt) * J + j) * rtp + c % rt] = V[e];
}

// ======================================================================= Procrustes
// Reciprocal and reciprocal square root in FP64 from the hardware estimates plus two Newton
// steps each (a few ulp; far shorter dependency chains than IEEE division and sqrt).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
// Jacobi rotation of the pair (p, q): t = tan(theta) of the smaller angle that annihilates
// a_pq, c = cos(theta), s = sin(theta). |tau| < 1e17 because a_pq is above the threshold, so
// 1 + tau^2 does not overflow.
__device__ __forceinline__ void jacobi_cs(double app, double aqq, double apq, double &t, double &c,
                                          double &s) {
  const double tau = (aqq - app) * rcp_nr(2.0 * apq);
  const double x = fma(tau, tau, 1.0);
  const double h = x * rsq_nr(x);  // sqrt(1 + tau^2)
  t = copysign(rcp_nr(fabs(tau) + h), tau);
  c = rsq_nr(fma(t, t, 1.0));
  s = t * c;
}

// Symmetric eigenproblem of size <= kNMax in registers (cyclic Jacobi, FP64). A is stored as a
// full array but only compile-time indices are used; on return A's diagonal holds the
// eigenvalues and V the eigenvectors (columns).
__device__ __forceinline__ void jacobi8(double (&A)[kNMax][kNMax], double (&V)[kNMax][kNMax]) {
#pragma unroll
  for (int i = 0; i < kNMax; ++i)
#pragma unroll
    for (int j = 0; j < kNMax; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  double scale = 0.0;
#pragma unroll
  for (int i = 0; i < kNMax; ++i) scale += fabs(A[i][i]);
  const double tiny = 1e-300 + 1e-17 * scale;
  for (int sweep = 0; sweep < 16; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int p = 0; p < kNMax - 1; ++p) {
#pragma unroll
      for (int q = p + 1; q < kNMax; ++q) {
        const double apq = A[p][q];
        if (fabs(apq) > tiny) {
          rotated = true;
          double t, c, s;
          jacobi_cs(A[p][p], A[q][q], apq, t, c, s);
#pragma unroll
          for (int k = 0; k < kNMax; ++k) {
            if (k == p || k == q) continue;
            const double akp = A[k][p], akq = A[k][q];
            const double nkp = c * akp - s * akq, nkq = s * akp + c * akq;
            A[k][p] = nkp;
            A[p][k] = nkp;
            A[k][q] = nkq;
            A[q][k] = nkq;
          }
          A[p][p] -= t * apq;
          A[q][q] += t * apq;
          A[p][q] = 0.0;
          A[q][p] = 0.0;
#pragma unroll
          for (int k = 0; k < kNMax; ++k) {
            const double vkp = V[k][p], vkq = V[k][q];
            V[k][p] = c * vkp - s * vkq;
            V[k][q] = s * vkp + c * vkq;
          }
        }
      }
    }
    if (!rotated) break;
  }
}

// Eigensolver on a packed upper triangle (N (N + 1) / 2 values), for the register-resident path;
// N is the padded problem size.
template <int N>
__host__ __device__ constexpr int triN(int i, int j) {
  return i <= j ? N * i - (i * (i - 1)) / 2 + (j - i) : N * j - (j * (j - 1)) / 2 + (i - j);
}

// Round-robin ("circle") order of the index pairs: with M players (N rounded up to even; an odd N
// adds one that sits out), round r pairs r with M - 1 and (r + m) with (r - m) mod (M - 1) for
// m = 1 .. M/2 - 1. Every pair meets once in M - 1 rounds and the pairs of a round are disjoint.
__host__ __device__ constexpr int rr_lo(int M, int r, int m) {
  const int a = m == 0 ? r : (r + m) % (M - 1), b = m == 0 ? M - 1 : (r - m + (M - 1)) % (M - 1);
  return a < b ? a : b;
}
__host__ __device__ constexpr int rr_hi(int M, int r, int m) {
  const int a = m == 0 ? r : (r + m) % (M - 1), b = m == 0 ? M - 1 : (r - m + (M - 1)) % (M - 1);
  return a < b ? b : a;
}

// Cyclic Jacobi in round-robin order. On entry V holds an orthogonal matrix and A = V^T G V; the
// rotations are accumulated onto V, so on return V holds the eigenvectors of G and A's diagonal
// its eigenvalues. The rotations of one round act on disjoint index pairs, so they commute: their
// angles are all taken from the matrix at the start of the round (independent dependency chains
// for the scheduler) and then applied one after the other. No branches: a pair whose entry is at
// or below the threshold gets the identity rotation. The sweep loop ends for the whole wavefront
// once no lane has an off-diagonal entry above the threshold.
template <int N>
__device__ __forceinline__ void jacobi_rr(double (&A)[N * (N + 1) / 2], double (&V)[N][N]) {
  constexpr int M = N + (N & 1);
  constexpr int P = M / 2;
  double scale = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) scale += fabs(A[triN<N>(i, i)]);
  const double tiny = 1e-300 + 1e-17 * scale;
  for (int sweep = 0; sweep < 16; ++sweep) {
    bool big = false;
#pragma unroll
    for (int p = 0; p < N - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < N; ++q) big = big || fabs(A[triN<N>(p, q)]) > tiny;
    if (!__any(big)) break;
#pragma unroll
    for (int r = 0; r < M - 1; ++r) {
      double tt[P], cc[P], ss[P];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        const int p = rr_lo(M, r, m), q = rr_hi(M, r, m);
        if (q >= N) continue;
        const double apq = A[triN<N>(p, q)];
        const bool on = fabs(apq) > tiny;
        double t, c, s;
        jacobi_cs(A[triN<N>(p, p)], A[triN<N>(q, q)], on ? apq : 1.0, t, c, s);
        tt[m] = on ? t : 0.0;
        cc[m] = on ? c : 1.0;
        ss[m] = on ? s : 0.0;
      }
#pragma unroll
      for (int m = 0; m < P; ++m) {
        const int p = rr_lo(M, r, m), q = rr_hi(M, r, m);
        if (q >= N) continue;
        const double t = tt[m], c = cc[m], s = ss[m];
        const double apq = A[triN<N>(p, q)];
#pragma unroll
        for (int k = 0; k < N; ++k) {
          if (k == p || k == q) continue;
          const double akp = A[triN<N>(k, p)], akq = A[triN<N>(k, q)];
          A[triN<N>(k, p)] = c * akp - s * akq;
          A[triN<N>(k, q)] = s * akp + c * akq;
        }
        A[triN<N>(p, p)] -= t * apq;
        A[triN<N>(q, q)] += t * apq;
        A[triN<N>(p, q)] = t != 0.0 ? 0.0 : apq;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

// E <- E (3 I - E^T E) / 2: one Newton-Schulz step towards the nearest orthogonal matrix, taking
// an FP32-rounded orthogonal matrix (deviation ~1e-7) to FP64 orthogonality (~1e-14).
template <int N>
__device__ __forceinline__ void orthonormalize(double (&E)[N][N]) {
  double Nm[N * (N + 1) / 2];
#pragma unroll
  for (int p = 0; p < N; ++p)
#pragma unroll
    for (int q = p; q < N; ++q) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) s += E[i][p] * E[i][q];
      Nm[triN<N>(p, q)] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double r[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < N; ++p) s += E[i][p] * Nm[triN<N>(p, q)];
      r[q] = 1.5 * E[i][q] - 0.5 * s;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) E[i][q] = r[q];
  }
}

static __global__ void k_eye8(float *__restrict__ Ew, int64_t K) {
  const int64_t n = K * kNMax * kNMax;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ent = e / K;
    Ew[e] = (ent / kNMax == ent % kNMax) ? 1.0f : 0.0f;
  }
}

// One subject per lane, eigenproblem size n = min(m, R) <= kNMax.
// A rows a_i = (t_i * w) H^T are computed in FP64 and kept as FP32 in the M buffer (free until
// the W update). Rows side (m <= R): Gram A A^T, Q = (A A^T)^{+1/2} A. Columns side (m > R):
// Gram A^T A, Q = A (A^T A)^{+1/2}. Eigenvalues at or below rtol^2 * lambda_max are dropped.
template <int R>
__global__ void __launch_bounds__(64)
    k_procrustes(int64_t K, int l, const int32_t *__restrict__ subj,
                 const int32_t *__restrict__ rk, const float *__restrict__ T,
                 float *__restrict__ Q, float *__restrict__ Abuf, const float *__restrict__ H,
                 const float *__restrict__ W, double rtol, FitScalars *sc) {
  __shared__ float sH[R * R];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sH[e] = H[e];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  int64_t base;
  int m, meff;
  if (l > 0) {
    base = k * l;
    m = l;
    meff = rk[k];
  } else {
    base = subj[k];
    m = subj[k + 1] - subj[k];
    meff = m;
  }
  if ((m < R ? m : R) > kNMax) return;  // one wavefront per subject handles these
  float w[R];
#pragma unroll
  for (int r = 0; r < R; ++r) w[r] = W[k * R + r];
  const bool rows_side = m <= R;
  double G[kNMax][kNMax];
#pragma unroll
  for (int i = 0; i < kNMax; ++i)
#pragma unroll
    for (int j = 0; j < kNMax; ++j) G[i][j] = 0.0;
  // stage 1: A rows; columns-side Gram on the fly
  for (int i = 0; i < m; ++i) {
    const float *t = T + (base + i) * R;
    float z[R];
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = t[r] * w[r];
    float a[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) s += (double)z[r] * (double)sH[c * R + r];
      a[c] = (float)s;
    }
    float *dst = Abuf + (base + i) * R;
#pragma unroll
    for (int c = 0; c < R; ++c) dst[c] = a[c];
    if (!rows_side) {
#pragma unroll
      for (int p = 0; p < kNMax; ++p)
#pragma unroll
        for (int q = 0; q < kNMax; ++q)
          if (p < R && q < R && q >= p) G[p][q] += (double)a[p < R ? p : 0] * a[q < R ? q : 0];
    }
  }
  if (rows_side) {
#pragma unroll
    for (int p = 0; p < kNMax; ++p) {
      if (p < m) {
        const float *ap = Abuf + (base + p) * R;
#pragma unroll
        for (int q = 0; q < kNMax; ++q) {
          if (q >= p && q < m) {
            const float *aq = Abuf + (base + q) * R;
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < R; ++c) s += (double)ap[c] * aq[c];
            G[p][q] = s;
          }
        }
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kNMax; ++p)
#pragma unroll
    for (int q = 0; q < p; ++q) G[p][q] = G[q][p];
  double E[kNMax][kNMax];
  jacobi8(G, E);
  double lmax = 0.0;
#pragma unroll
  for (int j = 0; j < kNMax; ++j) lmax = fmax(lmax, G[j][j]);
  double f[kNMax];
  int rank = 0;
#pragma unroll
  for (int j = 0; j < kNMax; ++j) {
    const bool keep = lmax > 0.0 && G[j][j] > rtol * rtol * lmax;
    f[j] = keep ? 1.0 / sqrt(G[j][j]) : 0.0;
    rank += keep ? 1 : 0;
  }
  // B = E diag(f) E^T  (overwrite G)
#pragma unroll
  for (int i = 0; i < kNMax; ++i)
#pragma unroll
    for (int j = 0; j < kNMax; ++j) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kNMax; ++q) s += E[i][q] * f[q] * E[j][q];
      G[i][j] = s;
    }
  if (rows_side) {
    // q_i = sum_j B(i,j) a_j
#pragma unroll
    for (int i = 0; i < kNMax; ++i) {
      if (i < m) {
        double acc[R];
#pragma unroll
        for (int c = 0; c < R; ++c) acc[c] = 0.0;
#pragma unroll
        for (int j = 0; j < kNMax; ++j) {
          if (j < m) {
            const float *aj = Abuf + (base + j) * R;
            const double b = G[i][j];
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] += b * aj[c];
          }
        }
        float *dst = Q + (base + i) * R;
#pragma unroll
        for (int c = 0; c < R; ++c) dst[c] = (float)acc[c];
      }
    }
  } else {
    for (int i = 0; i < m; ++i) {
      const float *ai = Abuf + (base + i) * R;
      float a[R];
#pragma unroll
      for (int c = 0; c < R; ++c) a[c] = ai[c];
      float *dst = Q + (base + i) * R;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < kNMax; ++j)
          if (j < R) s += (double)a[j < R ? j : 0] * G[j][c < kNMax ? c : 0];
        dst[c] = (float)s;
      }
    }
  }
  if (rank < (meff < R ? meff : R)) atomicAdd(&sc->rank_def_slot[sc->cur & 1], 1);
}

// Unsmoothed subjects whose eigenproblem n = min(I_k, R) exceeds what a lane holds: one
// wavefront per subject, n x n Gram and eigenvectors in LDS (FP64), cyclic Jacobi with every lane
// updating one row/column per rotation. Rows side (I_k <= R): A = T S H^T (I_k x R) in LDS,
// Gram A A^T, Q = B A. Columns side (I_k > R): Gamma = sum_i t_i^T t_i streamed, Gram
// H S Gamma S H^T, N = S H^T B and Q rows q_i = t_i N.
template <int R>
__global__ void __launch_bounds__(64)
    k_procrustes_wave(const int32_t *__restrict__ list, int nlist,
                      const int32_t *__restrict__ subj, const float *__restrict__ T,
                      float *__restrict__ Q, const float *__restrict__ H,
                      const float *__restrict__ W, double rtol, FitScalars *sc) {
  __shared__ double sG[R * R];
  __shared__ double sE[R * R];
  __shared__ double sA[R * R];  // A (rows side) or Gamma, then N (columns side)
  __shared__ double sw[R];
  __shared__ double sf[R];
  __shared__ float sH[R * R];
  const int lane = threadIdx.x;
  if ((int)blockIdx.x >= nlist) return;
  const int k = list[blockIdx.x];
  const int r0 = subj[k], m = subj[k + 1] - r0;
  const bool rows_side = m <= R;
  const int n = rows_side ? m : R;
  for (int e = lane; e < R * R; e += 64) sH[e] = H[e];
  for (int e = lane; e < R; e += 64) sw[e] = W[(int64_t)k * R + e];
  __syncthreads();
  if (rows_side) {
    // A(i, c) = sum_r t_i[r] w_r H(c, r)
    for (int e = lane; e < m * R; e += 64) {
      const int i = e / R, c = e % R;
      const float *t = T + (int64_t)(r0 + i) * R;
      double s = 0.0;
      for (int r = 0; r < R; ++r) s += (double)t[r] * sw[r] * (double)sH[c * R + r];
      sA[i * R + c] = (double)(float)s;
    }
    __syncthreads();
    for (int e = lane; e < n * n; e += 64) {
      const int p = e / n, q = e % n;
      double s = 0.0;
      for (int c = 0; c < R; ++c) s += sA[p * R + c] * sA[q * R + c];
      sG[p * n + q] = s;
    }
  } else {
    // Gamma = T^T T (lane a owns row a), then Z = Gamma o (w w^T) and G = H Z H^T
    double acc[R];
    for (int b = 0; b < R; ++b) acc[b] = 0.0;
    for (int i = 0; i < m; ++i) {
      const float *t = T + (int64_t)(r0 + i) * R;
      const double ta = lane < R ? (double)t[lane] : 0.0;
#pragma unroll
      for (int b = 0; b < R; ++b) acc[b] += ta * (double)t[b];
    }
    if (lane < R)
      for (int b = 0; b < R; ++b) sA[lane * R + b] = acc[b] * sw[lane] * sw[b];
    __syncthreads();
    // sE <- H Z
    for (int e = lane; e < R * R; e += 64) {
      const int a = e / R, b = e % R;
      double s = 0.0;
      for (int c = 0; c < R; ++c) s += (double)sH[a * R + c] * sA[c * R + b];
      sE[e] = s;
    }
    __syncthreads();
    for (int e = lane; e < R * R; e += 64) {
      const int a = e / R, b = e % R;
      double s = 0.0;
      for (int c = 0; c < R; ++c) s += sE[a * R + c] * (double)sH[b * R + c];
      sG[a * R + b] = s;
    }
  }
  __syncthreads();
  for (int e = lane; e < n * n; e += 64) sE[e] = (e / n == e % n) ? 1.0 : 0.0;
  double scale = 0.0;
  for (int i = 0; i < n; ++i) scale += fabs(sG[i * n + i]);
  const double tiny = 1e-300 + 1e-17 * scale;
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = sG[p * n + q];
        if (fabs(apq) > tiny) {
          rotated = true;
          const double app = sG[p * n + p], aqq = sG[q * n + q];
          double t, c, s;
          jacobi_cs(app, aqq, apq, t, c, s);
          __syncthreads();
          if (lane < n && lane != p && lane != q) {
            const double gkp = sG[lane * n + p], gkq = sG[lane * n + q];
            const double np_ = c * gkp - s * gkq, nq_ = s * gkp + c * gkq;
            sG[lane * n + p] = np_;
            sG[p * n + lane] = np_;
            sG[lane * n + q] = nq_;
            sG[q * n + lane] = nq_;
          }
          if (lane < n) {
            const double vkp = sE[lane * n + p], vkq = sE[lane * n + q];
            sE[lane * n + p] = c * vkp - s * vkq;
            sE[lane * n + q] = s * vkp + c * vkq;
          }
          if (lane == 0) {
            sG[p * n + p] = app - t * apq;
            sG[q * n + q] = aqq + t * apq;
            sG[p * n + q] = 0.0;
            sG[q * n + p] = 0.0;
          }
          __syncthreads();
        }
      }
    }
    if (!rotated) break;
  }
  double lmax = 0.0;
  for (int j = 0; j < n; ++j) lmax = fmax(lmax, sG[j * n + j]);
  int rank = 0;
  for (int j = 0; j < n; ++j) rank += (lmax > 0.0 && sG[j * n + j] > rtol * rtol * lmax) ? 1 : 0;
  if (lane < n) {
    const double lj = sG[lane * n + lane];
    sf[lane] = (lmax > 0.0 && lj > rtol * rtol * lmax) ? 1.0 / sqrt(lj) : 0.0;
  }
  __syncthreads();
  // B = E diag(f) E^T (n x n) into sG
  for (int e = lane; e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int q = 0; q < n; ++q) s += sE[i * n + q] * sf[q] * sE[j * n + q];
    sG[e] = s;
  }
  __syncthreads();
  if (rows_side) {
    // Q = B A
    for (int e = lane; e < m * R; e += 64) {
      const int i = e / R, c = e % R;
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += sG[i * n + j] * sA[j * R + c];
      Q[(int64_t)(r0 + i) * R + c] = (float)s;
    }
  } else {
    // N = S H^T B (R x R) into sA, then q_i = t_i N
    for (int e = lane; e < R * R; e += 64) {
      const int a = e / R, b = e % R;
      double s = 0.0;
      for (int c = 0; c < R; ++c) s += (double)sH[c * R + a] * sG[c * R + b];
      sA[e] = sw[a] * s;
    }
    __syncthreads();
    for (int i = 0; i < m; ++i) {
      const float *t = T + (int64_t)(r0 + i) * R;
      if (lane < R) {
        double s = 0.0;
        for (int r = 0; r < R; ++r) s += (double)t[r] * sA[r * R + lane];
        Q[(int64_t)(r0 + i) * R + lane] = (float)s;
      }
    }
  }
  if (lane == 0 && rank < (m < R ? m : R)) atomicAdd(&sc->rank_def_slot[sc->cur & 1], 1);
}

// Smoothed subjects (l <= N <= 8 projected rows) with R <= 16: one subject per lane, the
// eigenproblem in registers, A in LDS (FP64 where it fits), H in LDS as FP64 (N = l = 7 is the
// usual instance, N = 8 the general one; rows at or past l are zero). The 64 subjects of a block
// own one contiguous run of T rows and of Q rows, so both move through LDS (the A area, before
// and after A is live) with coalesced 16-byte loads and stores instead of each lane touching its
// own rows in memory. LDS stays at or below 40 KB, so four blocks fit a compute unit and a
// 50,000-subject launch is resident at once.
template <int R, int N>
struct ProcS {
  static constexpr bool kDoubleA = N * R * 64 * 8 + R * R * 8 <= 40960;
  using AT = std::conditional_t<kDoubleA, double, float>;
};

// dst[0, n) = src[0, n) by the 64 lanes of one wavefront, 16 bytes per lane per step with up to
// 8 steps in flight; both pointers 16-byte aligned
__device__ __forceinline__ void copy_run(float *__restrict__ dst, const float *__restrict__ src,
                                         int n, int lane) {
  const int n4 = n >> 2;
  const float4 *s4 = reinterpret_cast<const float4 *>(src);
  float4 *d4 = reinterpret_cast<float4 *>(dst);
  for (int e0 = 0; e0 < n4; e0 += 8 * 64) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 64 + lane;
      v[u] = s4[e < n4 ? e : 0];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 64 + lane;
      if (e < n4) d4[e] = v[u];
    }
  }
  for (int e = 4 * n4 + lane; e < n; e += 64) dst[e] = src[e];
}

template <int R, int N>
__global__ void __launch_bounds__(64)
    k_procrustes_s(int64_t K, int l, const int32_t *__restrict__ rk, const float *__restrict__ T,
                   float *__restrict__ Q, const float *__restrict__ H, const float *__restrict__ W,
                   float *__restrict__ Ew, double rtol, FitScalars *sc) {
  using AT = typename ProcS<R, N>::AT;
  constexpr int NT = N * (N + 1) / 2;
  __shared__ double sH[R * R];
  // A of this lane's subject, element (i, c) at (i R + c) 64 + lane; before that the block's T
  // rows and afterwards its Q rows (64 l R <= 64 N R floats)
  __shared__ __align__(16) AT sA[N * R * 64];
  float *sTQ = reinterpret_cast<float *>(sA);
  const int lane = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * 64;
  const int nsub = (int)(K - k0 < 64 ? K - k0 : 64);
  for (int e = lane; e < R * R; e += blockDim.x) sH[e] = (double)H[e];
  copy_run(sTQ, T + k0 * l * R, nsub * l * R, lane);
  __syncthreads();
  // lanes past the last subject redo the block's first subject and store nothing
  const bool live = lane < nsub;
  const int tl = live ? lane : 0;
  const int64_t k = k0 + tl;
  {
    float tv[N][R];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) tv[i][r] = sTQ[(tl * l + (i < l ? i : 0)) * R + r];
    __syncthreads();  // the T rows are in registers: the area takes A from here on
    float w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) w[r] = W[k * R + r];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double z[R];
#pragma unroll
      for (int r = 0; r < R; ++r) z[r] = (double)(tv[i][r] * w[r]);
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) s += z[r] * sH[c * R + r];
        sA[(i * R + c) * 64 + lane] = i < l ? (AT)s : (AT)0;
      }
    }
  }
  auto Aat = [&](int i, int c) -> double { return (double)sA[(i * R + c) * 64 + lane]; };
  const bool rows_side = l <= R;
  // Warm start: the Gram's eigenvectors change little between outer iterations, so the Jacobi
  // sweeps run on E^T G E with E = last iteration's eigenvectors (identity on the first), made
  // orthogonal to FP64 precision first. G = A A^T (rows side) or A^T A (columns side) is summed
  // from the rotated vectors E^T v over the columns (rows) v of A.
  double E[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) E[i][j] = (double)Ew[(int64_t)(i * kNMax + j) * K + k];
  orthonormalize<N>(E);
  double G[NT];
#pragma unroll
  for (int e = 0; e < NT; ++e) G[e] = 0.0;
  const int nv = rows_side ? R : N;
  for (int c = 0; c < nv; ++c) {
    double v[N], a[N];
#pragma unroll
    for (int p = 0; p < N; ++p) v[p] = rows_side ? Aat(p, c) : (p < R ? Aat(c, p) : 0.0);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double s = 0.0;
#pragma unroll
      for (int p = 0; p < N; ++p) s += E[p][q] * v[p];
      a[q] = s;
    }
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
      for (int q = p; q < N; ++q) G[triN<N>(p, q)] += a[p] * a[q];
  }
  jacobi_rr<N>(G, E);
  if (live) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) Ew[(int64_t)(i * kNMax + j) * K + k] = (float)E[i][j];
  }
  double lmax = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) lmax = fmax(lmax, G[triN<N>(j, j)]);
  double f[N];
  int rank = 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double lj = G[triN<N>(j, j)];
    const bool keep = lmax > 0.0 && lj > rtol * rtol * lmax;
    f[j] = keep ? rsq_nr(lj) : 0.0;
    rank += keep ? 1 : 0;
  }
  // B = E diag(f) E^T (symmetric) into the triangle
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < N; ++q) s += E[i][q] * f[q] * E[j][q];
      G[triN<N>(i, j)] = s;
    }
  float qv[N][R];
  if (rows_side) {
    // Q = B A, one column of A at a time
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double a[N];
#pragma unroll
      for (int j = 0; j < N; ++j) a[j] = Aat(j, c);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) s += G[triN<N>(i, j)] * a[j];
        qv[i][c] = (float)s;
      }
    }
  } else {
    // Q = A B (B is R x R, padded to N with zero rows and columns), one row of A at a time
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double a[N];
#pragma unroll
      for (int j = 0; j < N; ++j) a[j] = j < R ? Aat(i, j < R ? j : 0) : 0.0;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double s = 0.0;
        if (c < N) {
#pragma unroll
          for (int j = 0; j < N; ++j) s += a[j] * G[triN<N>(j, c < N ? c : 0)];
        }
        qv[i][c] = (float)s;
      }
    }
  }
  const int meff = rk[k];
  if (live && rank < (meff < R ? meff : R)) atomicAdd(&sc->rank_def_slot[sc->cur & 1], 1);
  __syncthreads();  // A is consumed: the area takes the Q rows
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i < l)
#pragma unroll
      for (int c = 0; c < R; ++c) sTQ[(lane * l + i) * R + c] = qv[i][c];
  __syncthreads();
  copy_run(Q + k0 * l * R, sTQ, nsub * l * R, lane);
}

// Smoothed subjects (l <= N <= 8 projected rows) with R > 16: one subject per lane, working on
// the subject's l x R block in LDS, which it transforms in place into the subject's Q rows:
//   Y = T_k S_k                                    (the rows scaled by W(k,:))
//   G = Y (H^T H) Y^T = A_k A_k^T                  (FP64; A_k = T_k S_k H^T)
//   G = E diag(lambda) E^T                         (FP64 Jacobi, warm-started from the last E)
//   P = B Y,  B = E diag(f) E^T,  f = lambda^{-1/2} on the kept eigenvalues   (column by column)
//   Q = P H^T = B A_k                              (row by row)
// Each lane's rows sit at a stride of l R + 1 words (odd, so the 64 lanes of a wavefront touch 64
// different banks); registers hold at most one R-long row beside the triangle of G and E. The
// block's T rows arrive, and its Q rows leave, as one contiguous run with coalesced accesses.
template <int R, int N>
__global__ void __launch_bounds__(64)
    k_procrustes_l(int64_t K, int l_arg, const int32_t *__restrict__ rk,
                   const float *__restrict__ T, float *__restrict__ Q, const float *__restrict__ H,
                   const float *__restrict__ W, float *__restrict__ Ew, double rtol,
                   FitScalars *sc) {
  constexpr int NT = N * (N + 1) / 2;
  const int l = l_arg;
  extern __shared__ double smem_d[];
  double *sHH = smem_d;                                       // H^T H, FP64
  float *sH = reinterpret_cast<float *>(smem_d + R * R);      // H, FP32
  float *sX = sH + R * R;                                     // 64 per-lane blocks
  const int lR = l * R, stride = lR + 1;
  // element f of the block's run sits at f + f / lR in sX (one pad word per lane block); the
  // quotient comes from a float reciprocal and one correction step (f < 2^24)
  const float inv_lR = 1.0f / (float)lR;
  auto at = [&](int f) {
    int q = (int)((float)f * inv_lR);
    const int r = f - q * lR;
    q += (r >= lR) - (r < 0);
    return f + q;
  };
  const int lane = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * 64;
  const int nsub = (int)(K - k0 < 64 ? K - k0 : 64);
  for (int e = lane; e < R * R; e += 64) sH[e] = H[e];
  {
    // contiguous run of nsub l R floats -> per-lane blocks (lanes past nsub get zeros), eight
    // loads in flight per lane
    const float *src = T + k0 * lR;
    const int n = nsub * lR, total = 64 * lR;
    for (int e0 = 0; e0 < total; e0 += 8 * 64) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 64 + lane;
        v[u] = e < n ? src[e] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 64 + lane;
        if (e < total) sX[at(e)] = v[u];
      }
    }
  }
  __syncthreads();
  for (int e = lane; e < R * R; e += 64) {
    const int a = e / R, b = e - a * R;
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += (double)sH[r * R + a] * (double)sH[r * R + b];
    sHH[e] = s;
  }
  const bool live = lane < nsub;
  const int64_t k = k0 + (live ? lane : 0);
  float *x = sX + lane * stride;
  __syncthreads();  // H^T H complete
  {
    float w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) w[r] = W[k * R + r];
#pragma unroll 1
    for (int i = 0; i < l; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) x[i * R + r] *= w[r];
  }
  // G = Y (H^T H) Y^T, one row z_j = y_j (H^T H) at a time
  double G[NT];
#pragma unroll
  for (int e = 0; e < NT; ++e) G[e] = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (j < l) {
      double z[R];
#pragma unroll
      for (int c = 0; c < R; ++c) z[c] = 0.0;
#pragma unroll 1
      for (int r = 0; r < R; ++r) {
        const double y = (double)x[j * R + r];
        const double *hh = sHH + r * R;
#pragma unroll
        for (int c = 0; c < R; ++c) z[c] = fma(y, hh[c], z[c]);
      }
#pragma unroll
      for (int i = 0; i <= j; ++i) {
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < R; ++c) s = fma((double)x[i * R + c], z[c], s);
        G[triN<N>(i, j)] = s;
      }
    }
  }
  // warm start: G' = E^T G E with E = last iteration's eigenvectors made orthogonal in FP64
  double E[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) E[i][j] = (double)Ew[(int64_t)(i * kNMax + j) * K + k];
  orthonormalize<N>(E);
  {
    double GE[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int q = 0; q < N; ++q) {
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < N; ++p) s = fma(G[triN<N>(i, p)], E[p][q], s);
        GE[i][q] = s;
      }
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
      for (int q = p; q < N; ++q) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) s = fma(E[i][p], GE[i][q], s);
        G[triN<N>(p, q)] = s;
      }
  }
  jacobi_rr<N>(G, E);
  if (live) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) Ew[(int64_t)(i * kNMax + j) * K + k] = (float)E[i][j];
  }
  double lmax = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) lmax = fmax(lmax, G[triN<N>(j, j)]);
  double f[N];
  int rank = 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double lj = G[triN<N>(j, j)];
    const bool keep = lmax > 0.0 && lj > rtol * rtol * lmax;
    f[j] = keep ? rsq_nr(lj) : 0.0;
    rank += keep ? 1 : 0;
  }
  // B = E diag(f) E^T into the triangle
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < N; ++q) s += E[i][q] * f[q] * E[j][q];
      G[triN<N>(i, j)] = s;
    }
  // P = B Y, column by column
#pragma unroll 1
  for (int r = 0; r < R; ++r) {
    double v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = i < l ? (double)x[i * R + r] : 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (i < l) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) s = fma(G[triN<N>(i, j)], v[j], s);
        x[i * R + r] = (float)s;
      }
  }
  // Q rows = P H^T, row by row
#pragma unroll 1
  for (int i = 0; i < l; ++i) {
    float p[R];
#pragma unroll
    for (int r = 0; r < R; ++r) p[r] = x[i * R + r];
#pragma unroll 1
    for (int c = 0; c < R; ++c) {
      const float *h = sH + c * R;
      float s = 0.0f;
#pragma unroll
      for (int r = 0; r < R; ++r) s = fmaf(p[r], h[r], s);
      x[i * R + c] = s;
    }
  }
  const int meff = rk[k];
  if (live && rank < (meff < R ? meff : R)) atomicAdd(&sc->rank_def_slot[sc->cur & 1], 1);
  __syncthreads();
  {
    float *dst = Q + k0 * lR;
    const int n = nsub * lR;
    for (int e0 = 0; e0 < n; e0 += 8 * 64) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 64 + lane;
        v[u] = e < n ? sX[at(e)] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 64 + lane;
        if (e < n) dst[e] = v[u];
      }
    }
  }
}

// Smoothed subjects with R > 16, four wavefronts per 64 subjects: the same steps as
// k_procrustes_l, with the R-long products split by columns over the four wavefronts (each takes
// a quarter of the columns of Y (H^T H), of P and of P H^T for all 64 subjects, the Gram partial
// sums added in wavefront order) and the l x l eigenproblems split by subjects (16 per
// wavefront). All four SIMDs of a compute unit work on a block.
template <int R, int N>
__global__ void __launch_bounds__(256)
    k_procrustes_m(int64_t K, int l_arg, const int32_t *__restrict__ rk,
                   const float *__restrict__ T, float *__restrict__ Q, const float *__restrict__ H,
                   const float *__restrict__ W, float *__restrict__ Ew, double rtol,
                   FitScalars *sc) {
  constexpr int NT = N * (N + 1) / 2;
  constexpr int RQ = (R + 3) / 4;  // columns per wavefront
  const int l = l_arg;
  extern __shared__ double smem_d[];
  double *sHH = smem_d;                                   // H^T H
  double *sG = sHH + R * R;                               // [NT x 64]: Gram, then B
  float *sH = reinterpret_cast<float *>(sG + NT * 64);    // H
  float *sX = sH + R * R;                                 // 64 per-subject blocks
  const int lR = l * R, stride = lR + 1;
  const float inv_lR = 1.0f / (float)lR;
  auto at = [&](int f) {
    int q = (int)((float)f * inv_lR);
    const int r = f - q * lR;
    q += (r >= lR) - (r < 0);
    return f + q;
  };
  const int t = threadIdx.x, s = t & 63, w = t >> 6;
  const int64_t k0 = (int64_t)blockIdx.x * 64;
  const int nsub = (int)(K - k0 < 64 ? K - k0 : 64);
  for (int e = t; e < R * R; e += 256) sH[e] = H[e];
  {
    const float *src = T + k0 * lR;
    const int n = nsub * lR, total = 64 * lR;
    for (int e0 = 0; e0 < total; e0 += 8 * 256) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + t;
        v[u] = e < n ? src[e] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + t;
        if (e < total) sX[at(e)] = v[u];
      }
    }
  }
  __syncthreads();
  for (int e = t; e < R * R; e += 256) {
    const int a = e / R, b = e - a * R;
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc += (double)sH[r * R + a] * (double)sH[r * R + b];
    sHH[e] = acc;
  }
  const bool live = s < nsub;
  const int64_t k = k0 + (live ? s : 0);
  float *x = sX + s * stride;
  const int c_lo = w * RQ;
  // Y = T_k S_k on this wavefront's columns
#pragma unroll 1
  for (int i = 0; i < l; ++i)
#pragma unroll
    for (int cc = 0; cc < RQ; ++cc)
      if (c_lo + cc < R) x[i * R + c_lo + cc] *= W[k * R + c_lo + cc];
  __syncthreads();
  {
    // partial Gram over this wavefront's columns: sum_c y_ic (Y (H^T H))_jc
    double Gp[NT];
#pragma unroll
    for (int e = 0; e < NT; ++e) Gp[e] = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (j < l) {
        double z[RQ];
#pragma unroll
        for (int cc = 0; cc < RQ; ++cc) z[cc] = 0.0;
#pragma unroll 1
        for (int r = 0; r < R; ++r) {
          const double y = (double)x[j * R + r];
          const double *hh = sHH + r * R + c_lo;
#pragma unroll
          for (int cc = 0; cc < RQ; ++cc)
            if (c_lo + cc < R) z[cc] = fma(y, hh[cc], z[cc]);
        }
#pragma unroll
        for (int i = 0; i <= j; ++i) {
          double acc = 0.0;
#pragma unroll
          for (int cc = 0; cc < RQ; ++cc)
            if (c_lo + cc < R) acc = fma((double)x[i * R + c_lo + cc], z[cc], acc);
          Gp[triN<N>(i, j)] = acc;
        }
      }
    }
    // add the four partial sums in wavefront order
#pragma unroll 1
    for (int ww = 0; ww < 4; ++ww) {
      if (w == ww) {
#pragma unroll
        for (int e = 0; e < NT; ++e) sG[e * 64 + s] = (ww == 0 ? 0.0 : sG[e * 64 + s]) + Gp[e];
      }
      __syncthreads();
    }
  }
  if ((t & 63) < 16) {
    // the eigenproblems: wavefront w takes subjects 16 w .. 16 w + 15
    const int sj = 16 * w + (t & 63);
    const bool lj = sj < nsub;
    const int64_t kj = k0 + (lj ? sj : 0);
    double G[NT];
#pragma unroll
    for (int e = 0; e < NT; ++e) G[e] = sG[e * 64 + sj];
    double E[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) E[i][j] = (double)Ew[(int64_t)(i * kNMax + j) * K + kj];
    orthonormalize<N>(E);
    {
      // G <- E^T G E, one column of G E at a time
      double Gn[NT];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        double ge[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          double acc = 0.0;
#pragma unroll
          for (int pp = 0; pp < N; ++pp) acc = fma(G[triN<N>(i, pp)], E[pp][q], acc);
          ge[i] = acc;
        }
#pragma unroll
        for (int pp = 0; pp <= q; ++pp) {
          double acc = 0.0;
#pragma unroll
          for (int i = 0; i < N; ++i) acc = fma(E[i][pp], ge[i], acc);
          Gn[triN<N>(pp, q)] = acc;
        }
      }
#pragma unroll
      for (int e = 0; e < NT; ++e) G[e] = Gn[e];
    }
    jacobi_rr<N>(G, E);
    if (lj) {
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) Ew[(int64_t)(i * kNMax + j) * K + kj] = (float)E[i][j];
    }
    double lmax = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) lmax = fmax(lmax, G[triN<N>(j, j)]);
    double f[N];
    int rank = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const double lv = G[triN<N>(j, j)];
      const bool keep = lmax > 0.0 && lv > rtol * rtol * lmax;
      f[j] = keep ? rsq_nr(lv) : 0.0;
      rank += keep ? 1 : 0;
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < N; ++q) acc += E[i][q] * f[q] * E[j][q];
        sG[triN<N>(i, j) * 64 + sj] = acc;
      }
    const int meff = rk[kj];
    if (lj && rank < (meff < R ? meff : R)) atomicAdd(&sc->rank_def_slot[sc->cur & 1], 1);
  }
  __syncthreads();
  {
    // P = B Y on this wavefront's columns
    double B[NT];
#pragma unroll
    for (int e = 0; e < NT; ++e) B[e] = sG[e * 64 + s];
#pragma unroll 1
    for (int cc = 0; cc < RQ; ++cc) {
      const int c = c_lo + cc;
      if (c < R) {
        double v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = i < l ? (double)x[i * R + c] : 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i)
          if (i < l) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) acc = fma(B[triN<N>(i, j)], v[j], acc);
            x[i * R + c] = (float)acc;
          }
      }
    }
  }
  __syncthreads();
  // Q rows = P H^T, row by row (every wavefront reads the whole row before any overwrites it)
#pragma unroll 1
  for (int i = 0; i < l; ++i) {
    float pr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) pr[r] = x[i * R + r];
    __syncthreads();
#pragma unroll 1
    for (int cc = 0; cc < RQ; ++cc) {
      const int c = c_lo + cc;
      if (c < R) {
        const float *h = sH + c * R;
        float acc = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) acc = fmaf(pr[r], h[r], acc);
        x[i * R + c] = acc;
      }
    }
  }
  __syncthreads();
  {
    float *dst = Q + k0 * lR;
    const int n = nsub * lR;
    for (int e0 = 0; e0 < n; e0 += 8 * 256) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + t;
        v[u] = e < n ? sX[at(e)] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + t;
        if (e < n) dst[e] = v[u];
      }
    }
  }
}

// Smoothed subjects with R > 16 in three launches, so that the l x l eigenproblems run without
// LDS at several wavefronts per SIMD:
//   k_proc_gram   A_k = T_k S_k H^T (FP32) and G_k = A_k A_k^T (FP64), entry-major per subject
//   k_proc_eigen  warm-started Jacobi on G_k (thread per subject), B_k = E diag(f) E^T
//   k_proc_q      A_k again from T_k (cheaper than storing it), then Q_k = B_k A_k
// Four wavefronts per 64 subjects in the first and last, a quarter of the columns each.

// Stages the rows t_i * w_k of the subjects k0 .. k0 + nsub - 1 (l R floats each) into LDS
// blocks of l R + 1 floats (the padding lets one lane per subject read its block without bank
// conflicts). When R % 4 == 0 a row is whole float4s, so eight float4 loads per thread are in
// flight at a time. Whole block.
template <int R>
__device__ __forceinline__ void stage_scaled_rows(const float *__restrict__ T,
                                                  const float *__restrict__ W, int64_t k0,
                                                  int nsub, int l, float *sX) {
  const int lR = l * R, stride = lR + 1;
  const int t = threadIdx.x;
  const bool aligned = (((uintptr_t)T | (uintptr_t)W) & 15) == 0;
  if (R % 4 == 0 && aligned) {
    constexpr int R4 = (R + 3) / 4, U = 8;
    const int lR4 = l * R4;
    const float4 *src = reinterpret_cast<const float4 *>(T + k0 * lR);
    const float4 *wsrc = reinterpret_cast<const float4 *>(W + k0 * R);
    const int n4 = nsub * lR4;
    for (int e0 = 0; e0 < n4; e0 += U * 256) {
      float4 v[U], w[U];
      int sj[U], off[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * 256 + t;
        const int ec = e < n4 ? e : 0;
        sj[u] = ec / lR4;
        off[u] = ec - sj[u] * lR4;
        v[u] = src[ec];
        w[u] = wsrc[sj[u] * R4 + off[u] % R4];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (e0 + u * 256 + t < n4) {
          float *d = sX + sj[u] * stride + off[u] * 4;
          d[0] = v[u].x * w[u].x;
          d[1] = v[u].y * w[u].y;
          d[2] = v[u].z * w[u].z;
          d[3] = v[u].w * w[u].w;
        }
      }
    }
  } else {
    const float *src = T + k0 * lR;
    const float *wsrc = W + k0 * R;
    const int n = nsub * lR;
    for (int e0 = 0; e0 < n; e0 += 8 * 256) {
      float v[8];
      int sj[8], off[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + t;
        const int ec = e < n ? e : 0;
        sj[u] = ec / lR;
        off[u] = ec - sj[u] * lR;
        v[u] = src[ec] * wsrc[sj[u] * R + off[u] % R];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (e0 + u * 256 + t < n) sX[sj[u] * stride + off[u]] = v[u];
    }
  }
}

// a_i = (t_i * w) H^T on the columns c_lo .. c_lo + RQ - 1, every row i < l of the lane's subject
// (x: its staged block): four entries of each H column at a time, applied to every row. With H in
// global memory and c_lo wavefront-uniform the H entries load into scalar registers; with H in
// LDS c_lo may differ between lanes.
template <int R, int N>
__device__ __forceinline__ void a_columns(const float *x, const float *__restrict__ H, int c_lo,
                                          int l, float (&a)[N][(R + 3) / 4]) {
  constexpr int RQ = (R + 3) / 4;
  constexpr bool kFullCols = R % 4 == 0;  // (then every wavefront's RQ columns exist)
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int cc = 0; cc < RQ; ++cc) a[i][cc] = 0.0f;
#pragma unroll
  for (int r0 = 0; r0 < R; r0 += 4) {
    float h[RQ][4];
#pragma unroll
    for (int cc = 0; cc < RQ; ++cc)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c_lo + cc, r = r0 + u;
        h[cc][u] = (r < R && (kFullCols || c < R)) ? H[c * R + r] : 0.0f;
      }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (i < l) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (r0 + u < R) {
            const float y = x[i * R + r0 + u];
#pragma unroll
            for (int cc = 0; cc < RQ; ++cc) a[i][cc] = fmaf(y, h[cc][u], a[i][cc]);
          }
        }
      }
    }
  }
}

// v summed over the lane's quad (lanes 4j .. 4j + 3) by two DPP exchanges; every lane of the quad
// gets the same (v0 + v1) + (v2 + v3), bit for bit.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffu), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}
__device__ __forceinline__ double quad_sum(double v) {
  v = v + dpp_d<0xB1>(v);  // quad_perm [1, 0, 3, 2]
  return v + dpp_d<0x4E>(v);  // quad_perm [2, 3, 0, 1]
}

// Four lanes per subject (64 per block), lane q of a quad a quarter of the columns: A_k's columns
// from the staged rows t_i * w_k with H from LDS, the partial FP64 Gram over them, the quad sum,
// and each lane stores a quarter of the subject's Gram entries (entry-major).
template <int R, int N>
__global__ void __launch_bounds__(256)
    k_proc_gram(int64_t K, int l, const float *__restrict__ T, const float *__restrict__ H,
                const float *__restrict__ W, double *__restrict__ Gk) {
  constexpr int NT = N * (N + 1) / 2;
  constexpr int RQ = (R + 3) / 4;
  extern __shared__ double smem_d[];
  float *sH = reinterpret_cast<float *>(smem_d);  // H (R x R)
  float *sX = sH + ((R * R + 3) & ~3);            // 64 per-subject blocks of l R + 1 floats
  const int lR = l * R, stride = lR + 1;
  const int t = threadIdx.x, s = t >> 2, q = t & 3;
  const int64_t k0 = (int64_t)blockIdx.x * 64;
  const int nsub = (int)(K - k0 < 64 ? K - k0 : 64);
  for (int e = t; e < R * R; e += 256) sH[e] = H[e];
  stage_scaled_rows<R>(T, W, k0, nsub, l, sX);
  __syncthreads();
  float a[N][RQ];
  a_columns<R, N>(sX + s * stride, sH, q * RQ, l, a);
  double Gp[NT];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int cc = 0; cc < RQ; ++cc)
        if (R % 4 == 0 || q * RQ + cc < R) acc = fma((double)a[i][cc], (double)a[j][cc], acc);
      Gp[triN<N>(i, j)] = quad_sum(acc);
    }
  if (s < nsub) {
#pragma unroll
    for (int e = 0; e < NT; ++e)
      if ((e & 3) == q) Gk[(int64_t)e * K + k0 + s] = Gp[e];
  }
}

template <int R, int N>
__global__ void __launch_bounds__(256)
    k_proc_eigen(int64_t K, int l, const int32_t *__restrict__ rk, double *__restrict__ Gk,
                 float *__restrict__ Ew, double rtol, FitScalars *sc) {
  constexpr int NT = N * (N + 1) / 2;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = k < K;
  const int64_t kk = live ? k : 0;
  double G[NT];
#pragma unroll
  for (int e = 0; e < NT; ++e) G[e] = Gk[(int64_t)e * K + kk];
  double E[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) E[i][j] = (double)Ew[(int64_t)(i * kNMax + j) * K + kk];
  orthonormalize<N>(E);
  {
    double Gn[NT];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double ge[N];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int pp = 0; pp < N; ++pp) acc = fma(G[triN<N>(i, pp)], E[pp][q], acc);
        ge[i] = acc;
      }
#pragma unroll
      for (int pp = 0; pp <= q; ++pp) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) acc = fma(E[i][pp], ge[i], acc);
        Gn[triN<N>(pp, q)] = acc;
      }
    }
#pragma unroll
    for (int e = 0; e < NT; ++e) G[e] = Gn[e];
  }
  jacobi_rr<N>(G, E);
  if (live) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j) Ew[(int64_t)(i * kNMax + j) * K + k] = (float)E[i][j];
  }
  double lmax = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) lmax = fmax(lmax, G[triN<N>(j, j)]);
  double f[N];
  int rank = 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double lv = G[triN<N>(j, j)];
    const bool keep = lmax > 0.0 && lv > rtol * rtol * lmax;
    f[j] = keep ? rsq_nr(lv) : 0.0;
    rank += keep ? 1 : 0;
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < N; ++q) acc += E[i][q] * f[q] * E[j][q];
        Gk[(int64_t)triN<N>(i, j) * K + k] = acc;
      }
    const int meff = rk[k];
    if (rank < (meff < R ? meff : R)) atomicAdd(&sc->rank_def_slot[sc->cur & 1], 1);
  }
}

template <int R, int N>
__global__ void __launch_bounds__(256)
    k_proc_q(int64_t K, int l, const float *__restrict__ T, const float *__restrict__ H,
             const float *__restrict__ W, const double *__restrict__ Bk, float *__restrict__ Q) {
  constexpr int NT = N * (N + 1) / 2;
  constexpr int RQ = (R + 3) / 4;
  extern __shared__ double smem_d[];
  float *sX = reinterpret_cast<float *>(smem_d);
  const int lR = l * R, stride = lR + 1;
  const float inv_lR = 1.0f / (float)lR;
  auto at = [&](int f) {
    int q = (int)((float)f * inv_lR);
    const int r = f - q * lR;
    q += (r >= lR) - (r < 0);
    return f + q;
  };
  const int t = threadIdx.x, s = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int64_t k0 = (int64_t)blockIdx.x * 64;
  const int nsub = (int)(K - k0 < 64 ? K - k0 : 64);
  const int64_t k = k0 + (s < nsub ? s : 0);
  double B[NT];
#pragma unroll
  for (int e = 0; e < NT; ++e) B[e] = Bk[(int64_t)e * K + k];
  stage_scaled_rows<R>(T, W, k0, nsub, l, sX);
  __syncthreads();
  float *x = sX + s * stride;
  const int c_lo = w * RQ;
  float a[N][RQ];
  a_columns<R, N>(x, H, c_lo, l, a);
  __syncthreads();  // (every wavefront has read the rows; the block now takes Q in their place)
#pragma unroll
  for (int cc = 0; cc < RQ; ++cc) {
    const int c = c_lo + cc;
    if (R % 4 == 0 || c < R) {
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (i < l) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < N; ++j)
            if (j < l) acc = fma(B[triN<N>(i, j)], (double)a[j][cc], acc);
          x[i * R + c] = (float)acc;
        }
    }
  }
  __syncthreads();
  {
    float *dst = Q + k0 * lR;
    const int n = nsub * lR;
    for (int e0 = 0; e0 < n; e0 += 8 * 256) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + t;
        v[u] = e < n ? sX[at(e)] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256 + t;
        if (e < n) dst[e] = v[u];
      }
    }
  }
}

// The three launches; `each` wraps every launch (per-kernel timing in the iteration, a plain call
// in the tuner).
template <int R, int N, typename F>
inline void launch_proc_split(copa_plan *p, const copa_state *st, hipStream_t s, F &&each) {
  constexpr int NT = N * (N + 1) / 2;
  const int64_t K = p->K;
  const unsigned nb = (unsigned)((K + 63) / 64);
  const size_t lds1 = (size_t)((R * R + 3) & ~3) * 4 + (size_t)64 * (p->l * R + 1) * 4;
  each(0, [&] { k_proc_gram<R, N><<<nb, 256, lds1, s>>>(K, p->l, p->T, st->H, st->W, p->pgb); });
  each(1, [&] {
    k_proc_eigen<R, N><<<(unsigned)((K + 255) / 256), 256, 0, s>>>(K, p->l, p->rk, p->pgb, p->Ew,
                                                                    p->opt.rank_rtol, p->scal);
  });
  const size_t lds3 = (size_t)64 * (p->l * R + 1) * 4;
  each(2, [&] {
    k_proc_q<R, N><<<nb, 256, lds3, s>>>(K, p->l, p->T, st->H, st->W, p->pgb, p->Q);
  });
}
struct PlainLaunch {
  template <typename L>
  void operator()(int, L &&launch) const { launch(); }
};

inline size_t procrustes_m_lds(int R, int l, int N) {
  return (size_t)R * R * 8 + (size_t)N * (N + 1) / 2 * 64 * 8 + (size_t)R * R * 4 +
         (size_t)64 * (l * R + 1) * 4;
}

// Dynamic LDS of k_procrustes_l: H^T H (FP64), H (FP32) and 64 blocks of l R + 1 floats.
inline size_t procrustes_l_lds(int R, int l) {
  return (size_t)R * R * 8 + (size_t)R * R * 4 + (size_t)64 * (l * R + 1) * 4;
}

// ======================================================================= ADMM helpers
// sGi <- (X * Y + rho I)^{-1} (Hadamard product, FP64, full R x R), rho = trace(X * Y) / R
// (Algorithm 1), by Gauss-Jordan elimination on [G + rho I | I] with the whole block: sL holds
// the left part and sGi the right part, and at step j every thread forms the new values of its
// entries of the R live columns (left columns j + 1 .. R - 1, right columns 0 .. j) from the old
// pivot row, then all write them. No pivoting is needed because the matrix is symmetric positive
// definite, and the rho shift bounds its condition number by R + 1, so the explicit inverse is as
// accurate as triangular solves and turns every later ADMM step into one matrix-vector product.
// Blocks of 256 threads. Returns false (and leaves Gi = I, rho = 1) when a pivot is not positive
// and finite.
template <int R>
__device__ __forceinline__ bool build_system(const double *__restrict__ X,
                                             const double *__restrict__ Y, double *sL,
                                             double *sGi, double *srho, int *sflag) {
  constexpr int RR = R * R;
  constexpr int NU = (RR + 255) / 256;  // entries per thread and step
  const int t = threadIdx.x;
  for (int e = t; e < RR; e += blockDim.x) {
    sL[e] = X[e] * Y[e];
    sGi[e] = e / R == e % R ? 1.0 : 0.0;
  }
  __syncthreads();
  double tr = 0.0;
  for (int i = 0; i < R; ++i) tr += sL[i * R + i];
  const double rho = tr / R;
  bool ok = isfinite(rho) && rho > 0.0;
  __syncthreads();  // every thread has read the diagonal
  if (t < R) sL[t * R + t] += rho;
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    const double piv = sL[j * R + j];
    ok = ok && piv > 0.0 && isfinite(piv);
    const double inv = rcp_nr(piv > 0.0 ? piv : 1.0);
    const int na = R - 1 - j;  // live left columns
    double nv[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = t + 256 * u;
      if (e < RR) {
        const int r = e / R, k = e - (e / R) * R;
        double *M = k < na ? sL : sGi;
        const int col = k < na ? j + 1 + k : k - na;
        const double old = M[r * R + col], pv = M[j * R + col];
        nv[u] = r == j ? old * inv : old - (sL[r * R + j] * inv) * pv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = t + 256 * u;
      if (e < RR) {
        const int r = e / R, k = e - (e / R) * R;
        double *M = k < na ? sL : sGi;
        const int col = k < na ? j + 1 + k : k - na;
        M[r * R + col] = nv[u];
      }
    }
    __syncthreads();
  }
  if (!ok)
    for (int e = t; e < RR; e += blockDim.x) sGi[e] = e / R == e % R ? 1.0 : 0.0;
  if (t == 0) {
    *srho = ok ? rho : 1.0;
    *sflag = ok ? 0 : 1;
  }
  __syncthreads();
  return *sflag == 0;
}

// ======================================================================= ADMM on rows by lanes
// One factor row spread over R lanes of a wavefront (lane c holds column c): the inner ADMM
// steps of Algorithm 1, Z = (F + rho (Zb + D)) (G + rho I)^{-1}, Zb = prox(Z - D), D += Zb - Z,
// with the row vector exchanged through this group's LDS slot xrow (wavefront-local: LDS
// operations of one wavefront complete in order, so a compiler barrier is enough).
template <int R>
__device__ __forceinline__ void admm_lanes(double F, float &Zb, float &D,
                                           const double *__restrict__ sGi, double rho, int kind,
                                           double lam, int iters, double *xrow, int c) {
  const double thr = lam / rho;
  for (int it = 0; it < iters; ++it) {
    xrow[c] = F + rho * ((double)Zb + (double)D);
    __builtin_amdgcn_wave_barrier();
    double z = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) z += xrow[k] * sGi[k * R + c];
    __builtin_amdgcn_wave_barrier();
    const double zb = prox_sel(z - (double)D, kind, lam, thr);
    D = (float)((double)D + zb - z);
    Zb = (float)zb;
  }
}

// The inner ADMM steps of admm_lanes in FP32 arithmetic (the system (G + rho I)^{-1} is formed in
// FP64 and rounded once; sGi: its FP32 copy in LDS, lanes of one column reading the same word),
// the product in four partial sums, which shortens the dependency chain of each step. The state
// Zb, D and the MTTKRP row F are FP32 values already.
template <int R>
__device__ __forceinline__ void admm_lanes_reg(float F, float &Zb, float &D,
                                               const float *__restrict__ sGi, float rho,
                                               int kind, float lam, int iters, float *xrow,
                                               int c) {
  const float thr = lam / rho;
  for (int it = 0; it < iters; ++it) {
    xrow[c] = fmaf(rho, Zb + D, F);
    __builtin_amdgcn_wave_barrier();
    float zs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k = 0; k < R; ++k) zs[k & 3] = fmaf(xrow[k], sGi[k * R + c], zs[k & 3]);
    const float z = (zs[0] + zs[1]) + (zs[2] + zs[3]);
    __builtin_amdgcn_wave_barrier();
    const float x = z - D;
    const float a1 = fabsf(x) - thr, a2 = x - thr;
    float zb = x;
    zb = kind == COPA_PROX_NONNEG ? (x > 0.0f ? x : 0.0f) : zb;
    zb = kind == COPA_PROX_L1 ? (a1 > 0.0f ? copysignf(a1, x) : 0.0f) : zb;
    zb = kind == COPA_PROX_L0 ? (x * x > lam ? x : 0.0f) : zb;
    zb = kind == COPA_PROX_NONNEG_L1 ? (a2 > 0.0f ? a2 : 0.0f) : zb;
    D = D + zb - z;
    Zb = zb;
  }
}

// ======================================================================= FIT of an iteration
// Inputs of the FIT and objective of outer iteration `it`, left as per-block partials by the V
// update and the W update of that iteration.
struct FitArgs {
  const double *vpart;    // [nvb x 4] <F_V, V>, |V|_1, zeros
  const double *vtvpart;  // [nvtv x R x R] V^T V: the V blocks' partials, or their sum (nvtv 1)
  int nvtv;
  int nvb;
  const double *wl1part;  // [nwb] |W|_1
  int nwb;
  double normX2;
  int64_t J;
  int proxV, proxW, proxH;
  double lamV, lamW, lamH;
};

// Whole block (256 threads; red: 6 x 256 doubles of LDS, sVtV: R x R of LDS). Adds the partials
// in block order, stores V^T V, and evaluates
//   FIT = 1 - (|X|^2 - 2 <F_V, V> + <Psi, V^T V>) / |X|^2   (Section "Evaluation Metrics")
// and the objective with the l1 penalties, with H = the factor of that iteration.
template <int R>
__device__ __forceinline__ void fit_finalize(const FitArgs &fa, int it, const float *H,
                                             double *small, FitScalars *sc, double (*red)[256],
                                             double *sVtV) {
  constexpr int RR = R * R;
  const int t = threadIdx.x;
  block_reduce_parts<RR>(fa.vtvpart, fa.nvtv, sVtV, red[0]);
  double dot = 0.0, l1 = 0.0, zeros = 0.0, wl1 = 0.0, hl1 = 0.0, quad = 0.0;
  for (int b = t; b < fa.nvb; b += blockDim.x) {
    dot += fa.vpart[b * 4 + 0];
    l1 += fa.vpart[b * 4 + 1];
    zeros += fa.vpart[b * 4 + 2];
  }
  // the W-update partials (one per block of that launch, thousands at large K): eight loads in
  // flight per thread, from clamped addresses
  {
    double w8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int nt = blockDim.x;
    for (int b0 = t; b0 < fa.nwb; b0 += 8 * nt) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + u * nt;
        const double x = fa.wl1part[b < fa.nwb ? b : 0];
        w8[u] += b < fa.nwb ? x : 0.0;
      }
    }
    wl1 = ((w8[0] + w8[1]) + (w8[2] + w8[3])) + ((w8[4] + w8[5]) + (w8[6] + w8[7]));
  }
  for (int e = t; e < RR; e += blockDim.x) {
    hl1 += fabs((double)H[e]);
    quad += small[kPsi * RR + e] * sVtV[e];
    small[kVtV * RR + e] = sVtV[e];
  }
  red[0][t] = dot;
  red[1][t] = l1;
  red[2][t] = zeros;
  red[3][t] = quad;
  red[4][t] = wl1;
  red[5][t] = hl1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int q = 0; q < 6; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  if (t == 0) {
    const double resid = fa.normX2 - 2.0 * red[0][0] + red[3][0];
    const double fit = fa.normX2 > 0.0 ? 1.0 - resid / fa.normX2 : 0.0;
    auto pen = [](int k, double la, double v) {
      return (k == COPA_PROX_L1 || k == COPA_PROX_NONNEG_L1) ? la * v : 0.0;
    };
    const double obj = 0.5 * resid + pen(fa.proxV, fa.lamV, red[1][0]) +
                       pen(fa.proxW, fa.lamW, red[4][0]) + pen(fa.proxH, fa.lamH, red[5][0]);
    if (!isfinite(fit) || !isfinite(obj)) atomicMin(&sc->fail_iter, it);
    if (it < kHistCap) {
      sc->hist_fit[it] = fit;
      sc->hist_obj[it] = obj;
    }
    sc->last_fit = fit;
    sc->last_obj = obj;
    sc->last_sparsity = fa.J > 0 ? red[2][0] / ((double)fa.J * R) : 0.0;
    sc->rank_deficient = sc->rank_def_slot[it & 1];
    sc->rank_def_slot[it & 1] = 0;
    sc->iter = it + 1;
  }
  __syncthreads();
}

template <int R>
__global__ void __launch_bounds__(256)
    k_fit(FitArgs fa, const float *H, double *small, FitScalars *sc) {
  __shared__ double red[6][256];
  __shared__ double sVtV[R * R];
  fit_finalize<R>(fa, sc->cur, H, small, sc, red, sVtV);
}

// The row Gram F_H = sum Q_row^T (T_row * w) (as k_rows_gram) with one extra block that takes
// the FIT of the previous outer iteration meanwhile (when the current iteration is not the first
// of its chunk).
template <int R, int WSEL>
__global__ void __launch_bounds__(256)
    k_rows_gram_fit(const float *__restrict__ A, const float *__restrict__ B, int64_t rows,
                    const float *__restrict__ W, int slot_rows,
                    const int32_t *__restrict__ rowsubj, double *__restrict__ part, int nb,
                    FitArgs fa, const float *__restrict__ H, double *small, FitScalars *sc) {
  if ((int)blockIdx.x == nb) {
    __shared__ double red[6][256];
    __shared__ double sVtV[R * R];
    const int it = sc->cur;
    if (it > 0) fit_finalize<R>(fa, it - 1, H, small, sc, red, sVtV);
    return;
  }
  rows_gram_block<R, WSEL>(A, B, rows, W, slot_rows, rowsubj, part, blockIdx.x, nb);
}

template <int R>
static void gram_fit(copa_plan *p, const float *A, const float *B, int64_t rows,
                     const float *W, int wsel, int slot, const FitArgs &fa, const float *H,
                     hipStream_t s) {
  const int64_t units = (rows + 63) / 64;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(p->gram_blocks, (units + 7) / 8));
  const unsigned grid = (unsigned)nb + 1u;
  double *p1 = gram_slot(p, slot);
  const int sr = p->slot_rows > 0 ? p->slot_rows : 1;
  if (wsel == 1)
    k_rows_gram_fit<R, 1><<<grid, 256, 0, s>>>(A, B, rows, W, sr, p->rowsubj, p1, nb, fa, H,
                                               p->small, p->scal);
  else
    k_rows_gram_fit<R, 2><<<grid, 256, 0, s>>>(A, B, rows, W, sr, p->rowsubj, p1, nb, fa, H,
                                               p->small, p->scal);
  k_gram_reduce<R * R><<<dim3((R * R + 3) / 4, 1), 256, 0, s>>>(p1, gram_total(p, slot), nullptr,
                                                                 nullptr, nb);
}

// ======================================================================= mode H (one block)
// G_H = W^TW * V^TV, rho, (G_H + rho I)^{-1}; inner ADMM on the R rows of H (R lanes per row);
// H^T H; then either the W-mode system G_W = H^TH * V^TV for the W update that follows (H first),
// or, with the new W's W^T W given (W first), the V-mode system G_V = H^TH * W^TW into modes[2].
template <int R>
__global__ void __launch_bounds__(256)
    k_mode_H(const double *FHtot, const double *WtWtot, double *small, ModeParams *modes,
             FitScalars *sc, float *H, float *DH, int kind, double lam, int iters, int build_w) {
  constexpr int RR = R * R;
  constexpr int G = kWave / R;
  __shared__ double sFH[RR], sX[RR], sY[RR], sL[RR], sGi[RR];
  __shared__ double xch[4][G + 1][R];
  __shared__ float sH[RR];
  __shared__ double srho;
  __shared__ int sflag;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane / R, c = lane % R;
  // W^T W: the stored one (H first) or the new W's total (W first)
  for (int e = t; e < RR; e += blockDim.x) {
    sFH[e] = FHtot[e];
    sX[e] = WtWtot ? WtWtot[e] : small[kWtW * RR + e];
    sY[e] = small[kVtV * RR + e];
  }
  __syncthreads();
  for (int e = t; e < RR; e += blockDim.x) {
    small[kFH * RR + e] = sFH[e];
    if (WtWtot) small[kWtW * RR + e] = sX[e];
  }
  bool ok = build_system<R>(sX, sY, sL, sGi, &srho, &sflag);
  if (t == 0 && !ok) atomicMin(&sc->fail_iter, sc->cur);
  const double rho = srho;
  for (int r0 = 0; r0 < R; r0 += 4 * G) {
    const int row = r0 + wave * G + g;
    const bool act = g < G && row < R;
    const int rc = act ? row : 0;
    float Zb = H[rc * R + c], D = DH[rc * R + c];
    admm_lanes<R>(sFH[rc * R + c], Zb, D, sGi, rho, kind, lam, iters, xch[wave][g], c);
    if (act) {
      H[row * R + c] = Zb;
      DH[row * R + c] = D;
      sH[row * R + c] = Zb;
    }
  }
  __syncthreads();
  for (int e = t; e < RR; e += blockDim.x) {
    const int a = e / R, b = e % R;
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) v += (double)sH[i * R + a] * (double)sH[i * R + b];
    sX[e] = v;
    small[kHtH * RR + e] = v;
  }
  __syncthreads();
  if (!build_w) {
    // W first: the next W system needs the new V, the V system of this iteration is known
    for (int e = t; e < RR; e += blockDim.x) sY[e] = WtWtot[e];
    __syncthreads();
    ok = build_system<R>(sX, sY, sL, sGi, &srho, &sflag);
    if (t == 0 && !ok) atomicMin(&sc->fail_iter, sc->cur);
    for (int e = t; e < RR; e += blockDim.x) modes[2].Gi[e] = sGi[e];
    if (t == 0) modes[2].rho = srho;
    return;
  }
  ok = build_system<R>(sX, sY, sL, sGi, &srho, &sflag);
  if (t == 0 && !ok) atomicMin(&sc->fail_iter, sc->cur);
  for (int e = t; e < RR; e += blockDim.x) modes[1].Gi[e] = sGi[e];
  if (t == 0) modes[1].rho = srho;
}

// ======================================================================= mode W (R lanes/subject)
// One subject per group of R lanes (lane c holds column c): F_W(k, c) = sum_i (q_i H)(c) t_i(c)
// (the q rows exchanged through wavefront-local LDS), the inner ADMM steps on W's row k (FP32, as
// admm_lanes_reg), then the M rows (q_i H) * w_k for pass 2 and the Psi Gram; per-block |W|_1 for
// the objective.
template <int R>
__global__ void __launch_bounds__(256)
    k_w_admm(int64_t K, int l, const int32_t *__restrict__ subj, const int32_t *__restrict__ rk,
             const float *__restrict__ T, const float *__restrict__ Q, float *__restrict__ M,
             const float *__restrict__ H, float *__restrict__ W, float *__restrict__ DW,
             float *__restrict__ FW, const ModeParams *__restrict__ modes, int kind, double lam,
             int iters, double *__restrict__ l1part) {
  constexpr int G = kWave / R;
  __shared__ float sGi[R * R];
  __shared__ float sH[R * R];
  __shared__ float xq[4][G + 1][kLMax][R];
  __shared__ float xch[4][G + 1][R];
  __shared__ double sred[256];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane / R, c = lane % R;
  for (int e = t; e < R * R; e += blockDim.x) {
    sGi[e] = (float)modes[1].Gi[e];
    sH[e] = H[e];
  }
  const int64_t k = ((int64_t)blockIdx.x * 4 + wave) * G + g;
  const bool act = g < G && k < K;
  const int64_t kc = act ? k : 0;
  float Zb = W[kc * R + c], D = DW[kc * R + c];
  int64_t base;
  int m;
  if (l > 0) {
    base = kc * l;
    m = rk[kc];
  } else {
    base = subj[kc];
    m = subj[kc + 1] - subj[kc];
  }
  if (!act) m = 0;
  __syncthreads();
  const float rho = (float)modes[1].rho;
  double F = 0.0;
  float qh[kLMax];  // smoothed: (q_i H)(c) of the l rows, kept for the M rows
  float(&xg)[kLMax][R] = xq[wave][g];
  if (l > 0) {
    float qv[kLMax], tv[kLMax];
#pragma unroll
    for (int i = 0; i < kLMax; ++i) {
      const int64_t ri = base + (i < l ? i : 0);
      qv[i] = Q[ri * R + c];
      tv[i] = T[ri * R + c];
    }
#pragma unroll
    for (int i = 0; i < kLMax; ++i) xg[i][c] = qv[i];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < kLMax; ++i) {
      double p = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) p += (double)xg[i][r] * (double)sH[r * R + c];
      F += i < m ? p * (double)tv[i] : 0.0;
      qh[i] = (float)p;
    }
  } else {
    for (int i = 0; i < m; ++i) {
      const float qv = Q[(base + i) * R + c], tv = T[(base + i) * R + c];
      __builtin_amdgcn_wave_barrier();
      xg[0][c] = qv;
      __builtin_amdgcn_wave_barrier();
      double p = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) p += (double)xg[0][r] * (double)sH[r * R + c];
      F += p * (double)tv;
    }
  }
  if (act) FW[k * R + c] = (float)F;
  admm_lanes_reg<R>((float)F, Zb, D, sGi, rho, kind, (float)lam, iters, xch[wave][g], c);
  double l1 = 0.0;
  if (act) {
    W[k * R + c] = Zb;
    DW[k * R + c] = D;
    l1 = fabs((double)Zb);
  }
  // M rows = (q_i H) * w_new
  if (l > 0) {
    if (act) {
#pragma unroll
      for (int i = 0; i < kLMax; ++i)
        if (i < l) M[(base + i) * R + c] = (float)((double)qh[i] * (double)Zb);
    }
  } else {
    for (int i = 0; i < m; ++i) {
      const float qv = Q[(base + i) * R + c];
      __builtin_amdgcn_wave_barrier();
      xg[0][c] = qv;
      __builtin_amdgcn_wave_barrier();
      double p = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) p += (double)xg[0][r] * (double)sH[r * R + c];
      M[(base + i) * R + c] = (float)(p * (double)Zb);
    }
  }
  sred[t] = l1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sred[t] += sred[t + w];
    __syncthreads();
  }
  if (t == 0) l1part[blockIdx.x] = sred[0];
}

// ======================================================================= W block first
// F_W(k, c) = sum_r H(r, c) P_k(r, c) for lane c: FP32 products of FP32 data in four partial sums.
template <int R>
__device__ __forceinline__ float column_dot(const float (&hcol)[R], const float (&pc)[R]) {
  float fs[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int r = 0; r < R; ++r) fs[r & 3] = fmaf(hcol[r], pc[r], fs[r & 3]);
  return (fs[0] + fs[1]) + (fs[2] + fs[3]);
}

// Adds the per-lane column accumulators acc[r] = X(r, c) of the 4 G lane groups of a block in a
// fixed order (groups of a wavefront in turn through LDS, then the four wavefronts) and stores
// the block's R x R partial. Whole block; red: 4 x R x R doubles of LDS.
template <int R>
__device__ __forceinline__ void block_columns_to_part(const double (&acc)[R], double (*red)[R * R],
                                                      double *__restrict__ part) {
  constexpr int G = kWave / R;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane / R, c = lane % R;
  for (int gg = 0; gg < G; ++gg) {
    if (g == gg) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        red[wave][r * R + c] = (gg == 0 ? 0.0 : red[wave][r * R + c]) + acc[r];
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  for (int e = t; e < R * R; e += blockDim.x)
    part[(int64_t)blockIdx.x * R * R + e] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
  __syncthreads();
}

// Block order W -> H -> V, one subject of the W block (R lanes, lane c holds column c): given
// F_W(k, c) and column c of P_k, the inner ADMM steps on W's row k, its store, and the lane's
// running sums of F_H(:, c) = sum_k P_k(:, c) w_k(c) and (W^T W)(:, c).
template <int R>
__device__ __forceinline__ void w_first_row(int64_t k, bool act, double F, const float (&pc)[R],
                                            float Zb, float D, const float *__restrict__ sGi,
                                            float rho, int kind, float lam, int iters,
                                            float *xrow, int c, float *__restrict__ W,
                                            float *__restrict__ DW, float *__restrict__ FW,
                                            double (&fh)[R], double (&wtw)[R], double &l1) {
  if (act) FW[k * R + c] = (float)F;
  admm_lanes_reg<R>((float)F, Zb, D, sGi, rho, kind, lam, iters, xrow, c);
  const double w = act ? (double)Zb : 0.0;
  if (act) {
    W[k * R + c] = Zb;
    DW[k * R + c] = D;
    l1 += fabs(w);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) fh[r] += (double)pc[r] * w;
  // W^T W: the new row through this group's LDS slot
  __builtin_amdgcn_wave_barrier();
  xrow[c] = (float)w;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < R; ++r) wtw[r] += (double)xrow[r] * w;
  __builtin_amdgcn_wave_barrier();
}

// Block order W -> H -> V: the W block right after the Procrustes step, then the H block's
// inputs. One subject per group of R lanes (lane c holds column c), each block striding over
// groups of 4 G subjects:
//   P_k = Q_k^T T_k (column c per lane), F_W(k, c) = sum_r H(r, c) P_k(r, c) with the H of the
//   previous outer iteration, the inner ADMM steps on W's row k with the W system built from
//   that H (modes[1]); then, with the new row w_k, the block's partials of
//   F_H = sum_k P_k diag(w_k), of W^T W and of |W|_1.
// The rows T_k and Q_k are read once; nothing per subject is written but W's row and F_W.
// Smoothed plans (l rows per subject) load the next subject's rows while the current one is
// processed.
// (two wavefronts per SIMD where the registers allow it without spills: R <= 20)
template <int R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(R <= 20 ? 2 : 1)))
    k_w_first(int64_t K, int l, const int32_t *__restrict__ subj, const int32_t *__restrict__ rk,
              const float *__restrict__ T, const float *__restrict__ Q,
              const float *__restrict__ H, float *__restrict__ W, float *__restrict__ DW,
              float *__restrict__ FW, const ModeParams *__restrict__ modes, int kind, double lam,
              int iters, double *__restrict__ l1part, double *__restrict__ fhpart,
              double *__restrict__ wtwpart) {
  constexpr int G = kWave / R;
  __shared__ float xq[4][G + 1][kLMax][R];
  __shared__ float xtq[4][G + 1][kLMax][R];
  __shared__ float xch[4][G + 1][R];
  __shared__ double red[4][R * R];
  __shared__ float sGi[R * R];
  __shared__ double sred[256];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane / R, c = lane % R;
  double fh[R], wtw[R];
  float hcol[R];
  for (int e = t; e < R * R; e += blockDim.x) sGi[e] = (float)modes[1].Gi[e];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    hcol[r] = H[r * R + c];
    fh[r] = 0.0;
    wtw[r] = 0.0;
  }
  const float rho = (float)modes[1].rho, lamf = (float)lam;
  __syncthreads();
  float(&xg)[kLMax][R] = xq[wave][g];
  float(&xt)[kLMax][R] = xtq[wave][g];
  float *xrow = xch[wave][g];
  double l1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 4 * G;
  const int64_t first = (int64_t)blockIdx.x * 4 * G + wave * G + g;
  if (l > 0) {
    // rows, W entry, dual and rank of subject kk (clamped to subject 0 past the end)
    float qv[kLMax], tv[kLMax], Zb, D;
    int m;
    // (the kLMax row slots from the subject's first row: rows past its l belong to the next
    // subject or to the buffers' slack rows, and are masked by the rank m <= l)
    auto fetch = [&](int64_t kk, float(&q)[kLMax], float(&tt)[kLMax], float &zb, float &d,
                     int &mm) {
      const bool a = g < G && kk < K;
      const int64_t kc = a ? kk : 0;
      const float *qb = Q + kc * l * R + c, *tb = T + kc * l * R + c;
#pragma unroll
      for (int i = 0; i < kLMax; ++i) {
        q[i] = qb[i * R];
        tt[i] = tb[i * R];
      }
      zb = W[kc * R + c];
      d = DW[kc * R + c];
      mm = a ? rk[kc] : 0;
    };
    if (first - wave * G - g < K) fetch(first, qv, tv, Zb, D, m);
    for (int64_t k = first; k - wave * G - g < K; k += stride) {
      const bool act = g < G && k < K;
      float qn[kLMax], tn[kLMax], Zn, Dn;
      int mn;
      fetch(k + stride, qn, tn, Zn, Dn, mn);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int i = 0; i < kLMax; ++i) {
        xg[i][c] = qv[i];
        xt[i][c] = tv[i];
      }
      __builtin_amdgcn_wave_barrier();
      float pc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) pc[r] = 0.0f;
      // P_k(:, c) from the rank-m rows (staged in LDS, which keeps the registers for the sums);
      // then F_W(k, c) = sum_r H(r, c) P_k(r, c)
#pragma unroll 1
      for (int i = 0; i < m; ++i) {
        const float ti = xt[i][c];
#pragma unroll
        for (int r = 0; r < R; ++r) pc[r] = fmaf(xg[i][r], ti, pc[r]);
      }
      const double F = column_dot<R>(hcol, pc);
      w_first_row<R>(k, act, F, pc, Zb, D, sGi, rho, kind, lamf, iters, xrow, c, W, DW, FW, fh,
                     wtw, l1);
#pragma unroll
      for (int i = 0; i < kLMax; ++i) {
        qv[i] = qn[i];
        tv[i] = tn[i];
      }
      Zb = Zn;
      D = Dn;
      m = mn;
    }
  } else {
    for (int64_t k = first; k - wave * G - g < K; k += stride) {
      const bool act = g < G && k < K;
      const int64_t kc = act ? k : 0;
      const float Zb = W[kc * R + c], D = DW[kc * R + c];
      const int64_t base = subj[kc];
      const int m = act ? subj[kc + 1] - subj[kc] : 0;
      float pc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) pc[r] = 0.0f;
      for (int i = 0; i < m; ++i) {
        const float qv = Q[(base + i) * R + c], ti = T[(base + i) * R + c];
        __builtin_amdgcn_wave_barrier();
        xg[0][c] = qv;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < R; ++r) pc[r] = fmaf(xg[0][r], ti, pc[r]);
      }
      const double F = column_dot<R>(hcol, pc);
      w_first_row<R>(k, act, F, pc, Zb, D, sGi, rho, kind, lamf, iters, xrow, c, W, DW, FW, fh,
                     wtw, l1);
    }
  }
  __syncthreads();
  block_columns_to_part<R>(fh, red, fhpart);
  block_columns_to_part<R>(wtw, red, wtwpart);
  sred[t] = l1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sred[t] += sred[t + w];
    __syncthreads();
  }
  if (t == 0) l1part[blockIdx.x] = sred[0];
}

// Block order W -> H -> V, after the H block: the M rows M_i = (q_i H) * w_k of every row i
// (subject k) for pass 2 and the block's partial of Psi = sum_i M_i^T M_i. Each group of R lanes
// takes kMRows consecutive rows at a time (their loads in flight together), each block striding
// over groups of 4 G kMRows rows.
constexpr int kMRows = 8;
template <int R>
__global__ void __launch_bounds__(256)
    k_m_rows(int64_t rows, int l, const int32_t *__restrict__ rowsubj,
             const float *__restrict__ Q, const float *__restrict__ H,
             const float *__restrict__ W, float *__restrict__ M, double *__restrict__ psipart) {
  constexpr int G = kWave / R;
  __shared__ float xq[4][G + 1][kMRows][R];
  __shared__ double red[4][R * R];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane / R, c = lane % R;
  double psi[R];
  float hcol[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    hcol[r] = H[r * R + c];
    psi[r] = 0.0;
  }
  float(&xr)[kMRows][R] = xq[wave][g];
  const int64_t step = (int64_t)4 * G * kMRows;
  for (int64_t i0 = (int64_t)blockIdx.x * step; i0 < rows; i0 += (int64_t)gridDim.x * step) {
    const int64_t ib = i0 + (int64_t)(wave * G + g) * kMRows;
    float q[kMRows], w[kMRows];
#pragma unroll
    for (int u = 0; u < kMRows; ++u) {
      const int64_t i = ib + u;
      const int64_t ic = g < G && i < rows ? i : 0;
      const int64_t k = l > 0 ? ic / l : (int64_t)rowsubj[ic];
      q[u] = Q[ic * R + c];
      w[u] = W[k * R + c];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < kMRows; ++u) xr[u][c] = q[u];
    __builtin_amdgcn_wave_barrier();
    float mv[kMRows];
#pragma unroll
    for (int u = 0; u < kMRows; ++u) {
      float p = 0.0f;
#pragma unroll
      for (int r = 0; r < R; ++r) p = fmaf(xr[u][r], hcol[r], p);
      const int64_t i = ib + u;
      const bool act = g < G && i < rows;
      mv[u] = act ? p * w[u] : 0.0f;
      if (act) M[i * R + c] = mv[u];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < kMRows; ++u) xr[u][c] = mv[u];
    __builtin_amdgcn_wave_barrier();
    // the kMRows rows' products summed in FP32, the running sum in FP64
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float s8 = 0.0f;
#pragma unroll
      for (int u = 0; u < kMRows; ++u) s8 = fmaf(xr[u][r], mv[u], s8);
      psi[r] += (double)s8;
    }
  }
  __syncthreads();
  block_columns_to_part<R>(psi, red, psipart);
}

// Block order W -> H -> V, end of an outer iteration (with_fit) or of the set-up: the FIT and
// objective of the iteration (fit_finalize, which also stores V^T V), then the W system of the
// next W block, (H^T H * V^T V + rho I)^{-1} with H^T H of the current H in FP64. One block.
template <int R>
__global__ void __launch_bounds__(256)
    k_finish_whv(FitArgs fa, int with_fit, const float *__restrict__ H, double *small,
                 ModeParams *modes, FitScalars *sc) {
  constexpr int RR = R * R;
  __shared__ double red[6][256];
  __shared__ double sVtV[RR], sX[RR], sL[RR], sGi[RR];
  __shared__ double srho;
  __shared__ int sflag;
  const int t = threadIdx.x;
  const int it = sc->cur;
  if (with_fit) {
    fit_finalize<R>(fa, it, H, small, sc, red, sVtV);
  } else {
    for (int e = t; e < RR; e += blockDim.x) sVtV[e] = small[kVtV * RR + e];
  }
  for (int e = t; e < RR; e += blockDim.x) {
    const int a = e / R, b = e % R;
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) v += (double)H[i * R + a] * (double)H[i * R + b];
    sX[e] = v;
  }
  __syncthreads();
  const bool ok = build_system<R>(sX, sVtV, sL, sGi, &srho, &sflag);
  if (t == 0 && !ok) atomicMin(&sc->fail_iter, it > 0 ? it : 0);
  for (int e = t; e < RR; e += blockDim.x) modes[1].Gi[e] = sGi[e];
  if (t == 0) modes[1].rho = srho;
}

// ======================================================================= mode V
// The V system of an outer iteration, G_V = H^TH * W^TW, rho and (G_V + rho I)^{-1}, into
// modes[2] (one block), built once for all blocks of k_v_admm.
template <int R>
__global__ void __launch_bounds__(256)
    k_v_system(const double *__restrict__ WtWtot, const double *__restrict__ small,
               ModeParams *modes, FitScalars *sc) {
  constexpr int RR = R * R;
  __shared__ double sX[RR], sY[RR], sL[RR], sGi[RR];
  __shared__ double srho;
  __shared__ int sflag;
  const int t = threadIdx.x;
  for (int e = t; e < RR; e += blockDim.x) {
    sX[e] = small[kHtH * RR + e];
    sY[e] = WtWtot[e];
  }
  __syncthreads();
  const bool ok = build_system<R>(sX, sY, sL, sGi, &srho, &sflag);
  if (t == 0 && !ok) atomicMin(&sc->fail_iter, sc->cur);
  for (int e = t; e < RR; e += blockDim.x) modes[2].Gi[e] = sGi[e];
  if (t == 0) modes[2].rho = srho;
}

// Every block: the V system from modes[2]; then its V rows, R lanes per row (inner ADMM, l1
// prox), the padded V tile copy for the next pass 1, and per-block partials of <F_V, V>, |V|_1,
// zeros and V^T V for the FIT (added by the next launch that needs them).
template <int R>
__global__ void __launch_bounds__(256)
    k_v_admm(int64_t J, const float *__restrict__ FV, float *__restrict__ V,
             float *__restrict__ DV, float *__restrict__ Vp, int rt, int rtp,
             const double *__restrict__ WtWtot, const double *__restrict__ Psitot, double *small,
             const ModeParams *__restrict__ modes, int kind, double lam, int iters,
             double *__restrict__ vpart, double *__restrict__ vtvpart) {
  constexpr int RR = R * R;
  constexpr int G = kWave / R;
  constexpr int RB = 4 * G;  // rows per block pass
  __shared__ double sGi[RR];
  __shared__ double xch[4][G + 1][R];
  __shared__ float sV[RB][R];
  __shared__ double red[3][256];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = lane / R, c = lane % R;
  const int slot = wave * G + g;
  for (int e = t; e < RR; e += blockDim.x) sGi[e] = modes[2].Gi[e];
  if (blockIdx.x == 0) {
    for (int e = t; e < RR; e += blockDim.x) {
      small[kWtW * RR + e] = WtWtot[e];
      small[kPsi * RR + e] = Psitot[e];
    }
  }
  __syncthreads();
  const double rho = modes[2].rho;
  double dot = 0.0, l1 = 0.0, zeros = 0.0;
  double vtv[(RR + 255) / 256];
#pragma unroll
  for (int u = 0; u < (RR + 255) / 256; ++u) vtv[u] = 0.0;
  for (int64_t j0 = (int64_t)blockIdx.x * RB; j0 < J; j0 += (int64_t)gridDim.x * RB) {
    const int64_t j = j0 + slot;
    const bool act = g < G && j < J;
    const int64_t jc = act ? j : 0;
    const double F = FV[jc * R + c];
    float Zb = V[jc * R + c], D = DV[jc * R + c];
    admm_lanes<R>(F, Zb, D, sGi, rho, kind, lam, iters, xch[wave][g], c);
    if (act) {
      V[j * R + c] = Zb;
      DV[j * R + c] = D;
      Vp[((int64_t)(c / rt) * J + j) * rtp + c % rt] = Zb;
      dot += F * (double)Zb;
      l1 += fabs((double)Zb);
      zeros += Zb == 0.0f ? 1.0 : 0.0;
    }
    if (g < G) sV[slot][c] = act ? Zb : 0.0f;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (RR + 255) / 256; ++u) {
      const int e = t + 256 * u;
      if (e < RR) {
        const int a = e / R, b = e % R;
        double v = 0.0;
#pragma unroll
        for (int s = 0; s < RB; ++s) v += (double)sV[s][a] * (double)sV[s][b];
        vtv[u] += v;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < (RR + 255) / 256; ++u) {
    const int e = t + 256 * u;
    if (e < RR) vtvpart[(int64_t)blockIdx.x * RR + e] = vtv[u];
  }
  red[0][t] = dot;
  red[1][t] = l1;
  red[2][t] = zeros;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < 3; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  if (t < 3) vpart[blockIdx.x * 4 + t] = red[t][0];
}

template <int R>
__global__ void __launch_bounds__(256)
    k_init_small(const double *__restrict__ partW, const double *__restrict__ partV, int nb,
                 double *small) {
  __shared__ double scratch[256];
  block_reduce_parts<R * R>(partW, nb, small + kWtW * R * R, scratch);
  block_reduce_parts<R * R>(partV, nb, small + kVtV * R * R, scratch);
}

static __global__ void k_zero(float *x, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0f;
}

static __global__ void k_reset_scalars(FitScalars *sc) {
  if (threadIdx.x == 0) {
    sc->cur = -1;  // pass 1 of the first iteration makes it 0
    sc->iter = 0;
    sc->fail_iter = INT_MAX;
    sc->rank_deficient = 0;
    sc->rank_def_slot[0] = 0;
    sc->rank_def_slot[1] = 0;
  }
}

// Qtilde rows: c_i Q_k (smoothed) or the Q row itself
template <int R>
__global__ void __launch_bounds__(256)
    k_qtilde(int64_t S, int l, const int32_t *__restrict__ rowsubj, const float *__restrict__ C,
             const float *__restrict__ Q, float *__restrict__ Qt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  if (l > 0) {
    const int64_t k = rowsubj[i];
    float c[kLMax];
#pragma unroll
    for (int a = 0; a < kLMax; ++a) c[a] = C[i * kLMax + a];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float s = 0.0f;
#pragma unroll
      for (int a = 0; a < kLMax; ++a)
        if (a < l) s += c[a] * Q[(k * l + a) * R + r];
      Qt[i * R + r] = s;
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) Qt[i * R + r] = Q[i * R + r];
  }
}

// ======================================================================= host launchers
template <int RT>
static void launch_pass1_rt(copa_plan *p, const float *, hipStream_t s) {
  constexpr int RTP = row4(RT);
  const int cg = p->tiles.cg;
  size_t lds = (size_t)cg * p->J * RTP * sizeof(float) + sizeof(float4);  // + the spare slot
  const int per_cu =
      std::max(1, std::min(p->p1_per_cu, (int)(160 * 1024 / std::max<size_t>(lds, 1))));
  const int nb = std::max(1, std::min((p->n_waves1 + 3) / 4, p->n_cu * per_cu));
  dim3 grid((unsigned)nb, (unsigned)(p->tiles.nt / cg)), block(256);
#define P1(SM, CP)                                                                              \
  k_pass1<RT, SM, CP><<<grid, block, lds, s>>>(p->waves1, p->n_waves1, p->order1, p->subj,       \
                                              p->row, p->col, p->val, p->xc, p->C, p->Vp, p->J, \
                                              p->R, p->l, cg, p->T, p->FV, p->scal)
  if (p->proj) {
    // the common basis size l = 7 has its own instances (fewer accumulators, no row guards)
    if (p->use_bf && p->l == 7)
      k_pass1p<RT, 8, true, 7><<<grid, block, lds, s>>>(p->waves1, p->n_waves1, p->order1, p->pp,
                                                         p->pairs1h, p->Vp, p->J, p->R, p->l, cg,
                                                         p->T, p->FV, p->scal);
    else if (p->use_bf)
      k_pass1p<RT, 8, true><<<grid, block, lds, s>>>(p->waves1, p->n_waves1, p->order1, p->pp,
                                                      p->pairs1h, p->Vp, p->J, p->R, p->l, cg,
                                                      p->T, p->FV, p->scal);
    else if (p->pw == 8 && p->l == 7)
      k_pass1p<RT, 8, false, 7><<<grid, block, lds, s>>>(p->waves1, p->n_waves1, p->order1,
                                                          p->pp, p->pairs1, p->Vp, p->J, p->R,
                                                          p->l, cg, p->T, p->FV, p->scal);
    else if (p->pw == 8)
      k_pass1p<RT, 8, false><<<grid, block, lds, s>>>(p->waves1, p->n_waves1, p->order1, p->pp,
                                                       p->pairs1, p->Vp, p->J, p->R, p->l, cg,
                                                       p->T, p->FV, p->scal);
    else
      k_pass1p<RT, 12, false><<<grid, block, lds, s>>>(p->waves1, p->n_waves1, p->order1, p->pp,
                                                        p->pairs1, p->Vp, p->J, p->R, p->l, cg,
                                                        p->T, p->FV, p->scal);
  } else if (p->l > 0) {
    if (p->compact) P1(true, true); else P1(true, false);
  } else {
    if (p->compact) P1(false, true); else P1(false, false);
  }
#undef P1
}

template <int RT>
static void launch_pass2c_rt(copa_plan *p, hipStream_t s) {
  if (p->proj)
    launch_pass2p<RT>(p, p->FV, s);
  else if (p->l > 0)
    launch_pass2c<RT, true>(p, p->M, p->FV, s);
  else
    launch_pass2c<RT, false>(p, p->M, p->FV, s);
}

// unchunked pass 2 (features past 2^16 or F_V tiles too wide for LDS): pass-1 tiling
template <int RT>
static void launch_pass2_rt(copa_plan *p, hipStream_t s) {
  dim3 grid((unsigned)((p->n_waves + 3) / 4), (unsigned)p->tiles.nt), block(256);
  if (p->l > 0)
    k_pass2<RT, true><<<grid, block, 0, s>>>(p->waves, p->n_waves, p->order, p->subj, p->row,
                                            p->col, p->val, p->C, p->M, p->J, p->R, p->l,
                                            p->FV);
  else
    k_pass2<RT, false><<<grid, block, 0, s>>>(p->waves, p->n_waves, p->order, p->subj, p->row,
                                             p->col, p->val, p->C, p->M, p->J, p->R, p->l,
                                             p->FV);
}

#define RT_SWITCH(rt, FN, ...)                                                               \
  switch (rt) {                                                                              \
    case 1: FN<1>(__VA_ARGS__); break;   case 2: FN<2>(__VA_ARGS__); break;                   \
    case 3: FN<3>(__VA_ARGS__); break;   case 4: FN<4>(__VA_ARGS__); break;                   \
    case 5: FN<5>(__VA_ARGS__); break;   case 6: FN<6>(__VA_ARGS__); break;                   \
    case 7: FN<7>(__VA_ARGS__); break;   case 8: FN<8>(__VA_ARGS__); break;                   \
    case 9: FN<9>(__VA_ARGS__); break;   case 10: FN<10>(__VA_ARGS__); break;                 \
    case 11: FN<11>(__VA_ARGS__); break; case 12: FN<12>(__VA_ARGS__); break;                 \
    case 13: FN<13>(__VA_ARGS__); break; case 14: FN<14>(__VA_ARGS__); break;                 \
    case 15: FN<15>(__VA_ARGS__); break; case 16: FN<16>(__VA_ARGS__); break;                 \
    default: break;                                                                          \
  }

// pass-2 widths: RT_SWITCH's and the wider tiles up to the rank (only widths <= R occur)
#define RT2_SWITCH(R, rt, FN, ...)                                                           \
  switch (rt) {                                                                              \
    case 20: if constexpr (R >= 20) FN<20>(__VA_ARGS__); break;                              \
    case 24: if constexpr (R >= 24) FN<24>(__VA_ARGS__); break;                              \
    case 32: if constexpr (R >= 32) FN<32>(__VA_ARGS__); break;                              \
    case 40: if constexpr (R >= 40) FN<40>(__VA_ARGS__); break;                              \
    default: RT_SWITCH(rt, FN, __VA_ARGS__); break;                                          \
  }


// Pass 2 in the plan's form: feature-sorted chunks (pairs or rows) or the unchunked row pass.
template <int R>
static void launch_pass2_any(copa_plan *p, hipStream_t s) {
  if (p->p2c || p->proj) {
    RT2_SWITCH(R, p->tiles2.rt, launch_pass2c_rt, p, s);
  } else {
    RT_SWITCH(p->tiles.rt, launch_pass2_rt, p, s);
  }
}

enum {
  kidPass1, kidProcrustes, kidGramFH, kidModeH, kidWadmm, kidGramWM, kidPass2, kidVadmm,
  kidWfirst, kidMrows, kidFinish, kidProcGram, kidProcEigen, kidProcQ
};

// Records a HIP event pair around one launch when the plan's timing is on.
template <typename F>
static inline void timed(copa_plan *p, hipStream_t s, int kid, F &&launch) {
  if (p->timing && p->ev_used + 2 <= (int)p->ev_pool.size()) {
    (void)hipEventRecord(p->ev_pool[p->ev_used], s);
    launch();
    (void)hipEventRecord(p->ev_pool[p->ev_used + 1], s);
    p->ev_kid.push_back(kid);
    p->ev_used += 2;
  } else {
    launch();
  }
}


// Blocks of the persistent W-first launch over `units` subjects (at most wf_blocks) and of the
// M-row launch over `units` groups of kMRows rows (at most wf_cap: its registers leave room for
// more wavefronts).
static int wf_grid(const copa_plan *p, int64_t units, bool mrows = false) {
  const int64_t per = 4 * (kWave / p->R);
  const int64_t cap = mrows ? p->mr_blocks : p->wf_blocks;
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (units + per - 1) / per));
}

static FitArgs fit_args(const copa_plan *p) {
  const copa_options &o = p->opt;
  FitArgs fa;
  fa.vpart = p->vpart;
  // many large V^T V partials are added by a launch of their own right after the V update
  fa.vtvpart = p->vtv_reduce ? gram_total(p, kSlotVtV) : gram_slot(p, kSlotVtV);
  fa.nvtv = p->vtv_reduce ? 1 : p->n_vblocks;
  fa.nvb = p->n_vblocks;
  fa.wl1part = p->wpart;
  fa.nwb = p->opt.order == COPA_ORDER_WHV ? wf_grid(p, p->K) : p->n_wblocks;
  fa.normX2 = p->normX2;
  fa.J = p->J;
  fa.proxV = o.prox_V;
  fa.proxW = o.prox_W;
  fa.proxH = o.prox_H;
  fa.lamV = o.lambda_V;
  fa.lamW = o.lambda_W;
  fa.lamH = o.lambda_H;
  return fa;
}

// The Procrustes step of one outer iteration (variant by l, R and the tuned proc_variant).
template <int R>
static void launch_procrustes_r(copa_plan *p, const copa_state *st, hipStream_t s) {
  const copa_options &o = p->opt;
  const int64_t K = p->K;
  if constexpr (R > 16) {
    if (p->l > 0 && p->proc_variant == 0) {
      const size_t lds = procrustes_l_lds(R, p->l);
      if (p->l == 7)
        k_procrustes_l<R, 7><<<(unsigned)((K + 63) / 64), 64, lds, s>>>(
            K, p->l, p->rk, p->T, p->Q, st->H, st->W, p->Ew, o.rank_rtol, p->scal);
      else
        k_procrustes_l<R, kLMax><<<(unsigned)((K + 63) / 64), 64, lds, s>>>(
            K, p->l, p->rk, p->T, p->Q, st->H, st->W, p->Ew, o.rank_rtol, p->scal);
      return;
    }
    if (p->l > 0 && p->proc_variant == 2) {
      if (p->l == 7)
        launch_proc_split<R, 7>(p, st, s, PlainLaunch{});
      else
        launch_proc_split<R, kLMax>(p, st, s, PlainLaunch{});
      return;
    }
    if (p->l > 0) {
      if (p->l == 7)
        k_procrustes_m<R, 7><<<(unsigned)((K + 63) / 64), 256, procrustes_m_lds(R, 7, 7),
                               s>>>(K, p->l, p->rk, p->T, p->Q, st->H, st->W, p->Ew,
                                    o.rank_rtol, p->scal);
      else
        k_procrustes_m<R, kLMax><<<(unsigned)((K + 63) / 64), 256,
                                   procrustes_m_lds(R, p->l, kLMax), s>>>(
            K, p->l, p->rk, p->T, p->Q, st->H, st->W, p->Ew, o.rank_rtol, p->scal);
      return;
    }
  }
  if constexpr (R <= 16) {
    if (p->l > 0) {
      if (p->l == 7)
        k_procrustes_s<R, 7><<<(unsigned)((K + 63) / 64), 64, 0, s>>>(
            K, p->l, p->rk, p->T, p->Q, st->H, st->W, p->Ew, o.rank_rtol, p->scal);
      else
        k_procrustes_s<R, kLMax><<<(unsigned)((K + 63) / 64), 64, 0, s>>>(
            K, p->l, p->rk, p->T, p->Q, st->H, st->W, p->Ew, o.rank_rtol, p->scal);
      return;
    }
  }
  k_procrustes<R><<<(unsigned)((K + 63) / 64), 64, 0, s>>>(
      K, p->l, p->subj, p->rk, p->T, p->Q, p->M, st->H, st->W, o.rank_rtol, p->scal);
  if (p->n_big > 0)
    k_procrustes_wave<R><<<(unsigned)p->n_big, 64, 0, s>>>(
        p->big_list, p->n_big, p->subj, p->T, p->Q, st->H, st->W, o.rank_rtol, p->scal);
    }

// One outer iteration; pass 1 advances the device iteration index and the later kernels read it,
// so the same launches serve every iteration (and one captured graph replays them).
// The Procrustes step of an iteration, timed per launch (the three-launch form as three kernels).
template <int R>
static void procrustes_step(copa_plan *p, const copa_state *st, hipStream_t s) {
  if (p->K == 0) return;
  if constexpr (R > 16) {
    if (p->l > 0 && p->proc_variant == 2) {
      auto each = [&](int part, auto &&launch) {
        timed(p, s, part == 0 ? kidProcGram : part == 1 ? kidProcEigen : kidProcQ, launch);
      };
      if (p->l == 7)
        launch_proc_split<R, 7>(p, st, s, each);
      else
        launch_proc_split<R, kLMax>(p, st, s, each);
      return;
    }
  }
  timed(p, s, kidProcrustes, [&] { launch_procrustes_r<R>(p, st, s); });
}

template <int R>
static void iteration_r(copa_plan *p, const copa_state *st, hipStream_t s) {
  const copa_options &o = p->opt;
  const int64_t K = p->K;
  timed(p, s, kidPass1, [&] { RT_SWITCH(p->tiles.rt, launch_pass1_rt, p, st->V, s); });
  procrustes_step<R>(p, st, s);
  timed(p, s, kidGramFH, [&] {
    // one more block of the same launch takes the FIT of the previous outer iteration
    const FitArgs fa = fit_args(p);
    gram_fit<R>(p, p->Q, p->T, p->rows_total, st->W, p->l > 0 ? 1 : 2, kSlotFH, fa, st->H, s);
  });
  timed(p, s, kidModeH, [&] {
    k_mode_H<R><<<1, 256, 0, s>>>(gram_total(p, kSlotFH), nullptr, p->small, p->modes, p->scal,
                                  st->H, st->D_H, o.prox_H, o.lambda_H, o.inner_iters, 1);
  });
  timed(p, s, kidWadmm, [&] {
    k_w_admm<R><<<(unsigned)p->n_wblocks, 256, 0, s>>>(K, p->l, p->subj, p->rk, p->T, p->Q, p->M, st->H, st->W,
                                   st->D_W, p->FW, p->modes, o.prox_W, o.lambda_W,
                                   o.inner_iters, p->wpart);
  });
  timed(p, s, kidGramWM, [&] {
    gram<R>(p, st->W, st->W, K, nullptr, 0, kSlotWtW, p->M, p->rows_total, kSlotPsi, s);
  });
  timed(p, s, kidPass2, [&] { launch_pass2_any<R>(p, s); });
  timed(p, s, kidVadmm, [&] {
    k_v_system<R><<<1, 256, 0, s>>>(gram_total(p, kSlotWtW), p->small, p->modes, p->scal);
    k_v_admm<R><<<p->n_vblocks, 256, 0, s>>>(
        p->J, p->FV, st->V, st->D_V, p->Vp, p->tiles.rt, row4(p->tiles.rt),
        gram_total(p, kSlotWtW), gram_total(p, kSlotPsi), p->small, p->modes, o.prox_V,
        o.lambda_V, o.inner_iters, p->vpart, gram_slot(p, kSlotVtV));
    if (p->vtv_reduce)
      k_gram_reduce<R * R><<<dim3((R * R + 3) / 4, 1), 256, 0, s>>>(
          gram_slot(p, kSlotVtV), gram_total(p, kSlotVtV), nullptr, nullptr, p->n_vblocks);
  });
}

// One outer iteration in the block order W -> H -> V: the W block runs right after the
// Procrustes step with the previous H (F_H and W^T W of the new W come out of the same launch),
// then the H block, the M rows and Psi, pass 2 and the V block; the FIT of the iteration and the
// next W system close it.
template <int R>
static void iteration_whv_r(copa_plan *p, const copa_state *st, hipStream_t s) {
  const copa_options &o = p->opt;
  const int64_t K = p->K;
  timed(p, s, kidPass1, [&] { RT_SWITCH(p->tiles.rt, launch_pass1_rt, p, st->V, s); });
  procrustes_step<R>(p, st, s);
  timed(p, s, kidWfirst, [&] {
    const int nb = wf_grid(p, K);
    k_w_first<R><<<(unsigned)nb, 256, 0, s>>>(
        K, p->l, p->subj, p->rk, p->T, p->Q, st->H, st->W, st->D_W, p->FW, p->modes, o.prox_W,
        o.lambda_W, o.inner_iters, p->wpart, gram_slot(p, kSlotFH), gram_slot(p, kSlotWtW));
    k_gram_reduce<R * R><<<dim3((R * R + 3) / 4, 2), 256, 0, s>>>(
        gram_slot(p, kSlotFH), gram_total(p, kSlotFH), gram_slot(p, kSlotWtW),
        gram_total(p, kSlotWtW), nb);
  });
  timed(p, s, kidModeH, [&] {
    k_mode_H<R><<<1, 256, 0, s>>>(gram_total(p, kSlotFH), gram_total(p, kSlotWtW), p->small,
                                  p->modes, p->scal, st->H, st->D_H, o.prox_H, o.lambda_H,
                                  o.inner_iters, 0);
  });
  timed(p, s, kidMrows, [&] {
    const int nb = wf_grid(p, (p->rows_total + kMRows - 1) / kMRows, true);
    k_m_rows<R><<<(unsigned)nb, 256, 0, s>>>(p->rows_total, p->l, p->rowsubj, p->Q, st->H,
                                             st->W, p->M, gram_slot(p, kSlotPsi));
    k_gram_reduce<R * R><<<dim3((R * R + 3) / 4, 1), 256, 0, s>>>(
        gram_slot(p, kSlotPsi), gram_total(p, kSlotPsi), nullptr, nullptr, nb);
  });
  timed(p, s, kidPass2, [&] { launch_pass2_any<R>(p, s); });
  timed(p, s, kidVadmm, [&] {
    k_v_admm<R><<<p->n_vblocks, 256, 0, s>>>(
        p->J, p->FV, st->V, st->D_V, p->Vp, p->tiles.rt, row4(p->tiles.rt),
        gram_total(p, kSlotWtW), gram_total(p, kSlotPsi), p->small, p->modes, o.prox_V,
        o.lambda_V, o.inner_iters, p->vpart, gram_slot(p, kSlotVtV));
    if (p->vtv_reduce)
      k_gram_reduce<R * R><<<dim3((R * R + 3) / 4, 1), 256, 0, s>>>(
          gram_slot(p, kSlotVtV), gram_total(p, kSlotVtV), nullptr, nullptr, p->n_vblocks);
  });
  timed(p, s, kidFinish, [&] {
    k_finish_whv<R><<<1, 256, 0, s>>>(fit_args(p), 1, st->H, p->small, p->modes, p->scal);
  });
}

template <int R>
static void init_grams_r(copa_plan *p, const copa_state *st, hipStream_t s) {
  constexpr int RR = R * R;
  k_reset_scalars<<<1, 64, 0, s>>>(p->scal);
  if (p->reset_warm && p->Ew && p->K > 0)
    k_eye8<<<(unsigned)std::min<int64_t>(4096, (p->K * kNMax * kNMax + 255) / 256), 256, 0, s>>>(
        p->Ew, p->K);
  if (p->J > 0)
    k_pad_V<R><<<(unsigned)((p->J * R + 255) / 256), 256, 0, s>>>(
        st->V, p->Vp, p->J, p->tiles.rt, row4(p->tiles.rt));
  gram<R>(p, st->W, st->W, p->K, nullptr, 0, kSlotWtW, st->V, p->J, kSlotVtV, s);
  k_init_small<R><<<1, 256, 0, s>>>(gram_total(p, kSlotWtW), gram_total(p, kSlotVtV), 1,
                                    p->small);
  if (p->opt.order == COPA_ORDER_WHV) {
    if (p->wf_blocks == 0) {
      // persistent grids of as many blocks as stay resident (a fixed count for a given build
      // and device, so that the fixed-order mode's summation order is fixed too)
      int b1 = 0, b2 = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, k_w_first<R>, 256, 0) != hipSuccess)
        b1 = 1;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, k_m_rows<R>, 256, 0) != hipSuccess)
        b2 = 1;
      const int ncu = std::max(1, p->n_cu);
      p->wf_blocks = std::max(1, std::min(p->wf_cap, std::max(1, b1) * ncu));
      p->mr_blocks = std::max(1, std::min(p->wf_cap, std::max(1, b2) * ncu));
    }
    // the first W system
    k_finish_whv<R><<<1, 256, 0, s>>>(fit_args(p), 0, st->H, p->small, p->modes, p->scal);
  }
}

// Per-rank entry points of the iteration; each rank is instantiated in one of the
// copa_iter_r*.hip translation units (compiled in parallel).
template <int R>
struct RankOps {
  static void iteration(copa_plan *p, const copa_state *st, hipStream_t s);
  static void fit(copa_plan *p, const copa_state *st, hipStream_t s);
  static void init_grams(copa_plan *p, const copa_state *st, hipStream_t s);
  static void qtilde(copa_plan *p, float *Qt, hipStream_t s);
  static copa_status tune(copa_plan *p, const copa_state *st, hipStream_t s);
};
// (defined out of the class so that they are not inline: the extern declarations below then
// keep every other translation unit from instantiating the kernels)
template <int R>
void RankOps<R>::iteration(copa_plan *p, const copa_state *st, hipStream_t s) {
  if (p->opt.order == COPA_ORDER_WHV)
    iteration_whv_r<R>(p, st, s);
  else
    iteration_r<R>(p, st, s);
}
template <int R>
void RankOps<R>::fit(copa_plan *p, const copa_state *st, hipStream_t s) {
  // (the W -> H -> V iteration takes its own FIT at its end)
  if (p->opt.order != COPA_ORDER_WHV)
    k_fit<R><<<1, 256, 0, s>>>(fit_args(p), st->H, p->small, p->scal);
}
template <int R>
void RankOps<R>::init_grams(copa_plan *p, const copa_state *st, hipStream_t s) {
  init_grams_r<R>(p, st, s);
}
// Autotuner: times candidate launch shapes of the passes, the Procrustes step and the row Grams
// on the plan's own data (the fit's starting point) and keeps the fastest of each. Every kernel
// timed here writes only buffers the iteration writes again before reading them (T, Q, the
// warm-start eigenvectors, which the fit then resets, F_V, the Gram slots), so the fit that
// follows is unaffected apart from the launch shapes.
template <int R>
copa_status RankOps<R>::tune(copa_plan *p, const copa_state *st, hipStream_t s) {
  hipEvent_t e0, e1;
  COPA_HIP(hipEventCreate(&e0));
  COPA_HIP(hipEventCreate(&e1));
  auto time_it = [&](auto &&launch) -> float {
    float best = 1e30f;
    launch();  // warm (first-touch, code load)
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(e0, s);
      launch();
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, ms);
    }
    return best;
  };
  k_reset_scalars<<<1, 64, 0, s>>>(p->scal);
  init_grams_r<R>(p, st, s);  // padded image of V, W^T W, V^T V
  // pass 1: persistent blocks per compute unit
  {
    int best_c = p->p1_per_cu;
    float best_t = 1e30f;
    for (int c : {1, 2, 3, 4}) {
      p->p1_per_cu = c;
      const float t = time_it([&] { RT_SWITCH(p->tiles.rt, launch_pass1_rt, p, st->V, s); });
      if (t < best_t) best_t = t, best_c = c;
    }
    p->p1_per_cu = best_c;
  }
  // T now holds the rows of the starting point: the Procrustes variants (smoothed, R > 16)
  if (R > 16 && p->l > 0 && p->K > 0) {
    int best_v = 0;
    float best_t = 1e30f;
    for (int v : {0, 1, 2}) {
      p->proc_variant = v;
      const float t = time_it([&] { launch_procrustes_r<R>(p, st, s); });
      if (t < best_t) best_t = t, best_v = v;
    }
    p->proc_variant = best_v;
  }
  // the row Grams (F_H's launch shape) and the pass-2 grid
  {
    int best_g = p->gram_blocks;
    float best_t = 1e30f;
    for (int g : {p->gmaxnb / 4, p->gmaxnb / 2, p->gmaxnb}) {
      if (g < 1) continue;
      p->gram_blocks = g;
      const float t = time_it([&] {
        gram<R>(p, p->Q, p->T, p->rows_total, st->W, p->l > 0 ? 1 : 2, kSlotFH, nullptr, 0, 0, s);
      });
      if (t < best_t) best_t = t, best_g = g;
    }
    p->gram_blocks = best_g;
  }
  if (p->p2c || p->proj) {
    int best_b = p->p2_blocks;
    float best_t = 1e30f;
    for (int b : {p->p2_blocks_cap / 4, p->p2_blocks_cap / 2, p->p2_blocks_cap}) {
      if (b < 1) continue;
      p->p2_blocks = b;
      const float t = time_it([&] { launch_pass2_any<R>(p, s); });
      if (t < best_t) best_t = t, best_b = b;
    }
    p->p2_blocks = best_b;
  }
  COPA_HIP(hipStreamSynchronize(s));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

template <int R>
void RankOps<R>::qtilde(copa_plan *p, float *Qt, hipStream_t s) {
  const unsigned nb = (unsigned)((p->S + 255) / 256);
  k_qtilde<R><<<nb, 256, 0, s>>>(p->S, p->l, p->rowsubj, p->C, p->Q, Qt);
}
#define COPA_EXTERN_RANK(r) extern template struct RankOps<r>;
COPA_R_LIST(COPA_EXTERN_RANK)
#undef COPA_EXTERN_RANK

}  // namespace copa
