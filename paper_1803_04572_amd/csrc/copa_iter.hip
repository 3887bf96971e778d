// One outer iteration of COPA (Algorithm 1) on the GPU, and the copa_fit / copa_mttkrp_last ABI.
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

#include "copa_common.h"

namespace copa {

#define COPA_R_LIST(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(15) X(16) X(20) X(24) X(32) X(40)

bool rank_supported(int R) {
  switch (R) {
#define CASE(r) case r:
    COPA_R_LIST(CASE)
#undef CASE
    return true;
    default: return false;
  }
}

Tiles choose_tiles(int R, int64_t J, int lds_limit) {
  int nt = (R + 15) / 16;
  for (;; ++nt) {
    int rt = (R + nt - 1) / nt;
    int rtp = (rt + 3) & ~3;
    if ((int64_t)J * rtp * 4 <= lds_limit || rt == 1) return Tiles{nt, rt};
  }
}

// small-buffer layout (FP64 R x R each)
enum { kFH = 0, kHtH = 1, kWtW = 2, kVtV = 3, kPsi = 4 };

// ======================================================================= streaming pass 1
// Wave list: each wave takes `cnt` subjects; G lanes per subject stride over its visit rows.
template <int RT, bool SMOOTH>
__global__ void __launch_bounds__(256)
    k_pass1(const WaveEntry *__restrict__ waves, int n_waves, const int32_t *__restrict__ order,
            const int32_t *__restrict__ subj, const int32_t *__restrict__ row,
            const int32_t *__restrict__ col, const float *__restrict__ val,
            const float *__restrict__ C, const float *__restrict__ V, int64_t J, int R, int l,
            float *__restrict__ T) {
  constexpr int RTP = (RT + 3) & ~3;
  extern __shared__ float4 smem4[];
  float *sV = reinterpret_cast<float *>(smem4);
  const int c0 = blockIdx.y * RT;
  for (int64_t e = threadIdx.x; e < J * RTP; e += blockDim.x) {
    int64_t j = e / RTP;
    int r = (int)(e - j * RTP);
    sV[e] = (r < RT && c0 + r < R) ? V[j * R + c0 + r] : 0.0f;
  }
  __syncthreads();
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wv >= n_waves) return;
  const int lane = threadIdx.x & 63;
  const WaveEntry we = waves[wv];
  const int lg = we.lg_count & 255, cnt = we.lg_count >> 8;
  const int G = 1 << lg, sidx = lane >> lg, sub = lane & (G - 1);
  const bool active = sidx < cnt;
  const int k = active ? order[we.first + sidx] : 0;
  const int r0 = active ? subj[k] : 0, r1 = active ? subj[k + 1] : 0;

  if constexpr (SMOOTH) {
    float acc[kLMax][RT];
#pragma unroll
    for (int a = 0; a < kLMax; ++a)
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[a][r] = 0.0f;
    for (int i = r0 + sub; i < r1; i += G) {
      float t[RTP];
#pragma unroll
      for (int r = 0; r < RTP; ++r) t[r] = 0.0f;
      const int e1 = row[i + 1];
      for (int e = row[i]; e < e1; ++e) {
        const float x = val[e];
        const float4 *v4 = reinterpret_cast<const float4 *>(sV + (int64_t)col[e] * RTP);
#pragma unroll
        for (int q = 0; q < RTP / 4; ++q) {
          float4 v = v4[q];
          t[4 * q + 0] += x * v.x;
          t[4 * q + 1] += x * v.y;
          t[4 * q + 2] += x * v.z;
          t[4 * q + 3] += x * v.w;
        }
      }
      const float4 *c4 = reinterpret_cast<const float4 *>(C + (int64_t)i * kLMax);
      float4 ca = c4[0], cb = c4[1];
      float c[kLMax] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
#pragma unroll
      for (int a = 0; a < kLMax; ++a)
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[a][r] += c[a] * t[r];
    }
    for (int m = 1; m < G; m <<= 1) {
#pragma unroll
      for (int a = 0; a < kLMax; ++a)
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[a][r] += shfl_xor_f(acc[a][r], m);
    }
    if (active) {
      float *dst = T + (int64_t)k * l * R + c0;
#pragma unroll
      for (int a = 0; a < kLMax; ++a)
#pragma unroll
        for (int r = 0; r < RT; ++r)
          if (a < l && c0 + r < R && ((a * RT + r) & (G - 1)) == sub) dst[a * R + r] = acc[a][r];
    }
  } else {
    if (!active) return;
    for (int i = r0 + sub; i < r1; i += G) {
      float t[RTP];
#pragma unroll
      for (int r = 0; r < RTP; ++r) t[r] = 0.0f;
      const int e1 = row[i + 1];
      for (int e = row[i]; e < e1; ++e) {
        const float x = val[e];
        const float4 *v4 = reinterpret_cast<const float4 *>(sV + (int64_t)col[e] * RTP);
#pragma unroll
        for (int q = 0; q < RTP / 4; ++q) {
          float4 v = v4[q];
          t[4 * q + 0] += x * v.x;
          t[4 * q + 1] += x * v.y;
          t[4 * q + 2] += x * v.z;
          t[4 * q + 3] += x * v.w;
        }
      }
      float *dst = T + (int64_t)i * R + c0;
#pragma unroll
      for (int r = 0; r < RT; ++r)
        if (c0 + r < R) dst[r] = t[r];
    }
  }
}

// ======================================================================= Procrustes
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
          const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
          const double t = copysign(1.0, tau) / (fabs(tau) + sqrt(1.0 + tau * tau));
          const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
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

// One subject per lane, eigenproblem size n = min(m, R) <= kNMax.
// A rows a_i = (t_i * w) H^T are computed in FP64 and kept as FP32 in the M buffer (free until
// the W update). Rows side (m <= R): Gram A A^T, Q = (A A^T)^{+1/2} A. Columns side (m > R):
// Gram A^T A, Q = A (A^T A)^{+1/2}. Eigenvalues at or below rtol^2 * lambda_max are dropped.
template <int R>
__global__ void __launch_bounds__(64)
    k_procrustes(int64_t K, int l, const int32_t *__restrict__ subj,
                 const int32_t *__restrict__ rk, const float *__restrict__ T,
                 float *__restrict__ Q, float *__restrict__ Abuf, const float *__restrict__ H,
                 const float *__restrict__ W, double rtol, int32_t *rank_def) {
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
  if (rank < (meff < R ? meff : R)) atomicAdd(rank_def, 1);
}

// ======================================================================= row Gram reductions
// part[b] = sum over rows of block b of A_row^T (B_row * w_subj(row)) (FP64, R x R).
// wsel: 0 = no scaling; 1 = scale B by W[row / slot_rows]; 2 = scale by W[rowsubj[row]].
template <int R>
__global__ void __launch_bounds__(256)
    k_rows_gram(const float *__restrict__ A, const float *__restrict__ B, int64_t rows,
                const float *__restrict__ W, int wsel, int slot_rows,
                const int32_t *__restrict__ rowsubj, double *__restrict__ part) {
  constexpr int CH = 64;
  constexpr int E = (R * R + 255) / 256;
  __shared__ float sA[CH * R];
  __shared__ float sB[CH * R];
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * per;
  const int64_t hi = lo + per < rows ? lo + per : rows;
  double acc[E];
#pragma unroll
  for (int s = 0; s < E; ++s) acc[s] = 0.0;
  for (int64_t c0 = lo; c0 < hi; c0 += CH) {
    const int n = (int)((hi - c0) < CH ? (hi - c0) : CH);
    __syncthreads();
    for (int e = threadIdx.x; e < n * R; e += blockDim.x) {
      const int64_t rr = c0 + e / R;
      const int c = e % R;
      sA[e] = A[rr * R + c];
      float bv = B[rr * R + c];
      if (wsel == 1) bv *= W[(rr / slot_rows) * R + c];
      else if (wsel == 2) bv *= W[(int64_t)rowsubj[rr] * R + c];
      sB[e] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int e = threadIdx.x + s * 256;
      if (e < R * R) {
        const int a = e / R, b = e % R;
        double v = 0.0;
        for (int rr = 0; rr < n; ++rr) v += (double)sA[rr * R + a] * (double)sB[rr * R + b];
        acc[s] += v;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int e = threadIdx.x + s * 256;
    if (e < R * R) part[(int64_t)blockIdx.x * R * R + e] = acc[s];
  }
}

// dst = sum_b part[b] in fixed order
__device__ void reduce_parts(const double *part, int nb, int RR, double *dst) {
  for (int e = threadIdx.x; e < RR; e += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * RR + e];
    dst[e] = s;
  }
}

// ======================================================================= ADMM helpers
// Cholesky of G + rho I in shared memory (FP64, lower triangle, row-major). Returns false
// (and leaves L = I) if a pivot is not positive and finite.
template <int R>
__device__ bool block_cholesky(double *sL, int *sflag) {
  if (threadIdx.x == 0) *sflag = 0;
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    if (threadIdx.x == 0) {
      double d = sL[j * R + j];
      if (!(d > 0.0) || !isfinite(d)) {
        *sflag = 1;
        d = 1.0;
      }
      sL[j * R + j] = sqrt(d);
    }
    __syncthreads();
    const double djj = sL[j * R + j];
    for (int i = j + 1 + threadIdx.x; i < R; i += blockDim.x) sL[i * R + j] /= djj;
    __syncthreads();
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
      const int i = e / R, c = e % R;
      if (i > j && c > j && c <= i) sL[i * R + c] -= sL[i * R + j] * sL[c * R + j];
    }
    __syncthreads();
  }
  const bool ok = *sflag == 0;
  if (!ok) {
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) sL[e] = (e / R == e % R) ? 1.0 : 0.0;
  }
  __syncthreads();
  return ok;
}

// Builds G = X * Y (Hadamard), rho = tr(G)/R and its Cholesky into `mp`; flags failure.
template <int R>
__device__ void mode_prepare(const double *X, const double *Y, ModeParams *mp, FitScalars *sc) {
  __shared__ double sL[R * R];
  __shared__ double srho;
  __shared__ int sflag;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sL[e] = X[e] * Y[e];
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0;
    for (int i = 0; i < R; ++i) tr += sL[i * R + i];
    srho = tr / R;
  }
  __syncthreads();
  const double rho = srho;
  for (int i = threadIdx.x; i < R; i += blockDim.x) sL[i * R + i] += rho;
  __syncthreads();
  const bool ok = block_cholesky<R>(sL, &sflag) && isfinite(rho) && rho > 0.0;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) mp->L[e] = sL[e];
  if (threadIdx.x == 0) {
    mp->rho = rho > 0.0 && isfinite(rho) ? rho : 1.0;
    if (!ok) atomicMin(&sc->fail_iter, sc->iter);
  }
}

// Inner ADMM steps on one row (Algorithm 1 inner loop):
//   Z = (F + rho (Zb + D)) (G + rho I)^{-1}  via L L^T,  Zb = prox(Z - D),  D += Zb - Z.
template <int R>
__device__ __forceinline__ void admm_row(const double (&F)[R], float (&Zb)[R], float (&D)[R],
                                         const double *__restrict__ sL, double rho, int kind,
                                         double lam, int iters) {
  for (int it = 0; it < iters; ++it) {
    double z[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double s = F[i] + rho * ((double)Zb[i] + (double)D[i]);
#pragma unroll
      for (int j = 0; j < i; ++j) s -= sL[i * R + j] * z[j];
      z[i] = s / sL[i * R + i];
    }
#pragma unroll
    for (int i = R - 1; i >= 0; --i) {
      double s = z[i];
#pragma unroll
      for (int j = i + 1; j < R; ++j) s -= sL[j * R + i] * z[j];
      z[i] = s / sL[i * R + i];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const double zb = prox_apply(z[i] - (double)D[i], kind, lam, rho);
      D[i] = (float)((double)D[i] + zb - z[i]);
      Zb[i] = (float)zb;
    }
  }
}

// ======================================================================= mode H (one block)
template <int R>
__global__ void __launch_bounds__(256)
    k_mode_H(const double *__restrict__ part, int nb, double *small, ModeParams *modes,
             FitScalars *sc, float *H, float *DH, int kind, double lam, int iters) {
  __shared__ double sFH[R * R];
  __shared__ double sL[R * R];
  reduce_parts(part, nb, R * R, sFH);
  __syncthreads();
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) small[kFH * R * R + e] = sFH[e];
  mode_prepare<R>(small + kWtW * R * R, small + kVtV * R * R, &modes[0], sc);
  __syncthreads();
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sL[e] = modes[0].L[e];
  __syncthreads();
  const double rho = modes[0].rho;
  if (threadIdx.x < R) {
    const int i = threadIdx.x;
    double F[R];
    float Zb[R], D[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      F[c] = sFH[i * R + c];
      Zb[c] = H[i * R + c];
      D[c] = DH[i * R + c];
    }
    admm_row<R>(F, Zb, D, sL, rho, kind, lam, iters);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      H[i * R + c] = Zb[c];
      DH[i * R + c] = D[c];
    }
  }
  __threadfence_block();
  __syncthreads();
  // H^T H from the stored FP32 values, then the W-mode system G_W = H^TH * V^TV
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int a = e / R, b = e % R;
    double s = 0.0;
    for (int i = 0; i < R; ++i) s += (double)H[i * R + a] * (double)H[i * R + b];
    small[kHtH * R * R + e] = s;
  }
  __syncthreads();
  mode_prepare<R>(small + kHtH * R * R, small + kVtV * R * R, &modes[1], sc);
}

// ======================================================================= mode W (lane/subject)
template <int R>
__global__ void __launch_bounds__(64)
    k_w_admm(int64_t K, int l, const int32_t *__restrict__ subj, const int32_t *__restrict__ rk,
             const float *__restrict__ T, const float *__restrict__ Q, float *__restrict__ M,
             const float *__restrict__ H, float *__restrict__ W, float *__restrict__ DW,
             float *__restrict__ FW, const ModeParams *__restrict__ modes, int kind, double lam,
             int iters, double *__restrict__ l1part) {
  __shared__ double sL[R * R];
  __shared__ float sH[R * R];
  __shared__ double sred[64];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    sL[e] = modes[1].L[e];
    sH[e] = H[e];
  }
  __syncthreads();
  const double rho = modes[1].rho;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l1 = 0.0;
  if (k < K) {
    int64_t base;
    int m;
    if (l > 0) {
      base = k * l;
      m = rk[k];
    } else {
      base = subj[k];
      m = subj[k + 1] - subj[k];
    }
    // F_W(k, c) = sum_i (q_i H)(c) t_i(c)
    double F[R];
#pragma unroll
    for (int c = 0; c < R; ++c) F[c] = 0.0;
    for (int i = 0; i < m; ++i) {
      const float *q = Q + (base + i) * R;
      const float *t = T + (base + i) * R;
      float qv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) qv[r] = q[r];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double p = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) p += (double)qv[r] * sH[r * R + c];
        F[c] += p * (double)t[c];
      }
    }
    float Zb[R], D[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      Zb[c] = W[k * R + c];
      D[c] = DW[k * R + c];
      FW[k * R + c] = (float)F[c];
    }
    admm_row<R>(F, Zb, D, sL, rho, kind, lam, iters);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      W[k * R + c] = Zb[c];
      DW[k * R + c] = D[c];
      l1 += fabs((double)Zb[c]);
    }
    // M rows = (q_i H) * w_new
    const int mall = l > 0 ? l : m;
    for (int i = 0; i < mall; ++i) {
      const float *q = Q + (base + i) * R;
      float qv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) qv[r] = q[r];
      float *dst = M + (base + i) * R;
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double p = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) p += (double)qv[r] * sH[r * R + c];
        dst[c] = (float)(p * (double)Zb[c]);
      }
    }
  }
  sred[threadIdx.x] = l1;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < 64; ++i) s += sred[i];
    l1part[blockIdx.x] = s;
  }
}

// ======================================================================= streaming pass 2
// F_V += x_ij * u_i with u_i = c_i M_k (smoothed) or the M row of visit i. LDS-private F_V tile
// per block (flushed as a per-block partial), or global atomics when the tile does not fit.
template <int RT, bool SMOOTH, bool LDSACC>
__global__ void __launch_bounds__(1024)
    k_pass2(const WaveEntry *__restrict__ waves, int n_waves, const int32_t *__restrict__ order,
            const int32_t *__restrict__ subj, const int32_t *__restrict__ row,
            const int32_t *__restrict__ col, const float *__restrict__ val,
            const float *__restrict__ C, const float *__restrict__ M, int64_t J, int R, int l,
            float *__restrict__ FVpart, float *__restrict__ FV) {
  extern __shared__ float4 smem4[];
  float *sF = reinterpret_cast<float *>(smem4);
  const int c0 = blockIdx.y * RT;
  if constexpr (LDSACC) {
    for (int64_t e = threadIdx.x; e < J * RT; e += blockDim.x) sF[e] = 0.0f;
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int nwb = blockDim.x >> 6;
  for (int wv = blockIdx.x * nwb + (threadIdx.x >> 6); wv < n_waves; wv += gridDim.x * nwb) {
    const WaveEntry we = waves[wv];
    const int lg = we.lg_count & 255, cnt = we.lg_count >> 8;
    const int G = 1 << lg, sidx = lane >> lg, sub = lane & (G - 1);
    if (sidx >= cnt) continue;
    const int k = order[we.first + sidx];
    const int r0 = subj[k], r1 = subj[k + 1];
    float mk[SMOOTH ? kLMax : 1][RT];
    if constexpr (SMOOTH) {
#pragma unroll
      for (int a = 0; a < kLMax; ++a)
#pragma unroll
        for (int r = 0; r < RT; ++r)
          mk[a][r] = (a < l && c0 + r < R) ? M[((int64_t)k * l + a) * R + c0 + r] : 0.0f;
    }
    for (int i = r0 + sub; i < r1; i += G) {
      float u[RT];
      if constexpr (SMOOTH) {
        const float4 *c4 = reinterpret_cast<const float4 *>(C + (int64_t)i * kLMax);
        float4 ca = c4[0], cb = c4[1];
        float c[kLMax] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          float s = 0.0f;
#pragma unroll
          for (int a = 0; a < kLMax; ++a) s += c[a] * mk[a][r];
          u[r] = s;
        }
      } else {
#pragma unroll
        for (int r = 0; r < RT; ++r) u[r] = (c0 + r < R) ? M[(int64_t)i * R + c0 + r] : 0.0f;
      }
      const int e1 = row[i + 1];
      for (int e = row[i]; e < e1; ++e) {
        const float x = val[e];
        const int64_t j = col[e];
        if constexpr (LDSACC) {
#pragma unroll
          for (int r = 0; r < RT; ++r) atomicAdd(&sF[j * RT + r], x * u[r]);
        } else {
#pragma unroll
          for (int r = 0; r < RT; ++r)
            if (c0 + r < R) atomicAdd(&FV[j * R + c0 + r], x * u[r]);
        }
      }
    }
  }
  if constexpr (LDSACC) {
    __syncthreads();
    float *dst = FVpart + (int64_t)blockIdx.x * J * R;
    for (int64_t e = threadIdx.x; e < J * RT; e += blockDim.x) {
      const int64_t j = e / RT;
      const int r = (int)(e - j * RT);
      if (c0 + r < R) dst[j * R + c0 + r] = sF[e];
    }
  }
}

// ======================================================================= mode V
template <int R>
__global__ void __launch_bounds__(256)
    k_mode_V_prep(const double *__restrict__ partW, const double *__restrict__ partPsi, int nb,
                  double *small, ModeParams *modes, FitScalars *sc) {
  reduce_parts(partW, nb, R * R, small + kWtW * R * R);
  reduce_parts(partPsi, nb, R * R, small + kPsi * R * R);
  __threadfence_block();
  __syncthreads();
  mode_prepare<R>(small + kHtH * R * R, small + kWtW * R * R, &modes[2], sc);
}

template <int R>
__global__ void __launch_bounds__(256)
    k_v_admm(int64_t J, const float *__restrict__ FVpart, int nparts, float *__restrict__ FV,
             float *__restrict__ V, float *__restrict__ DV, const ModeParams *__restrict__ modes,
             int kind, double lam, int iters, double *__restrict__ vpart) {
  __shared__ double sL[R * R];
  __shared__ double sred[3][256];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sL[e] = modes[2].L[e];
  __syncthreads();
  const double rho = modes[2].rho;
  double dot = 0.0, l1 = 0.0, zeros = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < J;
       j += (int64_t)gridDim.x * blockDim.x) {
    double F[R];
    if (FVpart) {
#pragma unroll
      for (int c = 0; c < R; ++c) F[c] = 0.0;
      for (int b = 0; b < nparts; ++b) {
        const float *src = FVpart + ((int64_t)b * J + j) * R;
#pragma unroll
        for (int c = 0; c < R; ++c) F[c] += (double)src[c];
      }
#pragma unroll
      for (int c = 0; c < R; ++c) FV[j * R + c] = (float)F[c];
    } else {
#pragma unroll
      for (int c = 0; c < R; ++c) F[c] = FV[j * R + c];
    }
    float Zb[R], D[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      Zb[c] = V[j * R + c];
      D[c] = DV[j * R + c];
    }
    admm_row<R>(F, Zb, D, sL, rho, kind, lam, iters);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      V[j * R + c] = Zb[c];
      DV[j * R + c] = D[c];
      dot += F[c] * (double)Zb[c];
      l1 += fabs((double)Zb[c]);
      zeros += Zb[c] == 0.0f ? 1.0 : 0.0;
    }
  }
  sred[0][threadIdx.x] = dot;
  sred[1][threadIdx.x] = l1;
  sred[2][threadIdx.x] = zeros;
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int i = 0; i < 256; ++i) s += sred[threadIdx.x][i];
    vpart[blockIdx.x * 4 + threadIdx.x] = s;
  }
}

// ======================================================================= finalize
template <int R>
__global__ void __launch_bounds__(256)
    k_finalize(const double *__restrict__ partV, int nb, const double *__restrict__ vpart,
               int nvb, const double *__restrict__ wl1part, int nwb, double *small,
               FitScalars *sc, const float *__restrict__ H, double normX2, int64_t J,
               int proxH, double lamH, int proxW, double lamW, int proxV, double lamV) {
  reduce_parts(partV, nb, R * R, small + kVtV * R * R);
  __threadfence_block();
  __syncthreads();
  if (threadIdx.x == 0) {
    double dot = 0.0, l1 = 0.0, zeros = 0.0, wl1 = 0.0, hl1 = 0.0;
    for (int b = 0; b < nvb; ++b) {
      dot += vpart[b * 4 + 0];
      l1 += vpart[b * 4 + 1];
      zeros += vpart[b * 4 + 2];
    }
    for (int b = 0; b < nwb; ++b) wl1 += wl1part[b];
    for (int e = 0; e < R * R; ++e) hl1 += fabs((double)H[e]);
    double quad = 0.0;
    for (int e = 0; e < R * R; ++e) quad += small[kPsi * R * R + e] * small[kVtV * R * R + e];
    const double resid = normX2 - 2.0 * dot + quad;
    const double fit = normX2 > 0.0 ? 1.0 - resid / normX2 : 0.0;
    auto pen = [](int kind, double lam, double a) {
      return (kind == COPA_PROX_L1 || kind == COPA_PROX_NONNEG_L1) ? lam * a : 0.0;
    };
    const double obj = 0.5 * resid + pen(proxV, lamV, l1) + pen(proxW, lamW, wl1) +
                       pen(proxH, lamH, hl1);
    const int it = sc->iter;
    if (!isfinite(fit) || !isfinite(obj)) atomicMin(&sc->fail_iter, it);
    if (it < kHistCap) {
      sc->hist_fit[it] = fit;
      sc->hist_obj[it] = obj;
    }
    sc->last_fit = fit;
    sc->last_obj = obj;
    sc->last_sparsity = J > 0 ? zeros / ((double)J * R) : 0.0;
    sc->rank_deficient = sc->rank_def_cur;
    sc->rank_def_cur = 0;
    sc->iter = it + 1;
  }
}

__global__ void k_zero(float *x, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0f;
}

__global__ void k_reset_scalars(FitScalars *sc) {
  if (threadIdx.x == 0) {
    sc->iter = 0;
    sc->fail_iter = INT_MAX;
    sc->rank_deficient = 0;
    sc->rank_def_cur = 0;
  }
}

template <int R>
__global__ void __launch_bounds__(256) k_reduce_into(const double *part, int nb, double *dst) {
  reduce_parts(part, nb, R * R, dst);
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
static void launch_pass1_rt(copa_plan *p, const float *V, hipStream_t s) {
  constexpr int RTP = (RT + 3) & ~3;
  dim3 grid((unsigned)((p->n_waves + 3) / 4), (unsigned)p->tiles.nt), block(256);
  size_t lds = (size_t)p->J * RTP * sizeof(float);
  if (p->l > 0)
    k_pass1<RT, true><<<grid, block, lds, s>>>(p->waves, p->n_waves, p->order, p->subj, p->row,
                                              p->col, p->val, p->C, V, p->J, p->R, p->l, p->T);
  else
    k_pass1<RT, false><<<grid, block, lds, s>>>(p->waves, p->n_waves, p->order, p->subj, p->row,
                                               p->col, p->val, p->C, V, p->J, p->R, p->l, p->T);
}

template <int RT>
static void launch_pass2_rt(copa_plan *p, hipStream_t s) {
  dim3 grid((unsigned)p->n_fv_blocks, (unsigned)p->tiles.nt), block(1024);
  if (p->fv_lds) {
    size_t lds = (size_t)p->J * RT * sizeof(float);
    if (p->l > 0)
      k_pass2<RT, true, true><<<grid, block, lds, s>>>(p->waves, p->n_waves, p->order, p->subj,
                                                       p->row, p->col, p->val, p->C, p->M, p->J,
                                                       p->R, p->l, p->FVpart, p->FV);
    else
      k_pass2<RT, false, true><<<grid, block, lds, s>>>(p->waves, p->n_waves, p->order, p->subj,
                                                        p->row, p->col, p->val, p->C, p->M,
                                                        p->J, p->R, p->l, p->FVpart, p->FV);
  } else {
    if (p->l > 0)
      k_pass2<RT, true, false><<<grid, block, 0, s>>>(p->waves, p->n_waves, p->order, p->subj,
                                                      p->row, p->col, p->val, p->C, p->M, p->J,
                                                      p->R, p->l, p->FVpart, p->FV);
    else
      k_pass2<RT, false, false><<<grid, block, 0, s>>>(p->waves, p->n_waves, p->order, p->subj,
                                                       p->row, p->col, p->val, p->C, p->M, p->J,
                                                       p->R, p->l, p->FVpart, p->FV);
  }
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

template <int R>
static void gram(copa_plan *p, const float *A, const float *B, int64_t rows, const float *W,
                 int wsel, double *part, hipStream_t s) {
  k_rows_gram<R><<<kGramBlocks, 256, 0, s>>>(A, B, rows, W, wsel, p->slot_rows > 0 ? p->slot_rows : 1,
                                             p->rowsubj, part);
}

template <int R>
static void iteration_r(copa_plan *p, const copa_state *st, hipStream_t s) {
  const copa_options &o = p->opt;
  const int64_t K = p->K;
  RT_SWITCH(p->tiles.rt, launch_pass1_rt, p, st->V, s);
  if (K > 0)
    k_procrustes<R><<<(unsigned)((K + 63) / 64), 64, 0, s>>>(
        K, p->l, p->subj, p->rk, p->T, p->Q, p->M, st->H, st->W, o.rank_rtol, &p->scal->rank_def_cur);
  gram<R>(p, p->Q, p->T, p->rows_total, st->W, p->l > 0 ? 1 : 2, p->gpart, s);
  k_mode_H<R><<<1, 256, 0, s>>>(p->gpart, kGramBlocks, p->small, p->modes, p->scal, st->H,
                                st->D_H, o.prox_H, o.lambda_H, o.inner_iters);
  const unsigned nwb = (unsigned)std::max<int64_t>(1, (K + 63) / 64);
  k_w_admm<R><<<nwb, 64, 0, s>>>(K, p->l, p->subj, p->rk, p->T, p->Q, p->M, st->H, st->W,
                                 st->D_W, p->FW, p->modes, o.prox_W, o.lambda_W, o.inner_iters,
                                 p->wpart);
  gram<R>(p, st->W, st->W, K, nullptr, 0, p->gpart, s);
  gram<R>(p, p->M, p->M, p->rows_total, nullptr, 0, p->gpart2, s);
  if (!p->fv_lds)
    k_zero<<<(unsigned)std::min<int64_t>(1024, (p->J * R + 255) / 256), 256, 0, s>>>(p->FV, p->J * R);
  RT_SWITCH(p->tiles.rt, launch_pass2_rt, p, s);
  k_mode_V_prep<R><<<1, 256, 0, s>>>(p->gpart, p->gpart2, kGramBlocks, p->small, p->modes,
                                     p->scal);
  k_v_admm<R><<<p->n_vblocks, 256, 0, s>>>(p->J, p->fv_lds ? p->FVpart : nullptr,
                                           p->n_fv_blocks, p->FV, st->V, st->D_V, p->modes,
                                           o.prox_V, o.lambda_V, o.inner_iters, p->vpart);
  gram<R>(p, st->V, st->V, p->J, nullptr, 0, p->gpart, s);
  k_finalize<R><<<1, 256, 0, s>>>(p->gpart, kGramBlocks, p->vpart, p->n_vblocks,
                                  p->wpart, (int)nwb, p->small, p->scal,
                                  st->H, p->normX2, p->J, o.prox_H, o.lambda_H, o.prox_W,
                                  o.lambda_W, o.prox_V, o.lambda_V);
}

template <int R>
static void init_grams_r(copa_plan *p, const copa_state *st, hipStream_t s) {
  k_reset_scalars<<<1, 64, 0, s>>>(p->scal);
  gram<R>(p, st->W, st->W, p->K, nullptr, 0, p->gpart, s);
  k_reduce_into<R><<<1, 256, 0, s>>>(p->gpart, kGramBlocks, p->small + kWtW * R * R);
  gram<R>(p, st->V, st->V, p->J, nullptr, 0, p->gpart2, s);
  k_reduce_into<R><<<1, 256, 0, s>>>(p->gpart2, kGramBlocks, p->small + kVtV * R * R);
}

copa_status launch_iteration(copa_plan *p, const copa_state *st, hipStream_t s) {
  switch (p->R) {
#define CASE(r) \
  case r: iteration_r<r>(p, st, s); break;
    COPA_R_LIST(CASE)
#undef CASE
    default: set_error("unsupported R"); return COPA_EUNSUPPORTED;
  }
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

copa_status launch_init_grams(copa_plan *p, const copa_state *st, hipStream_t s) {
  switch (p->R) {
#define CASE(r) \
  case r: init_grams_r<r>(p, st, s); break;
    COPA_R_LIST(CASE)
#undef CASE
    default: set_error("unsupported R"); return COPA_EUNSUPPORTED;
  }
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

copa_status launch_qtilde(copa_plan *p, float *Qt, hipStream_t s) {
  if (p->S == 0) return COPA_OK;
  const unsigned nb = (unsigned)((p->S + 255) / 256);
  switch (p->R) {
#define CASE(r) \
  case r: k_qtilde<r><<<nb, 256, 0, s>>>(p->S, p->l, p->rowsubj, p->C, p->Q, Qt); break;
    COPA_R_LIST(CASE)
#undef CASE
    default: set_error("unsupported R"); return COPA_EUNSUPPORTED;
  }
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

}  // namespace copa

using namespace copa;

extern "C" {

copa_status copa_fit(copa_plan *p, const copa_state *st, int32_t iters, float *Qtilde,
                     copa_report *rep, void *stream) {
  if (!p || !st || iters < 0) {
    set_error("plan/state is NULL or iters < 0");
    return COPA_EINVAL;
  }
  if (!st->H || !st->V || !st->D_H || !st->D_V || (p->K > 0 && (!st->W || !st->D_W))) {
    set_error("state array is NULL");
    return COPA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  COPA_HIP(hipSetDevice(p->device));
  copa_status cs = launch_init_grams(p, st, s);
  if (cs != COPA_OK) return cs;
  std::vector<double> hf, ho;
  FitScalars hs;
  int done = 0, chunk_start = 0, fail = -1;
  while (done < iters) {
    const int chunk = std::min(iters - done, kHistCap);
    if (done > 0) k_reset_scalars<<<1, 64, 0, s>>>(p->scal);
    for (int t = 0; t < chunk; ++t) {
      cs = launch_iteration(p, st, s);
      if (cs != COPA_OK) return cs;
    }
    COPA_HIP(hipMemcpyAsync(&hs, p->scal, sizeof(FitScalars), hipMemcpyDeviceToHost, s));
    COPA_HIP(hipStreamSynchronize(s));
    hf.insert(hf.end(), hs.hist_fit, hs.hist_fit + chunk);
    ho.insert(ho.end(), hs.hist_obj, hs.hist_obj + chunk);
    chunk_start = done;
    done += chunk;
    if (hs.fail_iter != INT_MAX) {
      fail = chunk_start + hs.fail_iter;
      break;
    }
  }
  if (Qtilde) {
    cs = launch_qtilde(p, Qtilde, s);
    if (cs != COPA_OK) return cs;
  }
  COPA_HIP(hipStreamSynchronize(s));
  if (rep) {
    rep->iters_done = done;
    rep->fail_iter = fail;
    if (done > 0) {
      rep->fit = hs.last_fit;
      rep->objective = hs.last_obj;
      rep->sparsity_V = hs.last_sparsity;
      rep->rank_deficient = hs.rank_deficient;
      if (rep->fit_history)
        for (int i = 0; i < done; ++i) rep->fit_history[i] = hf[i];
      if (rep->objective_history)
        for (int i = 0; i < done; ++i) rep->objective_history[i] = ho[i];
    }
  }
  if (fail >= 0) {
    set_error("non-finite value or Cholesky failure during the fit, iteration " +
              std::to_string(fail));
    return COPA_ENUMERIC;
  }
  return COPA_OK;
}

copa_status copa_mttkrp_last(copa_plan *p, float *F_H, float *F_W, float *F_V, void *stream) {
  if (!p) {
    set_error("plan is NULL");
    return COPA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int R = p->R;
  if (F_H) {
    std::vector<double> h(R * R);
    COPA_HIP(hipMemcpyAsync(h.data(), p->small + kFH * R * R, R * R * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    COPA_HIP(hipStreamSynchronize(s));
    std::vector<float> f(h.begin(), h.end());
    COPA_HIP(hipMemcpyAsync(F_H, f.data(), R * R * sizeof(float), hipMemcpyHostToDevice, s));
    COPA_HIP(hipStreamSynchronize(s));
  }
  if (F_W && p->K > 0)
    COPA_HIP(hipMemcpyAsync(F_W, p->FW, p->K * R * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (F_V)
    COPA_HIP(hipMemcpyAsync(F_V, p->FV, p->J * R * sizeof(float), hipMemcpyDeviceToDevice, s));
  return COPA_OK;
}

}  // extern "C"
