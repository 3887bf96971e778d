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
// Persistent blocks of 4 waves; each block stages one column tile of V (kept padded to RTP
// columns per row by the V update) in LDS once, then its waves walk the wave list: each wave takes
// `cnt` subjects and G lanes per subject stride over the subject's visit rows.
template <int RT, bool SMOOTH>
__global__ void __launch_bounds__(256)
    k_pass1(const WaveEntry *__restrict__ waves, int n_waves, const int32_t *__restrict__ order,
            const int32_t *__restrict__ subj, const int32_t *__restrict__ row,
            const int32_t *__restrict__ col, const float *__restrict__ val,
            const float *__restrict__ C, const float *__restrict__ Vp, int64_t J, int R, int l,
            float *__restrict__ T) {
  constexpr int RTP = (RT + 3) & ~3;
  extern __shared__ float4 smem4[];
  {
    const float4 *src = reinterpret_cast<const float4 *>(Vp + (int64_t)blockIdx.y * J * RTP);
    const int64_t n4 = J * RTP / 4;
    for (int64_t e = threadIdx.x; e < n4; e += blockDim.x) smem4[e] = src[e];
  }
  __syncthreads();
  const float *sV = reinterpret_cast<const float *>(smem4);
  const int c0 = blockIdx.y * RT;
  const int lane = threadIdx.x & 63;
  for (int wv = blockIdx.x * 4 + (threadIdx.x >> 6); wv < n_waves; wv += gridDim.x * 4) {
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
            const float4 v = v4[q];
            t[4 * q + 0] += x * v.x;
            t[4 * q + 1] += x * v.y;
            t[4 * q + 2] += x * v.z;
            t[4 * q + 3] += x * v.w;
          }
        }
        const float4 *c4 = reinterpret_cast<const float4 *>(C + (int64_t)i * kLMax);
        const float4 ca = c4[0], cb = c4[1];
        const float c[kLMax] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
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
    } else if (active) {
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
            const float4 v = v4[q];
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
// dst = sum over rows of A_row^T (B_row * w_subj(row)) (R x R, FP64), a dense contraction over
// the long row dimension done on the matrix cores: v_mfma_f64_16x16x4f64 takes 4 rows per
// instruction, lane l holding A[row0 + l/16][16 ti + l%16] and B[row0 + l/16][16 tj + l%16].
// wsel: 0 = no scaling; 1 = scale B by W[row / slot_rows]; 2 = scale by W[rowsubj[row]].
// Every block writes its partial; the last block to finish adds the partials in block order (the
// result does not depend on scheduling) into dst and resets the counter.
typedef double dbl4_t __attribute__((ext_vector_type(4)));

template <int R>
__global__ void __launch_bounds__(256)
    k_rows_gram(const float *__restrict__ A, const float *__restrict__ B, int64_t rows,
                const float *__restrict__ W, int wsel, int slot_rows,
                const int32_t *__restrict__ rowsubj, double *__restrict__ part,
                double *__restrict__ dst, int32_t *counter) {
  constexpr int NT = (R + 15) / 16;
  constexpr int RP = NT * 16;
  constexpr int RR = R * R;
  __shared__ double sacc[RP * RP];
  __shared__ int last;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m = lane & 15, kk = lane >> 4;
  for (int e = t; e < RP * RP; e += blockDim.x) sacc[e] = 0.0;
  const int64_t per = ((rows + gridDim.x - 1) / gridDim.x + 15) & ~(int64_t)15;
  const int64_t lo = blockIdx.x * per;
  const int64_t hi = lo + per < rows ? lo + per : rows;
  dbl4_t acc[NT][NT];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = dbl4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int64_t r0 = lo + 4 * wave; r0 < hi; r0 += 16) {
    const int64_t rr = r0 + kk;
    const bool ok = rr < hi;
    double av[NT], bv[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int c = q * 16 + m;
      const bool in = ok && c < R;
      av[q] = in ? (double)A[rr * R + c] : 0.0;
      double b = in ? (double)B[rr * R + c] : 0.0;
      if (in && wsel == 1) b *= (double)W[(rr / slot_rows) * R + c];
      else if (in && wsel == 2) b *= (double)W[(int64_t)rowsubj[rr] * R + c];
      bv[q] = b;
    }
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
  }
  __syncthreads();
  // D[ii][jj] of a 16 x 16 FP64 block: lane jj + 16 (ii % 4), element ii / 4
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ii = i * 16 + 4 * v + (lane >> 4), jj = j * 16 + (lane & 15);
            sacc[ii * RP + jj] += acc[i][j][v];
          }
    }
    __syncthreads();
  }
  for (int e = t; e < RR; e += blockDim.x)
    part[(int64_t)blockIdx.x * RR + e] = sacc[(e / R) * RP + e % R];
  __threadfence();
  __syncthreads();
  if (t == 0) last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int nb = gridDim.x;
  constexpr int G2 = RR >= 256 ? 1 : 256 / RR;
  double *sred = sacc;  // reuse (RP*RP >= 256 doubles)
  for (int e0 = 0; e0 < RR; e0 += 256 / G2) {
    const int e = e0 + t % (256 / G2 < RR ? 256 / G2 : RR);
    const int g = t / (256 / G2 < RR ? 256 / G2 : RR);
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (e < RR && g < G2) {
      int b = g;
      for (; b + 7 * G2 < nb; b += 8 * G2) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          s[u] += __hip_atomic_load(&part[(int64_t)(b + u * G2) * RR + e], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
      }
      for (; b < nb; b += G2)
        s[0] += __hip_atomic_load(&part[(int64_t)b * RR + e], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    sred[t] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    if (t < (256 / G2 < RR ? 256 / G2 : RR) && e0 + t < RR) {
      double v = 0.0;
      for (int q = 0; q < G2; ++q) v += sred[q * (256 / G2 < RR ? 256 / G2 : RR) + t];
      dst[e0 + t] = v;
    }
  }
  if (t == 0) *counter = 0;
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
    k_mode_H(double *small, ModeParams *modes, FitScalars *sc, float *H, float *DH, int kind,
             double lam, int iters) {
  __shared__ double sFH[R * R];
  __shared__ double sL[R * R];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sFH[e] = small[kFH * R * R + e];
  __syncthreads();
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
// F_V(j,:) += x_ij * u_i with u_i = c_i M_k (smoothed: basis row times Q_k H S_k) or the M row of
// visit i (plain). Chunked form: for every block of kChunkRows visit rows the plan stores the
// chunk's nonzeros sorted by feature (key = feature << 16 | row in chunk) and 9 split points
// that cut the sorted list into 8 slices on feature boundaries, one per wave. A block puts the
// chunk's u rows in LDS; each lane sums a contiguous run of its wave's slice feature by feature;
// a segmented scan over the lanes joins runs that share a feature, so every feature is added to
// the block's LDS copy of F_V by exactly one lane - no LDS atomics. The block's F_V tile goes to
// the global F_V with one atomic add per entry at the end.
template <int RT, bool SMOOTH>
__global__ void __launch_bounds__(512)
    k_pass2c(int nchunks, int64_t S, const int32_t *__restrict__ wsplit,
             const uint32_t *__restrict__ pkey, const float *__restrict__ pval,
             const int32_t *__restrict__ rowsubj, const float *__restrict__ C,
             const float *__restrict__ M, int64_t J, int R, int l, float *__restrict__ FV) {
  extern __shared__ float4 smem4[];
  float *sF = reinterpret_cast<float *>(smem4);
  float *sU = sF + J * RT;
  const int c0 = blockIdx.y * RT;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wave = t >> 6;
  for (int64_t e = t; e < J * RT; e += nt) sF[e] = 0.0f;
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int64_t r0 = (int64_t)c * kChunkRows;
    const int n = (int)((S - r0) < kChunkRows ? (S - r0) : kChunkRows);
    __syncthreads();
    for (int q = t; q < n; q += nt) {
      const int64_t i = r0 + q;
      float u[RT];
      if constexpr (SMOOTH) {
        const int64_t k = rowsubj[i];
        const float4 *c4 = reinterpret_cast<const float4 *>(C + i * kLMax);
        const float4 ca = c4[0], cb = c4[1];
        const float cr[kLMax] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
#pragma unroll
        for (int r = 0; r < RT; ++r) u[r] = 0.0f;
#pragma unroll
        for (int a = 0; a < kLMax; ++a) {
          if (a < l) {
            const float *mr = M + (k * l + a) * R + c0;
#pragma unroll
            for (int r = 0; r < RT; ++r)
              if (c0 + r < R) u[r] += cr[a] * mr[r];
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < RT; ++r) u[r] = (c0 + r < R) ? M[i * R + c0 + r] : 0.0f;
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) sU[q * RT + r] = u[r];
    }
    __syncthreads();
    const int s0 = wsplit[c * 9 + wave], s1 = wsplit[c * 9 + wave + 1];
    const int per = (s1 - s0 + 63) >> 6;
    const int a = s0 + lane * per;
    const int b = a + per < s1 ? a + per : s1;
    float acc[RT], head[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      acc[r] = 0.0f;
      head[r] = 0.0f;
    }
    int cur = -1, hkey = -1, nseg = 0;
    for (int e = a; e < b; ++e) {
      const uint32_t key = pkey[e];
      const int j = (int)(key >> 16);
      const float x = pval[e];
      const float *ur = sU + (key & 0xffffu) * RT;
      if (j != cur) {
        if (nseg == 1) {
          hkey = cur;
#pragma unroll
          for (int r = 0; r < RT; ++r) head[r] = acc[r];
        } else if (nseg > 1) {
          // a segment that starts and ends inside this lane's run: no other lane has it
#pragma unroll
          for (int r = 0; r < RT; ++r) sF[cur * RT + r] += acc[r];
        }
        cur = j;
        ++nseg;
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] = 0.0f;
      }
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[r] += x * ur[r];
    }
    // tail segment (cur, acc); the first key of this lane's run is hkey (several segments) or cur
    const int first = nseg > 1 ? hkey : cur;
    // inclusive segmented scan of the tails over lanes (keys are non-decreasing along lanes)
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int kprev = __shfl_up(cur, d, 64);
      float vprev[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) vprev[r] = __shfl_up(acc[r], d, 64);
      if (lane >= d && cur >= 0 && kprev == cur) {
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] += vprev[r];
      }
    }
    const int knext = __shfl_down(first, 1, 64);
    const int kprev1 = __shfl_up(cur, 1, 64);
    float carry[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) carry[r] = __shfl_up(acc[r], 1, 64);
    if (nseg > 1) {
      // head segment: complete once the previous lane's tail (if same feature) is added
      const bool join = lane > 0 && kprev1 == hkey;
#pragma unroll
      for (int r = 0; r < RT; ++r) sF[hkey * RT + r] += head[r] + (join ? carry[r] : 0.0f);
    }
    if (cur >= 0) {
      // tail: flushed unless the next lane's run starts with the same feature
      const bool cont = lane < 63 && knext == cur;
      if (!cont) {
#pragma unroll
        for (int r = 0; r < RT; ++r) sF[cur * RT + r] += acc[r];
      }
    }
  }
  __syncthreads();
  for (int64_t e = t; e < J * RT; e += nt) {
    const int64_t j = e / RT;
    const int r = (int)(e - j * RT);
    const float v = sF[e];
    if (c0 + r < R && v != 0.0f) unsafeAtomicAdd(&FV[j * R + c0 + r], v);
  }
}

// Unchunked fallback (features >= 2^16): global atomics per nonzero.
template <int RT, bool SMOOTH>
__global__ void __launch_bounds__(256)
    k_pass2(const WaveEntry *__restrict__ waves, int n_waves, const int32_t *__restrict__ order,
            const int32_t *__restrict__ subj, const int32_t *__restrict__ row,
            const int32_t *__restrict__ col, const float *__restrict__ val,
            const float *__restrict__ C, const float *__restrict__ M, int64_t J, int R, int l,
            float *__restrict__ FV) {
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wv >= n_waves) return;
  const int c0 = blockIdx.y * RT;
  const WaveEntry we = waves[wv];
  const int lg = we.lg_count & 255, cnt = we.lg_count >> 8;
  const int G = 1 << lg, sidx = lane >> lg, sub = lane & (G - 1);
  if (sidx >= cnt) return;
  const int k = order[we.first + sidx];
  const int r0 = subj[k], r1 = subj[k + 1];
  for (int i = r0 + sub; i < r1; i += G) {
    float u[RT];
    if constexpr (SMOOTH) {
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        float s = 0.0f;
        for (int a = 0; a < l; ++a)
          if (c0 + r < R) s += C[(int64_t)i * kLMax + a] * M[((int64_t)k * l + a) * R + c0 + r];
        u[r] = s;
      }
    } else {
#pragma unroll
      for (int r = 0; r < RT; ++r) u[r] = (c0 + r < R) ? M[(int64_t)i * R + c0 + r] : 0.0f;
    }
    for (int e = row[i]; e < row[i + 1]; ++e) {
      const float x = val[e];
      const int64_t j = col[e];
#pragma unroll
      for (int r = 0; r < RT; ++r)
        if (c0 + r < R) unsafeAtomicAdd(&FV[j * R + c0 + r], x * u[r]);
    }
  }
}

// ======================================================================= mode V
template <int R>
__global__ void __launch_bounds__(256)
    k_mode_V_prep(double *small, ModeParams *modes, FitScalars *sc) {
  mode_prepare<R>(small + kHtH * R * R, small + kWtW * R * R, &modes[2], sc);
}

template <int R>
__global__ void __launch_bounds__(256)
    k_v_admm(int64_t J, const float *__restrict__ FV, float *__restrict__ V,
             float *__restrict__ DV, float *__restrict__ Vp, int rt, int rtp,
             const ModeParams *__restrict__ modes, int kind, double lam, int iters,
             double *__restrict__ vpart) {
  __shared__ double sL[R * R];
  __shared__ double sred[3][256];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sL[e] = modes[2].L[e];
  __syncthreads();
  const double rho = modes[2].rho;
  double dot = 0.0, l1 = 0.0, zeros = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < J;
       j += (int64_t)gridDim.x * blockDim.x) {
    double F[R];
#pragma unroll
    for (int c = 0; c < R; ++c) F[c] = FV[j * R + c];
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
      Vp[((int64_t)(c / rt) * J + j) * rtp + c % rt] = Zb[c];
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
    k_finalize(const double *__restrict__ vpart, int nvb, const double *__restrict__ wl1part,
               int nwb, double *small, FitScalars *sc, const float *__restrict__ H, double normX2,
               int64_t J, int proxH, double lamH, int proxW, double lamW, int proxV,
               double lamV) {
  __shared__ double red[5][256];
  const int t = threadIdx.x;
  double dot = 0.0, l1 = 0.0, zeros = 0.0, wl1 = 0.0, quad = 0.0;
  for (int b = t; b < nvb; b += blockDim.x) {
    dot += vpart[b * 4 + 0];
    l1 += vpart[b * 4 + 1];
    zeros += vpart[b * 4 + 2];
  }
  for (int b = t; b < nwb; b += blockDim.x) wl1 += wl1part[b];
  for (int e = t; e < R * R; e += blockDim.x)
    quad += small[kPsi * R * R + e] * small[kVtV * R * R + e];
  red[0][t] = dot;
  red[1][t] = l1;
  red[2][t] = zeros;
  red[3][t] = wl1;
  red[4][t] = quad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < 5; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  if (t == 0) {
    dot = red[0][0];
    l1 = red[1][0];
    zeros = red[2][0];
    wl1 = red[3][0];
    quad = red[4][0];
    double hl1 = 0.0;
    for (int e = 0; e < R * R; ++e) hl1 += fabs((double)H[e]);
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
  constexpr int RTP = (RT + 3) & ~3;
  size_t lds = (size_t)p->J * RTP * sizeof(float);
  const int per_cu = std::max(1, std::min(4, (int)(160 * 1024 / std::max<size_t>(lds, 1))));
  const int nb = std::max(1, std::min((p->n_waves + 3) / 4, p->n_cu * per_cu));
  dim3 grid((unsigned)nb, (unsigned)p->tiles.nt), block(256);
  if (p->l > 0)
    k_pass1<RT, true><<<grid, block, lds, s>>>(p->waves, p->n_waves, p->order, p->subj, p->row,
                                              p->col, p->val, p->C, p->Vp, p->J, p->R, p->l,
                                              p->T);
  else
    k_pass1<RT, false><<<grid, block, lds, s>>>(p->waves, p->n_waves, p->order, p->subj, p->row,
                                               p->col, p->val, p->C, p->Vp, p->J, p->R, p->l,
                                               p->T);
}

template <int RT>
static void launch_pass2_rt(copa_plan *p, hipStream_t s) {
  if (p->p2c) {
    dim3 grid((unsigned)std::min(p->nchunks, std::max(1, p->n_cu)), (unsigned)p->tiles.nt),
        block(512);
    size_t lds = ((size_t)p->J * RT + (size_t)kChunkRows * RT) * sizeof(float);
    if (p->l > 0)
      k_pass2c<RT, true><<<grid, block, lds, s>>>(p->nchunks, p->S, p->wsplit, p->pkey, p->pval,
                                                  p->rowsubj, p->C, p->M, p->J, p->R, p->l,
                                                  p->FV);
    else
      k_pass2c<RT, false><<<grid, block, lds, s>>>(p->nchunks, p->S, p->wsplit, p->pkey, p->pval,
                                                   p->rowsubj, p->C, p->M, p->J, p->R, p->l,
                                                   p->FV);
  } else {
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
                 int wsel, int slot, double *dst, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kGramBlocks, (rows + 1023) / 1024));
  k_rows_gram<R><<<nb, 256, 0, s>>>(A, B, rows, W, wsel,
                                             p->slot_rows > 0 ? p->slot_rows : 1, p->rowsubj,
                                             p->gpart, dst, p->gcount + slot);
}

const char *const kernel_names[kNumKernels] = {
    "pass1", "procrustes", "gram_FH", "mode_H", "w_admm", "gram_W", "gram_M", "zero_FV",
    "pass2", "mode_V_prep", "v_admm", "gram_V", "finalize"};

enum { kidPass1, kidProcrustes, kidGramFH, kidModeH, kidWadmm, kidGramW, kidGramM, kidZeroFV,
       kidPass2, kidModeVPrep, kidVadmm, kidGramV, kidFinalize };

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

copa_status harvest_timing(copa_plan *p) {
  for (size_t e = 0; e < p->ev_kid.size(); ++e) {
    float ms = 0.0f;
    COPA_HIP(hipEventElapsedTime(&ms, p->ev_pool[2 * e], p->ev_pool[2 * e + 1]));
    p->t_ms[p->ev_kid[e]] += ms;
    p->t_cnt[p->ev_kid[e]] += 1;
  }
  p->ev_kid.clear();
  p->ev_used = 0;
  return COPA_OK;
}

template <int R>
static void iteration_r(copa_plan *p, const copa_state *st, hipStream_t s) {
  const copa_options &o = p->opt;
  const int64_t K = p->K;
  timed(p, s, kidPass1, [&] { RT_SWITCH(p->tiles.rt, launch_pass1_rt, p, st->V, s); });
  if (K > 0)
    timed(p, s, kidProcrustes, [&] {
      k_procrustes<R><<<(unsigned)((K + 63) / 64), 64, 0, s>>>(
          K, p->l, p->subj, p->rk, p->T, p->Q, p->M, st->H, st->W, o.rank_rtol,
          &p->scal->rank_def_cur);
    });
  timed(p, s, kidGramFH,
        [&] {
          gram<R>(p, p->Q, p->T, p->rows_total, st->W, p->l > 0 ? 1 : 2, 0,
                  p->small + kFH * R * R, s);
        });
  timed(p, s, kidModeH, [&] {
    k_mode_H<R><<<1, 256, 0, s>>>(p->small, p->modes, p->scal, st->H, st->D_H, o.prox_H,
                                  o.lambda_H, o.inner_iters);
  });
  const unsigned nwb = (unsigned)std::max<int64_t>(1, (K + 63) / 64);
  timed(p, s, kidWadmm, [&] {
    k_w_admm<R><<<nwb, 64, 0, s>>>(K, p->l, p->subj, p->rk, p->T, p->Q, p->M, st->H, st->W,
                                   st->D_W, p->FW, p->modes, o.prox_W, o.lambda_W,
                                   o.inner_iters, p->wpart);
  });
  timed(p, s, kidGramW,
        [&] { gram<R>(p, st->W, st->W, K, nullptr, 0, 1, p->small + kWtW * R * R, s); });
  timed(p, s, kidGramM, [&] {
    gram<R>(p, p->M, p->M, p->rows_total, nullptr, 0, 2, p->small + kPsi * R * R, s);
  });
  timed(p, s, kidZeroFV, [&] {
      k_zero<<<(unsigned)std::min<int64_t>(1024, (p->J * R + 255) / 256), 256, 0, s>>>(
          p->FV, p->J * R);
    });
  timed(p, s, kidPass2, [&] { RT_SWITCH(p->tiles.rt, launch_pass2_rt, p, s); });
  timed(p, s, kidModeVPrep, [&] {
    k_mode_V_prep<R><<<1, 256, 0, s>>>(p->small, p->modes, p->scal);
  });
  timed(p, s, kidVadmm, [&] {
    k_v_admm<R><<<p->n_vblocks, 256, 0, s>>>(p->J, p->FV, st->V, st->D_V, p->Vp, p->tiles.rt,
                                             (p->tiles.rt + 3) & ~3, p->modes, o.prox_V,
                                             o.lambda_V, o.inner_iters, p->vpart);
  });
  timed(p, s, kidGramV,
        [&] { gram<R>(p, st->V, st->V, p->J, nullptr, 0, 3, p->small + kVtV * R * R, s); });
  timed(p, s, kidFinalize, [&] {
    k_finalize<R><<<1, 256, 0, s>>>(p->vpart, p->n_vblocks, p->wpart, (int)nwb, p->small,
                                   p->scal, st->H, p->normX2, p->J,
                                    o.prox_H, o.lambda_H, o.prox_W, o.lambda_W, o.prox_V,
                                    o.lambda_V);
  });
}

template <int R>
static void init_grams_r(copa_plan *p, const copa_state *st, hipStream_t s) {
  k_reset_scalars<<<1, 64, 0, s>>>(p->scal);
  if (p->J > 0)
    k_pad_V<R><<<(unsigned)((p->J * R + 255) / 256), 256, 0, s>>>(
        st->V, p->Vp, p->J, p->tiles.rt, (p->tiles.rt + 3) & ~3);
  gram<R>(p, st->W, st->W, p->K, nullptr, 0, 4, p->small + kWtW * R * R, s);
  gram<R>(p, st->V, st->V, p->J, nullptr, 0, 5, p->small + kVtV * R * R, s);
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
    const int chunk = std::min(iters - done, p->timing ? kTimingChunk : kHistCap);
    if (done > 0) k_reset_scalars<<<1, 64, 0, s>>>(p->scal);
    for (int t = 0; t < chunk; ++t) {
      cs = launch_iteration(p, st, s);
      if (cs != COPA_OK) return cs;
    }
    COPA_HIP(hipMemcpyAsync(&hs, p->scal, sizeof(FitScalars), hipMemcpyDeviceToHost, s));
    COPA_HIP(hipStreamSynchronize(s));
    if (p->timing) {
      cs = harvest_timing(p);
      if (cs != COPA_OK) return cs;
    }
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

copa_status copa_set_timing(copa_plan *p, int32_t enable) {
  if (!p) {
    set_error("plan is NULL");
    return COPA_EINVAL;
  }
  COPA_HIP(hipSetDevice(p->device));
  if (enable && p->ev_pool.empty()) {
    p->ev_pool.resize((size_t)kTimingChunk * kNumKernels * 2);
    for (auto &e : p->ev_pool) COPA_HIP(hipEventCreate(&e));
  }
  p->timing = enable != 0;
  return COPA_OK;
}

copa_status copa_read_timing(copa_plan *p, double *ms, int64_t *launches) {
  if (!p) {
    set_error("plan is NULL");
    return COPA_EINVAL;
  }
  for (int k = 0; k < kNumKernels; ++k) {
    if (ms) ms[k] = p->t_ms[k];
    if (launches) launches[k] = p->t_cnt[k];
    p->t_ms[k] = 0.0;
    p->t_cnt[k] = 0;
  }
  return COPA_OK;
}

const char *copa_kernel_name(int32_t id) {
  return (id >= 0 && id < kNumKernels) ? kernel_names[id] : "unknown";
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
