// Reconstruction loss of the PARAFAC2 model and its hand-written adjoint (copa_loss_grad).
//
//   L = 1/2 sum_k ||X_k - Qt_k H S_k V^T||^2,  S_k = diag(W(k,:)),  Qt held fixed
//     (eq. Classic_PARAFAC2_obj_func with U_k = Qt_k H).
// With G = V^T V and, per visit row i of subject k,
//   t_i = x_i V,  a_i = qt_i H,  u_i = a_i * w_k (= qt_i H S_k),  z_i = u_i G,
// the terms of the loss and of its gradient are sums over rows:
//   <X_k, Qt_k H S_k V^T> = sum_i <u_i, t_i>,   ||Qt_k H S_k V^T||^2 = sum_i <z_i, u_i>,
//   dL/dH    = sum_i qt_i^T ((z_i - t_i) * w_k)                    (-P_k S_k + Pi_k H S_k G S_k)
//   dL/dV    = -sum_i x_i^T u_i + V sum_i u_i^T u_i                 (-X^T U + V Psi')
//   dL/dS_k  = sum_{i in k} a_i^T (z_i - t_i)                       (-H^T P_k + H^T Pi_k H S_k G)
//   dL/dW(k,r) = [dL/dS_k]_rr.
#include <climits>
#include <mutex>

#include "copa_common.h"
#include "copa_kernels.h"

namespace copa {

// Rows pass: U and D rows, dW (reduced over the lanes of each subject) and the two loss sums.
template <int R>
__global__ void __launch_bounds__(256)
    k_grad_rows(const WaveEntry *__restrict__ waves, int n_waves, const int32_t *__restrict__ order,
                const int32_t *__restrict__ subj, const int32_t *__restrict__ row,
                const int32_t *__restrict__ col, const float *__restrict__ val,
                const float *__restrict__ V, const float *__restrict__ H,
                const float *__restrict__ W, const float *__restrict__ Qt,
                const double *__restrict__ Gm, float *__restrict__ U, float *__restrict__ D,
                float *__restrict__ dW, double *__restrict__ lpart) {
  __shared__ float sH[R * R];
  __shared__ double sG[R * R];
  __shared__ double red[2][256];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    sH[e] = H[e];
    sG[e] = Gm[e];
  }
  __syncthreads();
  double lut = 0.0, lzu = 0.0;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wv < n_waves) {
    const int lane = threadIdx.x & 63;
    const WaveEntry we = waves[wv];
    const int lg = we.lg_count & 255, cnt = we.lg_count >> 8;
    const int G = 1 << lg, sidx = lane >> lg, sub = lane & (G - 1);
    const bool active = sidx < cnt;
    const int k = active ? order[we.first + sidx] : 0;
    const int r0 = active ? subj[k] : 0, r1 = active ? subj[k + 1] : 0;
    float w[R], dw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      w[r] = active ? W[(int64_t)k * R + r] : 0.0f;
      dw[r] = 0.0f;
    }
    for (int i = r0 + sub; i < r1; i += G) {
      float t[R];
#pragma unroll
      for (int r = 0; r < R; ++r) t[r] = 0.0f;
      const int e0 = row[i], e1 = row[i + 1];
      for (int eb = e0; eb < e1; eb += 4) {
        int cj[4];
        float xv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool ok = eb + q < e1;
          const int ec = ok ? eb + q : e0;
          cj[q] = col[ec];
          const float x = val[ec];
          xv[q] = ok ? x : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float *vr = V + (int64_t)cj[q] * R;
#pragma unroll
          for (int r = 0; r < R; ++r) t[r] += xv[q] * vr[r];
        }
      }
      float qv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) qv[r] = Qt[(int64_t)i * R + r];
      float a[R], u[R];
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) s += (double)qv[r] * (double)sH[r * R + c];
        a[c] = (float)s;
        u[c] = (float)(s * (double)w[c]);
      }
#pragma unroll
      for (int c = 0; c < R; ++c) {
        double z = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) z += (double)u[r] * sG[r * R + c];
        const double d = z - (double)t[c];
        U[(int64_t)i * R + c] = u[c];
        D[(int64_t)i * R + c] = (float)(d * (double)w[c]);
        dw[c] += (float)((double)a[c] * d);
        lut += (double)u[c] * (double)t[c];
        lzu += z * (double)u[c];
      }
    }
    for (int m = 1; m < G; m <<= 1) {
#pragma unroll
      for (int r = 0; r < R; ++r) dw[r] += shfl_xor_f(dw[r], m);
    }
    if (active && sub == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) dW[(int64_t)k * R + r] = dw[r];
    }
  }
  red[0][threadIdx.x] = lut;
  red[1][threadIdx.x] = lzu;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) lpart[blockIdx.x * 2 + threadIdx.x] = red[threadIdx.x][0];
}

// dV = -F + V Psi' (one row per thread); block 0 also writes dH and the loss.
template <int R>
__global__ void __launch_bounds__(256)
    k_grad_finish(int64_t J, const float *__restrict__ F, const float *__restrict__ V,
                  const double *__restrict__ partH, const double *__restrict__ partPsi, int nbp,
                  const double *__restrict__ lpart, int nlp, double normX2,
                  float *__restrict__ dV, float *__restrict__ dH, double *__restrict__ loss) {
  __shared__ double sPsi[R * R];
  __shared__ double sH[R * R];
  __shared__ double scratch[256];
  block_reduce_parts<R * R>(partPsi, nbp, sPsi, scratch);
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < J) {
    float v[R];
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = V[j * R + c];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double s = -(double)F[j * R + c];
#pragma unroll
      for (int r = 0; r < R; ++r) s += (double)v[r] * sPsi[r * R + c];
      dV[j * R + c] = (float)s;
    }
  }
  if (blockIdx.x == 0) {
    block_reduce_parts<R * R>(partH, nbp, sH, scratch);
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) dH[e] = (float)sH[e];
    if (threadIdx.x == 0) {
      double ut = 0.0, zu = 0.0;
      for (int b = 0; b < nlp; ++b) {
        ut += lpart[2 * b];
        zu += lpart[2 * b + 1];
      }
      *loss = 0.5 * (normX2 - 2.0 * ut + zu);
    }
  }
}

// Full dL/dS_k (optional): thread per (subject, slice of output rows); rows a in
// [a0, a0 + AR) of dS_k accumulated in registers over the subject's visit rows.
template <int R>
__global__ void __launch_bounds__(64)
    k_grad_dS(int64_t K, const int32_t *__restrict__ subj, const int32_t *__restrict__ row,
              const int32_t *__restrict__ col, const float *__restrict__ val,
              const float *__restrict__ V, const float *__restrict__ H,
              const float *__restrict__ W, const float *__restrict__ Qt,
              const double *__restrict__ Gm, float *__restrict__ dS) {
  constexpr int AR = R <= 12 ? R : (128 / R > 0 ? 128 / R : 1);
  constexpr int NP = (R + AR - 1) / AR;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= K * NP) return;
  const int64_t k = gid / NP;
  const int a0 = (int)(gid - k * NP) * AR;
  float w[R];
#pragma unroll
  for (int r = 0; r < R; ++r) w[r] = W[k * R + r];
  float acc[AR][R];
#pragma unroll
  for (int a = 0; a < AR; ++a)
#pragma unroll
    for (int c = 0; c < R; ++c) acc[a][c] = 0.0f;
  for (int i = subj[k]; i < subj[k + 1]; ++i) {
    float t[R];
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] = 0.0f;
    for (int e = row[i]; e < row[i + 1]; ++e) {
      const float x = val[e];
      const float *vr = V + (int64_t)col[e] * R;
#pragma unroll
      for (int r = 0; r < R; ++r) t[r] += x * vr[r];
    }
    float aa[R], e_[R];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) s += (double)Qt[(int64_t)i * R + r] * (double)H[r * R + c];
      aa[c] = (float)s;
    }
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double z = 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) z += (double)aa[r] * (double)w[r] * Gm[r * R + c];
      e_[c] = (float)(z - (double)t[c]);
    }
#pragma unroll
    for (int a = 0; a < AR; ++a) {
      const float av = (a0 + a < R) ? aa[a0 + a < R ? a0 + a : 0] : 0.0f;
#pragma unroll
      for (int c = 0; c < R; ++c) acc[a][c] += av * e_[c];
    }
  }
#pragma unroll
  for (int a = 0; a < AR; ++a)
    if (a0 + a < R)
#pragma unroll
      for (int c = 0; c < R; ++c) dS[(k * R + a0 + a) * R + c] = acc[a][c];
}

__global__ void k_zero_f(float *x, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0f;
}

// F += X^T U with U given per visit row (the plain-rows mode of the streaming scatter).
template <int RT>
static void scatter_c_rt(copa_plan *p, const float *U, float *F, hipStream_t s) {
  launch_pass2c<RT, false>(p, U, F, s);
}
template <int RT>
static void scatter_u_rt(copa_plan *p, const float *U, float *F, hipStream_t s) {
  dim3 grid((unsigned)((p->n_waves + 3) / 4), (unsigned)p->tiles.nt), block(256);
  k_pass2<RT, false><<<grid, block, 0, s>>>(p->waves, p->n_waves, p->order, p->subj, p->row,
                                            p->col, p->val, p->C, U, p->J, p->R, 0, F);
}

template <int R>
static void launch_scatter_rows(copa_plan *p, const float *U, float *F, hipStream_t s) {
  if (p->p2c) {
    switch (p->tiles2.rt) {
#define CASE(rt) \
  case rt: if constexpr (rt <= R) scatter_c_rt<rt>(p, U, F, s); break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11)
      CASE(12) CASE(13) CASE(14) CASE(15) CASE(16) CASE(20) CASE(24) CASE(32) CASE(40)
#undef CASE
      default: break;
    }
  } else {
    switch (p->tiles.rt) {
#define CASE(rt) \
  case rt: scatter_u_rt<rt>(p, U, F, s); break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10) CASE(11)
      CASE(12) CASE(13) CASE(14) CASE(15) CASE(16)
#undef CASE
      default: break;
    }
  }
}

// Work buffers of the adjoint: U and D rows (S x R each), F = X^T U (J x R), the per-block loss
// partials (2 doubles per block of the rows pass).
struct GradBufs {
  float *U, *D, *F;
  double *lpart;
};

static int grad_blocks(const copa_plan *p) { return std::max(1, (p->n_waves + 3) / 4); }

// floats of one contiguous GradBufs area (the partials 8-byte aligned at its end)
static size_t grad_floats(const copa_plan *p) {
  const size_t f = (((size_t)2 * p->S * p->R + (size_t)p->J * p->R) + 1) & ~(size_t)1;
  return f + (size_t)4 * grad_blocks(p);
}

static GradBufs grad_bufs_at(const copa_plan *p, float *base) {
  const size_t f = (((size_t)2 * p->S * p->R + (size_t)p->J * p->R) + 1) & ~(size_t)1;
  GradBufs b;
  b.U = base;
  b.D = base + (size_t)p->S * p->R;
  b.F = base + (size_t)2 * p->S * p->R;
  b.lpart = reinterpret_cast<double *>(base + f);
  return b;
}

template <int R>
static copa_status loss_grad_r(copa_plan *p, const float *H, const float *V, const float *W,
                               const float *Qt, float *dH, float *dV, float *dW, float *dS,
                               const GradBufs &bf, hipStream_t s) {
  // G = V^T V
  gram<R>(p, V, V, p->J, nullptr, 0, kSlotG, nullptr, 0, 0, s);
  const double *Gm = gram_total(p, kSlotG);
  float *U = bf.U;
  float *D = bf.D;
  const int nb = grad_blocks(p);
  k_grad_rows<R><<<nb, 256, 0, s>>>(p->waves, p->n_waves, p->order, p->subj, p->row, p->col,
                                    p->val, V, H, W, Qt, Gm, U, D, dW, bf.lpart);
  // dL/dH = Qt^T D and Psi' = U^T U in one launch
  gram<R>(p, Qt, D, p->S, nullptr, 0, kSlotFH, U, p->S, kSlotG2, s);
  // F = X^T U through the feature-sorted scatter
  float *F = bf.F;
  k_zero_f<<<(unsigned)std::min<int64_t>(1024, (p->J * R + 255) / 256), 256, 0, s>>>(F, p->J * R);
  launch_scatter_rows<R>(p, U, F, s);
  k_grad_finish<R><<<(unsigned)std::max<int64_t>(1, (p->J + 255) / 256), 256, 0, s>>>(
      p->J, F, V, gram_total(p, kSlotFH), gram_total(p, kSlotG2), 1, bf.lpart, nb, p->normX2,
      dV, dH, p->dloss);
  if (dS && p->K > 0) {
    constexpr int AR = R <= 12 ? R : (128 / R > 0 ? 128 / R : 1);
    constexpr int NP = (R + AR - 1) / AR;
    k_grad_dS<R><<<(unsigned)((p->K * NP + 63) / 64), 64, 0, s>>>(
        p->K, p->subj, p->row, p->col, p->val, V, H, W, Qt, Gm, dS);
  }
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

static copa_status ensure_grad_buffers(copa_plan *p) {
  if (!p->adjoint) {
    set_error("the plan was created without the adjoint's buffers (copa_options.adjoint = 0)");
    return COPA_EINVAL;
  }
  return COPA_OK;
}

static copa_status loss_grad_with(copa_plan *p, const float *H, const float *V, const float *W,
                                  const float *Qt, float *dH, float *dV, float *dW, float *dS,
                                  const GradBufs &bf, hipStream_t s) {
  switch (p->R) {
#define CASE(r) \
  case r: return loss_grad_r<r>(p, H, V, W, Qt, dH, dV, dW, dS, bf, s);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(10) CASE(12) CASE(15)
    CASE(16) CASE(20) CASE(24) CASE(32) CASE(40)
#undef CASE
    default: set_error("unsupported R"); return COPA_EUNSUPPORTED;
  }
}

static GradBufs plan_grad_bufs(const copa_plan *p) {
  GradBufs b;
  b.U = p->gradbuf;
  b.D = p->gradbuf + (size_t)p->S * p->R;
  b.F = p->gradbuf + (size_t)2 * p->S * p->R;
  b.lpart = p->lpart;
  return b;
}

copa_status launch_loss_grad(copa_plan *p, const float *H, const float *V, const float *W,
                             const float *Qt, float *dH, float *dV, float *dW, float *dS,
                             hipStream_t s) {
  const copa_status cs = ensure_grad_buffers(p);
  if (cs != COPA_OK) return cs;
  return loss_grad_with(p, H, V, W, Qt, dH, dV, dW, dS, plan_grad_bufs(p), s);
}

// ======================================================================= stationarity residual
// Per block: the steps rho_n = trace(G_n) / R from W^TW, V^TV (Gram totals) and H^TH (formed
// here), then sums over this block's share of the entries of H, W and V of
// (z - prox_n(z - g / rho_n))^2 and z^2 (g = dL/dz). part[block * 6 + 2n + {0, 1}].
template <int R>
__global__ void __launch_bounds__(256)
    k_stationarity(const float *__restrict__ H, const float *__restrict__ V,
                   const float *__restrict__ W, const float *__restrict__ dH,
                   const float *__restrict__ dV, const float *__restrict__ dW,
                   const double *__restrict__ VtV, const double *__restrict__ WtW, int64_t K,
                   int64_t J, int kH, double lH, int kW, double lW, int kV, double lV,
                   double *__restrict__ part) {
  __shared__ double red[6][256];
  __shared__ double srho[3];
  const int t = threadIdx.x;
  if (t < 3) {
    double tr = 0.0;
    for (int a = 0; a < R; ++a) {
      double hh = 0.0;
      for (int i = 0; i < R; ++i) hh += (double)H[i * R + a] * (double)H[i * R + a];
      const double vv = VtV[a * R + a], ww = WtW[a * R + a];
      tr += t == 0 ? ww * vv : (t == 1 ? hh * vv : hh * ww);
    }
    srho[t] = tr / R;
  }
  __syncthreads();
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t nH = (int64_t)R * R, nW = K * R, nV = J * R, n = nH + nW + nV;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + t; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    int m;
    double z, g;
    if (e < nH) {
      m = 0;
      z = H[e];
      g = dH[e];
    } else if (e < nH + nW) {
      m = 1;
      z = W[e - nH];
      g = dW[e - nH];
    } else {
      m = 2;
      z = V[e - nH - nW];
      g = dV[e - nH - nW];
    }
    const double rho = srho[m];
    const int kind = m == 0 ? kH : (m == 1 ? kW : kV);
    const double lam = m == 0 ? lH : (m == 1 ? lW : lV);
    const double d = z - prox_sel(z - g / rho, kind, lam, lam / rho);
    acc[2 * m] += d * d;
    acc[2 * m + 1] += z * z;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) red[q][t] = acc[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int q = 0; q < 6; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  if (t < 6) part[blockIdx.x * 6 + t] = red[t][0];
}

__global__ void k_stationarity_reduce(const double *__restrict__ part, int nb, double *res) {
  if (threadIdx.x < 3) {
    double num = 0.0, den = 0.0;
    for (int b = 0; b < nb; ++b) {
      num += part[b * 6 + 2 * threadIdx.x];
      den += part[b * 6 + 2 * threadIdx.x + 1];
    }
    res[threadIdx.x] = den > 0.0 ? sqrt(num / den) : 0.0;
  }
}

template <int R>
static copa_status stationarity_r(copa_plan *p, const float *H, const float *V, const float *W,
                                  const float *Qt, hipStream_t s) {
  float *dH = p->statbuf, *dV = dH + R * R, *dW = dV + p->J * R;
  double *part = reinterpret_cast<double *>(p->statbuf + p->statfloats);
  copa_status cs = loss_grad_r<R>(p, H, V, W, Qt, dH, dV, dW, nullptr, plan_grad_bufs(p), s);
  if (cs != COPA_OK) return cs;
  // W^T W into a slot the adjoint no longer needs (its V^T V stays in kSlotG)
  gram<R>(p, W, W, p->K, nullptr, 0, kSlotFH, nullptr, 0, 0, s);
  const copa_options &o = p->opt;
  k_stationarity<R><<<kStatBlocks, 256, 0, s>>>(
      H, V, W, dH, dV, dW, gram_total(p, kSlotG), gram_total(p, kSlotFH), p->K, p->J, o.prox_H,
      o.lambda_H, o.prox_W, o.lambda_W, o.prox_V, o.lambda_V, part);
  k_stationarity_reduce<<<1, 64, 0, s>>>(part, kStatBlocks, part + 6 * kStatBlocks);
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

copa_status launch_stationarity(copa_plan *p, const float *H, const float *V, const float *W,
                                const float *Qt, double *res_host, hipStream_t s) {
  copa_status cg = ensure_grad_buffers(p);
  if (cg != COPA_OK) return cg;
  copa_status cs;
  switch (p->R) {
#define CASE(r) \
  case r: cs = stationarity_r<r>(p, H, V, W, Qt, s); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(10) CASE(12) CASE(15)
    CASE(16) CASE(20) CASE(24) CASE(32) CASE(40)
#undef CASE
    default: set_error("unsupported R"); return COPA_EUNSUPPORTED;
  }
  if (cs != COPA_OK) return cs;
  const double *res = reinterpret_cast<double *>(p->statbuf + p->statfloats) + 6 * kStatBlocks;
  COPA_HIP(hipMemcpyAsync(res_host, res, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  COPA_HIP(hipStreamSynchronize(s));
  return COPA_OK;
}

}  // namespace copa

using namespace copa;

extern "C" copa_status copa_loss_grad(copa_plan *p, const float *H, const float *V, const float *W,
                                      const float *Qt, float *dH, float *dV, float *dW, float *dS,
                                      double *loss, void *stream) {
  if (!p || !H || !V || !Qt || !dH || !dV || !loss || (p->K > 0 && (!W || !dW))) {
    set_error("NULL argument");
    return COPA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  COPA_HIP(hipSetDevice(p->device));
  copa_status st = launch_loss_grad(p, H, V, W, Qt, dH, dV, dW, dS, s);
  if (st != COPA_OK) return st;
  COPA_HIP(hipMemcpyAsync(loss, p->dloss, sizeof(double), hipMemcpyDeviceToHost, s));
  COPA_HIP(hipStreamSynchronize(s));
  return COPA_OK;
}

extern "C" copa_status copa_stationarity(copa_plan *p, const float *H, const float *V,
                                         const float *W, const float *Qt, double *res,
                                         void *stream) {
  if (!p || !H || !V || !Qt || !res || (p->K > 0 && !W)) {
    set_error("NULL argument");
    return COPA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  COPA_HIP(hipSetDevice(p->device));
  return launch_stationarity(p, H, V, W, Qt, res, s);
}

// ======================================================================= no-allocation adjoint
// Work memory of copa_loss_grad_static: a file-scope device array, one copy per GPU, that every
// call on that GPU reuses (it keeps the last call's contents; calls that overlap on one GPU race
// on it). Host code never passes the array's name to a kernel: the device address of each GPU's
// copy comes from hipGetSymbolAddress on that call's first use of the device.
namespace copa {
constexpr size_t kStaticScratchFloats = (size_t)16 << 20;  // 64 MiB
static __device__ __align__(256) float scratch[kStaticScratchFloats];
static std::mutex g_scratch_mutex;
static float *g_scratch_ptr[64] = {};

static copa_status scratch_address(int device, float **out) {
  if (device < 0 || device >= 64) {
    set_error("device index outside 0..63");
    return COPA_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return COPA_EDEVICE;
    }
    g_scratch_ptr[device] = static_cast<float *>(ptr);
  }
  *out = g_scratch_ptr[device];
  return COPA_OK;
}
}  // namespace copa

extern "C" copa_status copa_loss_grad_static(copa_plan *p, const float *H, const float *V,
                                             const float *W, const float *Qt, float *dH,
                                             float *dV, float *dW, float *dS, double *loss,
                                             void *stream) {
  if (!p || !H || !V || !Qt || !dH || !dV || !loss || (p->K > 0 && (!W || !dW))) {
    set_error("NULL argument");
    return COPA_EINVAL;
  }
  const size_t need = grad_floats(p);
  if (need > kStaticScratchFloats) {
    set_error("copa_loss_grad_static needs " + std::to_string(need) +
              " floats of work memory (2 S R + J R + 4 per rows-pass block); its static scratch "
              "holds " + std::to_string(kStaticScratchFloats) + " (64 MiB)");
    return COPA_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  COPA_HIP(hipSetDevice(p->device));
  float *base = nullptr;
  copa_status st = scratch_address(p->device, &base);
  if (st != COPA_OK) return st;
  st = loss_grad_with(p, H, V, W, Qt, dH, dV, dW, dS, grad_bufs_at(p, base), s);
  if (st != COPA_OK) return st;
  COPA_HIP(hipMemcpyAsync(loss, p->dloss, sizeof(double), hipMemcpyDeviceToHost, s));
  COPA_HIP(hipStreamSynchronize(s));
  return COPA_OK;
}
