// Kernels shared by the fit (copa_iter.hip) and the adjoint (copa_grad.hip): the row-Gram
// contraction on the matrix cores and the feature-sorted streaming scatter F += X^T U.
#pragma once

#include <type_traits>

#include "copa_common.h"

namespace copa {

// ======================================================================= row Gram reductions
// dst[e] = sum_b part[b * RR + e] over b = 0..nb-1 in a fixed order, using the whole block
// (scratch: blockDim.x doubles of LDS). dst may be LDS or global memory.
template <int RR>
__device__ void block_reduce_parts(const double *__restrict__ part, int nb, double *dst,
                                   double *scratch) {
  const int t = threadIdx.x, nt = blockDim.x;
  auto ld = [&](int64_t i) { return part[i]; };
  if (RR <= nt) {
    const int G = nt / RR;
    const int e = t % RR, g = t / RR;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (g < G) {
      int b = g;
      for (; b + 7 * G < nb; b += 8 * G) {
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += ld((int64_t)(b + u * G) * RR + e);
      }
      for (; b < nb; b += G) s[0] += ld((int64_t)b * RR + e);
    }
    scratch[t] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    if (t < RR) {
      double v = 0.0;
      for (int q = 0; q < G; ++q) v += scratch[q * RR + t];
      dst[t] = v;
    }
    __syncthreads();
  } else {
    for (int e = t; e < RR; e += nt) {
      double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int b = 0;
      for (; b + 8 <= nb; b += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += ld((int64_t)(b + u) * RR + e);
      }
      for (; b < nb; ++b) s[0] += ld((int64_t)b * RR + e);
      dst[e] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    }
    __syncthreads();
  }
}

// part[block] = sum over the block's rows of A_row^T (B_row * w_subj(row)) (R x R, FP64): a dense
// contraction over the long row dimension on the matrix cores. v_mfma_f64_16x16x4f64 takes 4 rows
// per instruction, lane l holding A[row0 + l/16][16 ti + l%16] and B[row0 + l/16][16 tj + l%16];
// each wave loads BATCH such steps (64 rows; 32 for R > 16) before issuing their instructions.
// blockIdx.y == 1 computes a second, unscaled Gram A2^T A2 into part2 in the same launch (WSEL 0
// only). WSEL: 0 = no scaling; 1 = scale B by W[row / slot_rows]; 2 = scale by W[rowsubj[row]].
// The partials are added by k_gram_reduce, a separate launch: publishing a partial to other
// blocks of the same launch would take a device-scope release (an L2 write-back) per block.
typedef double dbl4_t __attribute__((ext_vector_type(4)));

// Block `bid` of `nblk` blocks: the partial of its share of the rows into part[bid].
template <int R, int WSEL>
__device__ __forceinline__ void rows_gram_block(const float *__restrict__ A,
                                                const float *__restrict__ B, int64_t rows,
                                                const float *__restrict__ W, int slot_rows,
                                                const int32_t *__restrict__ rowsubj,
                                                double *__restrict__ part, int bid, int nblk) {
  constexpr int NT = (R + 15) / 16;
  constexpr int RP = NT * 16;
  constexpr int RR = R * R;
  constexpr int BATCH = NT >= 2 ? 8 : 16;  // 4-row steps in flight per wave (registers)
  __shared__ double sacc[RP * RP];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
  const int m = lane & 15, kk = lane >> 4;
  for (int e = t; e < RP * RP; e += blockDim.x) sacc[e] = 0.0;
  const int64_t units = (rows + 4 * BATCH - 1) / (4 * BATCH);
  const int64_t upb = (units + nblk - 1) / nblk;
  const int64_t u0 = bid * upb;
  const int64_t u1 = u0 + upb < units ? u0 + upb : units;
  dbl4_t acc[NT][NT], acc2[NT][NT];
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      acc[i][j] = dbl4_t{0.0, 0.0, 0.0, 0.0};
      acc2[i][j] = dbl4_t{0.0, 0.0, 0.0, 0.0};
    }
  for (int64_t u = u0 + wave; u < u1; u += nw) {
    // every load goes to a clamped (always valid) address and is masked afterwards, so that the
    // whole batch is in flight at once
    int64_t rc[BATCH];
    bool ok[BATCH];
#pragma unroll
    for (int s = 0; s < BATCH; ++s) {
      const int64_t rr = u * (4 * BATCH) + 4 * s + kk;
      ok[s] = rr < rows;
      rc[s] = ok[s] ? rr : rows - 1;
    }
    int64_t wrow[BATCH];
#pragma unroll
    for (int s = 0; s < BATCH; ++s) {
      if constexpr (WSEL == 1)
        wrow[s] = (int64_t)((uint32_t)rc[s] / (uint32_t)slot_rows);
      else if constexpr (WSEL == 2)
        wrow[s] = rowsubj[rc[s]];
      else
        wrow[s] = 0;
    }
    double av[BATCH][NT], bv[BATCH][NT];
#pragma unroll
    for (int s = 0; s < BATCH; ++s) {
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        const int c = q * 16 + m;
        const bool in = ok[s] && c < R;
        const int cc = c < R ? c : R - 1;
        const float a = A[rc[s] * R + cc];
        const float b = B[rc[s] * R + cc];
        double bw = (double)b;
        if constexpr (WSEL != 0) bw *= (double)W[wrow[s] * R + cc];
        av[s][q] = in ? (double)a : 0.0;
        bv[s][q] = in ? bw : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < BATCH; s += 2)
#pragma unroll
      for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][i], bv[s][j], acc[i][j], 0, 0, 0);
          acc2[i][j] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(av[s + 1][i], bv[s + 1][j], acc2[i][j], 0, 0, 0);
        }
  }
#pragma unroll
  for (int i = 0; i < NT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] += acc2[i][j];
  __syncthreads();
  // D[ii][jj] of a 16 x 16 FP64 block: lane jj + 16 (ii % 4), element ii / 4; waves add in order
  for (int w = 0; w < nw; ++w) {
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
    part[(int64_t)bid * RR + e] = sacc[(e / R) * RP + e % R];
}

template <int R, int WSEL>
__global__ void __launch_bounds__(256)
    k_rows_gram(const float *__restrict__ A, const float *__restrict__ B, int64_t rows,
                const float *__restrict__ W, int slot_rows, const int32_t *__restrict__ rowsubj,
                double *__restrict__ part, const float *__restrict__ A2, int64_t rows2,
                double *__restrict__ part2) {
  if (WSEL == 0 && blockIdx.y == 1)
    rows_gram_block<R, 0>(A2, A2, rows2, W, slot_rows, rowsubj, part2, blockIdx.x, gridDim.x);
  else
    rows_gram_block<R, WSEL>(A, B, rows, W, slot_rows, rowsubj, part, blockIdx.x, gridDim.x);
}

// total[e] = sum_b part[b * RR + e] over the nb block partials in a fixed order: one block per
// group of 4 entries, 64 threads per entry, fixed-shape tree. blockIdx.y selects the launch half.
template <int RR>
__global__ void __launch_bounds__(256)
    k_gram_reduce(const double *__restrict__ part, double *__restrict__ total,
                  const double *__restrict__ part2, double *__restrict__ total2, int nb) {
  __shared__ double red[256];
  if (blockIdx.y == 1) {
    part = part2;
    total = total2;
  }
  const int t = threadIdx.x, lane = t & 63;
  const int e = blockIdx.x * 4 + (t >> 6);
  const int ec = e < RR ? e : RR - 1;
  // eight partials in flight per thread (clamped addresses, masked values), summed in a fixed order
  double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b0 = lane; b0 < nb; b0 += 8 * 64) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * 64;
      const double x = part[(int64_t)(b < nb ? b : 0) * RR + ec];
      s8[u] += b < nb ? x : 0.0;
    }
  }
  const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  red[t] = e < RR ? s : 0.0;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (lane < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (lane == 0 && e < RR) total[e] = red[t];
}

// Launches k_rows_gram and k_gram_reduce: A^T (B * w) into the total of `slot` and, when A2 is
// given, A2^T A2 into the total of `slot2`. wsel as WSEL of k_rows_gram (0 when A2 is given).
template <int R>
inline void gram(copa_plan *p, const float *A, const float *B, int64_t rows, const float *W,
                 int wsel, int slot, const float *A2, int64_t rows2, int slot2, hipStream_t s) {
  // about two 64-row units per wave of the 4-wave blocks
  const int64_t units = (std::max<int64_t>(rows, A2 ? rows2 : 0) + 63) / 64;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(p->gram_blocks, (units + 7) / 8));
  const dim3 grid(nb, A2 ? 2 : 1);
  double *p1 = gram_slot(p, slot), *p2 = A2 ? gram_slot(p, slot2) : nullptr;
  const int sr = p->slot_rows > 0 ? p->slot_rows : 1;
  if (wsel == 1)
    k_rows_gram<R, 1><<<grid, 256, 0, s>>>(A, B, rows, W, sr, p->rowsubj, p1, nullptr, 0, nullptr);
  else if (wsel == 2)
    k_rows_gram<R, 2><<<grid, 256, 0, s>>>(A, B, rows, W, sr, p->rowsubj, p1, nullptr, 0, nullptr);
  else
    k_rows_gram<R, 0><<<grid, 256, 0, s>>>(A, B, rows, W, sr, p->rowsubj, p1, A2, rows2, p2);
  k_gram_reduce<R * R><<<dim3((R * R + 3) / 4, A2 ? 2 : 1), 256, 0, s>>>(
      p1, gram_total(p, slot), p2, A2 ? gram_total(p, slot2) : nullptr, nb);
}

// ======================================================================= streaming pass 2
// F_V(j,:) += x_ij * u_i with u_i = c_i M_k (smoothed: basis row times Q_k H S_k) or the M row of
// visit i (plain). Chunked form: the plan cuts the visit rows into chunks of at most kChunkRows
// rows (and, smoothed, at most kChunkRows / l subjects), and stores each chunk's nonzeros sorted
// by feature (key = feature << 16 | row in chunk) with 9 split points that cut the sorted list
// into 8 slices on feature boundaries, one per wave. Per chunk a block issues every global load
// at once: the chunk's M rows (one contiguous block, staged in LDS), each row's basis row and
// subject, and each lane's first 8 keys and values; the next chunk's bounds are prefetched.
// Then the u rows are formed in LDS; each lane sums a contiguous run of its wave's slice feature
// by feature; a segmented scan over the lanes joins runs that share a feature, so every feature
// is added to the block's LDS copy of F_V by exactly one lane - no LDS atomics. The block's F_V
// tile goes to the global F_V with one atomic add per entry at the end.
template <int RT, bool SMOOTH>
__global__ void __launch_bounds__(512)
    k_pass2c(int nchunks, const int32_t *__restrict__ crow, const int32_t *__restrict__ cinfo,
             const int32_t *__restrict__ wsplit, const uint2 *__restrict__ pkv,
             const int32_t *__restrict__ rowsubj,
             const float *__restrict__ C, const float *__restrict__ M, int64_t J, int R, int l,
             float *__restrict__ FV, float *__restrict__ part) {
  // F_V tile and u rows with rows padded to RTP floats (16-byte LDS accesses; the pad stays 0)
  constexpr int RTP = row4(RT);
  extern __shared__ float4 smem4[];
  float *sF = reinterpret_cast<float *>(smem4);
  float *sU = sF + J * RTP;  // u rows of the chunk; first holds the chunk's M block (RT wide)
  const int c0 = blockIdx.y * RT;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wave = t >> 6;
  for (int64_t e = t; e < J * RTP; e += nt) sF[e] = 0.0f;
  int nr0 = 0, nr1 = 0, nk0 = 0, nns = 0, ns0 = 0, ns1 = 0;
  auto fetch = [&](int cc) {
    if (cc < nchunks) {
      nr0 = crow[cc];
      nr1 = crow[cc + 1];
      if constexpr (SMOOTH) {
        nk0 = cinfo[2 * cc];
        nns = cinfo[2 * cc + 1];
      }
      ns0 = wsplit[cc * 9 + wave];
      ns1 = wsplit[cc * 9 + wave + 1];
    }
  };
  fetch(blockIdx.x);
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int r0 = nr0, n = nr1 - nr0, k0 = nk0, nsub = nns, s0 = ns0, s1 = ns1;
    __syncthreads();  // the previous chunk is done with sU
    // ---- every global load of this chunk
    const int per = (s1 - s0 + 63) >> 6;
    const int a = s0 + lane * per;
    const int b = a + per < s1 ? a + per : s1;
    uint32_t kv[8];
    float xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint2 w = pkv[a + u < b ? a + u : 0];
      kv[u] = w.x;
      xv[u] = __uint_as_float(w.y);
    }
    const int tc = t < n ? t : 0;
    float cr[kLMax];
    int kl = 0;
    float u[RTP];
#pragma unroll
    for (int r = RT; r < RTP; ++r) u[r] = 0.0f;
    if constexpr (SMOOTH) {
      const int64_t i = r0 + tc;
      kl = rowsubj[i] - k0;
      const float4 *c4 = reinterpret_cast<const float4 *>(C + i * kLMax);
      const float4 ca = c4[0], cb = c4[1];
      cr[0] = ca.x; cr[1] = ca.y; cr[2] = ca.z; cr[3] = ca.w;
      cr[4] = cb.x; cr[5] = cb.y; cr[6] = cb.z; cr[7] = cb.w;
      // the chunk's M block (at most kChunkRows x RT floats): 4 loads in flight per thread per
      // step, from clamped addresses, stores masked
      const int nm = nsub * l * RT;
      const float *Mb = M + (int64_t)k0 * l * R + c0;
      for (int e0 = 0; e0 < nm; e0 += 4 * nt) {
        float mv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * nt + t;
          const int ec = e < nm ? e : nm - 1;
          const int q = ec / RT, r = ec - q * RT;
          mv[u] = Mb[(int64_t)q * R + (c0 + r < R ? r : R - 1 - c0)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          // M rows staged RTP apart (16-byte reads below); the spare slot past the u rows takes
          // the out-of-range lanes
          const int e = e0 + u * nt + t;
          const int q = e / RT;
          sU[e < nm ? q * RTP + (e - q * RT) : kChunkRows * RTP] = mv[u];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < RT; ++r) u[r] = M[(int64_t)(r0 + tc) * R + (c0 + r < R ? c0 + r : R - 1)];
    }
    fetch(c + gridDim.x);
    if constexpr (SMOOTH) {
      __syncthreads();
      // basis columns at or past l are zero: those M rows are skipped (l is uniform)
#pragma unroll
      for (int r = 0; r < RTP; ++r) u[r] = 0.0f;
#pragma unroll
      for (int q = 0; q < kLMax; ++q) {
        if (q < l) {
          float mv[RT];
          lds_row<RT>(sU + (kl * l + q) * RTP, mv);
#pragma unroll
          for (int r = 0; r < RT; ++r) u[r] += cr[q] * mv[r];
        }
      }
#pragma unroll
      for (int r = RT; r < RTP; ++r) u[r] = 0.0f;  // the staged rows' pad columns are not set
      __syncthreads();
    }
    if (t < n) {
      float4 *d4 = reinterpret_cast<float4 *>(sU + t * RTP);
#pragma unroll
      for (int q = 0; q < RTP / 4; ++q)
        d4[q] = make_float4(u[4 * q], u[4 * q + 1], u[4 * q + 2], u[4 * q + 3]);
    }
    __syncthreads();
    // sF[j] += v over the RT live entries of a padded row
    auto add_row = [&](int j, const float *v) { lds_row_add<RT>(sF + j * RTP, v); };
    float acc[RTP], head[RTP];
#pragma unroll
    for (int r = 0; r < RTP; ++r) {
      acc[r] = 0.0f;
      head[r] = 0.0f;
    }
    int cur = -1, hkey = -1, nseg = 0;
    for (int eb = a; eb < b; eb += 8) {
      if (eb > a) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint2 w = pkv[eb + q < b ? eb + q : a];
          kv[q] = w.x;
          xv[q] = __uint_as_float(w.y);
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (eb + q >= b) break;
        const uint32_t key = kv[q];
        const int j = (int)(key >> 16);
        const float x = xv[q];
        const float *ur = sU + (key & 0xffffu) * RTP;
        if (j != cur) {
          if (nseg == 1) {
            hkey = cur;
#pragma unroll
            for (int r = 0; r < RTP; ++r) head[r] = acc[r];
          } else if (nseg > 1) {
            // a segment that starts and ends inside this lane's run: no other lane has it
            add_row(cur, acc);
          }
          cur = j;
          ++nseg;
#pragma unroll
          for (int r = 0; r < RTP; ++r) acc[r] = 0.0f;
        }
        float uv[RT];
        lds_row<RT>(ur, uv);
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] += x * uv[r];
      }
    }
    // tail segment (cur, acc); the first key of this lane's run is hkey (several segments) or cur
    const int first = nseg > 1 ? hkey : cur;
    // inclusive segmented scan of the tails over lanes (keys are non-decreasing along lanes, so
    // equal keys at two lanes mean one segment between them): DPP shifts within rows of 16 lanes,
    // then the row broadcasts of lanes 15 and 31 (no LDS traffic)
    auto seg_step = [&](auto ctrl, auto mask) {
      constexpr int CT = decltype(ctrl)::value, MK = decltype(mask)::value;
      const int kp = dpp_i<CT, MK>(-1, cur);
      float vp[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) vp[r] = dpp_f<CT, MK>(0.0f, acc[r]);
      if (cur >= 0 && kp == cur) {
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] += vp[r];
      }
    };  // (the pad entries of acc stay zero)
    seg_step(std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xF>{});
    seg_step(std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xF>{});
    seg_step(std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xF>{});
    seg_step(std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xF>{});
    seg_step(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});
    seg_step(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});
    const int knext = dpp_i<0x130>(-1, first);   // lane + 1
    const int kprev1 = dpp_i<0x138>(-1, cur);    // lane - 1
    float carry[RTP];
#pragma unroll
    for (int r = 0; r < RTP; ++r) carry[r] = r < RT ? dpp_f<0x138>(0.0f, acc[r]) : 0.0f;
    if (nseg > 1) {
      // head segment: complete once the previous lane's tail (if same feature) is added
      const bool join = lane > 0 && kprev1 == hkey;
#pragma unroll
      for (int r = 0; r < RTP; ++r) head[r] += join ? carry[r] : 0.0f;
      add_row(hkey, head);
    }
    if (cur >= 0) {
      // tail: flushed unless the next lane's run starts with the same feature
      const bool cont = lane < 63 && knext == cur;
      if (!cont) add_row(cur, acc);
    }
  }
  __syncthreads();
  if (part) {
    // fixed-order mode: the block's tile goes to its own slice, summed in block order later
    float *dst = part + (int64_t)blockIdx.x * J * R;
    for (int64_t e = t; e < J * RTP; e += nt) {
      const int64_t j = e / RTP;
      const int r = (int)(e - j * RTP);
      if (r < RT && c0 + r < R) dst[j * R + c0 + r] = sF[e];
    }
    return;
  }
  for (int64_t e = t; e < J * RTP; e += nt) {
    const int64_t j = e / RTP;
    const int r = (int)(e - j * RTP);
    const float v = sF[e];
    if (r < RT && c0 + r < R && v != 0.0f) unsafeAtomicAdd(&FV[j * R + c0 + r], v);
  }
}

// F[e] += the sum over blocks b of part[b][e] in a fixed order (fixed-order mode): 64 entries per
// block of 512 threads, thread group g = 0..7 sums the slices b = g, g + 8, ... in that order (eight
// loads in flight), and the eight group sums are added as a fixed tree.
constexpr int kFvSumThreads = 512;
static __global__ void __launch_bounds__(kFvSumThreads)
    k_fv_sum(const float *__restrict__ part, int nb, int64_t n, float *__restrict__ F) {
  __shared__ float red[8][64];
  const int t = threadIdx.x, c = t & 63, g = t >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + c;
  float acc = 0.0f;
  if (e < n) {
    int b = g;
    for (; b + 56 < nb; b += 64) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + 8 * u) * n + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; b < nb; b += 8) acc += part[(int64_t)b * n + e];
  }
  red[g][c] = acc;
  __syncthreads();
  if (g == 0 && e < n)
    F[e] += ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c])) +
            ((red[4][c] + red[5][c]) + (red[6][c] + red[7][c]));
}

inline void launch_fv_sum(const float *part, int nb, int64_t n, float *F, hipStream_t s) {
  k_fv_sum<<<(unsigned)((n + 63) / 64), kFvSumThreads, 0, s>>>(part, nb, n, F);
}

// ------------------------------------------------------------------ projected pairs
// A smoothed plan with few nonzeros per visit row streams the projected data X'_k = C_k^T X_k
// instead of X and the basis rows: one record of PW floats per (subject, feature) pair that
// occurs, holding the l entries of that column of X'_k (FP32, formed in FP64 at plan creation),
// zeros, and a key in the last float.
template <int PW>
__device__ __forceinline__ void load_rec(const float *__restrict__ recs, int64_t q,
                                         float (&f)[PW]) {
  const float4 *r4 = reinterpret_cast<const float4 *>(recs + q * PW);
#pragma unroll
  for (int u = 0; u < PW / 4; ++u) {
    const float4 v = r4[u];
    f[4 * u] = v.x;
    f[4 * u + 1] = v.y;
    f[4 * u + 2] = v.z;
    f[4 * u + 3] = v.w;
  }
}

// Mixed precision: a 16-byte record of seven bfloat16 entries and a 16-bit tag (entry a in bits
// 16 (a & 1) of word a / 2, the tag in the high half of the last word). Unpacked into the layout
// of the FP32 records (PW = 8): f[0..6] the entries as FP32 (exact), f[7] the key bits, which are
// the tag (pass 1: the feature id) or, with `hi` given, hi[q] << 16 | tag (pass 2: feature and
// subject within the chunk).
__device__ __forceinline__ void load_rec_bf(const uint4 *__restrict__ recs,
                                            const uint16_t *__restrict__ hi, int64_t q,
                                            float (&f)[8]) {
  const uint4 w = recs[q];
  const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int a = 0; a < 7; ++a)
    f[a] = __uint_as_float((a & 1) ? (ws[a >> 1] & 0xffff0000u) : (ws[a >> 1] << 16));
  const uint32_t tag = w.w >> 16;
  f[7] = __uint_as_float(hi ? ((uint32_t)hi[q] << 16 | tag) : tag);
}

// the record of pair q as FP32 (BF: unpacked from the 16-byte mixed-precision form)
template <bool BF, int PW>
__device__ __forceinline__ void fetch_rec(const void *__restrict__ recs,
                                          const uint16_t *__restrict__ hi, int64_t q,
                                          float (&f)[PW]) {
  if constexpr (BF) {
    static_assert(PW == 8, "mixed-precision records hold seven entries");
    load_rec_bf(static_cast<const uint4 *>(recs), hi, q, f);
  } else {
    load_rec<PW>(static_cast<const float *>(recs), q, f);
  }
}

// Pass 2 on the projected pairs: F_V(j, :) += x'_j M_k for every pair (k, j), with the M rows of
// a chunk's subjects staged in LDS. A chunk is a run of at most kChunkRows / l subjects whose
// pairs are sorted by feature (key = feature << 16 | subject within the chunk) and cut into
// eight wave slices on feature boundaries; each lane sums a contiguous run of its wave's slice
// feature by feature, and the segmented scan over lanes of k_pass2c joins runs that share a
// feature, so each feature is added to the block's LDS copy of F_V by one lane.
template <int RT, int PW, bool BF, int LC = 0>
__global__ void __launch_bounds__(512)
    k_pass2p(int nchunks, const int32_t *__restrict__ cq, const int32_t *__restrict__ cinfo,
             const int32_t *__restrict__ wsplit, const void *__restrict__ recs,
             const uint16_t *__restrict__ feat_hi, const float *__restrict__ M, int64_t J, int R,
             int l_in, float *__restrict__ FV, float *__restrict__ part) {
  constexpr int RTP = row4(RT);
  const int l = LC > 0 ? LC : l_in;  // LC: the basis size fixed at compile time
  constexpr int PF = 4;  // records per lane loaded ahead of the chunk's M staging
  extern __shared__ float4 smem4[];
  float *sF = reinterpret_cast<float *>(smem4);
  float *sM = sF + J * RTP;  // the chunk's M rows, RTP apart
  const int c0 = blockIdx.y * RT;
  const int t = threadIdx.x, nt = blockDim.x, lane = t & 63, wave = t >> 6;
  for (int64_t e = t; e < J * RTP; e += nt) sF[e] = 0.0f;
  int nk0 = 0, nns = 0, ns0 = 0, ns1 = 0;
  auto fetch = [&](int cc) {
    if (cc < nchunks) {
      nk0 = cinfo[2 * cc];
      nns = cinfo[2 * cc + 1];
      ns0 = wsplit[cc * 9 + wave];
      ns1 = wsplit[cc * 9 + wave + 1];
    }
  };
  fetch(blockIdx.x);
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int k0 = nk0, nsub = nns, s0 = ns0, s1 = ns1;
    __syncthreads();  // the previous chunk is done with sM
    const int per = (s1 - s0 + 63) >> 6;
    const int a = s0 + lane * per;
    const int b = a + per < s1 ? a + per : s1;
    float pre[PF][PW];
#pragma unroll
    for (int u = 0; u < PF; ++u) fetch_rec<BF, PW>(recs, feat_hi, a + u < b ? a + u : 0, pre[u]);
    if (RT % 4 == 0 && RT == R && (((uintptr_t)M) & 15) == 0) {
      // the chunk's M block is nsub l whole rows, contiguous: float4 loads, up to eight per
      // thread in flight at once (rows of RT floats are RT / 4 float4s, RTP == RT)
      constexpr int R4 = RT / 4, U = 8;
      const int n4 = nsub * l * R4;
      const float4 *Mb4 = reinterpret_cast<const float4 *>(M + (int64_t)k0 * l * R);
      float4 *sM4 = reinterpret_cast<float4 *>(sM);
      for (int e0 = 0; e0 < n4; e0 += U * nt) {
        float4 mv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e0 + u * nt + t;
          mv[u] = Mb4[e < n4 ? e : 0];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e0 + u * nt + t;
          if (e < n4) sM4[e] = mv[u];
        }
      }
    } else {
      // the chunk's M block (nsub l rows of RT floats), 4 loads in flight per thread
      const int nm = nsub * l * RT;
      const float *Mb = M + (int64_t)k0 * l * R + c0;
      for (int e0 = 0; e0 < nm; e0 += 4 * nt) {
        float mv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * nt + t;
          const int ec = e < nm ? e : nm - 1;
          const int q = ec / RT, r = ec - q * RT;
          mv[u] = Mb[(int64_t)q * R + (c0 + r < R ? r : R - 1 - c0)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * nt + t;
          const int q = e / RT;
          sM[e < nm ? q * RTP + (e - q * RT) : kChunkRows * RTP] = mv[u];
        }
      }
    }
    fetch(c + gridDim.x);
    __syncthreads();
    auto add_row = [&](int j, const float *v) { lds_row_add<RT>(sF + j * RTP, v); };
    float acc[RTP], head[RTP];
#pragma unroll
    for (int r = 0; r < RTP; ++r) {
      acc[r] = 0.0f;
      head[r] = 0.0f;
    }
    int cur = -1, hkey = -1, nseg = 0;
    auto take = [&](const float (&f)[PW]) {
      const uint32_t key = __float_as_uint(f[PW - 1]);
      const int j = (int)(key >> 16);
      const float *mr = sM + (int)(key & 0xffffu) * l * RTP;
      if (j != cur) {
        if (nseg == 1) {
          hkey = cur;
#pragma unroll
          for (int r = 0; r < RTP; ++r) head[r] = acc[r];
        } else if (nseg > 1) {
          add_row(cur, acc);  // a segment inside this lane's run: no other lane has it
        }
        cur = j;
        ++nseg;
#pragma unroll
        for (int r = 0; r < RTP; ++r) acc[r] = 0.0f;
      }
#pragma unroll
      for (int q = 0; q < PW - 1; ++q) {
        if (q < l) {
          float mv[RT];
          lds_row<RT>(mr + q * RTP, mv);
#pragma unroll
          for (int r = 0; r < RT; ++r) acc[r] += f[q] * mv[r];
        }
      }
    };
#pragma unroll
    for (int u = 0; u < PF; ++u)
      if (a + u < b) take(pre[u]);
    for (int e = a + PF; e < b; e += PF) {
      float f[PF][PW];
#pragma unroll
      for (int u = 0; u < PF; ++u) fetch_rec<BF, PW>(recs, feat_hi, e + u < b ? e + u : e, f[u]);
#pragma unroll
      for (int u = 0; u < PF; ++u)
        if (e + u < b) take(f[u]);
    }
    const int first = nseg > 1 ? hkey : cur;
    auto seg_step = [&](auto ctrl, auto mask) {
      constexpr int CT = decltype(ctrl)::value, MK = decltype(mask)::value;
      const int kp = dpp_i<CT, MK>(-1, cur);
      float vp[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) vp[r] = dpp_f<CT, MK>(0.0f, acc[r]);
      if (cur >= 0 && kp == cur) {
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] += vp[r];
      }
    };
    seg_step(std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xF>{});
    seg_step(std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xF>{});
    seg_step(std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xF>{});
    seg_step(std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xF>{});
    seg_step(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});
    seg_step(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});
    const int knext = dpp_i<0x130>(-1, first);
    const int kprev1 = dpp_i<0x138>(-1, cur);
    float carry[RTP];
#pragma unroll
    for (int r = 0; r < RTP; ++r) carry[r] = r < RT ? dpp_f<0x138>(0.0f, acc[r]) : 0.0f;
    if (nseg > 1) {
      const bool join = lane > 0 && kprev1 == hkey;
#pragma unroll
      for (int r = 0; r < RTP; ++r) head[r] += join ? carry[r] : 0.0f;
      add_row(hkey, head);
    }
    if (cur >= 0) {
      const bool cont = lane < 63 && knext == cur;
      if (!cont) add_row(cur, acc);
    }
  }
  __syncthreads();
  if (part) {
    float *dst = part + (int64_t)blockIdx.x * J * R;
    for (int64_t e = t; e < J * RTP; e += nt) {
      const int64_t j = e / RTP;
      const int r = (int)(e - j * RTP);
      if (r < RT && c0 + r < R) dst[j * R + c0 + r] = sF[e];
    }
    return;
  }
  for (int64_t e = t; e < J * RTP; e += nt) {
    const int64_t j = e / RTP;
    const int r = (int)(e - j * RTP);
    const float v = sF[e];
    if (r < RT && c0 + r < R && v != 0.0f) unsafeAtomicAdd(&FV[j * R + c0 + r], v);
  }
}

template <int RT>
inline void launch_pass2p(const copa_plan *p, float *F, hipStream_t s) {
  const int gx = std::min(p->pnchunks, p->p2_blocks);
  const dim3 grid((unsigned)gx, (unsigned)p->tiles2.nt);
  const size_t lds = ((size_t)p->J * row4(RT) + (size_t)kChunkRows * row4(RT) + 4) * sizeof(float);
  float *part = p->opt.deterministic ? p->fvpart : nullptr;
  // the common basis size l = 7 has its own instances (no row guards)
  if (p->use_bf && p->l == 7)
    k_pass2p<RT, 8, true, 7><<<grid, 512, lds, s>>>(p->pnchunks, p->pcq, p->pcinfo, p->pwsplit,
                                                     p->pairs2h, p->feat2h, p->M, p->J, p->R,
                                                     p->l, F, part);
  else if (p->use_bf)
    k_pass2p<RT, 8, true><<<grid, 512, lds, s>>>(p->pnchunks, p->pcq, p->pcinfo, p->pwsplit,
                                                  p->pairs2h, p->feat2h, p->M, p->J, p->R, p->l,
                                                  F, part);
  else if (p->pw == 8 && p->l == 7)
    k_pass2p<RT, 8, false, 7><<<grid, 512, lds, s>>>(p->pnchunks, p->pcq, p->pcinfo, p->pwsplit,
                                                      p->pairs2, nullptr, p->M, p->J, p->R, p->l,
                                                      F, part);
  else if (p->pw == 8)
    k_pass2p<RT, 8, false><<<grid, 512, lds, s>>>(p->pnchunks, p->pcq, p->pcinfo, p->pwsplit,
                                                   p->pairs2, nullptr, p->M, p->J, p->R, p->l, F,
                                                   part);
  else
    k_pass2p<RT, 12, false><<<grid, 512, lds, s>>>(p->pnchunks, p->pcq, p->pcinfo, p->pwsplit,
                                                    p->pairs2, nullptr, p->M, p->J, p->R, p->l, F,
                                                    part);
  if (part) {
    const int64_t n = p->J * p->R;
    launch_fv_sum(part, gx, n, F, s);
  }
}

// Unchunked fallback (features >= 2^16): global atomics per nonzero.
// Launches k_pass2c on the plan's chunks: SMOOTH forms u rows from the basis and the M rows of
// each chunk's subjects; otherwise u_i is row i of Mrows (R wide).
// In fixed-order mode (deterministic) every block writes its F_V tile to its slice of fvpart and
// one more launch adds the slices to F in block order.
template <int RT, bool SMOOTH>
inline void launch_pass2c(const copa_plan *p, const float *Mrows, float *F, hipStream_t s) {
  const int gx = std::min(p->nchunks, p->p2_blocks);
  const dim3 grid((unsigned)gx, (unsigned)p->tiles2.nt);
  const size_t lds = ((size_t)p->J * row4(RT) + (size_t)kChunkRows * row4(RT) + 4) * sizeof(float);
  float *part = p->opt.deterministic ? p->fvpart : nullptr;
  k_pass2c<RT, SMOOTH><<<grid, 512, lds, s>>>(p->nchunks, p->crow, p->cinfo, p->wsplit, p->pkv,
                                             p->rowsubj, p->C, Mrows, p->J, p->R,
                                             SMOOTH ? p->l : 0, F, part);
  if (part) {
    const int64_t n = p->J * p->R;
    launch_fv_sum(part, gx, n, F, s);
  }
}

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

}  // namespace copa
