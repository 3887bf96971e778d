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
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "copa_iter_impl.h"

namespace copa {

bool rank_supported(int R) {
  switch (R) {
#define CASE(r) case r:
    COPA_R_LIST(CASE)
#undef CASE
    return true;
    default: return false;
  }
}

// Pass 1: column tiles of at most 16 (the width of the per-lane accumulators). A block stages cg
// tiles together and gives each a lane group of 64 / cg lanes, so X is streamed nt / cg times;
// the tiling with the fewest streams wins (then the fewest tiles).
Tiles choose_tiles(int R, int64_t J, int lds_limit) {
  Tiles best{0, 0, 0};
  int best_streams = INT_MAX;
  for (int nt = (R + 15) / 16; nt <= R && best_streams > 1; ++nt) {
    const int rt = (R + nt - 1) / nt;
    if ((nt - 1) * rt >= R) continue;  // the last tile would be empty
    const int64_t tile = J * row4(rt) * 4;
    for (int cg : {4, 2, 1}) {
      if (nt % cg != 0 || cg * tile + 16 > lds_limit) continue;
      if (nt / cg < best_streams) {
        best = Tiles{nt, rt, cg};
        best_streams = nt / cg;
      }
      break;
    }
  }
  if (best.nt == 0) best = Tiles{R, 1, 1};  // build_plan rejects J when even this does not fit
  return best;
}

// Widths pass 2 has kernels for.
bool pass2_width_supported(int rt) { return rt >= 1 && (rt <= 16 || rt == 20 || rt == 24 || rt == 32 || rt == 40); }

// Pass 2 keeps a block's F_V tile and one chunk of u rows in LDS: the fewest column tiles whose
// width has a kernel and fits; nt = 0 when none fits (pass 2 then runs unchunked).
Tiles choose_tiles2(int R, int64_t J, int lds_limit) {
  for (int nt = 1; nt <= R; ++nt) {
    const int rt = (R + nt - 1) / nt;
    if ((nt - 1) * rt >= R || !pass2_width_supported(rt)) continue;
    if ((J + kChunkRows) * row4(rt) * 4 + 16 <= (int64_t)lds_limit) return Tiles{nt, rt, 1};
  }
  return Tiles{0, 0, 0};
}

const char *const kernel_names[kNumKernels] = {
    "pass1", "procrustes", "gram_FH", "mode_H", "w_admm", "gram_WM", "pass2", "v_admm",
    "w_first", "m_rows", "finish", "proc_gram", "proc_eigen", "proc_q"};

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

copa_status launch_iteration(copa_plan *p, const copa_state *st, hipStream_t s) {
  switch (p->R) {
#define CASE(r) \
  case r: RankOps<r>::iteration(p, st, s); break;
    COPA_R_LIST(CASE)
#undef CASE
    default: set_error("unsupported R"); return COPA_EUNSUPPORTED;
  }
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

copa_status launch_fit(copa_plan *p, const copa_state *st, hipStream_t s) {
  switch (p->R) {
#define CASE(r) \
  case r: RankOps<r>::fit(p, st, s); break;
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
  case r: RankOps<r>::init_grams(p, st, s); break;
    COPA_R_LIST(CASE)
#undef CASE
    default: set_error("unsupported R"); return COPA_EUNSUPPORTED;
  }
  COPA_HIP(hipGetLastError());
  return COPA_OK;
}

copa_status launch_tune(copa_plan *p, const copa_state *st, hipStream_t s) {
  switch (p->R) {
#define CASE(r) \
  case r: return RankOps<r>::tune(p, st, s);
    COPA_R_LIST(CASE)
#undef CASE
    default: set_error("unsupported R"); return COPA_EUNSUPPORTED;
  }
}

copa_status launch_qtilde(copa_plan *p, float *Qt, hipStream_t s) {
  if (p->S == 0) return COPA_OK;
  switch (p->R) {
#define CASE(r) \
  case r: RankOps<r>::qtilde(p, Qt, s); break;
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

// Autotuner cache (optional): the file named by COPA_TUNE_CACHE holds one line per tuned shape,
//   <J> <R> <l> <projected> <precision> <log2 K> <compute units> : <pass-1 blocks per CU>
//   <Procrustes variant> <Gram blocks> <pass-2 blocks>
static std::string tune_key(const copa_plan *p) {
  int lk = 0;
  while ((int64_t)1 << (lk + 1) <= std::max<int64_t>(1, p->K)) ++lk;
  return std::to_string(p->J) + " " + std::to_string(p->R) + " " + std::to_string(p->l) + " " +
         std::to_string(p->proj ? 1 : 0) + " " + std::to_string(p->opt.precision) + " " +
         std::to_string(lk) + " " + std::to_string(p->n_cu);
}

static bool tune_from_cache(copa_plan *p) {
  const char *path = std::getenv("COPA_TUNE_CACHE");
  if (!path || !*path) return false;
  std::FILE *f = std::fopen(path, "r");
  if (!f) return false;
  const std::string key = tune_key(p);
  char line[512];
  bool hit = false;
  while (std::fgets(line, sizeof line, f)) {
    const char *colon = std::strchr(line, ':');
    if (!colon) continue;
    std::string k(line, colon - line);
    while (!k.empty() && k.back() == ' ') k.pop_back();
    int a, b, c, d;
    if (k == key && std::sscanf(colon + 1, "%d %d %d %d", &a, &b, &c, &d) == 4 && a >= 1 &&
        a <= 4 && b >= 0 && b <= 2 && c >= 1 && c <= p->gmaxnb && d >= 1 &&
        d <= p->p2_blocks_cap) {
      p->p1_per_cu = a, p->proc_variant = b, p->gram_blocks = c, p->p2_blocks = d;
      hit = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return hit;
}

static void tune_to_cache(const copa_plan *p) {
  const char *path = std::getenv("COPA_TUNE_CACHE");
  if (!path || !*path) return;
  std::FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s : %d %d %d %d\n", tune_key(p).c_str(), p->p1_per_cu, p->proc_variant,
               p->gram_blocks, p->p2_blocks);
  std::fclose(f);
}

// The launches of `chunk` outer iterations on stream s, and the FIT of the last one (the others
// are taken by the next iteration's F_H launch).
static copa_status launch_chunk(copa_plan *p, const copa_state *st, int chunk, hipStream_t s) {
  for (int t = 0; t < chunk; ++t) {
    copa_status cs = launch_iteration(p, st, s);
    if (cs != COPA_OK) return cs;
  }
  return launch_fit(p, st, s);
}

static bool same_state(const copa_state &a, const copa_state &b) {
  return a.H == b.H && a.W == b.W && a.V == b.V && a.D_H == b.D_H && a.D_W == b.D_W &&
         a.D_V == b.D_V;
}

// The same work with each outer iteration replayed from one hipGraph: the iteration is captured
// once per plan and state buffers on the plan's own stream (so that the caller's stream may be
// the null stream) and launched on s. None of the captured launches is a memset or a copy.
static copa_status run_chunk_graph(copa_plan *p, const copa_state *st, int chunk, hipStream_t s) {
  // one captured iteration per record precision (mixed-precision plans replay both)
  hipGraphExec_t &gx = p->use_bf ? p->gexec_bf : p->gexec;
  copa_state &gs = p->use_bf ? p->gstate_bf : p->gstate;
  if (!gx || !same_state(gs, *st)) {
    if (gx) {
      COPA_HIP(hipGraphExecDestroy(gx));
      gx = nullptr;
    }
    if (!p->cap_stream) COPA_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    COPA_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const copa_status cs = launch_iteration(p, st, p->cap_stream);
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (cs != COPA_OK) {
      if (g) (void)hipGraphDestroy(g);
      return cs;
    }
    COPA_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&gx, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    COPA_HIP(ei);
    gs = *st;
  }
  for (int t = 0; t < chunk; ++t) COPA_HIP(hipGraphLaunch(gx, s));
  return launch_fit(p, st, s);
}

copa_status copa_set_graph(copa_plan *p, int32_t enable) {
  if (!p) {
    set_error("plan is NULL");
    return COPA_EINVAL;
  }
  p->use_graph = enable != 0;
  return COPA_OK;
}

copa_status copa_fit(copa_plan *p, copa_state *st, int32_t iters, float *Qtilde,
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
  // the Procrustes warm start continues only for the state the previous call returned
  p->reset_warm = !(p->warm_valid && st->iter > 0 && same_state(p->last_state, *st) &&
                    p->last_state.iter == st->iter);
  p->warm_valid = false;
  copa_status cs;
  if (!p->tuned && p->opt.autotune && !p->opt.deterministic && iters > 0) {
    // launch shapes, once per plan: from the cache file, else timed on this fit's start
    if (tune_from_cache(p)) {
      p->tuned = 2;
    } else {
      const auto t0 = std::chrono::steady_clock::now();
      cs = launch_tune(p, st, s);
      if (cs != COPA_OK) return cs;
      p->tune_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0)
                       .count();
      p->tuned = 1;
      tune_to_cache(p);
    }
    if (p->gexec) {  // shapes captured before tuning are stale
      COPA_HIP(hipGraphExecDestroy(p->gexec));
      p->gexec = nullptr;
    }
    if (p->gexec_bf) {
      COPA_HIP(hipGraphExecDestroy(p->gexec_bf));
      p->gexec_bf = nullptr;
    }
  }
  cs = launch_init_grams(p, st, s);
  if (cs != COPA_OK) return cs;
  std::vector<double> hf, ho;
  FitScalars hs;
  int done = 0, chunk_start = 0, fail = -1;
  const bool check = p->opt.stop_tol > 0.0;
  const int every = p->opt.check_every > 0 ? p->opt.check_every : 10;
  double stat = -1.0;
  // mixed precision: the iterations stream the bfloat16 records, except the last mixed_refine of
  // the call, which stream the FP32 records (refinement)
  const bool mixed = p->opt.precision == COPA_PREC_MIXED && p->proj;
  const int n_bf = mixed ? std::max(0, iters - p->opt.mixed_refine) : 0;
  while (done < iters) {
    int chunk = std::min(iters - done, p->timing ? kTimingChunk : kHistCap);
    if (check) chunk = std::min(chunk, every);
    p->use_bf = done < n_bf;
    if (p->use_bf) chunk = std::min(chunk, n_bf - done);
    if (done > 0) k_reset_scalars<<<1, 64, 0, s>>>(p->scal);
    if (p->use_graph && !p->timing) {
      cs = run_chunk_graph(p, st, chunk, s);
      if (cs != COPA_OK) return cs;
    } else {
      cs = launch_chunk(p, st, chunk, s);
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
    if (check) {
      cs = launch_qtilde(p, p->qtbuf, s);
      if (cs != COPA_OK) return cs;
      double r[3];
      cs = launch_stationarity(p, st->H, st->V, st->W, p->qtbuf, r, s);
      if (cs != COPA_OK) return cs;
      stat = std::max(r[0], std::max(r[1], r[2]));
      if (stat < p->opt.stop_tol) break;
    }
  }
  p->use_bf = false;
  if (Qtilde) {
    cs = launch_qtilde(p, Qtilde, s);
    if (cs != COPA_OK) return cs;
  }
  COPA_HIP(hipStreamSynchronize(s));
  st->iter += done;
  if (fail < 0) {
    p->last_state = *st;
    p->warm_valid = true;
  }
  if (rep) {
    rep->iters_done = done;
    rep->fail_iter = fail;
    rep->stationarity = stat;
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

copa_status copa_plan_query(const copa_plan *p, int32_t what, int64_t *out) {
  if (!p || !out) {
    set_error("plan or out is NULL");
    return COPA_EINVAL;
  }
  switch (what) {
    case COPA_QUERY_COMPACT: *out = p->compact ? 1 : 0; return COPA_OK;
    case COPA_QUERY_CHUNKS: *out = p->proj ? p->pnchunks : (p->p2c ? p->nchunks : 0); return COPA_OK;
    case COPA_QUERY_PAIRS: *out = p->proj ? p->npairs : 0; return COPA_OK;
    case COPA_QUERY_TUNED: *out = p->tuned; return COPA_OK;
    case COPA_QUERY_PASS1_BLOCKS_PER_CU: *out = p->p1_per_cu; return COPA_OK;
    case COPA_QUERY_PROCRUSTES_VARIANT: *out = p->proc_variant; return COPA_OK;
    case COPA_QUERY_GRAM_BLOCKS: *out = p->gram_blocks; return COPA_OK;
    case COPA_QUERY_PASS2_BLOCKS: *out = p->p2_blocks; return COPA_OK;
    case COPA_QUERY_WFIRST_BLOCKS: *out = p->wf_blocks; return COPA_OK;
    case COPA_QUERY_MROWS_BLOCKS: *out = p->mr_blocks; return COPA_OK;
    case COPA_QUERY_WAVES: *out = p->n_waves; return COPA_OK;
    default: set_error("unknown query"); return COPA_EINVAL;
  }
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
