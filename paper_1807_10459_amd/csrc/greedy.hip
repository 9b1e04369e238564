// Greedy parent selection for one target (IDTxl Summary, network-inference paragraph):
// iterative conditioning on the candidate that maximises the CMI criterion, each inclusion
// gated by the max-statistic surrogate test, stopping at the first non-significant step,
// plus the optional omnibus test of the final source set.  With a learned null the step is
// first decided by the threshold network; only borderline steps pay for the surrogates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <vector>

#include "../../include/ksgcmi.h"
#include "internal.h"
#include "mlp.h"
#include "runtime.h"

using namespace ksg;


static int64_t round_up64(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

namespace {

struct Selector {
  ksg_ctx* c;
  const ksg_select_opts* o;
  int64_t N, n_pad;
  int C, L, P;
  const float* cand;  // [C][n_pad]
  const float* y;     // [n_pad]
  std::vector<int> selected, pool;

  Problem base_problem(int cidx, int p, int out_index) const {
    Problem q;
    std::memset(&q, 0, sizeof q);
    q.n = N;
    q.dx = 1;
    q.dy = 1;
    q.dz = (int)selected.size();
    q.k = o->k;
    q.col[0] = cand + (int64_t)cidx * n_pad;
    q.perm[0] = p > 0 ? o->perms + (int64_t)(p - 1) * N : nullptr;
    q.padded[0] = true;
    q.col[1] = y;
    q.padded[1] = true;
    for (size_t s = 0; s < selected.size(); ++s) {
      q.col[2 + s] = cand + (int64_t)selected[s] * n_pad;
      q.padded[2 + s] = true;
    }
    q.out_index = out_index;
    return q;
  }

  // Runs the CMI of every pooled candidate for rounds p0..p1-1 (round 0 = the original data)
  // into the [|pool|][P+1] table; other columns are left untouched.
  int step_cmis(int p0, int p1, double* d_cmi) {
    std::vector<Problem> probs;
    probs.reserve(pool.size() * (p1 - p0));
    for (size_t ci = 0; ci < pool.size(); ++ci)
      for (int p = p0; p < p1; ++p) probs.push_back(base_problem(pool[ci], p, (int)ci * (P + 1) + p));
    return c->run_batch(probs, d_cmi);
  }
};

}  // namespace

extern "C" int select_parents(ksg_ctx* c, const float* data, int32_t n_vars, int64_t T,
                              int32_t n_trials, int32_t target, const ksg_select_opts* o,
                              ksg_parent_set* out) {
  if (!c) return KSG_EINVAL;
  if (!data || !o || !out) return c->fail(KSG_EINVAL, "select_parents: null argument");
  if (o->k < 1 || o->k > KSG_MAX_K) return c->fail(KSG_EINVAL, "select_parents: k=%d outside [1,16]", o->k);
  if (o->max_lag < 1 || o->n_perm < 1 || o->n_perm > 4096 || !(o->alpha > 0 && o->alpha < 1) || !o->perms)
    return c->fail(KSG_EINVAL, "select_parents: need max_lag >= 1, 1 <= n_perm <= 4096, 0 < alpha < 1, perms");
  if (n_vars < 1 || n_trials < 1 || T <= o->max_lag || target < 0 || target >= n_vars)
    return c->fail(KSG_EINVAL, "select_parents: bad data shape");
  if (out->capacity < 0) return c->fail(KSG_EINVAL, "select_parents: negative capacity");
  if (o->max_cond < 0) return c->fail(KSG_EINVAL, "select_parents: max_cond must be >= 0");
  if (o->n_resume < 0 || (o->n_resume > 0 && !o->resume) || (o->n_resume > 0 && o->mode == KSG_MODE_BIVARIATE_TE))
    return c->fail(KSG_EINVAL, "select_parents: resume needs n_resume >= 0, a host array, and a multivariate mode");
  if (o->learned && !(o->margin_lo >= 0 && o->margin_hi >= 0))
    return c->fail(KSG_EINVAL, "select_parents: margins must be >= 0");
  if (o->learned && o->deep_dz != 0 && !(o->deep_dz > 0 && o->margin_lo_deep >= 0 && o->margin_hi_deep >= 0))
    return c->fail(KSG_EINVAL, "select_parents: deep_dz must be >= 0 and the deep margins >= 0");
  if (o->mode < KSG_MODE_MULTIVARIATE_TE || o->mode > KSG_MODE_MULTIVARIATE_MI || (o->prune != 0 && o->prune != 1) ||
      (o->sequential != 0 && o->sequential != 1))
    return c->fail(KSG_EINVAL, "select_parents: mode %d / prune %d / sequential %d not known", o->mode, o->prune,
                   o->sequential);
  KSG_HIP(c, hipSetDevice(c->device));

  Selector s;
  s.c = c;
  s.o = o;
  s.L = o->max_lag;
  s.P = o->n_perm;
  s.C = n_vars * s.L;
  s.N = (int64_t)n_trials * (T - s.L);
  if (s.N > (int64_t)INT32_MAX - 1024) return c->fail(KSG_EINVAL, "select_parents: N too large");
  if (s.N <= o->k) return c->fail(KSG_ETOOFEW, "select_parents: N=%lld <= k=%d", (long long)s.N, o->k);
  s.n_pad = round_up64(s.N, kPad);

  int st = c->reserve(c->embed, sizeof(float) * (size_t)(s.C + 1) * s.n_pad, "embedded columns");
  if (st) return st;
  float* cand = (float*)c->embed.ptr;
  float* y = cand + (int64_t)s.C * s.n_pad;
  s.cand = cand;
  s.y = y;
  KSG_HIP(c, launch_embed(data, n_vars, T, n_trials, target, s.L, cand, y, s.n_pad, c->stream));
  // Every later batch reads these columns in place or through gathers of them.
  const bool check = c->check_finite;
  if (check) {
    std::vector<PackJob> cols;
    for (int i = 0; i <= s.C; ++i)
      cols.push_back(PackJob{cand + (int64_t)i * s.n_pad, nullptr, cand + (int64_t)i * s.n_pad, (int)s.N, (int)s.N});
    KSG_HIP(c, hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
    KSG_HIP(c, launch_perm_check(o->perms, s.P, (int)s.N, c->d_flag, c->stream));
    st = c->check_columns_finite(cols, (int)s.n_pad);
    if (st) return st;
  }
  c->check_finite = false;
  struct Restore {
    ksg_ctx* c;
    bool v;
    ~Restore() { c->check_finite = v; }
  } restore{c, check};

  st = c->reserve(c->cmi, sizeof(double) * (size_t)s.C * (s.P + 1), "CMI table");
  if (st) return st;
  double* d_cmi = (double*)c->cmi.ptr;

  out->n = 0;
  out->truncated = 0;
  out->n_pruned = 0;
  out->n_steps = 0;
  out->n_fallback = 0;
  out->n_disagree = 0;
  out->n_gate_decided = 0;
  out->omnibus_tested = 0;
  out->omnibus_significant = 0;
  out->omnibus_cmi = 0;
  out->omnibus_pval = 0;
  out->n_cmi = 0;

  LearnedGate gate;
  if (o->learned) {
    st = gate.init(c, (const ksg_mlp*)o->learned, s.cand, s.n_pad, s.C, s.y, (int)s.N);
    if (st) return st;
  }

  // Inclusion over s.pool, conditioning on (and extending) s.selected; parents are recorded in
  // inclusion order.
  std::vector<int> incl;       // every included candidate, in order
  std::vector<double> incl_t;  // t_obs and p-value of its step
  std::vector<double> incl_p;
  // The conditioning set may hold at most cond_limit columns: the library's column limit less X
  // and Y (30; 14 under KSG algorithm 2), or the caller's smaller max_cond.  A selection whose
  // next step would need more stops there with truncated = 1: its last test was significant,
  // so the statistical stop was not reached.
  const int lib_cond = (c->algorithm == 2 ? kMaxDimsCompiled : KSG_MAX_DIMS) - 2;
  const int cond_limit = o->max_cond > 0 ? std::min(o->max_cond, lib_cond) : lib_cond;
  auto include_loop = [&]() -> int {
  while (!s.pool.empty() && (o->max_steps <= 0 || out->n_steps < o->max_steps)) {
    if ((int)s.selected.size() > cond_limit) {
      out->truncated = 1;
      break;
    }
    const int cands = (int)s.pool.size();
    char label[64];
    std::snprintf(label, sizeof label, "ksg greedy step %d (m=%d, %d candidates)", out->n_steps,
                  (int)s.selected.size(), cands);
    TraceRange step_range(label);
    int decision = -1;  // 1 include, 0 stop
    double t_obs = 0, pval = -1;
    int c_star = 0;
    bool run_full = true;
    int gate_verdict = 2, plain_decision = -1;
    float pred[2] = {NAN, NAN};
    if (o->learned) {
      // Originals only, then the gate on the device.
      st = s.step_cmis(0, 1, d_cmi);
      if (st) return st;
      out->n_cmi += cands;
      int verdict = 0;
      const bool deep = o->deep_dz > 0 && (int)s.selected.size() >= o->deep_dz;
      st = gate.decide(c, d_cmi, cands, s.P + 1, s.pool, 1, 1, (int)s.selected.size(), o->k, s.P,
                       deep ? o->margin_lo_deep : o->margin_lo, deep ? o->margin_hi_deep : o->margin_hi, &verdict,
                       &c_star, &t_obs, pred);
      if (st) return st;
      gate_verdict = verdict;
      if (verdict > 0 || (verdict < 0 && !o->verify_stop)) {
        decision = verdict > 0 ? 1 : 0;
        run_full = o->judge != 0;
        if (!o->judge) out->n_gate_decided++;
      } else {
        // borderline, or a predicted stop that the plain test confirms (verify_stop)
        out->n_fallback++;
      }
    }
    if (run_full) {
      st = s.step_cmis(o->learned ? 1 : 0, s.P + 1, d_cmi);
      if (st) return st;
      out->n_cmi += (int64_t)cands * (o->learned ? s.P : s.P + 1);
      st = c->maxstat_async(d_cmi, cands, s.P, o->alpha, 0);
      if (st) return st;
      KSG_HIP(c, hipStreamSynchronize(c->stream));
      const MaxStatOut& m = c->h_ms[0];
      const int plain = m.significant ? 1 : 0;
      plain_decision = plain;
      if (decision >= 0 && decision != plain) out->n_disagree++;
      if (decision >= 0 && o->judge) out->n_gate_decided++;
      decision = plain;
      t_obs = m.t_obs;
      pval = m.pval;
      c_star = m.c_star;
    }
    if (out->n_steps < out->step_capacity) {
      const int i = out->n_steps;
      if (out->step_tobs) out->step_tobs[i] = t_obs;
      if (out->step_pred) {
        out->step_pred[2 * i] = pred[0];
        out->step_pred[2 * i + 1] = pred[1];
      }
      if (out->step_verdict) out->step_verdict[i] = gate_verdict;
      if (out->step_plain) out->step_plain[i] = plain_decision;
    }
    out->n_steps++;
    if (decision != 1) break;
    const int chosen = s.pool[c_star];
    incl.push_back(chosen);
    incl_t.push_back(t_obs);
    incl_p.push_back(pval);
    s.selected.push_back(chosen);
    s.pool.erase(s.pool.begin() + c_star);
  }
  return KSG_OK;
  };

  const int n_vars_all = s.C / s.L;
  if (o->mode == KSG_MODE_BIVARIATE_TE) {
    for (int l = 0; l < s.L; ++l) s.pool.push_back(target * s.L + l);
    st = include_loop();
    if (st) return st;
    const std::vector<int> tgt_sel = s.selected;
    for (int v = 0; v < n_vars_all; ++v) {
      if (v == target) continue;
      s.selected = tgt_sel;
      s.pool.clear();
      for (int l = 0; l < s.L; ++l) s.pool.push_back(v * s.L + l);
      st = include_loop();
      if (st) return st;
    }
    // the parent set: the target past, then every source's lags
    s.selected = incl;
  } else {
    for (int i = 0; i < s.C; ++i)
      if (o->mode == KSG_MODE_MULTIVARIATE_TE || i / s.L != target) s.pool.push_back(i);
    // resume: the recorded inclusions of an earlier run come first, without their tests
    for (int r = 0; r < o->n_resume; ++r) {
      const auto it = std::find(s.pool.begin(), s.pool.end(), (int)o->resume[r]);
      if (it == s.pool.end())
        return c->fail(KSG_EINVAL, "select_parents: resume[%d] = %d is not an unselected candidate of this mode", r,
                       o->resume[r]);
      s.pool.erase(it);
      s.selected.push_back(o->resume[r]);
      incl.push_back(o->resume[r]);
      incl_t.push_back(NAN);
      incl_p.push_back(NAN);
    }
    st = include_loop();
    if (st) return st;
  }

  // ---- min-statistic pruning of the selected sources ----
  std::vector<int> kept = incl;
  std::vector<int> pruned;
  // Table [src][P+1] of I(c ; Y | kept \ {c}) for every source c in src, originals in column 0
  // and one surrogate per round (c's rows permuted), copied to the host.
  std::vector<double> h_tab;
  auto source_table = [&](const std::vector<int>& src) -> int {
    std::vector<Problem> probs;
    probs.reserve(src.size() * (s.P + 1));
    for (size_t i = 0; i < src.size(); ++i) {
      for (int p = 0; p <= s.P; ++p) {
        Problem q;
        std::memset(&q, 0, sizeof q);
        q.n = s.N;
        q.dx = 1;
        q.dy = 1;
        q.k = o->k;
        q.col[0] = cand + (int64_t)src[i] * s.n_pad;
        q.perm[0] = p > 0 ? o->perms + (int64_t)(p - 1) * s.N : nullptr;
        q.padded[0] = true;
        q.col[1] = y;
        q.padded[1] = true;
        int a = 2;
        for (int other : kept)
          if (other != src[i]) {
            q.col[a] = cand + (int64_t)other * s.n_pad;
            q.padded[a++] = true;
          }
        q.dz = a - 2;
        q.out_index = (int)i * (s.P + 1) + p;
        probs.push_back(q);
      }
    }
    int rc = c->run_batch(probs, d_cmi);
    if (rc) return rc;
    out->n_cmi += (int64_t)probs.size();
    h_tab.resize(probs.size());
    KSG_HIP(c, hipMemcpyAsync(h_tab.data(), d_cmi, sizeof(double) * h_tab.size(), hipMemcpyDeviceToHost,
                              c->stream));
    KSG_HIP(c, hipStreamSynchronize(c->stream));
    return KSG_OK;
  };
  auto sources_of = [&]() {
    std::vector<int> src;
    for (int cidx : kept)
      if (cidx / s.L != target) src.push_back(cidx);
    return src;
  };
  if (o->prune) {
    TraceRange prune_range("ksg pruning");
    for (;;) {
      const std::vector<int> src = sources_of();
      if (src.empty()) break;
      st = source_table(src);
      if (st) return st;
      // minimum statistic: T_min over the originals (lowest index on ties), per-round minima
      int c_min = 0;
      for (size_t i = 1; i < src.size(); ++i)
        if (h_tab[i * (s.P + 1)] < h_tab[(size_t)c_min * (s.P + 1)]) c_min = (int)i;
      const double t_min = h_tab[(size_t)c_min * (s.P + 1)];
      int count = 0;
      for (int p = 1; p <= s.P; ++p) {
        double m = h_tab[p];
        for (size_t i = 1; i < src.size(); ++i) m = std::min(m, h_tab[i * (s.P + 1) + p]);
        if (m >= t_min) ++count;
      }
      if ((double)count / s.P < o->alpha) break;  // significant: keep the rest
      pruned.push_back(src[c_min]);
      kept.erase(std::find(kept.begin(), kept.end(), src[c_min]));
    }
    s.selected = kept;
  }
  out->n_pruned = (int32_t)pruned.size();
  for (size_t i = 0; i < pruned.size() && (int)i < out->capacity; ++i)
    if (out->pruned) out->pruned[i] = pruned[i];

  if (o->omnibus) {
    TraceRange omni_range("ksg omnibus test");
    std::vector<int> src, tgt;
    for (int cidx : s.selected) (cidx / s.L == target ? tgt : src).push_back(cidx);
    if (!src.empty() && (int)(src.size() + 1 + tgt.size()) <= lib_cond + 2) {
      std::vector<Problem> probs(s.P + 1);
      for (int p = 0; p <= s.P; ++p) {
        Problem& q = probs[p];
        std::memset(&q, 0, sizeof q);
        q.n = s.N;
        q.dx = (int)src.size();
        q.dy = 1;
        q.dz = (int)tgt.size();
        q.k = o->k;
        int a = 0;
        for (int cidx : src) {
          q.col[a] = cand + (int64_t)cidx * s.n_pad;
          q.perm[a] = p > 0 ? o->perms + (int64_t)(p - 1) * s.N : nullptr;
          q.padded[a] = true;
          ++a;
        }
        q.col[a] = y;
        q.padded[a++] = true;
        for (int cidx : tgt) {
          q.col[a] = cand + (int64_t)cidx * s.n_pad;
          q.padded[a++] = true;
        }
        q.out_index = p;
      }
      st = c->run_batch(probs, d_cmi);
      if (st) return st;
      out->n_cmi += s.P + 1;
      st = c->maxstat_async(d_cmi, 1, s.P, o->alpha, 0);
      if (st) return st;
      KSG_HIP(c, hipStreamSynchronize(c->stream));
      out->omnibus_tested = 1;
      out->omnibus_significant = c->h_ms[0].significant;
      out->omnibus_cmi = c->h_ms[0].t_obs;
      out->omnibus_pval = c->h_ms[0].pval;
    }
  }
  // ---- sequential max-statistic test of the kept sources (after a significant omnibus test) ----
  std::vector<int> seq_removed;
  std::vector<std::pair<int, double>> seq_p;  // (source, p-value) of every tested source
  if (o->sequential && (!o->omnibus || !out->omnibus_tested || out->omnibus_significant)) {
    TraceRange seq_range("ksg sequential test");
    const std::vector<int> src = sources_of();
    if (!src.empty()) {
      st = source_table(src);
      if (st) return st;
      std::vector<int32_t> sig(src.size());
      std::vector<double> pv(src.size());
      if (ksg_maxstat_sequential(h_tab.data(), (int32_t)src.size(), s.P, o->alpha, sig.data(), pv.data()))
        return c->fail(KSG_EINVAL, "select_parents: sequential test");
      // removed sources in rank order (descending original CMI, lower row first on ties)
      std::vector<int> rank(src.size());
      for (size_t i = 0; i < src.size(); ++i) rank[i] = (int)i;
      std::stable_sort(rank.begin(), rank.end(),
                       [&](int a, int b) { return h_tab[(size_t)a * (s.P + 1)] > h_tab[(size_t)b * (s.P + 1)]; });
      for (int i : rank)
        if (!sig[i]) seq_removed.push_back(src[i]);
      for (size_t i = 0; i < src.size(); ++i) seq_p.emplace_back(src[i], pv[i]);
      for (int r : seq_removed) kept.erase(std::find(kept.begin(), kept.end(), r));
      s.selected = kept;
    }
  }
  out->n_seq_removed = (int32_t)seq_removed.size();
  for (size_t i = 0; i < seq_removed.size() && (int)i < out->capacity; ++i)
    if (out->seq_removed) out->seq_removed[i] = seq_removed[i];

  // parents: the kept candidates in inclusion order, with their inclusion step's statistics
  for (size_t i = 0; i < incl.size(); ++i) {
    if (std::find(kept.begin(), kept.end(), incl[i]) == kept.end()) continue;
    if (out->n < out->capacity) {
      if (out->var) out->var[out->n] = incl[i] / s.L;
      if (out->lag) out->lag[out->n] = incl[i] % s.L + 1;
      if (out->cmi) out->cmi[out->n] = incl_t[i];
      if (out->pval) out->pval[out->n] = incl_p[i];
      if (out->seq_pval) {
        double v = -1.0;
        for (const auto& e : seq_p)
          if (e.first == incl[i]) v = e.second;
        out->seq_pval[out->n] = v;
      }
    }
    out->n++;
  }

  KSG_HIP(c, hipStreamSynchronize(c->stream));
  if (out->n > out->capacity)
    return c->fail(KSG_EBUFSMALL, "select_parents: %d parents, capacity %d", out->n, out->capacity);
  return KSG_OK;
}

extern "C" int ksg_greedy_step(ksg_ctx* c, const float* cand, const float* y, int64_t N,
                               const int32_t* pool, int32_t n_pool, const int32_t* cond,
                               int32_t n_cond, const int32_t* perms, int32_t n_perm, int32_t k,
                               double alpha, double* cmi_out, ksg_maxstat_result* result) {
  if (!c) return KSG_EINVAL;
  if (!cand || !y || !pool || (n_cond > 0 && !cond) || !cmi_out || !result || (n_perm > 0 && !perms))
    return c->fail(KSG_EINVAL, "ksg_greedy_step: null argument");
  if (n_pool < 1 || n_cond < 0 || 2 + n_cond > KSG_MAX_DIMS || n_perm < 1 || n_perm > 4096)
    return c->fail(KSG_EINVAL, "ksg_greedy_step: need n_pool >= 1, 0 <= n_cond <= %d, 1 <= n_perm <= 4096",
                   KSG_MAX_DIMS - 2);
  for (int i = 0; i < n_pool; ++i)
    if (pool[i] < 0) return c->fail(KSG_EINVAL, "ksg_greedy_step: negative candidate index");
  for (int i = 0; i < n_cond; ++i)
    if (cond[i] < 0) return c->fail(KSG_EINVAL, "ksg_greedy_step: negative conditioning index");
  KSG_HIP(c, hipSetDevice(c->device));
  std::vector<Problem> probs;
  probs.reserve((size_t)n_pool * (n_perm + 1));
  for (int ci = 0; ci < n_pool; ++ci) {
    for (int p = 0; p <= n_perm; ++p) {
      Problem q;
      std::memset(&q, 0, sizeof q);
      q.n = N;
      q.dx = 1;
      q.dy = 1;
      q.dz = n_cond;
      q.k = k;
      q.col[0] = cand + (int64_t)pool[ci] * N;
      q.perm[0] = p > 0 ? perms + (int64_t)(p - 1) * N : nullptr;
      q.col[1] = y;
      for (int s = 0; s < n_cond; ++s) q.col[2 + s] = cand + (int64_t)cond[s] * N;
      q.out_index = ci * (n_perm + 1) + p;
      probs.push_back(q);
    }
  }
  int st = c->run_batch(probs, cmi_out);
  if (st) return st;
  st = c->maxstat_async(cmi_out, n_pool, n_perm, alpha, 0);
  if (st) return st;
  KSG_HIP(c, hipStreamSynchronize(c->stream));
  const MaxStatOut& m = c->h_ms[0];
  result->c_star = m.c_star;
  result->count = m.count;
  result->significant = m.significant;
  result->n_perm = m.n_perm;
  result->t_obs = m.t_obs;
  result->pval = m.pval;
  result->tau05 = m.tau05;
  result->tau01 = m.tau01;
  return KSG_OK;
}
