// Splitting schemes for i psi_t = (H1 + V2) psi (paper Sec. 5.1): A = H1 is
// applied exactly by the separable propagator, B = V2 pointwise.
//
// The scheme is written out as a sequence of factors e^{-i t A} / e^{-i t B},
// adjacent factors of the same operator are merged (their times add, exactly:
// e^{-i a X} e^{-i b X} = e^{-i (a+b) X}), and every remaining B factor is
// fused into the load or store of the neighbouring A factor.  This is the
// merged schedule of Remark rem:cost_naive_merged: one A propagation per
// Strang step, three A and three B per Yoshida step, M per approximated qHOP
// step and 3M per approximated Magnus-2 step (M >= 2, asymptotically in the
// number of steps).
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ts.h"
#include "ts_apply.h"
#include "ts_internal.h"
#include "ts_small.h"
#include "ts_tasks.h"

namespace ts {

// Factor list of nsteps steps, in the order the factors act on psi;
// 'A' = propagator of H1, 'B' = potential factor.
std::vector<std::pair<char, double>> split_factors(int scheme, double dt, int nsteps) {
  std::vector<std::pair<char, double>> ops;
  const double c = std::cbrt(2.0);
  const double g1 = 1.0 / (2.0 - c), g2 = -c / (2.0 - c);
  auto strang = [&](double h, bool bab) {
    if (bab) {
      ops.push_back({'B', h / 2});
      ops.push_back({'A', h});
      ops.push_back({'B', h / 2});
    } else {
      ops.push_back({'A', h / 2});
      ops.push_back({'B', h});
      ops.push_back({'A', h / 2});
    }
  };
  for (int i = 0; i < nsteps; ++i) {
    switch (scheme) {
      case TS_STRANG_BAB: strang(dt, true); break;
      case TS_STRANG_ABA: strang(dt, false); break;
      case TS_YOSHIDA_BAB: strang(g1 * dt, true); strang(g2 * dt, true); strang(g1 * dt, true); break;
      case TS_YOSHIDA_ABA: strang(g1 * dt, false); strang(g2 * dt, false); strang(g1 * dt, false); break;
    }
  }
  return merge_factors(ops);
}

std::vector<std::pair<char, double>> merge_factors(const std::vector<std::pair<char, double>>& ops) {
  std::vector<std::pair<char, double>> merged;
  for (auto& o : ops) {
    if (!merged.empty() && merged.back().first == o.first) merged.back().second += o.second;
    else merged.push_back(o);
  }
  return merged;
}

// M-point Gauss-Legendre rule on [0, 1]: nodes ascending, weights summing to
// one.  Newton's method on P_M, evaluated by the three-term recurrence
// (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}, with P_M' = M (x P_M - P_{M-1}) /
// (x^2 - 1); starting points cos(pi (i + 3/4) / (M + 1/2)) lie close to the
// roots.  Weight on [-1, 1]: 2 / ((1 - x^2) P_M'(x)^2).
bool gauss_legendre01(int M, double* s, double* w) {
  if (M < 1 || M > kMaxQuadNodes) return false;
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < M; ++i) {
    double x = std::cos(pi * (i + 0.75) / (M + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 1; k < M; ++k) {
        double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      dp = M * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    // evaluate P_M' once more at the converged root
    double p0 = 1.0, p1 = x;
    for (int k = 1; k < M; ++k) {
      double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
      p0 = p1;
      p1 = p2;
    }
    dp = M * (x * p1 - p0) / (x * x - 1.0);
    // roots come out descending; store ascending on [0, 1]
    s[M - 1 - i] = 0.5 * (x + 1.0);
    w[M - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);  // (2 / ((1-x^2) P'^2)) / 2
  }
  return true;
}

// Approximated qHOP step of size h (Sec. 5.1, eq. (qhop_product)) in the
// merged form of Remark rem:cost_naive_merged:
//   e^{-iA (h - s_M)} e^{-i w_M h B} e^{-iA (s_M - s_{M-1})} ... e^{-i w_1 h B} e^{-iA s_1},
// the rightmost factor acting first; s_k = h * node_k, w_k the normalised
// weights.  Magnus-2 (eq. (yoshida)) chains three such steps of sizes
// g1 dt, g2 dt, g1 dt.  Factors of the same operator that meet at step and
// sub-step boundaries are merged.
std::vector<std::pair<char, double>> qhop_factors(double dt, int nsteps, int M, bool magnus2) {
  std::vector<std::pair<char, double>> ops;
  double node[kMaxQuadNodes], wt[kMaxQuadNodes];
  if (!gauss_legendre01(M, node, wt)) return ops;
  const double c = std::cbrt(2.0);
  const double g1 = 1.0 / (2.0 - c), g2 = -c / (2.0 - c);
  auto step = [&](double h) {
    double prev = 0.0;
    for (int k = 0; k < M; ++k) {
      ops.push_back({'A', h * node[k] - prev});
      ops.push_back({'B', wt[k] * h});
      prev = h * node[k];
    }
    ops.push_back({'A', h - prev});
  };
  for (int i = 0; i < nsteps; ++i) {
    if (magnus2) {
      step(g1 * dt);
      step(g2 * dt);
      step(g1 * dt);
    } else {
      step(dt);
    }
  }
  return merge_factors(ops);
}

namespace {

int check_common(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int dtype, int prec) {
  if (!plan || !V2 || !psi) { set_error("null argument"); return TS_ERR_INVALID; }
  if (nsteps < 0 || !std::isfinite(dt)) { set_error("bad dt or nsteps"); return TS_ERR_INVALID; }
  if (dtype != TS_C128 && dtype != TS_C64) { set_error("splitting needs TS_C128 or TS_C64 data"); return TS_ERR_INVALID; }
  if (prec < TS_PREC_FP64 || prec > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  return TS_OK;
}

int check_split(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int scheme, int dtype, int prec) {
  if (scheme < TS_STRANG_BAB || scheme > TS_YOSHIDA_ABA) { set_error("unknown scheme"); return TS_ERR_INVALID; }
  return check_common(plan, V2, psi, dt, nsteps, dtype, prec);
}

int check_qhop(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int M, int dtype, int prec) {
  if (M < 1 || M > kMaxQuadNodes) { set_error("M must be in 1..64"); return TS_ERR_INVALID; }
  return check_common(plan, V2, psi, dt, nsteps, dtype, prec);
}

// Runs the merged factor list a few A factors per unit.
class SplitTask : public Task {
 public:
  SplitTask(ts_plan* p, const void* V2, void* psi, std::vector<std::pair<char, double>> ops, int nsteps,
            int dtype, int prec, ExecCtx& c)
      : p_(p), V2_(V2), psi_(psi), dtype_(dtype), prec_(prec), c_(c), ops_(std::move(ops)) {
    for (int i = 0; i < (int)ops_.size(); ++i)
      if (ops_[i].first == 'A') lastA_ = i;
    iters = nsteps;
  }
  int start(hipStream_t st) override {
    if (lastA_ < 0) {  // nsteps = 0 or only potential factors
      for (auto& o : ops_) {
        hipError_t e = launch_phase(psi_, V2_, o.second, p_->N, dtype_ == TS_C128, st);
        if (e != hipSuccess) { set_error("phase launch failed"); return TS_ERR_DEVICE; }
      }
      pos_ = (int)ops_.size();
      return TS_OK;
    }
    return unit(st);
  }
  int advance(hipStream_t st, bool* done) override {
    *done = pos_ > lastA_;
    if (*done) return TS_OK;
    return unit(st);
  }

 private:
  int unit(hipStream_t st) {
    int applied = 0;
    Phases ph;
    ph.V2 = V2_;
    while (pos_ <= lastA_ && applied < kPerUnit) {
      const auto& o = ops_[pos_];
      if (o.first == 'B') {
        ph.pre = true;
        ph.th_pre = o.second;
        ++pos_;
        continue;
      }
      if (pos_ == lastA_ && pos_ + 1 < (int)ops_.size()) {  // trailing potential factor
        ph.post = true;
        ph.th_post = ops_[pos_ + 1].second;
      }
      int rc = apply_exp_phased(p_, o.second, psi_, dtype_, prec_, ph, st, c_);
      if (rc) return rc;
      ph.pre = ph.post = false;
      ++pos_;
      ++applied;
    }
    return TS_OK;
  }

  static constexpr int kPerUnit = 4;
  ts_plan* p_;
  const void* V2_;
  void* psi_;
  int dtype_, prec_;
  ExecCtx& c_;
  std::vector<std::pair<char, double>> ops_;
  int lastA_ = -1, pos_ = 0;
};

}  // namespace

std::unique_ptr<Task> make_split_task(ts_plan* p, const void* V2, void* psi, double dt, int nsteps, int scheme,
                                      int dtype, int prec, ExecCtx& c) {
  return std::unique_ptr<Task>(new SplitTask(p, V2, psi, split_factors(scheme, dt, nsteps), nsteps, dtype, prec, c));
}

std::unique_ptr<Task> make_qhop_task(ts_plan* p, const void* V2, void* psi, double dt, int nsteps, int M,
                                     bool magnus2, int dtype, int prec, ExecCtx& c) {
  return std::unique_ptr<Task>(
      new SplitTask(p, V2, psi, qhop_factors(dt, nsteps, M, magnus2), nsteps, dtype, prec, c));
}

int split_run(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int scheme, int dtype, int prec,
              hipStream_t st, ExecCtx& c) {
  int rc = check_split(plan, V2, psi, dt, nsteps, scheme, dtype, prec);
  if (rc) return rc;
  SplitTask t(plan, V2, psi, split_factors(scheme, dt, nsteps), nsteps, dtype, prec, c);
  return run_blocking(t, st);
}

int qhop_run(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int M, bool magnus2, int dtype,
             int prec, hipStream_t st, ExecCtx& c) {
  int rc = check_qhop(plan, V2, psi, dt, nsteps, M, dtype, prec);
  if (rc) return rc;
  SplitTask t(plan, V2, psi, qhop_factors(dt, nsteps, M, magnus2), nsteps, dtype, prec, c);
  return run_blocking(t, st);
}

int qhop_check(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int M, int dtype, int prec) {
  return check_qhop(plan, V2, psi, dt, nsteps, M, dtype, prec);
}

int split_check(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int scheme, int dtype, int prec) {
  return check_split(plan, V2, psi, dt, nsteps, scheme, dtype, prec);
}

}  // namespace ts

extern "C" int ts_qhop_step(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int M, int magnus2,
                            int dtype, int prec, void* hip_stream) {
  if (!plan) { ts::set_error("null plan"); return TS_ERR_INVALID; }
  return ts::qhop_run(plan, V2, psi, dt, nsteps, M, magnus2 != 0, dtype, prec, (hipStream_t)hip_stream, plan->ctx);
}

extern "C" int ts_gauss_legendre(int M, double* nodes, double* weights) {
  if (!nodes || !weights) { ts::set_error("null argument"); return TS_ERR_INVALID; }
  if (!ts::gauss_legendre01(M, nodes, weights)) { ts::set_error("M must be in 1..64"); return TS_ERR_INVALID; }
  return TS_OK;
}

extern "C" int ts_split_step(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int scheme,
                             int dtype, int prec, void* hip_stream) {
  if (!plan) { ts::set_error("null plan"); return TS_ERR_INVALID; }
  return ts::split_run(plan, V2, psi, dt, nsteps, scheme, dtype, prec, (hipStream_t)hip_stream, plan->ctx);
}
