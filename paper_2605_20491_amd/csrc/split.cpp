// Splitting schemes for i psi_t = (H1 + V2) psi (paper Sec. 5.1): A = H1 is
// applied exactly by the separable propagator, B = V2 pointwise.
//
// The scheme is written out as a sequence of factors e^{-i t A} / e^{-i t B},
// adjacent factors of the same operator are merged (their times add, exactly:
// e^{-i a X} e^{-i b X} = e^{-i (a+b) X}), and every remaining B factor is
// fused into the load or store of the neighbouring A factor.  This is the
// merged schedule of Remark rem:cost_naive_merged: one A propagation per
// Strang step, three A and three B per Yoshida step.
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ts.h"
#include "ts_apply.h"
#include "ts_internal.h"
#include "ts_small.h"

namespace ts {

// Factor list of nsteps steps; 'A' = propagator of H1, 'B' = potential factor.
std::vector<std::pair<char, double>> split_factors(int scheme, double dt, int nsteps) {
  std::vector<std::pair<char, double>> ops;
  const double c = std::cbrt(2.0);
  const double g1 = 1.0 / (2.0 - c), g2 = -c / (2.0 - c);
  auto strang = [&](double h, bool bab) {
    // listed in the order the factors act on psi
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
  std::vector<std::pair<char, double>> merged;
  for (auto& o : ops) {
    if (!merged.empty() && merged.back().first == o.first) merged.back().second += o.second;
    else merged.push_back(o);
  }
  return merged;
}

}  // namespace ts

using namespace ts;

extern "C" int ts_split_step(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int scheme,
                             int dtype, int prec, void* hip_stream) {
  if (!plan || !V2 || !psi) { set_error("null argument"); return TS_ERR_INVALID; }
  if (nsteps < 0 || !std::isfinite(dt)) { set_error("bad dt or nsteps"); return TS_ERR_INVALID; }
  if (scheme < TS_STRANG_BAB || scheme > TS_YOSHIDA_ABA) { set_error("unknown scheme"); return TS_ERR_INVALID; }
  if (dtype != TS_C128 && dtype != TS_C64) { set_error("splitting needs TS_C128 or TS_C64 data"); return TS_ERR_INVALID; }
  if (prec < TS_PREC_FP64 || prec > TS_PREC_BF16) { set_error("bad precision"); return TS_ERR_INVALID; }
  if (prec == TS_PREC_FP64 && dtype != TS_C128) { set_error("FP64 transforms need TS_C128 data"); return TS_ERR_INVALID; }
  hipStream_t st = (hipStream_t)hip_stream;
  auto ops = split_factors(scheme, dt, nsteps);
  int lastA = -1;
  for (int i = 0; i < (int)ops.size(); ++i)
    if (ops[i].first == 'A') lastA = i;
  const bool fp64_data = dtype == TS_C128;
  if (lastA < 0) {
    for (auto& o : ops) {
      hipError_t e = launch_phase(psi, V2, o.second, plan->N, fp64_data, st);
      if (e != hipSuccess) { set_error("phase launch failed"); return TS_ERR_DEVICE; }
    }
    return TS_OK;
  }
  Phases ph;
  ph.V2 = V2;
  for (int i = 0; i < (int)ops.size(); ++i) {
    if (ops[i].first == 'B') {
      if (i > lastA) break;  // trailing factor: fused into the last A below
      ph.pre = true;
      ph.th_pre = ops[i].second;
      continue;
    }
    if (i == lastA && i + 1 < (int)ops.size()) {
      ph.post = true;
      ph.th_post = ops[i + 1].second;
    }
    int rc = apply_exp_phased(plan, ops[i].second, psi, dtype, prec, ph, st, nullptr);
    if (rc) return rc;
    ph.pre = ph.post = false;
  }
  return TS_OK;
}
