// Host planner of the grouped small-extent passes: partitions the axes into
// groups whose tiles fit in LDS, sizes the tiles, builds the FP64 diagonal
// tables of the slowest group and launches the 2g - 1 passes of one apply.
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ts.h"
#include "ts_internal.h"
#include "ts_small.h"

namespace ts {

bool plan_is_small(const ts_plan* p) {
  for (int k = 0; k < p->d; ++k)
    if (p->n[k] > kSmallMaxN) return false;
  return true;
}

namespace {

struct Group {
  int a, b;       // axes a..b (inclusive), a slower than b
  int64_t G;
};

// Groups from the fastest axis down.  The fastest group's tile holds whole
// groups (R = components); the others need at least rt_min contiguous values
// per tile row.
std::vector<Group> make_groups(const ts_plan* p, int ncomp, int64_t budget, int64_t rt_min) {
  std::vector<Group> gs;
  int k = p->d - 1;
  bool fastest = true;
  while (k >= 0) {
    Group g{k, k, p->n[k]};
    const int64_t need_r = fastest ? ncomp : rt_min;
    while (g.a - 1 >= 0 && (g.b - g.a + 1) < 4 && g.G * p->n[g.a - 1] * need_r <= budget) {
      g.a -= 1;
      g.G *= p->n[g.a];
    }
    gs.push_back(g);
    k = g.a - 1;
    fastest = false;
  }
  std::reverse(gs.begin(), gs.end());  // gs[0] is the slowest group
  return gs;
}

}  // namespace

size_t small_table_bytes(const ts_plan* p, bool cplx, bool fp64, bool exp) {
  (void)fp64;
  // size for either compute precision (their groupings differ)
  size_t worst = 0;
  for (int64_t eb : {4, 8}) {
    std::vector<Group> gs = make_groups(p, cplx ? 2 : 1, kSmallTileBytes / eb, 64 / eb);
    const int64_t G = gs[0].G;
    worst = std::max(worst, (size_t)(G + p->N / G));
  }
  return worst * (exp ? sizeof(double2) : sizeof(double)) + 256;
}

int run_small_apply(ts_plan* p, const SmallApply& s, hipStream_t st, ExecCtx& c) {
  const int d = p->d;
  const int ncomp = s.cplx ? 2 : 1;
  const size_t eb = s.fp64 ? 8 : 4;
  const int64_t budget = kSmallTileBytes / (int64_t)eb;
  const int64_t rt_min = 64 / (int64_t)eb;  // 64-byte runs
  std::vector<Group> gs = make_groups(p, ncomp, budget, rt_min);
  const int m = (int)gs.size();

  // diagonal tables of the slowest group: axes [0, b0] vs (b0, d)
  const Group& g0 = gs[0];
  const int64_t nlo = g0.G, nhi = p->N / g0.G;
  void* tab = nullptr;
  const size_t tb = (size_t)(nlo + nhi) * (s.epi == Epi::Exp ? sizeof(double2) : sizeof(double));
  int rc = ctx_get(c, kSlotTab, tb, &tab);
  if (rc) return rc;
  RangeTableArgs ra;
  ra.d = d;
  ra.split = g0.b + 1;
  ra.mode = s.epi == Epi::Exp ? 1 : 0;
  for (int k = 0; k < d; ++k) {
    ra.n[k] = p->n[k];
    ra.lam[k] = p->ax[k]->lam;
  }
  ra.tau = s.tau;
  ra.n_lo = nlo;
  ra.n_hi = nhi;
  if (ra.mode == 0) {
    ra.L_lo = (double*)tab;
    ra.L_hi = ra.L_lo + nlo;
  } else {
    ra.E_lo = (double2*)tab;
    ra.E_hi = ra.E_lo + nlo;
  }
  hipError_t e = launch_range_tables(ra, st);
  if (e != hipSuccess) { set_error("table launch failed"); return TS_ERR_DEVICE; }

  // pass list: forward over groups m-1..1, the slowest group (forward, scale,
  // backward), backward over groups 1..m-1
  struct PassDesc { int gi; bool fwd, bwd; };
  std::vector<PassDesc> passes;
  for (int gi = m - 1; gi >= 1; --gi) passes.push_back({gi, true, false});
  passes.push_back({0, true, true});
  for (int gi = 1; gi < m; ++gi) passes.push_back({gi, false, true});

  for (size_t pi = 0; pi < passes.size(); ++pi) {
    const Group& g = gs[passes[pi].gi];
    GroupArgs a;
    a.Xin = pi == 0 ? s.in : s.out;
    a.Xout = s.out;
    a.P = 1;
    for (int k = 0; k < g.a; ++k) a.P *= p->n[k];
    a.R = ncomp;
    for (int k = g.b + 1; k < d; ++k) a.R *= p->n[k];
    a.G = (int)g.G;
    if (g.b == d - 1) {  // fastest group: whole groups per tile
      a.RT = (int)a.R;
      a.PB = (int)std::max<int64_t>(1, std::min<int64_t>(a.P, budget / (g.G * a.R)));
    } else {
      a.PB = 1;
      int64_t rt = std::min<int64_t>(a.R, budget / g.G);
      if (rt >= rt_min) rt = rt / rt_min * rt_min;
      if (s.cplx && (rt & 1)) rt -= 1;
      a.RT = (int)std::max<int64_t>(rt, ncomp);
    }
    a.tile_elems = a.PB * a.G * a.RT;
    a.rtiles = (a.R + a.RT - 1) / a.RT;
    a.nblocks = ((a.P + a.PB - 1) / a.PB) * a.rtiles;
    int nmax = 0;
    int ns = 0;
    auto add_steps = [&](bool forward) {
      // forward over the group's axes fastest first, backward slowest first
      for (int i = 0; i <= g.b - g.a; ++i) {
        const int k = forward ? g.b - i : g.a + i;
        const AxisFactor* F = (s.sym ? p->ax_sym : p->ax)[k].get();
        GroupStep& S = a.step[ns++];
        if (s.fp64) S.Q = forward ? (const void*)F->Q64 : (const void*)F->QT64;
        else S.Q = forward ? (const void*)F->Q32 : (const void*)F->QT32;
        S.ld = F->ld;
        S.n = (int)p->n[k];
        int64_t stride = 1;
        for (int m2 = k + 1; m2 <= g.b; ++m2) stride *= p->n[m2];
        S.stride = (int)stride;
        nmax = std::max(nmax, small_nmax(p->n[k]));
      }
    };
    if (passes[pi].fwd) add_steps(true);
    if (passes[pi].fwd && passes[pi].bwd) {
      a.scale_after = ns - 1;
      if (s.epi == Epi::Exp) {
        a.Eg = (const double2*)tab;
        a.Er = a.Eg + nlo;
      } else {
        a.Lg = (const double*)tab;
        a.Lr = a.Lg + nlo;
        a.shift = s.shift;
      }
    }
    if (passes[pi].bwd) add_steps(false);
    a.nsteps = ns;
    a.V2 = s.V2;
    if (pi == 0 && s.pre) { a.pre = 1; a.th_pre = s.th_pre; }
    if (pi + 1 == passes.size() && s.post) { a.post = 1; a.th_post = s.th_post; }
    a.skip = s.skip;
    e = launch_group(a, s.tio, s.fp64, s.cplx, nmax, st);
    if (e != hipSuccess) {
      set_error(std::string("grouped pass launch failed: ") + hipGetErrorString(e));
      return TS_ERR_DEVICE;
    }
  }
  return TS_OK;
}

}  // namespace ts
