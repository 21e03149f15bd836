// Small-extent grouped passes (modeprod_small.hip) and their host planner.
#pragma once

#include "ts_internal.h"

namespace ts {

constexpr int64_t kSmallMaxN = 32;          // every axis at most this long -> grouped path
constexpr int kSmallTileBytes = 48 * 1024;  // LDS tile budget per block

struct GroupStep {
  const void* Q = nullptr;  // factor (Q for forward, Q^T for backward), compute precision, [ld][ld]
  int64_t ld = 0;
  int n = 0;
  int stride = 1;           // stride of this axis inside the group index
  uint32_t wmul = 0;        // ceil(2^32 / (stride x RT)), 0 when that is 1 (set by the launcher)
};

struct GroupArgs {
  const void* Xin = nullptr;
  void* Xout = nullptr;
  int64_t P = 1, R = 1;     // tensor viewed as [P][G][R] (R counts real values)
  int G = 1;
  int PB = 1, RT = 1;       // tile: PB x G x RT
  int flat = 0;             // tile is one contiguous run (RT = R; set by the launcher)
  int tile_elems = 0;
  int64_t rtiles = 1, nblocks = 0;
  int nsteps = 0;
  GroupStep step[8];
  int scale_after = -1;     // apply the diagonal after this step (slowest group only)
  const double* Lg = nullptr;  // inverse: 1 / (Lg[g] + Lr[q] + shift)
  const double* Lr = nullptr;
  double shift = 0.0;
  const double2* Eg = nullptr; // propagator: Eg[g] * Er[q]
  const double2* Er = nullptr;
  const void* V2 = nullptr;    // real, same precision as the data
  double th_pre = 0.0, th_post = 0.0;
  int pre = 0, post = 0;
  const int* skip = nullptr;
};

struct RangeTableArgs {
  int d = 0, split = 0, mode = 0;
  int64_t n[TS_MAX_D] = {};
  const double* lam[TS_MAX_D] = {};
  double tau = 0.0;
  int64_t n_lo = 0, n_hi = 0;
  double* L_lo = nullptr;
  double* L_hi = nullptr;
  double2* E_lo = nullptr;
  double2* E_hi = nullptr;
};

int small_nmax(int64_t n);
hipError_t launch_group(const GroupArgs& a, DT tio, bool fp64_compute, bool cplx, int nmax, hipStream_t st);
hipError_t launch_phase(void* psi, const void* V2, double theta, int64_t N, bool fp64, hipStream_t st);
hipError_t launch_range_tables(const RangeTableArgs& a, hipStream_t st);

// True if every axis of the plan takes the grouped path.
bool plan_is_small(const ts_plan* p);

// Apply through grouped passes.  cplx: interleaved complex data; epi: Inv or
// Exp; V2 / th_pre / th_post: optional fused potential factors (complex only).
struct SmallApply {
  const void* in = nullptr;
  void* out = nullptr;
  DT tio = DT::F64;
  bool fp64 = true;
  bool cplx = false;
  Epi epi = Epi::Inv;
  double shift = 0.0;
  double tau = 0.0;
  const void* V2 = nullptr;
  double th_pre = 0.0, th_post = 0.0;
  bool pre = false, post = false;
  const int* skip = nullptr;
  bool sym = false;  // the plan's orthogonal (solver) factors
};
int run_small_apply(ts_plan* p, const SmallApply& s, hipStream_t st, ExecCtx& c);
// Bytes of the diagonal tables of one grouped apply.
size_t small_table_bytes(const ts_plan* p, bool cplx, bool fp64, bool exp);

}  // namespace ts
