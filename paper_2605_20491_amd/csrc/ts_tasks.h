// Non-blocking solver tasks.  A task enqueues one unit of work at a time on
// its stream; its driver records an event after each unit and, once the event
// has completed, calls advance() so the task can read its pinned scalar
// mirror and enqueue the next unit.  The blocking entry points and the
// serving loop drive the same tasks, so a request computes the same thing
// alone and inside a mix.
#pragma once

#include <memory>
#include <utility>
#include <vector>

#include "ts_internal.h"
#include "ts_vec.h"

namespace ts {

class Task {
 public:
  virtual ~Task() = default;
  // Enqueue the first unit.  Returns a ts_status.
  virtual int start(hipStream_t st) = 0;
  // The last enqueued unit has completed.  Either enqueue the next unit
  // (*done = false) or finish (*done = true, status/iters/relres final).
  virtual int advance(hipStream_t st, bool* done) = 0;
  int status = 0;
  int iters = 0;
  double relres = 0.0;
};

// Run a task to completion on `st`, waiting on an event between units.
int run_blocking(Task& t, hipStream_t st);

// scale_io: for SEM plans, f and x are in the caller's variables and are
// moved to and from the symmetric form's variables M^{1/2} x.
std::unique_ptr<Task> make_pcg_task(ts_plan* p, const double* V2, double s_op, double s_pc, const double* f,
                                    double* x, double rtol, int maxit, int prec, ExecCtx& c, bool scale_io = true);
std::unique_ptr<Task> make_refine_task(ts_plan* p, double sigma, const double* f, double* u, int inner,
                                       double rtol, int maxit, ExecCtx& c);
std::unique_ptr<Task> make_inverse_task(ts_plan* p, double shift, const void* b, void* u, int dtype, int prec,
                                        ExecCtx& c);
std::unique_ptr<Task> make_exp_task(ts_plan* p, double tau, const void* in, void* out, int dtype, int prec,
                                    ExecCtx& c);
std::unique_ptr<Task> make_split_task(ts_plan* p, const void* V2, void* psi, double dt, int nsteps, int scheme,
                                      int dtype, int prec, ExecCtx& c);

std::vector<std::pair<char, double>> split_factors(int scheme, double dt, int nsteps);
std::vector<std::pair<char, double>> merge_factors(const std::vector<std::pair<char, double>>& ops);
constexpr int kMaxQuadNodes = 64;
bool gauss_legendre01(int M, double* s, double* w);
std::vector<std::pair<char, double>> qhop_factors(double dt, int nsteps, int M, bool magnus2);
std::unique_ptr<Task> make_qhop_task(ts_plan* p, const void* V2, void* psi, double dt, int nsteps, int M,
                                     bool magnus2, int dtype, int prec, ExecCtx& c);
int qhop_check(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int M, int dtype, int prec);
int split_check(ts_plan* plan, const void* V2, void* psi, double dt, int nsteps, int scheme, int dtype, int prec);

}  // namespace ts
