// Internal interface of the GMRES driver (solver.cpp) shared by the C ABI (api.cpp)
// and the packed multi-problem solve (pack.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "problem.h"

namespace vc {

constexpr double kEps0 = 8.8541878128e-12;   // F/m (CODATA 2018)

struct SolveSpec {
  vc_precision mvp;     // VC_FP64 or VC_FP32 product
  int transpose;
  int precond;          // 0 none, 1 block-diagonal-diagonal, 2 diagonal
  double rtol;
  int restart, max_iter;
  // relaxed mixed form: the product precision is chosen per segment of Arnoldi steps
  // (FP32 once every iterating column's residual estimate is <= relax_thr); cycle
  // starts (residuals) and updates use mvp, which is then VC_FP64
  int relax = 0;
  double relax_thr = 0.0;
};

// views of the cycle state for one (nrhs, restart) solve
struct Cyc {
  double *H, *cs, *sn, *g, *bn, *rn, *rre, *scal, *rtol;
  int *kd, *iters, *act_cycle, *act_step, *skip, *bad;
};

double now_s();
vc_status ensure_workspace(vc_problem* P, int nrhs, int restart);
Cyc cycle_views(vc_problem* P, int nrhs, int m);
vc_status op_with_precond(vc_problem* P, const SolveSpec& sp, const double* v, double* z, double* w, int nrhs,
                          hipStream_t st, const int* skip = nullptr, const int* act = nullptr);
vc_status residual(vc_problem* P, const SolveSpec& sp, const double* b, const double* x, double* r, int nrhs,
                   hipStream_t st, const int* skip = nullptr);
vc_status col_norms(vc_problem* P, const double* w, int64_t N, int nrhs, double* d_out, std::vector<double>& h,
                    hipStream_t st);
vc_status issue_cycle(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs, hipStream_t st,
                      int part);
vc_status cycle_graph(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs, hipStream_t st,
                      int part, hipGraph_t* g_out, hipGraphExec_t* e_out);
vc_status gmres(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs, std::vector<int>& iters,
                std::vector<double>& rre, hipStream_t st, int* steps32 = nullptr, bool x_zero = false);
hipStream_t get_solve_stream(vc_problem* P);
vc_status solve(vc_problem* P, const vc_solve_opts& o, int transpose, const double* b, double* x, int nrhs,
                vc_stats* stats, hipStream_t st, std::vector<int>* it_out = nullptr,
                std::vector<double>* rre_out = nullptr);
vc_solve_opts fill_defaults(const vc_solve_opts* in);
// vc_capacitance in two parts (api.cpp): argument checks and defaults; then, with the
// workspace regions in place (P->ws) and st the stream, the solve, the reduction of
// eq. (8) and the copies of C (and rho) out
vc_status capacitance_check(vc_problem* p, const vc_solve_opts* opts, const double* C, vc_solve_opts* o);
vc_status capacitance_run(vc_problem* p, const vc_solve_opts& o, double* C, double* rho_dev, vc_stats* stats,
                          hipStream_t st, std::vector<double>* rho_host, double t0);
// packed sets (pack.cpp): members must outlive the combined problem
vc_status pack_create(vc_problem* const* problems, int n, vc_problem** out);
vc_status pack_capacitance(vc_problem* q, const vc_solve_opts* opts, double* const* C_out, vc_stats* stats);
void pack_info(const vc_problem* q, int32_t out[6]);

}  // namespace vc
