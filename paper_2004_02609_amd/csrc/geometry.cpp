// Panel extraction (Sec. II.A, eq. 3) and the index maps used by the FFT product.
//
// A face of the voxel grid is a conductor panel when exactly one of its two voxels is a
// conductor and a dielectric panel when neither is and their permittivities differ;
// outside the box is the background medium.  Faces are visited in (axis, i, j, k)
// order, which is the library's panel order, so the panels of every (axis, i, j) line
// along z are contiguous.
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "mvp_kernels.h"
#include "problem.h"

namespace vc {

bool smooth7(int n) {
  if (n <= 0) return false;
  for (int f : {2, 3, 5, 7})
    while (n % f == 0) n /= f;
  return n == 1;
}

// Radix schedule of one FFT length: the fewest stages from the radices the engine
// implements (composite ones run as Cooley-Tukey in registers), ties broken towards
// balanced radices; max_radix bounds per-thread registers.
static void plan_search(int n, int max_radix, int depth, int* cur, int* best, int* best_n, double* best_score) {
  static const int kRad[] = {27, 25, 21, 20, 18, 16, 15, 14, 12, 10, 9, 8, 7, 6, 5, 4, 3, 2};
  if (n == 1) {
    double score = 0.0;   // prefer fewer stages, then a larger smallest radix
    int mn = 1 << 30;
    for (int i = 0; i < depth; ++i) mn = cur[i] < mn ? cur[i] : mn;
    score = -1000.0 * depth + mn;
    if (score > *best_score) {
      *best_score = score;
      *best_n = depth;
      for (int i = 0; i < depth; ++i) best[i] = cur[i];
    }
    return;
  }
  if (depth >= kMaxStages || depth >= 6) return;
  for (int r : kRad) {
    if (r > max_radix || n % r) continue;
    if (depth > 0 && r > cur[depth - 1]) continue;   // non-increasing order: one visit per multiset
    cur[depth] = r;
    plan_search(n / r, max_radix, depth + 1, cur, best, best_n, best_score);
  }
}

AxisPlan make_plan(int L, int max_radix) {
  AxisPlan pl{};
  pl.L = L;
  int cur[kMaxStages], best[kMaxStages];
  int nbest = -1;
  double score = -1e30;
  plan_search(L, max_radix, 0, cur, best, &nbest, &score);
  pl.nst = nbest;
  for (int i = 0; i < nbest; ++i) pl.rad[i] = best[i];
  return pl;
}

// Sandwich plan: radices in non-increasing order, the last one (the register stage)
// at most rs_max and leaving at most max_tl butterflies per column; fewest stages,
// then the largest register radix (fewest threads per column).
static void sand_search(int n, int rmax, int rmid, int rs_max, int max_tl, int L, int depth, int* cur, int* best,
                        int* best_n, double* best_score) {
  static const int kRad[] = {27, 25, 21, 20, 18, 16, 15, 14, 12, 10, 9, 8, 7, 6, 5, 4, 3, 2};
  if (n == 1) {
    const int rs = cur[depth - 1];
    if (rs > rs_max || L / rs > max_tl) return;
    for (int s = 1; s + 1 < depth; ++s)
      if (cur[s] > rmid) return;
    const double score = -1000.0 * depth + 10.0 * rs;
    if (score > *best_score) {
      *best_score = score;
      *best_n = depth;
      for (int i = 0; i < depth; ++i) best[i] = cur[i];
    }
    return;
  }
  if (depth >= kSandMaxStages) return;
  for (int r : kRad) {
    if (r > rmax || n % r) continue;
    if (depth > 0 && r > cur[depth - 1]) continue;
    cur[depth] = r;
    sand_search(n / r, rmax, rmid, rs_max, max_tl, L, depth + 1, cur, best, best_n, best_score);
  }
}

AxisPlan make_sandwich_plan(int L, int rmax, int rmid, int rs_max, int max_tl) {
  AxisPlan pl{};
  pl.L = L;
  int cur[kMaxStages], best[kMaxStages];
  int nbest = -1;
  double score = -1e30;
  if (L >= 2) sand_search(L, rmax, rmid, rs_max, max_tl, L, 0, cur, best, &nbest, &score);
  pl.nst = nbest;
  for (int i = 0; i < nbest; ++i) pl.rad[i] = best[i];
  return pl;
}

vc_status panelize(vc_problem* P) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const int n[3] = {nx, ny, nz};
  auto vid = [&](int i, int j, int k) -> int64_t { return ((int64_t)i * ny + j) * nz + k; };
  // validation
  int32_t maxid = -1;
  for (size_t v = 0; v < P->cond_id.size(); ++v) {
    const int32_t c = P->cond_id[v];
    if (c < -1) { set_error("cond_id %d < -1 at voxel %zu", c, v); return VC_ERR_GEOMETRY; }
    if (c > maxid) maxid = c;
    if (c == -1 && !(P->eps_r[v] > 0.0 && std::isfinite(P->eps_r[v]))) {
      set_error("eps_r must be > 0 at voxel %zu", v);
      return VC_ERR_GEOMETRY;
    }
  }
  if (maxid < 0) { set_error("no conductor voxel"); return VC_ERR_GEOMETRY; }
  if (!(P->eps_b > 0.0)) { set_error("eps_background must be > 0"); return VC_ERR_GEOMETRY; }
  std::vector<char> used(maxid + 1, 0);
  for (int32_t c : P->cond_id)
    if (c >= 0) used[c] = 1;
  for (int c = 0; c <= maxid; ++c)
    if (!used[c]) { set_error("conductor ids must be dense: id %d unused", c); return VC_ERR_GEOMETRY; }
  P->m = maxid + 1;
  P->panels.clear();
  for (int a = 0; a < 3; ++a) {
    const int lim[3] = {nx + (a == 0), ny + (a == 1), nz + (a == 2)};
    for (int i = 0; i < lim[0]; ++i)
      for (int j = 0; j < lim[1]; ++j)
        for (int k = 0; k < lim[2]; ++k) {
          int idx[3] = {i, j, k};
          int lo[3] = {i, j, k};
          lo[a] -= 1;
          const bool lo_in = idx[a] >= 1;
          const bool hi_in = idx[a] < n[a];
          const int32_t clo = lo_in ? P->cond_id[vid(lo[0], lo[1], lo[2])] : -1;
          const int32_t chi = hi_in ? P->cond_id[vid(i, j, k)] : -1;
          const double elo = lo_in ? P->eps_r[vid(lo[0], lo[1], lo[2])] : P->eps_b;
          const double ehi = hi_in ? P->eps_r[vid(i, j, k)] : P->eps_b;
          vc_panel pn{};
          pn.i = i; pn.j = j; pn.k = k; pn.dir = (int8_t)a;
          if (clo >= 0 && chi >= 0) {
            if (clo != chi) {
              set_error("conductors %d and %d share the face (%d,%d,%d) normal %d", clo, chi, i, j, k, a);
              return VC_ERR_GEOMETRY;
            }
            continue;
          }
          if (clo >= 0 || chi >= 0) {
            pn.kind = 0;
            pn.cond = clo >= 0 ? clo : chi;
            pn.eps_lo = clo >= 0 ? 0.0 : elo;
            pn.eps_hi = chi >= 0 ? 0.0 : ehi;
            pn.eps_adj = clo >= 0 ? ehi : elo;
            P->panels.push_back(pn);
          } else if (elo != ehi) {
            pn.kind = 1;
            pn.cond = -1;
            pn.eps_lo = elo;
            pn.eps_hi = ehi;
            pn.eps_adj = 0.0;
            P->panels.push_back(pn);
          }
        }
  }
  const int64_t N = (int64_t)P->panels.size();
  if (N >= (int64_t)1 << 31) { set_error("too many panels"); return VC_ERR_ARG; }
  P->n_cond = P->n_diel = 0;
  for (auto& pn : P->panels) (pn.kind == 0 ? P->n_cond : P->n_diel)++;
  // index maps
  const int n1x = nx + 1, n1y = ny + 1;
  P->n1[0] = n1x; P->n1[1] = n1y; P->n1[2] = nz + 1;
  const int64_t nlines = 3LL * n1x * n1y;
  P->line_ptr.assign(nlines + 1, 0);
  P->lflag.assign(nlines, 0);
  P->pflag.assign(3 * n1x, 0);
  P->pk.resize(N);
  P->pkind.resize(N);
  P->diag.resize(N);
  P->weight.assign(N, 0.0);
  for (int64_t p = 0; p < N; ++p) {
    const vc_panel& pn = P->panels[p];
    const int64_t line = ((int64_t)pn.dir * n1x + pn.i) * n1y + pn.j;
    P->line_ptr[line + 1]++;
    P->lflag[line] |= (pn.kind == 0) ? 1 : 2;
    P->pflag[pn.dir * n1x + pn.i] |= (pn.kind == 0) ? 1 : 2;
    P->pk[p] = pn.k;
    P->pkind[p] = pn.kind;
    P->diag[p] = pn.kind == 1 ? 2.0 * M_PI * (pn.eps_lo + pn.eps_hi) / (pn.eps_lo - pn.eps_hi) : 0.0;
    if (pn.kind == 0) P->weight[p] = pn.eps_adj;
  }
  for (int64_t l = 0; l < nlines; ++l) P->line_ptr[l + 1] += P->line_ptr[l];
  P->items.clear();
  for (int64_t l = 0; l < nlines; ++l)
    if (P->line_ptr[l + 1] > P->line_ptr[l]) P->items.push_back((int32_t)l);
  // conductor panels grouped by id
  P->cond_ptr.assign(P->m + 1, 0);
  for (auto& pn : P->panels)
    if (pn.kind == 0) P->cond_ptr[pn.cond + 1]++;
  for (int c = 0; c < P->m; ++c) P->cond_ptr[c + 1] += P->cond_ptr[c];
  P->cond_panels.assign(P->n_cond, 0);
  std::vector<int32_t> fill(P->cond_ptr.begin(), P->cond_ptr.end() - 1);
  for (int64_t p = 0; p < N; ++p)
    if (P->panels[p].kind == 0) P->cond_panels[fill[P->panels[p].cond]++] = (int32_t)p;
  return VC_OK;
}

vc_status choose_sizes(vc_problem* P, const int32_t* fft) {
  const int n[3] = {P->nx, P->ny, P->nz};
  for (int a = 0; a < 3; ++a) {
    const int need = 2 * n[a] + 1;
    int M = fft ? fft[a] : 0;
    if (M == 0) {
      M = need + (need & 1);
      while (!smooth7(M)) M += 2;
    } else if (M < need || (M & 1) || !smooth7(M)) {
      set_error("fft_size[%d] = %d must be even, 7-smooth and >= %d", a, M, need);
      return VC_ERR_ARG;
    }
    P->M[a] = M;
  }
  P->H = P->M[2] / 2 + 1;
  P->Hx = P->M[0] / 2 + 1;
  P->Hy = P->M[1] / 2 + 1;
  return VC_OK;
}

}  // namespace vc
