// Several independent problems of different sizes solved as one (the uneven batch of
// the capacitance extraction, Sec. II and eq. (8) per member).
//
// The members' right-hand sides (one per conductor) become the columns of one block
// whose rows are the largest member's panel count; a member's columns are zero past its
// own panels and stay zero (no product, preconditioner or Krylov update writes there).
// One GMRES runs over all columns, each column freezing on its own tolerance, so a
// restart cycle of the whole set is one captured graph.  Every pass of the product of
// eq. (11) and of the preconditioner of eq. (14) is ONE launch over all members: the
// launch's workgroups are split between the members by a device table of their
// arguments (first workgroup, sizes, plans, array pointers), and a workgroup whose
// column has already converged returns at once.  The x pass groups members by its
// compiled register radix, so it takes one launch per distinct (outputs, radix) pair.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "mvp_kernels.h"
#include "problem.h"
#include "solver.h"

namespace vc {

int pair_odd_bits(int q);

struct PackPass {   // one multi-member launch
  DevMem tab;
  int n = 0, nblk = 0, nthr = 64;
  size_t lds = 0;
  int rs = 0, nout = 0;   // x-pass groups only
};

struct PackPrec {
  bool ok = false;
  PackPass zf, yf, yi, zi;   // yf / yi: members on the LDS-tile y kernel
  std::vector<PackPass> yfr, yir;   // members on the register-edge y kernel, by last radix
  std::vector<PackPass> sand;
};

struct PackData {
  std::vector<vc_problem*> mem;
  std::vector<int> c0;   // first column of each member
  int R = 0;             // columns
  PackPrec p32, p64;
  DevMem dinv, dinv_diag;   // [R][rows] diagonal parts of eq. (14), zero on padding rows
  DevMem box_ptr, box_panels, box_block, block_off, block_n, blocks, box_c0, box_nc;
  int nbox = 0;
  DevMem b;                 // unit-potential right-hand sides [R][rows]
};

static int lg2(int n) {
  int l = 0;
  while ((1 << (l + 1)) <= n) ++l;
  return l;
}

template <typename S>
static vc_status upload_tab(PackPass& pp, const std::vector<S>& v) {
  pp.n = (int)v.size();
  VC_HIP(pp.tab.alloc(std::max<size_t>(v.size(), 1) * sizeof(S)));
  if (!v.empty()) VC_HIP(hipMemcpy(pp.tab.p, v.data(), v.size() * sizeof(S), hipMemcpyHostToDevice));
  return VC_OK;
}

static void grow(PackPass& pp, int nthr, size_t lds) {
  pp.nthr = std::max(pp.nthr, nthr);
  pp.lds = std::max(pp.lds, lds);
}

// The launch tables of one precision: the same tiles and x-pass plans a member's own
// product would use (default plan, no timing), laid out back to back.
template <typename T>
static vc_status build_tables(PackData& D, PackPrec& pp) {
  const int eb = 2 * (int)sizeof(T);
  const size_t budget = kLdsBudget;
  std::vector<ZScene> zf, zi;
  std::vector<StridedScene> yf, yi;
  std::map<std::pair<int, int>, std::vector<SandScene>> sg;   // (outputs, register radix) -> members
  std::map<std::pair<int, int>, PackPass> sgp;
  std::map<int, std::vector<YScene>> ygf, ygi;                 // register radix -> members (y forward / inverse)
  std::map<int, PackPass> ypf, ypi;
  int bzf = 0, bzi = 0, byf = 0, byi = 0;
  for (size_t k = 0; k < D.mem.size(); ++k) {
    vc_problem* P = D.mem[k];
    PrecTables& tb = sizeof(T) == 8 ? P->t64 : P->t32;
    const int m = P->m, c0 = D.c0[k];
    const int n1x = P->n1[0], n1y = P->n1[1];
    const int Mx = P->M[0], My = P->M[1], Mz = P->M[2], H = P->H;
    const int nitems = (int)P->items.size();
    const bool diel = P->n_diel > 0;
    int ncol = 0, nthr = 0;
    // 1. scatter + z transform (two right-hand sides per complex transform)
    ZScene z{};
    z.items = P->d_items.as<int32_t>();
    z.line_ptr = P->d_line_ptr.as<int32_t>();
    z.pk = P->d_pk.as<int32_t>();
    z.pkind = P->d_pkind.as<int8_t>();
    z.diag = P->d_diag.as<double>();
    z.lflag = P->d_lflag.as<uint8_t>();
    z.tw = tb.ax[2].tw.p;
    z.ph = tb.ax[2].ph.p;   // the z-normal components' half-voxel shift
    z.pl = tb.ax[2].plan;
    z.comp_stride = P->comp_stride;
    z.rhs_stride = P->rhs_stride;
    z.nitems = nitems;
    z.nrhs = m;
    z.n1x = n1x; z.n1y = n1y; z.My = My; z.H = H;
    z.c0 = c0;
    if (nitems > 0) {
      if (!pick_tile(Mz, eb, Tune<T>::emax, nitems, &ncol, &nthr, budget, (m + 1) / 2)) return VC_ERR_ARG;
      ZScene f = z;
      f.F = P->work_F.p;
      f.lgc = lg2(ncol);
      f.gx = (nitems + ncol - 1) / ncol;
      f.blk0 = bzf;
      bzf += f.gx * ((m + 1) / 2);
      zf.push_back(f);
      grow(pp.zf, nthr, zs_lds_bytes((int)sizeof(T), Mz, ncol));
    }
    // 2. y transform of the three input components
    StridedScene y{};
    y.a.comp_stride = P->comp_stride;
    y.a.rhs_stride = P->rhs_stride;
    y.a.plane_stride = (int64_t)My * H;
    y.a.row_stride = H;
    y.a.ncols = H;
    y.a.nrhs = m;
    y.a.n1x = n1x;
    y.a.n1y = n1y;
    y.a.ph = tb.ax[1].ph.p;   // the y-normal components' half-voxel shift
    y.a.phax = 1;
    y.pl = tb.ax[1].plan;
    y.tw = tb.ax[1].tw.p;
    y.lflag = P->d_lflag.as<uint8_t>();
    y.pflag = P->d_pflag.as<uint8_t>();
    y.c0 = c0;
    y.gy = n1x;
    // the register-edge y kernel when its default tile covers at least 32 bytes of a row
    // (the member's own default), else the LDS-tile kernel
    auto yreg = [&](const CompSet& cs, int nin, int nout, int inverse, void* data,
                    std::map<int, std::vector<YScene>>& grp, std::map<int, PackPass>& gp) -> bool {
      YScene ys{};
      YArgs& ya = ys.a;
      ya.comp_stride = P->comp_stride; ya.rhs_stride = P->rhs_stride; ya.plane_stride = (int64_t)My * H;
      ya.row_stride = H; ya.ncols = H; ya.nrhs = m; ya.n1x = n1x; ya.n1y = n1y;
      ya.cs = cs; ya.nin = nin; ya.nout = nout; ya.inverse = inverse;
      ya.ph = tb.ax[1].ph.p;
      ya.phax = 1;
      int ythr = 0;
      size_t lds = 0;
      if (!ypass_config(My, (int)sizeof(T), H, budget, &ya, &ythr) || ya.ncol * eb < 32 ||
          !ypass_args_ok<T>(ya, ythr, true, &lds))
        return false;
      ys.data = data;
      ys.tw = tb.ax[1].tw.p;
      ys.lflag = P->d_lflag.as<uint8_t>();
      ys.pflag = P->d_pflag.as<uint8_t>();
      ys.c0 = c0;
      ys.gx = (H + ya.ncol - 1) / ya.ncol;
      ys.gy = n1x;
      const int rs = (int)((ya.radpack >> (5 * (ya.nst - 1))) & 31u);
      grp[rs].push_back(ys);
      PackPass& g = gp[rs];
      g.rs = rs;
      grow(g, ythr, lds);
      return true;
    };
    {
      StridedScene f = y;
      f.cs.n = 3;
      for (int a = 0; a < 3; ++a) { f.cs.comp[a] = a; f.cs.axis[a] = a; f.cs.min_[a] = 3; f.cs.mout[a] = 0; }
      if (!yreg(f.cs, n1y, My, 0, P->work_F.p, ygf, ypf)) {
        if (!pick_tile(My, eb, Tune<T>::emax, H, &ncol, &nthr, budget, (int64_t)n1x * 3 * m)) return VC_ERR_ARG;
        f.a.ncol = ncol; f.a.lgc = lg2(ncol); f.a.nin = n1y; f.a.nout = My; f.a.inverse = 0;
        f.data = P->work_F.p;
        f.gx = (H + ncol - 1) / ncol;
        f.blk0 = byf;
        byf += f.gx * f.gy * f.cs.n * m;
        yf.push_back(f);
        grow(pp.yf, nthr, zs_lds_bytes((int)sizeof(T), My, ncol));
      }
    }
    // 3. x transform + block multiply + inverse x transform
    {
      SandScene sc{};
      SandArgs& xa = sc.a;
      xa.comp_stride = P->comp_stride;
      xa.rhs_stride = P->rhs_stride;
      xa.pair_stride = (int64_t)P->Hy * H * P->Hx;
      xa.nrhs = m; xa.n1x = n1x; xa.Mx = Mx; xa.My = My; xa.H = H; xa.Hx = P->Hx; xa.Hy = P->Hy;
      for (int q = 0; q < 15; ++q) xa.oddmask |= (uint64_t)pair_odd_bits(q) << (3 * q);
      xa.adjoint = 0;
      xa.nin = 3;
      xa.nout = diel ? 6 : 3;
      SandCfg cfg;
      if (!sandwich_default(Mx, (int)sizeof(T), 3, n1x, budget, &cfg)) {
        set_error("x transform length %d too long for the sandwich kernel", Mx);
        return VC_ERR_ARG;
      }
      xa.nst = cfg.nst; xa.radpack = cfg.radpack; xa.tl = cfg.tl; xa.ncol = cfg.ncol;
      sc.Fin = P->work_F.p;
      sc.Fout = P->work_O.p;
      sc.R = tb.R.p;
      sc.tw = tb.ax[0].tw.p;
      sc.phx = tb.ax[0].ph.p;
      sc.pflag = P->d_pflag.as<uint8_t>();
      sc.c0 = c0;
      sc.ntiles = (My * H + cfg.ncol - 1) / cfg.ncol;
      const int rs = (int)((cfg.radpack >> (5 * (cfg.nst - 1))) & 31u);
      const std::pair<int, int> key(xa.nout, rs);
      sg[key].push_back(sc);
      PackPass& g = sgp[key];
      g.rs = rs;
      g.nout = xa.nout;
      grow(g, cfg.nthr, sandwich_lds_bytes(Mx, cfg.ncol, (int)sizeof(T), n1x));
    }
    // 4. inverse y transform of the outputs
    {
      StridedScene f = y;
      const int no = diel ? 6 : 3;
      f.cs.n = no;
      for (int o = 0; o < no; ++o) { f.cs.comp[o] = o; f.cs.axis[o] = o % 3; f.cs.min_[o] = 0; f.cs.mout[o] = o < 3 ? 1 : 2; }
      if (!yreg(f.cs, My, n1y, 1, P->work_O.p, ygi, ypi)) {
        if (!pick_tile(My, eb, Tune<T>::emax, H, &ncol, &nthr, budget, (int64_t)n1x * no * m)) return VC_ERR_ARG;
        f.a.ncol = ncol; f.a.lgc = lg2(ncol); f.a.nin = My; f.a.nout = n1y; f.a.inverse = 1;
        f.data = P->work_O.p;
        f.gx = (H + ncol - 1) / ncol;
        f.blk0 = byi;
        byi += f.gx * f.gy * no * m;
        yi.push_back(f);
        grow(pp.yi, nthr, zs_lds_bytes((int)sizeof(T), My, ncol));
      }
    }
    // 5. inverse z transform + gather + jump term
    if (nitems > 0) {
      if (!pick_tile(Mz, eb, Tune<T>::emax, nitems, &ncol, &nthr, budget, m)) return VC_ERR_ARG;
      ZScene f = z;
      f.F = P->work_O.p;
      f.lgc = lg2(ncol);
      f.gx = (nitems + ncol - 1) / ncol;
      f.blk0 = bzi;
      bzi += f.gx * m;
      zi.push_back(f);
      grow(pp.zi, nthr, zs_lds_bytes((int)sizeof(T), Mz, ncol));
    }
  }
  pp.zf.nblk = bzf;
  pp.yf.nblk = byf;
  pp.yi.nblk = byi;
  pp.zi.nblk = bzi;
  for (PackPass* q : {&pp.zf, &pp.yf, &pp.yi, &pp.zi})
    if (q->lds > lds_ext_budget() || q->nthr > 1024) { set_error("packed pass exceeds the launch limits"); return VC_ERR_ARG; }
  vc_status s;
  if ((s = upload_tab(pp.zf, zf)) != VC_OK || (s = upload_tab(pp.yf, yf)) != VC_OK ||
      (s = upload_tab(pp.yi, yi)) != VC_OK || (s = upload_tab(pp.zi, zi)) != VC_OK)
    return s;
  // register-edge y groups: workgroups laid out member after member
  for (int dir = 0; dir < 2; ++dir) {
    auto& grp = dir == 0 ? ygf : ygi;
    auto& gp = dir == 0 ? ypf : ypi;
    std::vector<PackPass>& out = dir == 0 ? pp.yfr : pp.yir;
    out.clear();
    for (auto& kv : grp) {
      PackPass g = std::move(gp[kv.first]);
      int blk = 0;
      for (YScene& ys : kv.second) {
        size_t lds = 0;
        if (!ypass_args_ok<T>(ys.a, g.nthr, true, &lds)) {
          set_error("packed y-pass configuration rejected");
          return VC_ERR_ARG;
        }
        ys.blk0 = blk;
        blk += ys.gx * ys.gy * ys.a.cs.n * ys.a.nrhs;
      }
      g.nblk = blk;
      if (g.lds > lds_ext_budget() || g.nthr > 1024) {
        set_error("packed pass exceeds the launch limits");
        return VC_ERR_ARG;
      }
      if ((s = upload_tab(g, kv.second)) != VC_OK) return s;
      out.push_back(std::move(g));
    }
  }
  pp.sand.clear();
  for (auto& kv : sg) {
    PackPass g = std::move(sgp[kv.first]);
    int blk = 0;
    for (SandScene& sc : kv.second) {
      if (!sandwich_args_ok<T>(sc.a, g.nthr)) { set_error("packed x-pass configuration rejected"); return VC_ERR_ARG; }
      sc.blk0 = blk;
      blk += sc.ntiles * sc.a.nrhs;
    }
    g.nblk = blk;
    if ((s = upload_tab(g, kv.second)) != VC_OK) return s;
    pp.sand.push_back(std::move(g));
  }
  pp.ok = true;
  return VC_OK;
}

template <typename T>
static vc_status pack_apply_t(PackPrec& pp, int64_t N, const double* x, double* y, hipStream_t st, const int* skip,
                              const int* act) {
  VC_HIP(launch_zfwd_multi<T>(pp.zf.tab.as<ZScene>(), pp.zf.n, pp.zf.nblk, x, N, skip, act, pp.zf.nthr, pp.zf.lds, st));
  VC_HIP(launch_strided_multi<T>(pp.yf.tab.as<StridedScene>(), pp.yf.n, pp.yf.nblk, skip, act, pp.yf.nthr, pp.yf.lds,
                                 st));
  for (PackPass& g : pp.yfr)
    VC_HIP(launch_ypass_multi<T>(g.tab.as<YScene>(), g.n, g.nblk, g.rs, g.nthr, g.lds, skip, act, st));
  for (PackPass& g : pp.sand) {
    if (g.nout == 6)
      VC_HIP((launch_sandwich_multi_v<T, 3, 6>(g.tab.as<SandScene>(), g.n, g.nblk, skip, act, g.nthr, g.lds, g.rs, st)));
    else
      VC_HIP((launch_sandwich_multi_v<T, 3, 3>(g.tab.as<SandScene>(), g.n, g.nblk, skip, act, g.nthr, g.lds, g.rs, st)));
  }
  VC_HIP(launch_strided_multi<T>(pp.yi.tab.as<StridedScene>(), pp.yi.n, pp.yi.nblk, skip, act, pp.yi.nthr, pp.yi.lds,
                                 st));
  for (PackPass& g : pp.yir)
    VC_HIP(launch_ypass_multi<T>(g.tab.as<YScene>(), g.n, g.nblk, g.rs, g.nthr, g.lds, skip, act, st));
  VC_HIP(launch_zinv_multi<T>(pp.zi.tab.as<ZScene>(), pp.zi.n, pp.zi.nblk, x, y, N, skip, act, pp.zi.nthr, pp.zi.lds,
                              st));
  return VC_OK;
}

vc_status pack_apply(vc_problem* Q, int transpose, vc_precision prec, const double* x, double* y, int nrhs,
                     hipStream_t st, const int* skip, const int* act) {
  PackData& D = *Q->pack;
  if (transpose) { set_error("a packed set has no transposed product"); return VC_ERR_ARG; }
  if (nrhs != D.R) { set_error("a packed product takes all %d columns (got %d)", D.R, nrhs); return VC_ERR_ARG; }
  PackPrec& pp = prec == VC_FP32 ? D.p32 : D.p64;
  if (!pp.ok) {
    set_error("the packed problems lack the %s spectra", prec == VC_FP32 ? "FP32" : "FP64");
    return VC_ERR_STATE;
  }
  Q->mvp_count++;
  return prec == VC_FP32 ? pack_apply_t<float>(pp, Q->pack_rows, x, y, st, skip, act)
                         : pack_apply_t<double>(pp, Q->pack_rows, x, y, st, skip, act);
}

vc_status pack_precond(vc_problem* Q, const double* x, double* y, int nrhs, hipStream_t st, const int* skip) {
  PackData& D = *Q->pack;
  const int64_t N = Q->pack_rows;
  if (Q->pc.mode == 3) { set_error("packed sets use the block-diagonal-diagonal or diagonal preconditioner"); return VC_ERR_ARG; }
  if (Q->pc.mode == 2) {
    VC_HIP(launch_diag_scale(x, y, D.dinv_diag.as<double>(), N, nrhs, skip, st, N));
    return VC_OK;
  }
  VC_HIP(launch_diag_scale(x, y, D.dinv.as<double>(), N, nrhs, skip, st, N));
  VC_HIP(launch_block_apply(x, y, N, nrhs, D.box_ptr.as<int32_t>(), D.box_panels.as<int32_t>(),
                            D.box_block.as<int32_t>(), D.block_off.as<int64_t>(), D.block_n.as<int32_t>(),
                            D.blocks.as<double>(), D.nbox, skip, st, D.box_c0.as<int32_t>(), D.box_nc.as<int32_t>()));
  return VC_OK;
}

template <typename T>
static vc_status upload_vec(DevMem& d, const std::vector<T>& h) {
  VC_HIP(d.alloc(std::max<size_t>(h.size(), 1) * sizeof(T)));
  if (!h.empty()) VC_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return VC_OK;
}

vc_status pack_create(vc_problem* const* probs, int n, vc_problem** out) {
  if (!probs || n <= 0 || !out) { set_error("bad packed-set arguments"); return VC_ERR_ARG; }
  auto D = std::make_shared<PackData>();
  int64_t N = 0;
  int R = 0, dev = -1;
  bool all32 = true, all64 = true;
  for (int k = 0; k < n; ++k) {
    vc_problem* P = probs[k];
    if (!P || !P->setup_done || P->hip_failed || P->pack) {
      set_error("member %d: not a problem after vc_setup", k);
      return VC_ERR_STATE;
    }
    if (!P->tk.empty()) { set_error("member %d: packed sets need uncompressed spectra", k); return VC_ERR_ARG; }
    if (P->m < 1 || P->m > P->max_rhs) { set_error("member %d: setup max_rhs below its conductor count", k); return VC_ERR_STATE; }
    if (dev >= 0 && P->device != dev) { set_error("members on different devices"); return VC_ERR_ARG; }
    if (!P->pc.built) { set_error("member %d: preconditioner not built", k); return VC_ERR_STATE; }
    dev = P->device;
    D->mem.push_back(P);
    D->c0.push_back(R);
    R += P->m;
    N = std::max(N, npanels(P));
    all32 = all32 && P->have32;
    all64 = all64 && P->have64;
  }
  if (R > 256) { set_error("a packed set holds at most 256 conductors (got %d)", R); return VC_ERR_ARG; }
  D->R = R;
  VC_HIP(hipSetDevice(dev));
  std::unique_ptr<vc_problem> Q(new vc_problem);
  Q->device = dev;
  Q->m = R;
  Q->max_rhs = R;
  Q->pack_rows = N;
  Q->have32 = all32;
  Q->have64 = all64;
  vc_status s;
  if (all64 && (s = build_tables<double>(*D, D->p64)) != VC_OK) return s;
  if (all32 && (s = build_tables<float>(*D, D->p32)) != VC_OK) return s;
  // eq. (14): per-column diagonals and the members' boxes, each box tagged with its columns
  VC_HIP(D->dinv.alloc((size_t)R * N * sizeof(double)));
  VC_HIP(D->dinv_diag.alloc((size_t)R * N * sizeof(double)));
  VC_HIP(hipMemset(D->dinv.p, 0, D->dinv.bytes));
  VC_HIP(hipMemset(D->dinv_diag.p, 0, D->dinv_diag.bytes));
  std::vector<int32_t> bp(1, 0), bpan, bblk, bn, bc0, bnc;
  std::vector<int64_t> boff;
  std::vector<double> blocks;
  std::vector<double> B((size_t)R * N, 0.0);
  for (size_t k = 0; k < D->mem.size(); ++k) {
    vc_problem* P = D->mem[k];
    const Precond& pc = P->pc;
    const int64_t Nk = npanels(P);
    const int c0 = D->c0[k];
    for (int j = 0; j < P->m; ++j) {
      VC_HIP(hipMemcpy(D->dinv.as<double>() + (size_t)(c0 + j) * N, pc.dinv.p, Nk * sizeof(double),
                       hipMemcpyDeviceToDevice));
      VC_HIP(hipMemcpy(D->dinv_diag.as<double>() + (size_t)(c0 + j) * N, pc.dinv_diag.p, Nk * sizeof(double),
                       hipMemcpyDeviceToDevice));
    }
    const int blk_base = (int)bn.size();
    const int64_t dbl_base = (int64_t)blocks.size();
    for (int b = 0; b < pc.nbox; ++b) {
      const int p0 = pc.h_box_ptr[b], p1 = pc.h_box_ptr[b + 1];
      bpan.insert(bpan.end(), pc.h_box_panels.begin() + p0, pc.h_box_panels.begin() + p1);
      bp.push_back((int32_t)bpan.size());
      bblk.push_back(pc.h_box_block[b] + blk_base);
      bc0.push_back(c0);
      bnc.push_back(P->m);
    }
    for (size_t q = 0; q < pc.h_block_n.size(); ++q) {
      bn.push_back(pc.h_block_n[q]);
      boff.push_back(pc.h_block_off[q] + dbl_base);
    }
    blocks.insert(blocks.end(), pc.h_blocks.begin(), pc.h_blocks.end());
    for (int64_t i = 0; i < Nk; ++i)
      if (P->panels[i].kind == 0) B[(size_t)(c0 + P->panels[i].cond) * N + i] = 1.0;
  }
  D->nbox = (int)bblk.size();
  if ((s = upload_vec(D->box_ptr, bp)) != VC_OK || (s = upload_vec(D->box_panels, bpan)) != VC_OK ||
      (s = upload_vec(D->box_block, bblk)) != VC_OK || (s = upload_vec(D->block_off, boff)) != VC_OK ||
      (s = upload_vec(D->block_n, bn)) != VC_OK || (s = upload_vec(D->blocks, blocks)) != VC_OK ||
      (s = upload_vec(D->box_c0, bc0)) != VC_OK || (s = upload_vec(D->box_nc, bnc)) != VC_OK ||
      (s = upload_vec(D->b, B)) != VC_OK)
    return s;
  Q->pc.built = 1;
  Q->pack = D;
  Q->setup_done = true;
  *out = Q.release();
  return VC_OK;
}

double pack_product_bytes(vc_problem* Q, int elem) {
  double b = 0.0;
  if (Q && Q->pack)
    for (vc_problem* P : Q->pack->mem) b += product_bytes_model(P, elem, P->m);
  return b;
}

vc_status pack_capacitance(vc_problem* Q, const vc_solve_opts* opts, double* const* C_out, vc_stats* stats) {
  if (!Q || !Q->pack) { set_error("not a packed set"); return VC_ERR_ARG; }
  PackData& D = *Q->pack;
  if (!C_out) { set_error("null C_out"); return VC_ERR_ARG; }
  vc_solve_opts o = fill_defaults(opts);
  if ((o.prec == VC_FP32 || o.prec == VC_MIXED) && !Q->have32) { set_error("FP32 spectra not built"); return VC_ERR_STATE; }
  if (o.prec != VC_FP32 && !Q->have64) { set_error("FP64 spectra not built"); return VC_ERR_STATE; }
  VC_HIP(hipSetDevice(Q->device));
  const double t0 = now_s();
  hipStream_t st = get_solve_stream(Q);
  if (!st) { set_error("could not create the solve stream"); return VC_ERR_HIP; }
  const int R = D.R;
  const int64_t N = Q->pack_rows;
  Q->mvp_count = 0;
  vc_status s = ensure_workspace(Q, R, o.restart);
  if (s != VC_OK) return s;
  std::vector<int> it;
  std::vector<double> rre;
  vc_stats all{};
  s = solve(Q, o, 0, D.b.as<double>(), Q->ws.x, R, &all, st, &it, &rre);
  if (s != VC_OK && s != VC_ERR_NOT_CONVERGED) return s;
  // eq. (8) per member, from its columns of the packed solution
  std::vector<int64_t> coff(D.mem.size() + 1, 0);
  for (size_t k = 0; k < D.mem.size(); ++k) coff[k + 1] = coff[k] + (int64_t)D.mem[k]->m * D.mem[k]->m;
  DevMem dC;
  VC_HIP(dC.alloc((size_t)coff.back() * sizeof(double)));
  for (size_t k = 0; k < D.mem.size(); ++k) {
    vc_problem* P = D.mem[k];
    VC_HIP(launch_cap_reduce_n(Q->ws.x + (size_t)D.c0[k] * N, N, P->m, P->m,
                               P->d_cond_panels.as<int32_t>(), P->d_cond_ptr.as<int32_t>(), P->d_weight.as<double>(),
                               4.0 * M_PI * kEps0 * P->dv, dC.as<double>() + coff[k], st));
  }
  std::vector<double> hC((size_t)coff.back());
  VC_HIP(hipMemcpyAsync(hC.data(), dC.p, hC.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  VC_HIP(hipStreamSynchronize(st));
  const double t_solve = now_s() - t0;
  for (size_t k = 0; k < D.mem.size(); ++k) {
    vc_problem* P = D.mem[k];
    if (C_out[k]) std::memcpy(C_out[k], hC.data() + coff[k], (size_t)P->m * P->m * sizeof(double));
    if (stats) {
      vc_stats& sk = stats[k];
      std::memset(&sk, 0, sizeof(vc_stats));
      for (int j = 0; j < P->m && j < 64; ++j) {
        sk.iters[j] = D.c0[k] + j < (int)it.size() ? it[D.c0[k] + j] : 0;
        sk.final_rre[j] = D.c0[k] + j < (int)rre.size() ? rre[D.c0[k] + j] : 0.0;
      }
      sk.ir_steps = all.ir_steps;
      sk.mixed_form = all.mixed_form;
      sk.steps_fp32 = all.steps_fp32;
      sk.mvp_count = Q->mvp_count;
      sk.t_setup_s = P->t_setup;
      sk.t_solve_s = t_solve;
      sk.spectra_bytes = P->spectra_bytes;
    }
  }
  return s;
}

// kernel launches of one packed product: the z passes, the y passes (LDS-tile launch if
// any member uses it, one register-edge launch per last radix) and the x-pass groups
static int32_t pack_launches(const PackPrec& pp) {
  if (!pp.ok) return 0;
  return (pp.zf.n > 0) + (pp.zi.n > 0) + (pp.yf.n > 0) + (pp.yi.n > 0) + (int32_t)pp.yfr.size() +
         (int32_t)pp.yir.size() + (int32_t)pp.sand.size();
}

void pack_info(const vc_problem* Q, int32_t out[6]) {
  const PackData& D = *Q->pack;
  out[0] = (int32_t)D.mem.size();
  out[1] = D.R;
  out[2] = (int32_t)Q->pack_rows;
  out[3] = pack_launches(D.p64);
  out[4] = pack_launches(D.p32);
  out[5] = 2;
}

}  // namespace vc
