// Persistent cache of the x- and y-pass autotuners: the timed choices for one problem
// shape are written to a text file and read back by later problems of the same shape on
// the same GPU architecture, so they skip the timing (and compute bitwise the same
// products: the choices decide the kernels' arithmetic order).  One line per choice:
//   vc-xpass 1 <arch> <elem bytes> <transpose> <nrhs> <Mx> <My> <H> <n1x> <nin> <nout>
//            <nst> <r0> .. <r5> <cols> <ms>
//   vc-ypass 1 <arch> <elem bytes> <transpose> <inverse> <nrhs> <My> <H> <n1x> <n1y>
//            <dielectrics> <kernel> <cols> <xcd group> <lds ms> <register ms>
// The shape fields are everything the candidates and their timing depend on.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "mvp_kernels.h"
#include "problem.h"

using namespace vc;

namespace {

struct Entry {
  std::string arch;
  int elem = 0, transpose = 0, nrhs = 0, Mx = 0, My = 0, H = 0, n1x = 0, nin = 0, nout = 0;
  int nst = 0, rad[6] = {0, 0, 0, 0, 0, 0}, cols = 0;
  double ms = 0.0;
  bool same_key(const Entry& o) const {
    return arch == o.arch && elem == o.elem && transpose == o.transpose && nrhs == o.nrhs && Mx == o.Mx &&
           My == o.My && H == o.H && n1x == o.n1x && nin == o.nin && nout == o.nout;
  }
};

bool parse(const std::string& line, Entry* e) {
  std::istringstream is(line);
  std::string tag;
  int ver = 0;
  if (!(is >> tag >> ver) || tag != "vc-xpass" || ver != 1) return false;
  if (!(is >> e->arch >> e->elem >> e->transpose >> e->nrhs >> e->Mx >> e->My >> e->H >> e->n1x >> e->nin >>
        e->nout >> e->nst))
    return false;
  for (int s = 0; s < 6; ++s)
    if (!(is >> e->rad[s])) return false;
  return static_cast<bool>(is >> e->cols >> e->ms);
}

std::string format(const Entry& e) {
  char buf[512];
  std::snprintf(buf, sizeof buf, "vc-xpass 1 %s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %.6f",
                e.arch.c_str(), e.elem, e.transpose, e.nrhs, e.Mx, e.My, e.H, e.n1x, e.nin, e.nout, e.nst, e.rad[0],
                e.rad[1], e.rad[2], e.rad[3], e.rad[4], e.rad[5], e.cols, e.ms);
  return buf;
}

// one y-pass choice (key of vc_problem::y_choice: nrhs << 3 | transpose << 2 | inverse << 1 | fp64)
struct YEntry {
  std::string arch;
  int elem = 0, transpose = 0, inverse = 0, nrhs = 0, My = 0, H = 0, n1x = 0, n1y = 0, diel = 0;
  int impl = 0, cols = 0, xg = 1;
  double ms0 = 0.0, ms1 = 0.0;
  bool same_key(const YEntry& o) const {
    return arch == o.arch && elem == o.elem && transpose == o.transpose && inverse == o.inverse && nrhs == o.nrhs &&
           My == o.My && H == o.H && n1x == o.n1x && n1y == o.n1y && diel == o.diel;
  }
};

bool parse_y(const std::string& line, YEntry* e) {
  std::istringstream is(line);
  std::string tag;
  int ver = 0;
  if (!(is >> tag >> ver) || tag != "vc-ypass" || ver != 1) return false;
  return static_cast<bool>(is >> e->arch >> e->elem >> e->transpose >> e->inverse >> e->nrhs >> e->My >> e->H >>
                           e->n1x >> e->n1y >> e->diel >> e->impl >> e->cols >> e->xg >> e->ms0 >> e->ms1);
}

std::string format_y(const YEntry& e) {
  char buf[512];
  std::snprintf(buf, sizeof buf, "vc-ypass 1 %s %d %d %d %d %d %d %d %d %d %d %d %d %.6f %.6f", e.arch.c_str(),
                e.elem, e.transpose, e.inverse, e.nrhs, e.My, e.H, e.n1x, e.n1y, e.diel, e.impl, e.cols, e.xg, e.ms0,
                e.ms1);
  return buf;
}

YEntry yshape_of(const vc_problem* p, const std::string& arch, int key) {
  YEntry e;
  e.arch = arch;
  e.elem = (key & 1) ? 8 : 4;
  e.inverse = (key >> 1) & 1;
  e.transpose = (key >> 2) & 1;
  e.nrhs = key >> 3;
  e.My = p->M[1];
  e.H = p->H;
  e.n1x = p->n1[0];
  e.n1y = p->n1[1];
  e.diel = p->n_diel > 0 ? 1 : 0;
  return e;
}

bool arch_of(int device, std::string* out) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return false;
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');   // drop feature suffixes
  *out = c == std::string::npos ? a : a.substr(0, c);
  return !out->empty();
}

// the shape part of a cache key for one sand_choice key of this problem
Entry shape_of(const vc_problem* p, const std::string& arch, int key) {
  Entry e;
  e.arch = arch;
  e.elem = (key & 1) ? 8 : 4;
  e.transpose = (key >> 1) & 1;
  e.nrhs = key >> 2;
  e.Mx = p->M[0];
  e.My = p->M[1];
  e.H = p->H;
  e.n1x = p->n1[0];
  const bool diel = p->n_diel > 0;
  e.nin = (e.transpose && diel) ? 6 : 3;
  e.nout = e.transpose ? 3 : (diel ? 6 : 3);
  return e;
}

}  // namespace

extern "C" {

vc_status vc_tuning_save(vc_problem* p, const char* path, int32_t* n_saved) {
  if (!p || !path) { set_error("null argument"); return VC_ERR_ARG; }
  if (!p->setup_done) { set_error("vc_setup first"); return VC_ERR_STATE; }
  std::string arch;
  if (!arch_of(p->device, &arch)) { set_error("could not query the device architecture"); return VC_ERR_HIP; }
  std::vector<Entry> mine;
  for (const auto& kv : p->sand_choice) {
    const auto& c = kv.second;
    if (!c.tuned) continue;   // only timed choices are worth keeping
    Entry e = shape_of(p, arch, kv.first);
    e.nst = c.nst;
    for (int s = 0; s < c.nst && s < 6; ++s) e.rad[s] = (int)((c.radpack >> (5 * s)) & 31u);
    e.cols = c.stage ? -c.ncol : c.ncol;   // negative: the staged form
    e.ms = c.ms_best;
    mine.push_back(e);
  }
  std::vector<YEntry> ymine;
  for (const auto& kv : p->y_choice) {
    const auto& c = kv.second;
    if (!c.tuned) continue;
    YEntry e = yshape_of(p, arch, kv.first);
    e.impl = c.impl;
    e.cols = c.ncol;
    e.xg = c.xg;
    e.ms0 = c.ms[0];
    e.ms1 = c.ms[1];
    ymine.push_back(e);
  }
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
      Entry e;
      YEntry ye;
      bool replaced = false;
      if (parse(line, &e)) {
        for (const Entry& m : mine) replaced = replaced || m.same_key(e);
      } else if (parse_y(line, &ye)) {
        for (const YEntry& m : ymine) replaced = replaced || m.same_key(ye);
      } else {
        continue;   // unreadable lines are dropped
      }
      if (!replaced) keep.push_back(line);
    }
  }
  for (const Entry& m : mine) keep.push_back(format(m));
  for (const YEntry& m : ymine) keep.push_back(format_y(m));
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) { set_error("cannot write %s", tmp.c_str()); return VC_ERR_ARG; }
    for (const std::string& l : keep) out << l << "\n";
    if (!out) { set_error("write to %s failed", tmp.c_str()); return VC_ERR_ARG; }
  }
  if (std::rename(tmp.c_str(), path) != 0) { set_error("cannot replace %s", path); return VC_ERR_ARG; }
  if (n_saved) *n_saved = (int32_t)(mine.size() + ymine.size());
  return VC_OK;
}

vc_status vc_tuning_load(vc_problem* p, const char* path, int32_t* n_loaded) {
  if (!p || !path) { set_error("null argument"); return VC_ERR_ARG; }
  if (!p->setup_done) { set_error("vc_setup first"); return VC_ERR_STATE; }
  if (n_loaded) *n_loaded = 0;
  std::ifstream in(path);
  if (!in) return VC_OK;   // no cache yet
  std::string arch;
  if (!arch_of(p->device, &arch)) { set_error("could not query the device architecture"); return VC_ERR_HIP; }
  int32_t count = 0;
  std::string line;
  while (std::getline(in, line)) {
    YEntry ye;
    if (parse_y(line, &ye)) {
      if (ye.nrhs <= 0 || ye.nrhs > p->max_rhs || (ye.elem != 4 && ye.elem != 8) || (ye.transpose != 0 && ye.transpose != 1) ||
          (ye.inverse != 0 && ye.inverse != 1) || (ye.impl != 0 && ye.impl != 1) || ye.cols < 0 || ye.cols > 32 ||
          (ye.cols & (ye.cols - 1)) || !(ye.xg == 1 || ye.xg == 2 || ye.xg == 4 || ye.xg == -1))
        continue;
      if (ye.transpose && p->n_diel == 0) continue;
      const int ykey = (ye.nrhs << 3) | (ye.transpose << 2) | (ye.inverse << 1) | (ye.elem == 8 ? 1 : 0);
      if (!yshape_of(p, arch, ykey).same_key(ye)) continue;
      vc_problem::YChoice ch{ye.impl, false, {ye.ms0, ye.ms1}, ye.cols, ye.xg};
      ch.from_file = true;
      p->y_choice[ykey] = ch;
      ++count;
      continue;
    }
    Entry e;
    if (!parse(line, &e)) continue;
    if (e.nrhs <= 0 || e.nrhs > p->max_rhs || (e.elem != 4 && e.elem != 8) || (e.transpose != 0 && e.transpose != 1))
      continue;
    if (e.transpose && p->n_diel == 0) continue;   // the symmetric operator has no transposed pass
    const int key = (e.nrhs << 2) | (e.transpose << 1) | (e.elem == 8 ? 1 : 0);
    if (!shape_of(p, arch, key).same_key(e)) continue;
    // accept it only as one of this problem's own candidates
    const std::vector<SandCfg> cand = xpass_candidate_list(p, e.elem, e.nin);
    for (const SandCfg& g : cand) {
      bool same = e.nst == g.nst && e.cols == (g.stage ? -g.ncol : g.ncol);
      for (int s = 0; s < 6 && same; ++s)
        same = e.rad[s] == (s < g.nst ? (int)((g.radpack >> (5 * s)) & 31u) : 0);
      if (!same) continue;
      vc_problem::SandChoice ch{g.nst, g.tl, g.ncol, g.nthr, g.radpack, true, e.ms, 0.0};
      ch.from_file = true;
      ch.stage = g.stage;
      p->sand_choice[key] = ch;
      ++count;
      break;
    }
  }
  if (n_loaded) *n_loaded = count;
  return VC_OK;
}

}  // extern "C"
