// Internal state of one capacitance problem (host + device) -- not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/voxcap.h"
#include "fft_core.hpp"

namespace vc {

void set_error(const char* fmt, ...);
struct SandCfg;
// tk_npairs > 0: the Tucker-fused x pass of that many stored pairs (its LDS holds the
// tile's spectra, Hx rows each)
std::vector<SandCfg> sandwich_candidates(int L, int elem, int nin, int n1x, size_t budget, int tk_npairs = 0,
                                         int Hx = 0);
bool sandwich_default(int L, int elem, int nin, int n1x, size_t budget, SandCfg* cfg, int tk_npairs = 0, int Hx = 0);
// every x-pass configuration a problem's product can use in precision elem with nin
// input components: the fused form's (Tucker spectra), or the per-RHS workgroups' and
// then the staged form's (stored spectra; SandCfg::stage)
std::vector<SandCfg> xpass_candidate_list(::vc_problem* p, int elem, int nin);

// Owning device allocation.
struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  DevMem(DevMem&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevMem& operator=(DevMem&& o) noexcept {
    if (this != &o) {
      reset();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevMem() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t n) {
    reset();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    else p = nullptr;
    return e;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// FFT tables of one axis in one precision.
struct AxisTables {
  AxisPlan plan{};
  DevMem tw;   // L complex: exp(-2 pi i t / L)
  DevMem ph;   // L complex: exp(+i pi k / L), the half-voxel shift
};

struct PrecTables {
  AxisTables ax[3];
  DevMem R;    // [15][Hx][Hy][H] real spectra, kz contiguous (pairs not stored left unset)
};

// Tucker form of one stored spectrum pair (eq. 13): core r0 x r1 x r2 and factors
// D_m x r_m (row-major), FP64 and FP32 copies.
struct TuckerPair {
  int r[3] = {0, 0, 0};
  DevMem S64, U64[3], S32, U32[3];
  // the fused x pass's copies of U1: FP64 with rows padded to r1p = r1 rounded up to 4
  // (zero filled; a row is read as whole 16-byte vectors), FP32 transposed, [r1q][hxp]
  // (r1q = r1 rounded up to 16, hxp = Hx rounded up to 64, zero filled)
  int r1p = 0, r1q = 0, hxp = 0;
  DevMem U1p64, U1t32;
};

// The conventional block-diagonal preconditioner the paper compares against (Sec. III.A):
// every panel (conductor and dielectric) belongs to one box, and each box's block of the
// full eq. (4) matrix is inverted; dielectric rows make the blocks unsymmetric, so the
// transposed apply reads them transposed.
struct FullBlocks {
  int built = 0;
  int nbox = 0;
  int nblock = 0;
  int64_t block_doubles = 0;
  DevMem box_ptr, box_panels, box_block, block_off, block_n, blocks;
};

struct Precond {
  int built = 0;
  int mode = 1;   // 1 = block-diagonal-diagonal, 2 = diagonal only, 3 = block-diagonal (all panels)
  FullBlocks full;
  int nbox = 0;
  int nblock = 0;
  int64_t block_doubles = 0;
  double pself = 0.0;   // eq. (5) self term of a panel (conductor rows of the diagonal preconditioner)
  DevMem box_ptr, box_panels, box_block, block_off, block_n, blocks, dinv, dinv_diag;
  std::vector<int32_t> h_box_ptr, h_box_panels, h_box_block, h_block_n;
  std::vector<int64_t> h_block_off;
  std::vector<double> h_blocks;
};

constexpr int kToeplitzPairs = 15;   // 6 pairs of eq. (5), 9 of eq. (6)

struct PackData;   // several problems solved as one (pack.cpp)

// Device arrays of one GMRES solve (solver.cpp), all regions of one block: either the
// problem's own allocation or the library's static scratch array (noalloc.cpp).
struct SolveWs {
  double *V = nullptr, *w = nullptr, *z = nullptr, *r = nullptr, *b = nullptr, *x = nullptr, *tmp = nullptr;
  double *rr = nullptr, *dd = nullptr, *h = nullptr, *y2 = nullptr, *partial = nullptr, *norm = nullptr;
  double *cyc = nullptr;       // device-side GMRES cycle state (doubles)
  double *dC = nullptr;        // m x m capacitance of the last reduction
  double *rx = nullptr;        // 2 + nrhs doubles the relaxed mixed form reads per segment
  int *active = nullptr, *cyci = nullptr;
  unsigned* cnt = nullptr;     // completion counters of the fused Gram-Schmidt step (rest at 0)
  int nrhs = 0, restart = 0;   // the largest solve shape the regions hold
};
// byte size of the regions for nrhs columns of N rows and restart r, laid out from base
// (256-byte aligned regions) into *ws when base is not null
size_t solve_ws_layout(int64_t N, int nrhs, int r, char* base, SolveWs* ws);

}  // namespace vc

// Tucker-compressed Toeplitz octants of every pair over a largest grid (toeplitz.cpp):
// device core and factors (FP64) plus their host copies for saving
struct vc_toeplitz_cache {
  int device = 0;
  int nmax[3] = {0, 0, 0};
  double tol = 0.0;
  double build_s = 0.0;   // seconds taken by the build or the load
  vc::TuckerPair pair[vc::kToeplitzPairs];
  std::vector<double> hS[vc::kToeplitzPairs];
  std::vector<double> hU[vc::kToeplitzPairs][3];
};

struct vc_problem {
  int device = 0;
  int nx = 0, ny = 0, nz = 0;
  double dv = 0.0, eps_b = 1.0;
  std::vector<int32_t> cond_id;
  std::vector<double> eps_r;
  // panels in library order (sorted by dir, i, j, k)
  std::vector<vc_panel> panels;
  int64_t n_cond = 0, n_diel = 0;
  int m = 0;
  int n1[3] = {0, 0, 0};
  int M[3] = {0, 0, 0};
  int H = 0, Hx = 0, Hy = 0;
  // host index maps
  std::vector<int32_t> line_ptr;    // 3*n1x*n1y + 1
  std::vector<int32_t> items;       // lines holding panels
  std::vector<uint8_t> lflag;       // per line: 1 conductor panel, 2 dielectric panel
  std::vector<uint8_t> pflag;       // per (axis, x plane): OR of line flags
  std::vector<int32_t> pk;          // z index per panel
  std::vector<int8_t> pkind;
  std::vector<double> diag;         // eq. (7) term, +axis convention (0 on conductor panels)
  std::vector<int32_t> cond_ptr, cond_panels;   // conductor panels grouped by id
  std::vector<double> weight;       // eps_adj on conductor panels
  // where setup takes the Toeplitz tensors from: nullptr = the panel integrals, else a
  // cache restored and cropped to this grid (vc_setup_toeplitz_source)
  const vc_toeplitz_cache* tz_cache = nullptr;
  double t_toeplitz = 0.0;          // seconds of the last setup spent on the Toeplitz tensors
  // setup state
  bool setup_done = false;
  bool hip_failed = false;
  bool have64 = false, have32 = false;
  int max_rhs = 0;
  int nv[3] = {8, 8, 8};
  double t_setup = 0.0;
  double spectra_bytes = 0.0;
  double extract_resid = 0.0;
  // Tucker compression of the stored spectra (tucker_tol > 0): the strips T1, T2 are
  // rebuilt before each product and the x pass builds each tile's spectra from them
  double tucker_tol = 0.0;
  std::vector<vc::TuckerPair> tk;
  // rebuild scratch, one region per stored pair: T1 (shared by the precisions, rewritten
  // whole by each rebuild) and T2 per precision ([0] FP32, [1] FP64: their zero padding
  // past r1 must stay zero)
  vc::DevMem tk_T1, tk_T2[2];
  std::vector<int64_t> tk_o1, tk_o2;  // element offsets of each pair's regions
  struct TkTables {                 // device tables of the two batched strip GEMMs (T1, T2)
    bool built = false;
    vc::DevMem tab[2];
    int n[2] = {0, 0}, nblk[2] = {0, 0};
  } tk_tab[2];                      // [0] FP32, [1] FP64
  vc::DevMem tk_dev[2];             // per stored pair {U1, T2, r1} of the fused x pass ([0] FP32, [1] FP64)
  double tk_ms = 0.0;
  int tk_count = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tk_pending;
  // device mirrors
  vc::DevMem d_line_ptr, d_items, d_lflag, d_pflag, d_pk, d_pkind, d_diag, d_cond_ptr, d_cond_panels, d_weight, d_gl;
  vc::DevMem d_pcond;               // conductor id per panel (-1 on dielectric panels)
  vc::PrecTables t64, t32;
  vc::DevMem work_F, work_O;        // spectral work arrays (sized for FP64, reused by FP32)
  int64_t rhs_stride = 0, comp_stride = 0;
  int ncomp_F = 0, ncomp_O = 0;
  vc::Precond pc;
  // solver workspace: the regions the solver uses (ws) and the problem's own block they
  // point into, unless a call without allocation points them at the static scratch
  vc::DevMem s_all;
  vc::SolveWs ws, ws_own;
  bool ws_static = false;           // set for the duration of vc_capacitance_static
  // restart cycles captured as graphs, keyed by what their kernel arguments bake in
  bool use_graphs = true;
  struct GraphKey {
    int mvp, transpose, precond, nrhs, restart;
    int part;   // 0: cycle start, 1..nseg: segments of Arnoldi steps, nseg + 1: the update
    const double* b;
    double* x;
    int relax;  // segments of the relaxed mixed form end with the state read-back kernel
    bool operator==(const GraphKey& o) const {
      return mvp == o.mvp && transpose == o.transpose && precond == o.precond && nrhs == o.nrhs &&
             restart == o.restart && part == o.part && b == o.b && x == o.x && relax == o.relax;
    }
  };
  struct GraphEntry {
    GraphKey key;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipGraphExec_t find_graph(const GraphKey& k) const {
    for (const auto& e : graphs)
      if (e.key == k) return e.exec;
    return nullptr;
  }
  void add_graph(const GraphKey& k, hipGraph_t g, hipGraphExec_t e) {
    if (graphs.size() >= 32) {   // bounded cache (a solve shape holds a few segments): drop the oldest
      (void)hipGraphExecDestroy(graphs.front().exec);
      (void)hipGraphDestroy(graphs.front().graph);
      graphs.erase(graphs.begin());
    }
    graphs.push_back(GraphEntry{k, g, e});
  }
  void drop_graphs() {
    for (auto& e : graphs) {
      (void)hipGraphExecDestroy(e.exec);
      (void)hipGraphDestroy(e.graph);
    }
    graphs.clear();
  }
  hipStream_t solve_stream = nullptr;   // blocking stream of the solves (graphs cannot use the null stream)
  int mvp_count = 0;
  // x-pass launch configuration per (precision, direction, nrhs) key
  bool autotune = false;
  struct SandChoice {
    int nst, tl, ncol, nthr;
    uint32_t radpack;
    bool tuned;
    double ms_best, ms_default;
    bool from_file = false;   // read from a tuning cache (vc_tuning_load)
    int stage = 0;            // the staged form (SandArgs::stage)
  };
  std::map<int, SandChoice> sand_choice;
  // y-pass kernel per (precision, direction, transposed product, nrhs) key:
  // 0 = LDS Stockham tiles (k_strided), 1 = register-edge stages (k_ypass)
  struct YChoice {
    int impl;
    bool tuned;
    double ms[2];
    int ncol;   // register-edge tile width (0: the heuristic's)
    int xg;     // consecutive tiles per XCD (YArgs::xg)
    bool from_file = false;   // read from the tuning cache file
  };
  std::map<int, YChoice> y_choice;
  std::string tune_cache;   // tuning cache file of vc_setup_opts (empty: none)
  // per-pass timing (measurement)
  int prof = 0;   // 0 off, 1 every pass, 2 the x pass only
  std::vector<hipEvent_t> ev_free;
  std::vector<std::vector<hipEvent_t>> ev_pending;
  double pass_bytes[5] = {0, 0, 0, 0, 0};
  // set on the combined problem of a packed set: its rows are the largest member's
  // panel count and its products / preconditioner run over every member at once
  std::shared_ptr<vc::PackData> pack;
  int64_t pack_rows = 0;
  ~vc_problem() {
    drop_graphs();
    if (solve_stream) (void)hipStreamDestroy(solve_stream);
    for (auto& v : ev_pending)
      for (hipEvent_t e : v)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : tk_pending) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
  }
};

namespace vc {
inline int64_t npanels(const vc_problem* p) { return p->pack ? p->pack_rows : (int64_t)p->panels.size(); }
vc_status panelize(vc_problem* p);
vc_status choose_sizes(vc_problem* p, const int32_t* fft_size);
vc_status build_spectra(vc_problem* p, int want64, int want32, double tucker_tol, hipStream_t st);
vc_status build_precond(vc_problem* p, hipStream_t st);
vc_status build_precond_full(vc_problem* p, hipStream_t st);
// FP64 sequentially truncated HOSVD of a device tensor (D1 x D2 x D3 row-major) into
// tp.S64 / tp.U64 (tucker.cpp)
vc_status tucker_compress_tensor(const double* X, int D1, int D2, int D3, double tol, TuckerPair& tp,
                                 hipStream_t st);
void gauss_legendre_table(std::vector<double>& gl);
// Toeplitz octants (toeplitz.cpp): n[a] voxels per axis -> (n0+1)(n1+1)(n2+1) doubles
vc_status toeplitz_restore(const vc_toeplitz_cache* C, int q, const int n[3], double* out, hipStream_t st);
vc_status toeplitz_octant(int q, const int n[3], double* out, const double* gl, hipStream_t st);
void pair_axes(int q, int* a, int* b, int* want);
vc_status tucker_begin(vc_problem* p, double tol);
vc_status tucker_compress_pair(vc_problem* p, const double* X, hipStream_t st);
vc_status tucker_end(vc_problem* p);
// T1 = S x3 U3 and T2 = T1 x2 U2 of every stored pair (the x pass applies U1)
template <typename T>
vc_status tucker_rebuild(vc_problem* p, hipStream_t st, const int* skip = nullptr);
// algorithmic bytes of one forward product of nrhs columns, every pass (elem: 4 or 8)
double product_bytes_model(vc_problem* p, int elem, int nrhs);
// the same summed over the members of a packed set (one product of all their columns)
double pack_product_bytes(vc_problem* q, int elem);
vc_status apply_op(vc_problem* p, int transpose, vc_precision prec, const double* x, double* y, int nrhs,
                   hipStream_t st, const int* skip = nullptr, const int* act = nullptr);
// the same over a packed set (pack.cpp)
vc_status pack_apply(vc_problem* q, int transpose, vc_precision prec, const double* x, double* y, int nrhs,
                     hipStream_t st, const int* skip, const int* act);
vc_status pack_precond(vc_problem* q, const double* x, double* y, int nrhs, hipStream_t st, const int* skip);
vc_status apply_precond(vc_problem* p, int transpose, const double* x, double* y, int nrhs, hipStream_t st,
                        const int* skip = nullptr);
AxisPlan make_plan(int L, int max_radix);
bool pick_tile(int L, int elem_bytes, int emax, int ncols_total, int* ncol, int* nthr, size_t budget,
               int64_t other_blocks, int max_thr = 1024);
bool smooth7(int n);
}  // namespace vc

#define VC_HIP(expr)                                                                          \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess) {                                                                   \
      vc::set_error("HIP error %s at %s:%d (%s)", hipGetErrorString(_e), __FILE__, __LINE__, #expr); \
      return VC_ERR_HIP;                                                                      \
    }                                                                                         \
  } while (0)
