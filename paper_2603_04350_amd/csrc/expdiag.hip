// Host side of the Exp-ParaDiag library: handles, symbol tables, launch
// plans, hipGraph capture, and the C ABI declared in include/expdiag.h.
//
// Spectral state.  Inside a handle the space-time iterate lives in Fourier
// space as its half spectrum Uh[l][kappa], l = 0..Nt-1 (slices 1..Nt),
// kappa = 0..Nk-1 in rfftn order; the ABI is physical, so each solve does
// one forward batched FFT on entry and one inverse on exit.
//
// One fixed-point iteration (Sec. 3, eq. pcond-1st-order with the lagged
// nonlinearity of Sec. 6.2) is
//   pass A (nonlinear only, per slice):  N^_l = FFT N(IFFT Uh_{l-1})
//   pass B (per kappa tile, all Nt rows): residual, steps (a)-(c), update,
//          norms, convergence state (device side).
// An iteration is a fixed list of launches (a "plan"): launches are grouped
// by stage and kernel signature and each carries a device job table, so a
// batch of instances of any shapes costs one launch per group.  The plan is
// captured once into a hipGraph and replayed; finished instances and
// off-phase jobs exit at their first instruction.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/expdiag.h"
#include "kernels_dense.hpp"
#include "kernels_bdf.hpp"
#include "kernels_fft.hpp"
#include "kernels_krylov.hpp"
#include "kernels_passb.hpp"

using namespace expdiag;

namespace {

constexpr int HIST_CAP = 4096;
// grid points per axis: powers of two NMIN..NMAX; row transforms of
// length NMAX/2 (half spectrum), column transforms of length NMAX; the
// 2C-column workgroups only up to WIDE_LMAX (LDS)
constexpr int NMAX = 4096;
constexpr int WIDE_LMAX = 1024;
constexpr int NPROF = 5;
constexpr double BULK_TOL = 1e-6;
enum ProfClass { P_COL = 0, P_ROW = 1, P_PASSB = 2, P_RED = 3, P_KRY = 4 };

struct EventPair {
  hipEvent_t a, b;
  int cls;
};

// K_X*: boundary-transform stages (entry / exit of a batch): fp64 rows in
// the group's row mode, fp64 columns in the group's direction, and fp64 ->
// fp32 copies (a ColJob with `outer` complex elements)
enum Kind {
  K_ROW = 0, K_COL = 1, K_PASSB = 2, K_XROW = 3, K_XCOL = 4, K_XNARROW = 5,
  K_XWIDEN = 6, K_XZERO = 7
};
bool kind_rows(int k) { return k == K_ROW || k == K_XROW; }
bool kind_cols(int k) {
  return k == K_COL || k == K_XCOL || k == K_XNARROW || k == K_XWIDEN ||
         k == K_XZERO;
}

// One launch of a plan: jobs of the same kernel signature.
// Algorithmic bytes of one job of an iteration launch in each precision
// phase (PH_BULK, PH_SWITCH, PH_FP64) of its instance, and the instance's
// host mirror (profiling resolves a launch's bytes from the phases its
// instances were in, once the solve has ended).
struct JobBytes {
  const Ctl* hm;
  double b[3];
};

struct Group {
  int stage, kind, tcode, len, mode, ti, to;  // signature
  int wide = 0;  // column stages: 1 = the 2C-column workgroup variant
  std::vector<RowJob> rj;
  std::vector<ColJob> cj;
  std::vector<PassBArgs> pj;
  std::vector<int> start;  // njobs + 1
  // instances whose convergence reduction this launch performs (the
  // hosting column stage: before its transform blocks; pass B: as a
  // ctl_reduce launch right after)
  std::vector<PassBArgs> red;
  double bytes = 0;        // algorithmic bytes of one full launch
  // per job, when built for an instance with a host mirror (profiling)
  std::vector<JobBytes> jb;
  void* djobs = nullptr;
  int* dstart = nullptr;
  void* dred = nullptr;
  int grid() const { return start.empty() ? 0 : start.back(); }
  int njobs() const { return static_cast<int>(start.size()) - 1; }
  std::tuple<int, int, int, int, int, int, int, int> key() const {
    return std::make_tuple(stage, kind, tcode, len, mode, ti, to, wide);
  }
};

struct Plan {
  std::vector<Group> groups;
  bool uploaded = false;
  // host mirror of the instance whose launches are being added (set by
  // plan_iteration while it builds; null: no per-phase bytes)
  const Ctl* cur_hm = nullptr;
  // one device arena (and pinned staging) for every group's job table,
  // grown on demand and reused across rebuilds
  char* arena = nullptr;
  char* staging = nullptr;
  size_t cap = 0;
  // arena and staging provided by the caller: never grown or freed here
  bool fixed = false;
  // the pass-B groups' convergence reductions as one list on the device,
  // reduced by one launch after the last pass-B group of an iteration
  void* dred_pb = nullptr;
  int nred_pb = 0;
  double red_pb_bytes = 0;
};

}  // namespace

struct expdiag_ctx {
  int dim = 1;
  int n[3] = {0, 0, 0};
  int Nt = 0;
  double dt = 0, alpha = 0;
  int scheme = 1;
  expdiag_problem p{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  long Ns = 0, Nk = 0;
  int nh = 0;
  bool nonlinear = false;
  bool mixed = false;
  int restart_cap = 0;
  int tvariant = 0;  // time transform: 0 radix FFT, 1 dense MFMA GEMM
  int col_wide = 0;  // pass-A column stages: 1 = 2C-column workgroups
  bool cplx = false;  // complex symbols (advection): E, c1, c2 not real
  // complex state (complex coefficients): physical arrays are complex, the
  // spectral state is the full spectrum (Nk = Ns, nh = n_last)
  bool cstate = false;
  bool light = false;  // no plan / graph of its own (batch, server)

  // device buffers
  cx<double>* Uh = nullptr;   // [Nt][Nk]
  cx<double>* Nh = nullptr;   // [Nt][Nk] fp64; fp32 view in its 2nd half
  cx<double>* T = nullptr;    // [Nt][Nk] scratch
  cx<double>* T2 = nullptr;   // [Nt][Nk] scratch (GMRES / Newton)
  cx<float>* T32 = nullptr;   // [Nt][Nk] fp32 pass-A scratch (mixed, d >= 2)
  cx<float>* U32 = nullptr;   // [Nt][Nk] fp32 bulk-phase iterate (same)
  double* Uphys = nullptr;    // [Nt][Ns] physical iterate (Newton)
  float* Uphys32 = nullptr;   // [Nt][Ns] its fp32 copy (mixed Newton)
  cx<double>* u0h = nullptr;  // [Nk]
  cx<double> *E = nullptr, *c1 = nullptr, *c2 = nullptr;  // [Nk]
  double *gam = nullptr, *igam = nullptr;             // [Nt]
  cx<double>* lam = nullptr;                          // [Nt]
  cx<double>* tw64 = nullptr;                         // [TW_N]
  cx<float>* tw32 = nullptr;                          // [TW_N]
  cx<double>* roots = nullptr;  // e^{+2 pi i j/N}, j < N (EBDF dense transform)
  double* partials = nullptr;                         // [maxblocks][4]
  int max_partials = 0;
  double* red_out = nullptr;  // [8]
  Ctl* ctl = nullptr;
  double* hist = nullptr;     // [HIST_CAP][2]
  cx<double>* V = nullptr;    // Krylov basis [(restart+1)][Nt][Nk]
  double* kdots = nullptr;    // [4 (restart+2)]
  double* kpart = nullptr;    // [blocks][restart+2]
  int kpart_blocks = 0;

  // pinned host memory
  Ctl* h_ctl = nullptr;       // staging for control-block uploads
  Ctl* h_mirror = nullptr;    // host-mapped mirror written by the device
  Ctl* d_mirror = nullptr;    // its device address
  double* h_red = nullptr;
  double* h_kdots = nullptr;

  // completion events of the (at most two) chunks of iterations in flight,
  // and the iterations the previous solve of this handle took (the first
  // chunk's size; 0 before the first solve)
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};
  int last_iters = 0;

  // iteration plan and its graph
  Plan plan;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool use_graph = true;
  // solves start from U = 0 whatever U holds (expdiag_set_zero_guess)
  bool zero_guess = false;

  // profiling
  bool prof = false;
  int prof_mask = 0;  // classes whose launches are bracketed by events
  long prof_all[NPROF] = {0, 0, 0, 0, 0};  // launches of every class
  std::vector<EventPair> events;
  size_t ev_used = 0;
  double prof_ms[NPROF] = {0, 0, 0, 0, 0};
  long prof_cnt[NPROF] = {0, 0, 0, 0, 0};
  double prof_bytes[NPROF] = {0, 0, 0, 0, 0};
  // iteration launches of the solve being profiled: their index (1-based)
  // and the per-phase bytes of their jobs, resolved at the solve's end
  struct PendingBytes {
    int cls, k;
    std::vector<JobBytes> jobs;
  };
  int prof_iter = 0;
  std::vector<PendingBytes> prof_pending;

  std::string err;
  size_t bytes = 0;

  // device buffers carved from a caller-provided fixed workspace instead of
  // hipMalloc (the no-allocation entry point); such a handle is never
  // released with hipFree
  char* arena = nullptr;
  size_t arena_cap = 0, arena_off = 0;
};

namespace {

thread_local std::string g_create_err;

int fail(expdiag_ctx* h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h != nullptr)
    h->err = buf;
  else
    g_create_err = buf;
  return code;
}

#define HIPCHK(h, expr)                                                   \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return fail((h), EXPDIAG_EHIP, "%s: %s (%s:%d)", #expr,             \
                  hipGetErrorString(e_), __FILE__, __LINE__);             \
  } while (0)

#define RCHK(expr)          \
  do {                      \
    int r_ = (expr);        \
    if (r_ != 0) return r_; \
  } while (0)

bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

template <int LO, int HI, typename F>
bool dispatch_pow2(int v, F&& f) {
  if constexpr (LO > HI) {
    return false;
  } else {
    if (v == LO) {
      f(std::integral_constant<int, LO>{});
      return true;
    }
    return dispatch_pow2<LO * 2, HI>(v, f);
  }
}

template <typename T>
constexpr int tcode_of() {
  return std::is_same<T, double>::value ? 0 : 1;
}

// ---------------------------------------------------------------- profiling
// Brackets one launch with events when profiling is on and accounts the
// launch's algorithmic bytes (what the kernel must read and write once).
// With `ext` the launch itself carries the events (klaunch) and they time
// the kernel's execution; otherwise they are recorded on the stream around
// it (which adds the dispatch latency).
struct ProfScope {
  expdiag_ctx* h;
  int cls;
  bool ext;
  EventPair* ep = nullptr;
  ProfScope(expdiag_ctx* h_, int c, double bytes, bool ext_ = false)
      : h(h_), cls(c), ext(ext_) {
    if (h == nullptr || !h->prof) return;
    h->prof_bytes[c] += bytes;
    h->prof_all[c] += 1;
    if (((h->prof_mask >> c) & 1) && h->ev_used < h->events.size()) {
      ep = &h->events[h->ev_used++];
      ep->cls = cls;
      if (!ext) (void)hipEventRecord(ep->a, h->stream);
    }
  }
  ~ProfScope() {
    if (ep != nullptr && !ext) (void)hipEventRecord(ep->b, h->stream);
  }
};

// Launch `kernel` on `st`.  When `ps` (made with ext) brackets this launch,
// its start and stop events are attached to the dispatch itself, so they
// record when the kernel starts and ends on the GPU.
template <typename... KArgs, typename... Args>
void klaunch(const ProfScope& ps, void (*kernel)(KArgs...), dim3 grid,
             dim3 block, hipStream_t st, Args... args) {
  if (ps.ep != nullptr)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, ps.ep->a, ps.ep->b, 0,
                          args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
}

Ctl read_mirror(const Ctl* p);

// Bytes a profiled launch of group g adds now: its static bytes, or, for
// an iteration launch built with per-phase bytes, none yet (recorded with
// the launch's iteration index and resolved by prof_resolve).
double prof_group_bytes(expdiag_ctx* ph, const Group& g, int cls) {
  if (ph == nullptr || !ph->prof || g.jb.empty()) return g.bytes;
  ph->prof_pending.push_back({cls, ph->prof_iter, g.jb});
  return 0.0;
}

// Start of a profiled solve: iteration launches count from 1 again.
void prof_begin(expdiag_ctx* ph) {
  if (ph == nullptr) return;
  ph->prof_iter = 0;
  ph->prof_pending.clear();
}

// End of a profiled solve (stream synchronised, mirrors final): each
// recorded iteration launch k adds, per job, the bytes of the phase its
// instance was in at its k-th iteration (bulk through its switch_iter-th
// iteration, the switch iteration next, fp64 after), nothing once the
// instance had finished.  Exact when every instance launched runs from the
// solve's first iteration on (fixed-count solves, compaction of finished
// instances); an instance a batch schedule paused is counted as if it had
// run.
void prof_resolve(expdiag_ctx* ph) {
  if (ph == nullptr) return;
  for (const auto& r : ph->prof_pending) {
    double b = 0;
    for (const auto& j : r.jobs) {
      const Ctl c = read_mirror(j.hm);
      if (r.k > c.iters) continue;
      // the first iteration of a solve from zero skips its pass A
      if (r.k == 1 && c.zstart && (r.cls == P_COL || r.cls == P_ROW))
        continue;
      const int s = c.switch_iter;
      const int phase = (s == 0 || r.k <= s) ? PH_BULK
                        : (r.k == s + 1)    ? PH_SWITCH
                                            : PH_FP64;
      b += j.b[phase];
    }
    ph->prof_bytes[r.cls] += b;
  }
  ph->prof_pending.clear();
}

template <typename T>
const cx<T>* twid_table(expdiag_ctx* h) {
  if constexpr (std::is_same<T, double>::value)
    return h->tw64;
  else
    return h->tw32;
}

// ------------------------------------------------------- job constructors
int row_blocks(int M, long nrows) {
  long b = 0;
  dispatch_pow2<2, NMAX / 2>(M, [&](auto Mc) {
    constexpr int MM = decltype(Mc)::value;
    b = (nrows + RowShape<MM>::RPB - 1) / RowShape<MM>::RPB;
  });
  return static_cast<int>(b);
}
int col_blocks(int L, long outer, long inner, int wide = 0) {
  long b = 0;
  dispatch_pow2<4, NMAX>(L, [&](auto Lc) {
    constexpr int LL = decltype(Lc)::value;
    const long C = (wide && LL <= WIDE_LMAX) ? ColShape<LL, 2>::C
                                             : ColShape<LL>::C;
    b = outer * ((inner + C - 1) / C);
  });
  return static_cast<int>(b);
}
int passb_blocks_nt(int Nt, long Nk) {
  long b = 0;
  dispatch_pow2<2, 512>(Nt, [&](auto Nc) {
    constexpr int NN = decltype(Nc)::value;
    b = (Nk + PassBShape<NN>::C - 1) / PassBShape<NN>::C;
  });
  return static_cast<int>(b);
}
constexpr int DENSE_NT_MIN = 8, DENSE_NT_MAX = 128;
bool dense_ok(int Nt) {
  return is_pow2(Nt) && Nt >= DENSE_NT_MIN && Nt <= DENSE_NT_MAX;
}
// blocks of the first-order dense (DFT on MFMA) pass B
int dft_blocks(int Nt, long Nk) {
  long b = 0;
  dispatch_pow2<DENSE_NT_MIN, DENSE_NT_MAX>(Nt, [&](auto Nc) {
    constexpr int NN = decltype(Nc)::value;
    b = (Nk + DftShape<NN>::C - 1) / DftShape<NN>::C;
  });
  return static_cast<int>(b);
}
// Order s of an exponential BDF scheme (EBDF2, EBDF3..EBDF6), else 0.
int bdf_order(int scheme) {
  if (scheme == EXPDIAG_EBDF2) return 2;
  if (scheme >= EXPDIAG_EBDF3 && scheme <= EXPDIAG_EBDF6)
    return scheme - EXPDIAG_EBDF3 + 3;
  return 0;
}
// Time points of the transform in pass B: Nt, or Nt - s + 1 for an order-s
// exponential BDF, whose window rows 0..s-2 are the fixed starts A^m u_0.
int time_len(const expdiag_ctx* h) {
  const int s = bdf_order(h->scheme);
  return s > 0 ? h->Nt - s + 1 : h->Nt;
}
// Pass A: the slices whose N the residual needs and the N^ slot of the
// first.  ETD: u_0..u_{Nt-1} for rows 0..Nt-1, u_0 from the initial
// condition (slot 0, prepare_u0), so U slices 0..Nt-2 go to slots 1..Nt-1.
// IF1 (N(u_l) in row l): all Nt slices of U to slots 0..Nt-1.
long pass_a_slices(const expdiag_ctx* h) {
  return h->scheme == EXPDIAG_IF1 ? h->Nt : h->Nt - 1;
}
long pass_a_slot(const expdiag_ctx* h) {
  return h->scheme == EXPDIAG_IF1 ? 0 : 1;
}
// Order-s exponential BDF windows take the radix FFT when N = Nt - s + 1
// is a power of two (2..512) and the dense transform when Nt is one
// (8..128, N >= 2).
bool bdf_fft_ok(int Nt, int s) {
  const int N = Nt - s + 1;
  return N >= 2 && N <= 512 && is_pow2(N);
}
bool bdf_ok(int Nt, int s) {
  return bdf_fft_ok(Nt, s) || (dense_ok(Nt) && Nt - s + 1 >= 2);
}
// f(std::integral_constant<int, SC>) for an order s = 2..6 (false
// otherwise): the radix pass B of orders 2..4 is compiled for its order
// (SC = s); orders 5 and 6 take the kernel that reads s per job (SC = 0),
// because compiled in they spill (96 and 168 bytes per lane at N = 64) and
// measured 37 and 49 us against 31 and 32 us per launch.
template <typename F>
bool dispatch_bdf_order(int s, F&& f) {
  switch (s) {
    case 2: f(std::integral_constant<int, 2>{}); return true;
    case 3: f(std::integral_constant<int, 3>{}); return true;
    case 4: f(std::integral_constant<int, 4>{}); return true;
    case 5:
    case 6: f(std::integral_constant<int, 0>{}); return true;
    default: return false;
  }
}
// Spectral index width the kernels weight inner products by: entries at
// kl = kappa % nh in {0, nh - 1} count once, the others twice (Parseval on
// a half spectrum).  A full spectrum (complex state) weights every entry
// once, which nh = 1 gives (kl is then always 0).
int parseval_nh(const expdiag_ctx* h) { return h->cstate ? 1 : h->nh; }

// Whether a mixed-precision instance keeps its bulk-phase iterate in fp32
// (its buffer U32): first-order schemes with the radix pass B on grids of
// d >= 2 (whose pass A starts with a column stage).
bool bulk_u32(const expdiag_ctx* h) {
  return h->mixed && h->nonlinear && h->dim >= 2 && !h->cstate &&
         (h->scheme == EXPDIAG_ETD1 || h->scheme == EXPDIAG_ETD2) &&
         h->tvariant == 0 && h->U32 != nullptr;
}
cx<float>* u32_view(expdiag_ctx* h) { return h->U32; }
int passb_blocks(expdiag_ctx* h) {
  if (h->tvariant == 1)
    return dft_blocks(h->Nt, h->Nk);
  return passb_blocks_nt(time_len(h), h->Nk);
}

double row_bytes(int M, int mode, long nrows, size_t si, size_t so) {
  const double realb = static_cast<double>(nrows) * 2 * M;
  const double cplxb = static_cast<double>(nrows) * (M + 1) * 2;
  if (mode == ROW_R2C || mode == ROW_NR2C) return realb * si + cplxb * so;
  if (mode == ROW_C2R) return cplxb * si + realb * so;
  return cplxb * (si + so) + (mode == ROW_JVP ? realb * si : 0.0);
}

RowJob make_row(expdiag_ctx* h, const void* in, void* out, long nrows,
                long in_pitch, long out_pitch, double scale, const Ctl* ctl,
                int phase_req, const void* aux = nullptr, long aux_pitch = 0) {
  RowJob j{};
  j.in = in;
  j.out = out;
  j.aux = aux;
  j.nrows = nrows;
  j.in_pitch = in_pitch;
  j.out_pitch = out_pitch;
  j.aux_pitch = aux_pitch;
  j.scale = scale;
  j.n1 = h->p.n1;
  j.n2 = h->p.n2;
  j.n3 = h->p.n3;
  j.ctl = ctl;
  j.phase_req = phase_req;
  return j;
}

ColJob make_col(const void* in, void* out, long outer, long inner,
                double scale, const Ctl* ctl, int phase_req) {
  ColJob j{};
  j.in = in;
  j.out = out;
  j.outer = outer;
  j.inner = inner;
  j.scale = scale;
  j.ctl = ctl;
  j.phase_req = phase_req;
  return j;
}

PassBArgs passb_args(expdiag_ctx* h) {
  PassBArgs a{};
  a.U = h->Uh;
  a.U32 = bulk_u32(h) ? u32_view(h) : nullptr;
  a.Nh = h->Nh;
  a.Nh32 = nullptr;
  a.u0h = h->u0h;
  a.E = h->E;
  a.c1 = h->c1;
  a.c2 = h->c2;
  a.gam = h->gam;
  a.igam = h->igam;
  a.lam = h->lam;
  a.partials = h->partials;
  a.ctl = nullptr;
  a.hmirror = nullptr;
  a.hist = nullptr;
  a.tw = h->tw64;
  a.roots = h->roots;
  a.Nk = h->Nk;
  a.nh = parseval_nh(h);
  a.nonlinear = h->nonlinear ? 1 : 0;
  a.etd2 = h->scheme == EXPDIAG_ETD2 ? 1 : 0;
  a.nblocks = passb_blocks(h);
  a.inv_ns = 1.0 / static_cast<double>(h->Ns);
  a.same_slice = h->scheme == EXPDIAG_IF1 ? 1 : 0;
  a.bdf_s = bdf_order(h->scheme);
  a.jac_mode = h->scheme == EXPDIAG_IF1 ? h->p.jacobian : 0;
  a.sigma = 0.0;
  a.jac_c[0] = h->dt * h->p.n1;
  a.jac_c[1] = 2.0 * h->dt * h->p.n2;
  a.jac_c[2] = 3.0 * h->dt * h->p.n3;
  a.inv_ntns = 1.0 / (static_cast<double>(h->Nt) * h->Ns);
  // the same long-double values as the gamma table
  const int N = time_len(h);
  const int R = std::min(N, 4), tpl = N / R;
  const long double la = logl(static_cast<long double>(h->alpha));
  for (int s = 0; s < 4; ++s) {
    const long double g = s < R ? expl(la * (s * tpl) / N) : 1.0L;
    a.gstep[s] = static_cast<double>(g);
    a.igstep[s] = static_cast<double>(1.0L / g);
  }
  return a;
}

// ------------------------------------------------------ single launches
template <typename T, int MODE, typename TI, typename TO>
int launch_row1(expdiag_ctx* h, const RowJob& jb) {
  const int M = h->n[h->dim - 1] / 2;
  ProfScope ps(h, P_ROW, row_bytes(M, MODE, jb.nrows, sizeof(TI), sizeof(TO)));
  bool ok = dispatch_pow2<2, NMAX / 2>(M, [&](auto Mc) {
    constexpr int MM = decltype(Mc)::value;
    using S = RowShape<MM>;
    const long blocks = (jb.nrows + S::RPB - 1) / S::RPB;
    hipLaunchKernelGGL((row_kernel1<T, MM, MODE, TI, TO>), dim3(blocks),
                       dim3(S::THREADS), 0, h->stream, jb, twid_table<T>(h));
  });
  if (!ok) return fail(h, EXPDIAG_EUNSUPPORTED, "row length %d", 2 * M);
  HIPCHK(h, hipGetLastError());
  return 0;
}

template <typename T, int S, typename TI, typename TO>
int launch_col1(expdiag_ctx* h, int L, const ColJob& jb) {
  ProfScope ps(h, P_COL, static_cast<double>(jb.outer) * L * jb.inner * 2 *
                             (sizeof(TI) + sizeof(TO)));
  bool ok = dispatch_pow2<4, NMAX>(L, [&](auto Lc) {
    constexpr int LL = decltype(Lc)::value;
    using SH = ColShape<LL>;
    const long tiles = (jb.inner + SH::C - 1) / SH::C;
    hipLaunchKernelGGL((col_kernel1<T, LL, S, TI, TO>),
                       dim3(jb.outer * tiles), dim3(SH::THREADS), 0,
                       h->stream, jb, twid_table<T>(h));
  });
  if (!ok) return fail(h, EXPDIAG_EUNSUPPORTED, "column length %d", L);
  HIPCHK(h, hipGetLastError());
  return 0;
}

double passb_bytes(const PassBArgs& a, int Nt, int mode, size_t nb) {
  const double ent = static_cast<double>(Nt) * a.Nk;
  double bytes = static_cast<double>(a.Nk) * (sizeof(double) * 3 + 16);
  const double nbytes = a.nonlinear ? static_cast<double>(nb) : 0.0;
  if (mode == PB_PRECOND) return bytes + ent * 32;
  // the iterate read and written (fp32 in the bulk phase when kept so)
  const double ubytes = (mode == PB_ITERATE && a.U32 != nullptr) ? 16 : 32;
  return bytes + ent * (ubytes + nbytes);
}

// Blocks (partial sums) of the single-instance pass B of mode `mode`: the
// first-order schemes run every mode but the dense-variant PB_PRECOND on
// the radix kernel.
int passb1_blocks(expdiag_ctx* h, int mode) {
  if (bdf_order(h->scheme) == 0 && !(mode == PB_PRECOND && h->tvariant == 1))
    return passb_blocks_nt(h->Nt, h->Nk);
  return passb_blocks(h);
}

template <int MODE, typename TN>
int launch_passb1(expdiag_ctx* h, const PassBArgs& a) {
  ProfScope ps(h, P_PASSB, passb_bytes(a, h->Nt, MODE, sizeof(cx<TN>)));
  if constexpr (MODE == PB_PRECRES) {
    if (bdf_order(h->scheme) > 0)
      return fail(h, EXPDIAG_EUNSUPPORTED, "fused residual for EBDF");
  } else if (const int s = bdf_order(h->scheme); s > 0) {
    // radix FFT: one instantiation per order; dense (MFMA-bound either way):
    // order 2 has its own, 3..6 share one that reads s
    bool ok = false;
    if (h->tvariant == 1) {
      ok = dispatch_pow2<DENSE_NT_MIN, DENSE_NT_MAX>(h->Nt, [&](auto Nc) {
        constexpr int NN = decltype(Nc)::value;
        const dim3 grid(dft_blocks(NN, h->Nk)), th(DENSE_THREADS);
        if (s == 2)
          hipLaunchKernelGGL((passb_bdf_kernel1<NN, 2, MODE>), grid, th, 0,
                             h->stream, a);
        else
          hipLaunchKernelGGL((passb_bdf_kernel1<NN, 0, MODE>), grid, th, 0,
                             h->stream, a);
      });
    } else {
      ok = dispatch_pow2<2, 512>(time_len(h), [&](auto Nc) {
        constexpr int NN = decltype(Nc)::value;
        const dim3 grid(passb_blocks_nt(NN, h->Nk));
        const dim3 th(PassBShape<NN>::THREADS);
        ok = dispatch_bdf_order(s, [&](auto Sc) {
          constexpr int SS = decltype(Sc)::value;
          hipLaunchKernelGGL((passb_bdf_fft_kernel1<NN, SS, MODE>), grid, th,
                             0, h->stream, a);
        });
      });
    }
    if (!ok)
      return fail(h, EXPDIAG_EUNSUPPORTED, "EBDF%d Nt %d", s, h->Nt);
    HIPCHK(h, hipGetLastError());
    return 0;
  }
  if (MODE == PB_PRECOND && h->tvariant == 1) {
    const bool ok = dispatch_pow2<DENSE_NT_MIN, DENSE_NT_MAX>(h->Nt, [&](auto Nc) {
      constexpr int NN = decltype(Nc)::value;
      hipLaunchKernelGGL((passb_dense_kernel1<NN, PB_PRECOND, double>),
                         dim3(dft_blocks(NN, h->Nk)), dim3(DENSE_THREADS), 0,
                         h->stream, a);
    });
    if (!ok) return fail(h, EXPDIAG_EUNSUPPORTED, "dense Nt %d", h->Nt);
    HIPCHK(h, hipGetLastError());
    return 0;
  }
  bool ok = dispatch_pow2<2, 512>(h->Nt, [&](auto Nc) {
    constexpr int NN = decltype(Nc)::value;
    using SH = PassBShape<NN>;
    const long blocks = (h->Nk + SH::C - 1) / SH::C;
    if (h->cplx)
      hipLaunchKernelGGL((passb_kernel1<NN, MODE, TN, true>), dim3(blocks),
                         dim3(SH::THREADS), 0, h->stream, a);
    else
      hipLaunchKernelGGL((passb_kernel1<NN, MODE, TN, false>), dim3(blocks),
                         dim3(SH::THREADS), 0, h->stream, a);
  });
  if (!ok) return fail(h, EXPDIAG_EUNSUPPORTED, "Nt %d", h->Nt);
  HIPCHK(h, hipGetLastError());
  return 0;
}

int launch_reduce(expdiag_ctx* h, int nblocks) {
  ProfScope ps(h, P_RED, static_cast<double>(nblocks) * 32);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(RED_THREADS), 0, h->stream,
                     h->partials, nblocks, 1.0 / static_cast<double>(h->Ns),
                     h->red_out);
  HIPCHK(h, hipGetLastError());
  return 0;
}

// real physical slices [ns][Ns] -> half spectra [ns][Nk].  ROWMODE is
// ROW_R2C or ROW_NR2C (apply N pointwise first).  Uses h->T as scratch.
// Complex rows of the last axis, length n_last: dst = scale * FFT_S(src).
template <int S>
int launch_row_c2c(expdiag_ctx* h, const cx<double>* src, cx<double>* dst,
                   long rows, double scale) {
  const int M = h->n[h->dim - 1];
  ProfScope ps(h, P_ROW, static_cast<double>(rows) * M * 32);
  const bool ok = dispatch_pow2<4, NMAX>(M, [&](auto Mc) {
    constexpr int MM = decltype(Mc)::value;
    using SH = RowShape<MM>;
    const long blocks = (rows + SH::RPB - 1) / SH::RPB;
    hipLaunchKernelGGL((row_c2c_kernel<MM, S>), dim3(blocks),
                       dim3(SH::THREADS), 0, h->stream, src, dst, rows,
                       scale, h->tw64);
  });
  if (!ok) return fail(h, EXPDIAG_EUNSUPPORTED, "row length %d", M);
  HIPCHK(h, hipGetLastError());
  return 0;
}

// Complex-state slices, physical [ns][Ns] complex <-> full spectra
// [ns][Ns]: C2C transforms along every axis (forward: the last axis first;
// inverse: the last axis last, scaled by 1/Ns).  Uses h->T as scratch.
int fwd_slices_c2c(expdiag_ctx* h, const cx<double>* src, cx<double>* dst,
                   long ns) {
  const int d = h->dim;
  const int nl = h->n[d - 1];
  if (d == 1) return launch_row_c2c<-1>(h, src, dst, ns, 1.0);
  RCHK(launch_row_c2c<-1>(h, src, h->T, ns * (h->Ns / nl), 1.0));
  if (d == 2)
    return launch_col1<double, -1, double, double>(
        h, h->n[0], make_col(h->T, dst, ns, nl, 1.0, nullptr, -1));
  RCHK((launch_col1<double, -1, double, double>(
      h, h->n[1], make_col(h->T, h->T, ns * h->n[0], nl, 1.0, nullptr, -1))));
  return launch_col1<double, -1, double, double>(
      h, h->n[0],
      make_col(h->T, dst, ns, static_cast<long>(h->n[1]) * nl, 1.0, nullptr,
               -1));
}

int inv_slices_c2c(expdiag_ctx* h, const cx<double>* src, cx<double>* dst,
                   long ns) {
  const int d = h->dim;
  const int nl = h->n[d - 1];
  const double sc = 1.0 / static_cast<double>(h->Ns);
  if (d == 1) return launch_row_c2c<1>(h, src, dst, ns, sc);
  if (d == 2) {
    RCHK((launch_col1<double, 1, double, double>(
        h, h->n[0], make_col(src, h->T, ns, nl, 1.0, nullptr, -1))));
  } else {
    RCHK((launch_col1<double, 1, double, double>(
        h, h->n[0],
        make_col(src, h->T, ns, static_cast<long>(h->n[1]) * nl, 1.0,
                 nullptr, -1))));
    RCHK((launch_col1<double, 1, double, double>(
        h, h->n[1], make_col(h->T, h->T, ns * h->n[0], nl, 1.0, nullptr,
                             -1))));
  }
  return launch_row_c2c<1>(h, h->T, dst, ns * (h->Ns / nl), sc);
}

template <int ROWMODE>
int fwd_slices(expdiag_ctx* h, const double* src, cx<double>* dst, long ns) {
  if constexpr (ROWMODE == ROW_R2C) {
    if (h->cstate)
      return fwd_slices_c2c(h, reinterpret_cast<const cx<double>*>(src), dst,
                            ns);
  }
  const int d = h->dim;
  const long nh2 = 2L * h->nh;
  const int nl = h->n[d - 1];
  if (d == 1)
    return launch_row1<double, ROWMODE, double, double>(
        h, make_row(h, src, dst, ns, nl, nh2, 1.0, nullptr, -1));
  const long rows = ns * (h->Ns / nl);
  RCHK((launch_row1<double, ROWMODE, double, double>(
      h, make_row(h, src, h->T, rows, nl, nh2, 1.0, nullptr, -1))));
  if (d == 2)
    return launch_col1<double, -1, double, double>(
        h, h->n[0], make_col(h->T, dst, ns, h->nh, 1.0, nullptr, -1));
  RCHK((launch_col1<double, -1, double, double>(
      h, h->n[1], make_col(h->T, h->T, ns * h->n[0], h->nh, 1.0, nullptr, -1))));
  return launch_col1<double, -1, double, double>(
      h, h->n[0],
      make_col(h->T, dst, ns, static_cast<long>(h->n[1]) * h->nh, 1.0,
               nullptr, -1));
}

// half spectra [ns][Nk] -> real physical slices [ns][Ns] (normalised).
// `src` may be h->T.
int inv_slices(expdiag_ctx* h, const cx<double>* src, double* dst, long ns) {
  if (h->cstate)
    return inv_slices_c2c(h, src, reinterpret_cast<cx<double>*>(dst), ns);
  const int d = h->dim;
  const long nh2 = 2L * h->nh;
  const int nl = h->n[d - 1];
  const double sc = 1.0 / static_cast<double>(h->Ns);
  if (d == 1)
    return launch_row1<double, ROW_C2R, double, double>(
        h, make_row(h, src, dst, ns, nh2, nl, sc, nullptr, -1));
  if (d == 2) {
    RCHK((launch_col1<double, 1, double, double>(
        h, h->n[0], make_col(src, h->T, ns, h->nh, 1.0, nullptr, -1))));
  } else {
    RCHK((launch_col1<double, 1, double, double>(
        h, h->n[0],
        make_col(src, h->T, ns, static_cast<long>(h->n[1]) * h->nh, 1.0,
                 nullptr, -1))));
    RCHK((launch_col1<double, 1, double, double>(
        h, h->n[1],
        make_col(h->T, h->T, ns * h->n[0], h->nh, 1.0, nullptr, -1))));
  }
  const long rows = ns * (h->Ns / nl);
  return launch_row1<double, ROW_C2R, double, double>(
      h, make_row(h, h->T, dst, rows, nh2, nl, sc, nullptr, -1));
}

// Storage of N^ in precision T.  The fp64 array fills the allocation; the
// fp32 array of the mixed bulk phase lives in its second half, so it never
// overlaps fp64 slot 0 (N^_0 of the initial condition; Nt >= 2).
template <typename T>
cx<T>* nh_view(expdiag_ctx* h) {
  if constexpr (std::is_same<T, double>::value) {
    return h->Nh;
  } else {
    return reinterpret_cast<cx<float>*>(reinterpret_cast<char*>(h->Nh) +
                                        static_cast<size_t>(h->Nt) * h->Nk *
                                            sizeof(cx<float>));
  }
}

// Elementwise boundary kernels (copies between precisions, clearing): 256
// threads per block, each thread XPT elements 256 apart, so a block covers
// XPB consecutive elements (far fewer blocks than one element per thread,
// whose launch rate, not memory, bounded these kernels)
constexpr int XPT = 8;
constexpr int XPB = 256 * XPT;
int xblocks(long n) { return static_cast<int>((n + XPB - 1) / XPB); }

__global__ void narrow_kernel(const cx<double>* __restrict__ in,
                              cx<float>* __restrict__ out, long n) {
  const long b = static_cast<long>(blockIdx.x) * XPB + threadIdx.x;
#pragma unroll
  for (int k = 0; k < XPT; ++k) {
    const long i = b + k * 256;
    if (i < n) out[i] = cvt<float>(in[i]);
  }
}

// The iterate as the bulk phase keeps it: fp32 copy of Uh (after the entry
// transform of a solve), and back (before the exit transform) when the
// instance's control block says the fp32 copy is the current iterate
// (phase PH_BULK or PH_SWITCH after the last iteration).
__global__ void widen_bulk_kernel(const Ctl* __restrict__ ctl,
                                  const cx<float>* __restrict__ in,
                                  cx<double>* __restrict__ out, long n) {
  if (ctl->phase > PH_SWITCH) return;
  const long b = static_cast<long>(blockIdx.x) * XPB + threadIdx.x;
#pragma unroll
  for (int k = 0; k < XPT; ++k) {
    const long i = b + k * 256;
    if (i < n) out[i] = cvt<double>(in[i]);
  }
}

// n 8-byte words of device memory set to zero by a kernel (a memset node
// would misbehave where a caller captures the stream into a graph)
__global__ void zero_words_kernel(double* __restrict__ p, long n) {
  const long b = static_cast<long>(blockIdx.x) * XPB + threadIdx.x;
#pragma unroll
  for (int k = 0; k < XPT; ++k) {
    const long e = b + k * 256;
    if (e < n) p[e] = 0.0;
  }
}

int zero_words(expdiag_ctx* h, void* p, long n, hipStream_t st) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(zero_words_kernel, dim3(xblocks(n)), dim3(256), 0, st,
                     static_cast<double*>(p), n);
  HIPCHK(h, hipGetLastError());
  return 0;
}

int enter_bulk_state(expdiag_ctx* h, hipStream_t st) {
  if (!bulk_u32(h)) return 0;
  const long n = static_cast<long>(h->Nt) * h->Nk;
  hipLaunchKernelGGL(narrow_kernel, dim3(xblocks(n)), dim3(256), 0, st,
                     h->Uh, u32_view(h), n);
  HIPCHK(h, hipGetLastError());
  return 0;
}

int leave_bulk_state(expdiag_ctx* h, const Ctl* ctl, hipStream_t st) {
  if (!bulk_u32(h)) return 0;
  const long n = static_cast<long>(h->Nt) * h->Nk;
  hipLaunchKernelGGL(widen_bulk_kernel, dim3(xblocks(n)), dim3(256), 0, st,
                     ctl, u32_view(h), h->Uh, n);
  HIPCHK(h, hipGetLastError());
  return 0;
}

// Whether a fixed-point solve from U = 0 may skip its first pass A: the
// first-order exponential schemes take N at U's slices only into slots
// 1..Nt-1 of N^ (slot 0 is N(u_0)), and N(0) = 0.
bool zero_start_ok(const expdiag_ctx* h) {
  return h->nonlinear &&
         (h->scheme == EXPDIAG_ETD1 || h->scheme == EXPDIAG_ETD2);
}

// Slot region [offset, count) in words of N^ that the first pass B of a
// solve from U = 0 reads for U's slices: fp32 slots 1..Nt-1 in the bulk
// phase of a mixed instance (the fp32 view shares the allocation's second
// half, so fp64 slots are left alone), else fp64 slots 1..Nt-1.
void zero_start_region(expdiag_ctx* h, void** p, long* words) {
  const long n1 = static_cast<long>(h->Nt - 1) * h->Nk;
  if (h->mixed) {
    *p = nh_view<float>(h) + h->Nk;
    *words = n1;
  } else {
    *p = h->Nh + h->Nk;
    *words = 2 * n1;
  }
}

// The initial guess as the solve's spectral iterate Uh (and, with `bulk`,
// its fp32 bulk copy where the instance keeps one): the forward transform
// of U on h's stream, or, for a solve from U = 0 (`zero`), zeros, which is
// what that transform would give, without reading U; with `bulk` and a
// scheme that allows it, also the N^ rows the first pass B reads, so that
// the first iteration's pass A can be skipped (Ctl::zstart).
int enter_guess(expdiag_ctx* h, const double* U, bool bulk, bool zero) {
  const long n = static_cast<long>(h->Nt) * h->Nk;
  if (zero) {
    // an instance that keeps the fp32 bulk iterate reads Uh only after
    // writing all of it (the switch iteration's pass B, or the exit's
    // widening of the fp32 iterate when the solve stops before that)
    if (!(bulk && bulk_u32(h)))
      RCHK(zero_words(h, h->Uh, 2 * n, h->stream));
    if (bulk && bulk_u32(h)) RCHK(zero_words(h, u32_view(h), n, h->stream));
    if (bulk && zero_start_ok(h)) {
      void* p = nullptr;
      long w = 0;
      zero_start_region(h, &p, &w);
      RCHK(zero_words(h, p, w, h->stream));
    }
    return 0;
  }
  RCHK(fwd_slices<ROW_R2C>(h, U, h->Uh, h->Nt));
  return bulk ? enter_bulk_state(h, h->stream) : 0;
}

// u0 -> u0h, N^_0 = FFT N(u0) (fp64 slot 0) and, for mixed precision, its
// fp32 copy in slot 0 of the fp32 view.
int prepare_u0(expdiag_ctx* h, const double* u0) {
  RCHK(fwd_slices<ROW_R2C>(h, u0, h->u0h, 1));
  // (IF1 takes N at every slice of U, never at u_0)
  if (!h->nonlinear || h->scheme == EXPDIAG_IF1) return 0;
  RCHK(fwd_slices<ROW_NR2C>(h, u0, h->Nh, 1));
  if (h->mixed) {
    hipLaunchKernelGGL(narrow_kernel, dim3(xblocks(h->Nk)), dim3(256), 0,
                       h->stream, h->Nh, nh_view<float>(h), h->Nk);
    HIPCHK(h, hipGetLastError());
  }
  return 0;
}

// ----------------------------------------------------------------- plans
Group& plan_group(Plan& P, int stage, int kind, int tcode, int len, int mode,
                  int ti, int to, int wide = 0) {
  for (auto& g : P.groups)
    if (g.key() ==
        std::make_tuple(stage, kind, tcode, len, mode, ti, to, wide))
      return g;
  Group g{};
  g.stage = stage;
  g.kind = kind;
  g.tcode = tcode;
  g.len = len;
  g.mode = mode;
  g.ti = ti;
  g.to = to;
  g.wide = wide;
  g.start.push_back(0);
  P.groups.push_back(g);
  return P.groups.back();
}

template <typename T, typename TI, typename TO>
void plan_row(Plan& P, int stage, int M, int mode, const RowJob& j) {
  Group& g = plan_group(P, stage, K_ROW, tcode_of<T>(), M, mode,
                        tcode_of<TI>(), tcode_of<TO>());
  g.rj.push_back(j);
  g.start.push_back(g.start.back() + row_blocks(M, j.nrows));
  g.bytes += row_bytes(M, mode, j.nrows, sizeof(TI), sizeof(TO));
}

template <typename T, int S, typename TI, typename TO>
void plan_col(Plan& P, int stage, int L, const ColJob& j) {
  Group& g = plan_group(P, stage, K_COL, tcode_of<T>(), L, S,
                        tcode_of<TI>(), tcode_of<TO>());
  g.cj.push_back(j);
  g.start.push_back(g.start.back() + col_blocks(L, j.outer, j.inner));
  g.bytes += static_cast<double>(j.outer) * L * j.inner * 2 *
             (sizeof(TI) + sizeof(TO));
}

// `len` keys the group (the transform length of the radix kernels, the
// window length of the dense ones); `rows` is the window length.
void plan_passb(Plan& P, int stage, int len, int rows, const PassBArgs& a,
                size_t nb, int variant, bool reduce_after) {
  Group& g = plan_group(P, stage, K_PASSB, variant, len, PB_ITERATE, 0, 0);
  g.pj.push_back(a);
  if (reduce_after) g.red.push_back(a);
  g.start.push_back(g.start.back() + a.nblocks);
  g.bytes += passb_bytes(a, rows, PB_ITERATE, nb);
  if (P.cur_hm != nullptr) {
    // per entry: U read and written, N^ read (fp32 in the bulk phase; the
    // fp32 iterate in the bulk phase and read by the switch iteration)
    const double base = static_cast<double>(a.Nk) * (sizeof(double) * 3 + 16);
    const double ent = static_cast<double>(rows) * a.Nk;
    JobBytes j{P.cur_hm, {0, 0, 0}};
    if (!a.nonlinear) {
      j.b[0] = j.b[1] = j.b[2] = base + ent * 32;
    } else if (a.Nh32 == nullptr) {
      j.b[0] = j.b[1] = j.b[2] = base + ent * 48;
    } else if (a.U32 != nullptr) {
      j.b[0] = base + ent * 24;
      j.b[1] = base + ent * 40;
      j.b[2] = base + ent * 48;
    } else {
      j.b[0] = base + ent * 40;
      j.b[1] = j.b[2] = base + ent * 48;
    }
    g.jb.push_back(j);
  }
}

// pass A of one instance in precision T, gated on phase `ph`
template <typename T>
void plan_pass_a(Plan& P, expdiag_ctx* h, const Ctl* ctl, int ph) {
  const int d = h->dim;
  const long ns = pass_a_slices(h);
  const long nh2 = 2L * h->nh;
  const int nl = h->n[d - 1];
  const double sc = 1.0 / static_cast<double>(h->Ns);
  cx<T>* Tt = reinterpret_cast<cx<T>*>(h->T);
  cx<T>* N1 = nh_view<T>(h) + pass_a_slot(h) * h->Nk;
  if (d == 1) {
    plan_row<T, double, T>(P, 2, nl / 2, ROW_FUSED,
                           make_row(h, h->Uh, N1, ns, nh2, nh2, sc, ctl, ph));
    return;
  }
  const long in2 = d == 3 ? static_cast<long>(h->n[1]) * h->nh : h->nh;
  plan_col<T, 1, double, T>(P, 0, h->n[0],
                            make_col(h->Uh, Tt, ns, in2, 1.0, ctl, ph));
  if (d == 3)
    plan_col<T, 1, T, T>(P, 1, h->n[1],
                         make_col(Tt, Tt, ns * h->n[0], h->nh, 1.0, ctl, ph));
  plan_row<T, T, T>(P, 2, nl / 2, ROW_FUSED,
                    make_row(h, Tt, Tt, ns * (h->Ns / nl), nh2, nh2, sc, ctl,
                             ph));
  if (d == 3)
    plan_col<T, -1, T, T>(P, 3, h->n[1],
                          make_col(Tt, Tt, ns * h->n[0], h->nh, 1.0, ctl, ph));
  plan_col<T, -1, T, T>(P, 4, h->n[0], make_col(Tt, N1, ns, in2, 1.0, ctl, ph));
}

// Pass A of one instance in an iteration plan (tcode 2 groups hold the
// instance's fp32 job for the mixed-precision bulk phase and its fp64 job
// side by side, picked per block from the control block; ti names the fp32
// job's input type).  For d >= 2 the first stage, the inverse transform of
// Uh along axis 0, may perform the instance's convergence reduction of the
// previous iteration (`red`, when `host`): it then runs in fp64 in both
// phases (tcode 3; its blocks cannot see the phase that reduction sets),
// and the bulk phase reads that fp64 intermediate in the next stage before
// continuing in fp32 through T32.  Not hosted, the first stage picks its
// phase like the others and writes T32 in the bulk phase (16 bytes less
// per complex entry in the bulk phase, for one reduction launch after
// pass B).  Returns whether the reduction is hosted (1D pass A is one row
// stage that depends on the phase: never hosted).  Instances without a
// bulk phase carry their fp64 job in both slots.  A group's byte count is
// that of the phase the instance spends most iterations in (fp32 when
// mixed).
bool plan_pass_a_mp(Plan& P, expdiag_ctx* h, const Ctl* ctl,
                    const PassBArgs& red, bool host) {
  const int d = h->dim;
  const long ns = pass_a_slices(h);
  const long nh2 = 2L * h->nh;
  const int nl = h->n[d - 1];
  const int M = nl / 2;
  const double sc = 1.0 / static_cast<double>(h->Ns);
  const bool mx = h->mixed;
  cx<double>* T64 = h->T;
  cx<float>* T32 = h->T32;
  cx<double>* N64 = nh_view<double>(h) + pass_a_slot(h) * h->Nk;
  cx<float>* N32 = nh_view<float>(h) + pass_a_slot(h) * h->Nk;
  auto row2 = [&](int stage, const RowJob& j32, const RowJob& j64,
                  int ti32) {
    Group& g = plan_group(P, stage, K_ROW, 2, M, ROW_FUSED, ti32, 1);
    g.rj.push_back(mx ? j32 : j64);
    g.rj.push_back(j64);
    g.start.push_back(g.start.back() + row_blocks(M, j64.nrows));
    const double b64 =
        row_bytes(M, ROW_FUSED, j64.nrows, sizeof(double), sizeof(double));
    const double b32 = row_bytes(
        M, ROW_FUSED, j32.nrows, ti32 == 0 ? sizeof(double) : sizeof(float),
        sizeof(float));
    g.bytes += mx ? b32 : b64;
    if (P.cur_hm != nullptr)
      g.jb.push_back({P.cur_hm, {mx ? b32 : b64, b64, b64}});
  };
  const int wd = h->col_wide;
  auto col2 = [&](int stage, int L, int S, const ColJob& j32,
                  const ColJob& j64, int ti32) {
    const int wdl = L <= WIDE_LMAX ? wd : 0;
    Group& g = plan_group(P, stage, K_COL, 2, L, S, ti32, 1, wdl);
    g.cj.push_back(mx ? j32 : j64);
    g.cj.push_back(j64);
    g.start.push_back(g.start.back() +
                      col_blocks(L, j64.outer, j64.inner, wdl));
    const double ent = static_cast<double>(j64.outer) * L * j64.inner * 2;
    const double b64 = ent * 2 * sizeof(double);
    const double b32 =
        ent * ((ti32 == 0 ? sizeof(double) : sizeof(float)) + sizeof(float));
    // the switch iteration's first stage reads the fp32 iterate
    const double bsw =
        j64.in32 != nullptr ? ent * (sizeof(float) + sizeof(double)) : b64;
    g.bytes += mx ? b32 : b64;
    if (P.cur_hm != nullptr)
      g.jb.push_back({P.cur_hm, {mx ? b32 : b64, mx ? bsw : b64, b64}});
  };
  if (d == 1) {
    row2(2, make_row(h, h->Uh, N32, ns, nh2, nh2, sc, ctl, -1),
         make_row(h, h->Uh, N64, ns, nh2, nh2, sc, ctl, -1), 0);
    return false;
  }
  const int n0 = h->n[0];
  const long in2 = d == 3 ? static_cast<long>(h->n[1]) * h->nh : h->nh;
  host = host || !mx;
  if (host) {
    const ColJob j = make_col(h->Uh, T64, ns, in2, 1.0, ctl, -1);
    const int wd0 = n0 <= WIDE_LMAX ? wd : 0;
    Group& g = plan_group(P, 0, K_COL, 3, n0, 1, 0, 0, wd0);
    g.cj.push_back(j);
    g.red.push_back(red);
    g.start.push_back(g.start.back() + col_blocks(n0, ns, in2, wd0));
    const double b64 =
        static_cast<double>(ns) * n0 * in2 * 2 * 2 * sizeof(double);
    g.bytes += b64;
    if (P.cur_hm != nullptr) g.jb.push_back({P.cur_hm, {b64, b64, b64}});
  } else if (bulk_u32(h)) {
    // the bulk phase reads its fp32 iterate, and so does the fp64 job of
    // the switch iteration
    ColJob j64 = make_col(h->Uh, T64, ns, in2, 1.0, ctl, -1);
    j64.in32 = u32_view(h);
    col2(0, n0, 1, make_col(u32_view(h), T32, ns, in2, 1.0, ctl, -1), j64,
         1);
  } else {
    col2(0, n0, 1, make_col(h->Uh, T32, ns, in2, 1.0, ctl, -1),
         make_col(h->Uh, T64, ns, in2, 1.0, ctl, -1), 0);
  }
  // input type of the next stage's fp32 job: fp64 after the hosted stage
  const int ti1 = host ? 0 : 1;
  const void* tin32 = host ? static_cast<const void*>(T64)
                           : static_cast<const void*>(T32);
  const long rows = ns * (h->Ns / nl);
  if (d == 2) {
    row2(2, make_row(h, tin32, T32, rows, nh2, nh2, sc, ctl, -1),
         make_row(h, T64, T64, rows, nh2, nh2, sc, ctl, -1), ti1);
  } else {
    const int n1 = h->n[1];
    col2(1, n1, 1, make_col(tin32, T32, ns * n0, h->nh, 1.0, ctl, -1),
         make_col(T64, T64, ns * n0, h->nh, 1.0, ctl, -1), ti1);
    row2(2, make_row(h, T32, T32, rows, nh2, nh2, sc, ctl, -1),
         make_row(h, T64, T64, rows, nh2, nh2, sc, ctl, -1), 1);
    col2(3, n1, -1, make_col(T32, T32, ns * n0, h->nh, 1.0, ctl, -1),
         make_col(T64, T64, ns * n0, h->nh, 1.0, ctl, -1), 1);
  }
  col2(4, n0, -1, make_col(T32, N32, ns, in2, 1.0, ctl, -1),
       make_col(T64, N64, ns, in2, 1.0, ctl, -1), 1);
  return host;
}

// All launches of one fixed-point iteration of instance h, with control
// block `ctl` (device) and host mirror `mirror` (device address).  A
// mixed-precision instance takes its convergence reduction as a launch of
// its own after pass B (its first pass-A stage then writes fp32 in the bulk
// phase); an fp64 one has it ride on that stage (one launch less per
// iteration).  The choice depends on the instance only, so a batched
// instance runs the same kernels on the same data as it does alone.
void plan_iteration(Plan& P, expdiag_ctx* h, Ctl* ctl, Ctl* mirror,
                    double* hist, const Ctl* host_mirror = nullptr) {
  P.cur_hm = host_mirror;
  PassBArgs a = passb_args(h);
  a.ctl = ctl;
  a.hmirror = mirror;
  a.hist = hist;
  if (h->nonlinear && h->mixed) a.Nh32 = nh_view<float>(h);
  const bool hosted =
      h->nonlinear && plan_pass_a_mp(P, h, ctl, a, !h->mixed);
  // pass B variant: 0 radix FFT, 1 dense, 2 EBDF2 dense, 3 EBDF2 radix FFT,
  // 4 radix FFT with complex symbols, 5 the dense kernel of EBDF3..6 (the
  // order read per job), 30 + s the radix FFT kernel of EBDFs (the group
  // length is the transform length for the radix kernels)
  int variant = h->tvariant;
  const int s = bdf_order(h->scheme);
  if (s == 2)
    variant = h->tvariant == 1 ? 2 : 3;
  else if (s > 2)
    variant = h->tvariant == 1 ? 5 : 30 + s;
  else if (variant == 0 && h->cplx)
    variant = 4;
  const int len = variant == 3 || variant > 30 ? time_len(h) : h->Nt;
  plan_passb(P, 5, len, h->Nt, a, sizeof(cx<double>), variant, !hosted);
  P.cur_hm = nullptr;
}

// Whether an iteration replays its captured graph by default.  Measured on
// this GPU with the host enqueueing iterations ahead of the device, the
// replay was slower than launching the same kernels one by one at every
// iterate size, by 3.4-6.5 us per iteration (the 1D 64 x 16 window to the
// 256^2 x 64 instance, fp64 and mixed), with the kernels' own durations
// unchanged: the graph stays captured for callers that ask for it
// (expdiag_set_graph), and a batch measures both on its inputs
// (expdiag_batch_autotune).
constexpr bool GRAPH_REPLAY_DEFAULT = false;

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// Copy every group's job table into the plan's device arena (stream-ordered
// on `st`; the staging buffer is reused only after `st` has synchronised,
// which every caller does before rebuilding a plan).
int plan_upload(expdiag_ctx* h, Plan& P, hipStream_t st) {
  // failure-path tests force an upload failure from the host (as a failed
  // arena allocation would leave it: no device tables)
  if (std::getenv("EXPDIAG_FAIL_PLAN_UPLOAD") != nullptr) {
    P.uploaded = false;
    return fail(h, EXPDIAG_EHIP, "plan upload failed (forced)");
  }
  std::stable_sort(P.groups.begin(), P.groups.end(),
                   [](const Group& x, const Group& y) {
                     return x.stage < y.stage;
                   });
  size_t need = 0;
  for (auto& g : P.groups) {
    const size_t jb = kind_rows(g.kind)   ? g.rj.size() * sizeof(RowJob)
                      : kind_cols(g.kind) ? g.cj.size() * sizeof(ColJob)
                                          : g.pj.size() * sizeof(PassBArgs);
    need += align256(jb) + align256(g.start.size() * sizeof(int)) +
            align256(g.red.size() * sizeof(PassBArgs));
  }
  if (need > P.cap && P.fixed)
    return fail(h, EXPDIAG_EINVAL,
                "launch tables need %zu bytes of a fixed %zu", need, P.cap);
  if (need > P.cap) {
    if (P.arena != nullptr) (void)hipFree(P.arena);
    if (P.staging != nullptr) (void)hipHostFree(P.staging);
    P.arena = nullptr;
    P.staging = nullptr;
    P.cap = 0;
    const size_t cap = std::max<size_t>(need * 2, 64 << 10);
    HIPCHK(h, hipMalloc(&P.arena, cap));
    HIPCHK(h, hipHostMalloc(&P.staging, cap));
    P.cap = cap;
  }
  size_t off = 0;
  for (auto& g : P.groups) {
    size_t jb = 0;
    const void* src = nullptr;
    if (kind_rows(g.kind)) {
      jb = g.rj.size() * sizeof(RowJob);
      src = g.rj.data();
    } else if (kind_cols(g.kind)) {
      jb = g.cj.size() * sizeof(ColJob);
      src = g.cj.data();
    } else {
      jb = g.pj.size() * sizeof(PassBArgs);
      src = g.pj.data();
    }
    std::memcpy(P.staging + off, src, jb);
    g.djobs = P.arena + off;
    off += align256(jb);
    const size_t sb = g.start.size() * sizeof(int);
    std::memcpy(P.staging + off, g.start.data(), sb);
    g.dstart = reinterpret_cast<int*>(P.arena + off);
    off += align256(sb);
    g.dred = nullptr;
    if (!g.red.empty() && g.kind != K_PASSB) {
      const size_t rb = g.red.size() * sizeof(PassBArgs);
      std::memcpy(P.staging + off, g.red.data(), rb);
      g.dred = P.arena + off;
      off += align256(rb);
    }
  }
  // the pass-B groups' reductions in one list (the space the per-group
  // sizes above reserved covers it)
  P.dred_pb = nullptr;
  P.nred_pb = 0;
  P.red_pb_bytes = 0;
  size_t rb_pb = 0;
  for (auto& g : P.groups) {
    if (g.kind != K_PASSB || g.red.empty()) continue;
    const size_t rb = g.red.size() * sizeof(PassBArgs);
    std::memcpy(P.staging + off + rb_pb, g.red.data(), rb);
    rb_pb += rb;
    P.nred_pb += static_cast<int>(g.red.size());
    P.red_pb_bytes += static_cast<double>(g.grid()) * 32;
  }
  if (rb_pb > 0) {
    P.dred_pb = P.arena + off;
    off += align256(rb_pb);
  }
  HIPCHK(h, hipMemcpyAsync(P.arena, P.staging, off, hipMemcpyHostToDevice, st));
  P.uploaded = true;
  return 0;
}

// Drop the plan's groups; keep (keep_arena) or free its arena.
void plan_clear(Plan& P, bool keep_arena) {
  P.groups.clear();
  P.uploaded = false;
  if (!keep_arena && !P.fixed) {
    if (P.arena != nullptr) (void)hipFree(P.arena);
    if (P.staging != nullptr) (void)hipHostFree(P.staging);
    P.arena = nullptr;
    P.staging = nullptr;
    P.cap = 0;
  }
}

void plan_free(Plan& P) { plan_clear(P, false); }

// Launch every group of the plan on `st` in stage order.  `ph` is the handle
// used for profiling and error text (nullable).
int plan_launch(expdiag_ctx* ph, Plan& P, hipStream_t st,
                const cx<double>* tw64, const cx<float>* tw32) {
  // a plan whose job tables are not on the device is never launched
  if (!P.uploaded) return fail(ph, EXPDIAG_EHIP, "plan not uploaded");
  if (ph != nullptr && ph->prof) ++ph->prof_iter;
  for (auto& g : P.groups) {
    const int grid = g.grid();
    if (grid == 0) continue;
    const int nj = g.njobs();
    bool ok = false;
    if (g.kind == K_ROW) {
      ProfScope ps(ph, P_ROW, prof_group_bytes(ph, g, P_ROW), true);
      const RowJob* J = static_cast<const RowJob*>(g.djobs);
      ok = dispatch_pow2<2, NMAX / 2>(g.len, [&](auto Mc) {
        constexpr int MM = decltype(Mc)::value;
        const dim3 th(RowShape<MM>::THREADS);
        if (g.ti == 0)  // 1D: the fp32 job reads the fp64 spectrum
          klaunch(ps, row_kernel_mp<MM, ROW_FUSED, double>, dim3(grid), th, st,
                  J, g.dstart, nj, tw32, tw64);
        else
          klaunch(ps, row_kernel_mp<MM, ROW_FUSED, float>, dim3(grid), th, st,
                  J, g.dstart, nj, tw32, tw64);
      });
    } else if (g.kind == K_COL && g.tcode == 3) {
      ProfScope ps(ph, P_COL, prof_group_bytes(ph, g, P_COL), true);
      const ColJob* J = static_cast<const ColJob*>(g.djobs);
      const PassBArgs* RJ = static_cast<const PassBArgs*>(g.dred);
      const int nred = static_cast<int>(g.red.size());
      ok = dispatch_pow2<4, NMAX>(g.len, [&](auto Lc) {
        constexpr int LL = decltype(Lc)::value;
        if constexpr (LL <= WIDE_LMAX) {
          if (g.wide) {
            klaunch(ps, col_kernel_host<LL, 1, 2>, dim3(grid + nred),
                    dim3(ColShape<LL, 2>::THREADS), st, J, g.dstart, nj, RJ,
                    nred, tw64);
            return;
          }
        }
          klaunch(ps, col_kernel_host<LL, 1>, dim3(grid + nred),
                  dim3(ColShape<LL>::THREADS), st, J, g.dstart, nj, RJ, nred,
                  tw64);
      });
    } else if (g.kind == K_COL) {
      ProfScope ps(ph, P_COL, prof_group_bytes(ph, g, P_COL), true);
      const ColJob* J = static_cast<const ColJob*>(g.djobs);
      auto run = [&](auto Lc, auto Wc) {
        constexpr int LL = decltype(Lc)::value;
        constexpr int WW = decltype(Wc)::value;
        const dim3 th(ColShape<LL, WW>::THREADS);
        // first inverse stage reads the fp64 spectrum; the others read the
        // stage before in the job's own precision
        if (g.mode == 1 && g.ti == 0)
          klaunch(ps, col_kernel_mp<LL, 1, double, WW>, dim3(grid), th, st,
                  J, g.dstart, nj, tw32, tw64);
        else if (g.mode == 1)
          klaunch(ps, col_kernel_mp<LL, 1, float, WW>, dim3(grid), th, st,
                  J, g.dstart, nj, tw32, tw64);
        else
          klaunch(ps, col_kernel_mp<LL, -1, float, WW>, dim3(grid), th, st,
                  J, g.dstart, nj, tw32, tw64);
      };
      ok = dispatch_pow2<4, NMAX>(g.len, [&](auto Lc) {
        constexpr int LL = decltype(Lc)::value;
        if constexpr (LL <= WIDE_LMAX) {
          if (g.wide) {
            run(Lc, std::integral_constant<int, 2>());
            return;
          }
        }
        run(Lc, std::integral_constant<int, 1>());
      });
    } else {
      const PassBArgs* J = static_cast<const PassBArgs*>(g.djobs);
      {
        ProfScope ps(ph, P_PASSB, prof_group_bytes(ph, g, P_PASSB), true);
        if (g.tcode == 1) {
          ok = dispatch_pow2<DENSE_NT_MIN, DENSE_NT_MAX>(g.len, [&](auto Nc) {
            constexpr int NN = decltype(Nc)::value;
            klaunch(ps, passb_dense_kernel<NN, PB_ITERATE, double>, dim3(grid),
                    dim3(DENSE_THREADS), st, J, g.dstart, nj);
          });
        } else if (g.tcode == 2 || g.tcode == 5) {
          ok = dispatch_pow2<DENSE_NT_MIN, DENSE_NT_MAX>(g.len, [&](auto Nc) {
            constexpr int NN = decltype(Nc)::value;
            if (g.tcode == 2)
              klaunch(ps, passb_bdf_kernel<NN, 2>, dim3(grid),
                      dim3(DENSE_THREADS), st, J, g.dstart, nj);
            else
              klaunch(ps, passb_bdf_kernel<NN, 0>, dim3(grid),
                      dim3(DENSE_THREADS), st, J, g.dstart, nj);
          });
        } else if (g.tcode == 3 || g.tcode > 30) {
          ok = dispatch_pow2<2, 512>(g.len, [&](auto Nc) {
            constexpr int NN = decltype(Nc)::value;
            ok = dispatch_bdf_order(g.tcode == 3 ? 2 : g.tcode - 30,
                                    [&](auto Sc) {
              constexpr int SS = decltype(Sc)::value;
              klaunch(ps, passb_bdf_fft_kernel<NN, SS>, dim3(grid),
                      dim3(PassBShape<NN>::THREADS), st, J, g.dstart, nj);
            });
          });
        } else {
          ok = dispatch_pow2<2, 512>(g.len, [&](auto Nc) {
            constexpr int NN = decltype(Nc)::value;
            if (g.tcode == 4)
              klaunch(ps, passb_kernel<NN, PB_ITERATE, double, true>,
                      dim3(grid), dim3(PassBShape<NN>::THREADS), st, J,
                      g.dstart, nj);
            else
              klaunch(ps, passb_kernel<NN, PB_ITERATE, double, false>,
                      dim3(grid), dim3(PassBShape<NN>::THREADS), st, J,
                      g.dstart, nj);
          });
        }
      }
    }
    if (!ok) return fail(ph, EXPDIAG_EUNSUPPORTED, "plan length %d", g.len);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      return fail(ph, EXPDIAG_EHIP, "plan launch: %s", hipGetErrorString(e));
  }
  // the reductions that follow pass B (mixed instances, whose next first
  // stage reads the phase; instances with no pass A) in one launch after
  // the last pass-B group: pass B is the plan's last stage and every
  // instance has its pass B in exactly one group
  if (P.nred_pb > 0) {
    ProfScope pr(ph, P_RED, P.red_pb_bytes, true);
    klaunch(pr, ctl_reduce_kernel, dim3(P.nred_pb), dim3(CTL_THREADS), st,
            static_cast<const PassBArgs*>(P.dred_pb), P.nred_pb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      return fail(ph, EXPDIAG_EHIP, "reduce launch: %s",
                  hipGetErrorString(e));
  }
  return 0;
}

// ------------------------------------------- batched boundary transforms
// fp32 -> fp64 copies of the jobs whose control block says the fp32 copy
// is the current iterate (see widen_bulk_kernel)
__global__ void widen_kernel_jt(const ColJob* __restrict__ jobs,
                                const int* __restrict__ start, int njobs) {
  const int i = find_job(start, njobs);
  const ColJob jb = jobs[i];
  if (jb.ctl->phase > PH_SWITCH) return;
  const long b = static_cast<long>(blockIdx.x - start[i]) * XPB + threadIdx.x;
#pragma unroll
  for (int k = 0; k < XPT; ++k) {
    const long e = b + k * 256;
    if (e < jb.outer)
      static_cast<cx<double>*>(jb.out)[e] =
          cvt<double>(static_cast<const cx<float>*>(jb.in)[e]);
  }
}

// zeros into job j's `outer` 8-byte words at `out`
__global__ void zero_kernel_jt(const ColJob* __restrict__ jobs,
                               const int* __restrict__ start, int njobs) {
  const int i = find_job(start, njobs);
  const ColJob jb = jobs[i];
  const long b = static_cast<long>(blockIdx.x - start[i]) * XPB + threadIdx.x;
#pragma unroll
  for (int k = 0; k < XPT; ++k) {
    const long e = b + k * 256;
    if (e < jb.outer) static_cast<double*>(jb.out)[e] = 0.0;
  }
}

// fp64 -> fp32 copies, job j copying `outer` complex elements
__global__ void narrow_kernel_jt(const ColJob* __restrict__ jobs,
                                 const int* __restrict__ start, int njobs) {
  const int i = find_job(start, njobs);
  const ColJob jb = jobs[i];
  const long b = static_cast<long>(blockIdx.x - start[i]) * XPB + threadIdx.x;
#pragma unroll
  for (int k = 0; k < XPT; ++k) {
    const long e = b + k * 256;
    if (e < jb.outer)
      static_cast<cx<float>*>(jb.out)[e] =
          cvt<float>(static_cast<const cx<double>*>(jb.in)[e]);
  }
}

void plan_xrow(Plan& P, int stage, int M, int mode, const RowJob& j) {
  Group& g = plan_group(P, stage, K_XROW, 0, M, mode, 0, 0);
  g.rj.push_back(j);
  g.start.push_back(g.start.back() + row_blocks(M, j.nrows));
  g.bytes += row_bytes(M, mode, j.nrows, sizeof(double), sizeof(double));
}

void plan_xcol(Plan& P, int stage, int L, int S, const ColJob& j) {
  Group& g = plan_group(P, stage, K_XCOL, 0, L, S, 0, 0);
  g.cj.push_back(j);
  g.start.push_back(g.start.back() + col_blocks(L, j.outer, j.inner));
  g.bytes += static_cast<double>(j.outer) * L * j.inner * 32;
}

// ns real slices at src -> their half spectra at dst: rows written straight
// into dst, then the column stages in place there (stages stage0..+2)
void plan_xfwd(Plan& P, expdiag_ctx* h, int stage0, int rowmode,
               const double* src, cx<double>* dst, long ns) {
  const int d = h->dim;
  const long nh2 = 2L * h->nh;
  const int nl = h->n[d - 1];
  plan_xrow(P, stage0, nl / 2, rowmode,
            make_row(h, src, dst, ns * (h->Ns / nl), nl, nh2, 1.0, nullptr,
                     -1));
  if (d == 2) {
    plan_xcol(P, stage0 + 1, h->n[0], -1,
              make_col(dst, dst, ns, h->nh, 1.0, nullptr, -1));
  } else if (d == 3) {
    plan_xcol(P, stage0 + 1, h->n[1], -1,
              make_col(dst, dst, ns * h->n[0], h->nh, 1.0, nullptr, -1));
    plan_xcol(P, stage0 + 2, h->n[0], -1,
              make_col(dst, dst, ns, static_cast<long>(h->n[1]) * h->nh, 1.0,
                       nullptr, -1));
  }
}

// What expdiag_iterate does before its iterations (prepare_u0 and the
// forward transform of U), as plan stages 0..3; real states only.
// Entry transforms of one instance as plan stages; `zero`: the solve starts
// from U = 0, so its spectral iterate (or its fp32 bulk copy, where the
// instance keeps one) is cleared rather than transformed from U
// (enter_guess)
void plan_entry(Plan& P, expdiag_ctx* h, const double* u0, const double* U,
                bool zero) {
  plan_xfwd(P, h, 0, ROW_R2C, u0, h->u0h, 1);
  if (h->nonlinear && h->scheme != EXPDIAG_IF1) {
    plan_xfwd(P, h, 0, ROW_NR2C, u0, h->Nh, 1);
    if (h->mixed) {
      Group& g = plan_group(P, 3, K_XNARROW, 0, 0, 0, 0, 0);
      g.cj.push_back(make_col(h->Nh, nh_view<float>(h), h->Nk, 1, 1.0,
                              nullptr, -1));
      g.start.push_back(g.start.back() +
                        xblocks(h->Nk));
    }
  }
  const long n = static_cast<long>(h->Nt) * h->Nk;
  if (zero) {
    Group& g = plan_group(P, 3, K_XZERO, 0, 0, 0, 0, 0);
    auto add = [&](void* p, long words) {
      g.cj.push_back(make_col(nullptr, p, words, 1, 1.0, nullptr, -1));
      g.start.push_back(g.start.back() +
                        xblocks(words));
    };
    // (Uh of an instance that keeps the fp32 bulk iterate is written
    // before it is read: enter_guess)
    if (bulk_u32(h))
      add(u32_view(h), n);
    else
      add(h->Uh, 2 * n);
    if (zero_start_ok(h)) {
      void* p = nullptr;
      long w = 0;
      zero_start_region(h, &p, &w);
      add(p, w);
    }
    return;
  }
  plan_xfwd(P, h, 0, ROW_R2C, U, h->Uh, h->Nt);
  if (bulk_u32(h)) {
    Group& g = plan_group(P, 3, K_XNARROW, 0, 0, 0, 0, 0);
    g.cj.push_back(make_col(h->Uh, u32_view(h), n, 1, 1.0, nullptr, -1));
    g.start.push_back(g.start.back() + xblocks(n));
  }
}

// leave_bulk_state (stage 0, gated on the control block `ctl`) and
// inv_slices(h, h->Uh, U, Nt) (stages 1..3, through h->T) as plan stages
void plan_exit(Plan& P, expdiag_ctx* h, double* U, const Ctl* ctl) {
  const int d = h->dim;
  const long nh2 = 2L * h->nh;
  const int nl = h->n[d - 1];
  const double sc = 1.0 / static_cast<double>(h->Ns);
  const long ns = h->Nt;
  if (bulk_u32(h)) {
    Group& g = plan_group(P, 0, K_XWIDEN, 0, 0, 0, 0, 0);
    const long n = ns * h->Nk;
    g.cj.push_back(make_col(u32_view(h), h->Uh, n, 1, 1.0, ctl, -1));
    g.start.push_back(g.start.back() + xblocks(n));
  }
  if (d == 1) {
    plan_xrow(P, 3, nl / 2, ROW_C2R,
              make_row(h, h->Uh, U, ns, nh2, nl, sc, nullptr, -1));
    return;
  }
  if (d == 2) {
    plan_xcol(P, 1, h->n[0], 1,
              make_col(h->Uh, h->T, ns, h->nh, 1.0, nullptr, -1));
  } else {
    plan_xcol(P, 1, h->n[0], 1,
              make_col(h->Uh, h->T, ns, static_cast<long>(h->n[1]) * h->nh,
                       1.0, nullptr, -1));
    plan_xcol(P, 2, h->n[1], 1,
              make_col(h->T, h->T, ns * h->n[0], h->nh, 1.0, nullptr, -1));
  }
  plan_xrow(P, 3, nl / 2, ROW_C2R,
            make_row(h, h->T, U, ns * (h->Ns / nl), nh2, nl, sc, nullptr,
                     -1));
}

// Launch the groups of a boundary-transform plan in stage order.
int plan_launch_x(expdiag_ctx* ph, Plan& P, hipStream_t st,
                  const cx<double>* tw64) {
  if (!P.uploaded) return fail(ph, EXPDIAG_EHIP, "plan not uploaded");
  for (auto& g : P.groups) {
    const int grid = g.grid();
    if (grid == 0) continue;
    const int nj = g.njobs();
    bool ok = false;
    if (g.kind == K_XROW) {
      const RowJob* J = static_cast<const RowJob*>(g.djobs);
      ok = dispatch_pow2<2, NMAX / 2>(g.len, [&](auto Mc) {
        constexpr int MM = decltype(Mc)::value;
        const dim3 th(RowShape<MM>::THREADS);
        if (g.mode == ROW_R2C)
          hipLaunchKernelGGL((row_kernel_jt<MM, ROW_R2C>), dim3(grid), th, 0,
                             st, J, g.dstart, nj, tw64);
        else if (g.mode == ROW_NR2C)
          hipLaunchKernelGGL((row_kernel_jt<MM, ROW_NR2C>), dim3(grid), th,
                             0, st, J, g.dstart, nj, tw64);
        else
          hipLaunchKernelGGL((row_kernel_jt<MM, ROW_C2R>), dim3(grid), th, 0,
                             st, J, g.dstart, nj, tw64);
      });
    } else if (g.kind == K_XCOL) {
      const ColJob* J = static_cast<const ColJob*>(g.djobs);
      ok = dispatch_pow2<4, NMAX>(g.len, [&](auto Lc) {
        constexpr int LL = decltype(Lc)::value;
        const dim3 th(ColShape<LL>::THREADS);
        if (g.mode == 1)
          hipLaunchKernelGGL((col_kernel_jt<LL, 1>), dim3(grid), th, 0, st,
                             J, g.dstart, nj, tw64);
        else
          hipLaunchKernelGGL((col_kernel_jt<LL, -1>), dim3(grid), th, 0, st,
                             J, g.dstart, nj, tw64);
      });
    } else if (g.kind == K_XNARROW) {
      hipLaunchKernelGGL(narrow_kernel_jt, dim3(grid), dim3(256), 0, st,
                         static_cast<const ColJob*>(g.djobs), g.dstart, nj);
      ok = true;
    } else if (g.kind == K_XWIDEN) {
      hipLaunchKernelGGL(widen_kernel_jt, dim3(grid), dim3(256), 0, st,
                         static_cast<const ColJob*>(g.djobs), g.dstart, nj);
      ok = true;
    } else if (g.kind == K_XZERO) {
      hipLaunchKernelGGL(zero_kernel_jt, dim3(grid), dim3(256), 0, st,
                         static_cast<const ColJob*>(g.djobs), g.dstart, nj);
      ok = true;
    }
    if (!ok) return fail(ph, EXPDIAG_EUNSUPPORTED, "transform length %d",
                         g.len);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      return fail(ph, EXPDIAG_EHIP, "transform launch: %s",
                  hipGetErrorString(e));
  }
  return 0;
}

// After the last iteration of a chunk: the convergence reduction of every
// instance whose pass B has not been reduced yet (those hosted by the next
// iteration's first stage), so the control blocks are current when the
// host looks.
int plan_finish(expdiag_ctx* ph, Plan& P, hipStream_t st) {
  if (!P.uploaded) return fail(ph, EXPDIAG_EHIP, "plan not uploaded");
  for (auto& g : P.groups) {
    if (g.kind != K_PASSB || g.njobs() == 0) continue;
    ProfScope pr(ph, P_RED, static_cast<double>(g.grid()) * 32, true);
    klaunch(pr, ctl_reduce_kernel, dim3(g.njobs()), dim3(CTL_THREADS), st,
            static_cast<const PassBArgs*>(g.djobs), g.njobs());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      return fail(ph, EXPDIAG_EHIP, "reduce launch: %s",
                  hipGetErrorString(e));
  }
  return 0;
}

// Capture one iteration of plan P into an executable graph.
int plan_capture(expdiag_ctx* h, Plan& P, hipStream_t cap,
                 const cx<double>* tw64, const cx<float>* tw32,
                 hipGraph_t* graph, hipGraphExec_t* exec) {
  HIPCHK(h, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  int rc = plan_launch(nullptr, P, cap, tw64, tw32);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cap, &g);
  if (rc != 0) {
    if (g != nullptr) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess)
    return fail(h, EXPDIAG_EHIP, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(h, EXPDIAG_EHIP, "graph instantiate: %s",
                hipGetErrorString(e));
  }
  *graph = g;
  return 0;
}

// ------------------------------------------------------------------ tables
long double phi1l(long double z) {
  if (z == 0.0L) return 1.0L;
  return expm1l(z) / z;
}

// 1/n!, n = 0..39 (once per process)
const long double* inv_factorials() {
  static const std::vector<long double> f = [] {
    std::vector<long double> v(40);
    long double fact = 1.0L;
    for (int i = 0; i < 40; ++i) {
      if (i > 0) fact *= i;
      v[i] = 1.0L / fact;
    }
    return v;
  }();
  return f.data();
}

long double phi2l(long double z) {
  if (fabsl(z) < 1.0L) {
    // sum_{j>=0} z^j / (j+2)!, Horner from the tail
    const long double* inv = inv_factorials();
    long double acc = 0.0L;
    for (int j = 35; j >= 0; --j) acc = acc * z + inv[j + 2];
    return acc;
  }
  return (expm1l(z) - z) / (z * z);
}

// exp(-2 pi i j / TW_N), j < TW_N, in fp64 and fp32 (once per process)
struct TwiddleTables {
  std::vector<cx<double>> d;
  std::vector<cx<float>> f;
};
const TwiddleTables& twiddle_tables() {
  static const TwiddleTables t = [] {
    TwiddleTables r;
    r.d.resize(TW_N);
    r.f.resize(TW_N);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int j = 0; j < TW_N; ++j) {
      const long double th = -2.0L * pi * j / TW_N;
      const long double cr = cosl(th), si = sinl(th);
      r.d[j] = mk<double>(static_cast<double>(cr), static_cast<double>(si));
      r.f[j] = mk<float>(static_cast<float>(cr), static_cast<float>(si));
    }
    return r;
  }();
  return t;
}

using cld = std::complex<long double>;

// phi1, phi2 of a complex argument: power series for |z| < 1 (Horner from
// the tail, 36 terms), the closed forms beyond.
cld phi1c(cld z) {
  const long double* inv = inv_factorials();
  if (std::abs(z) < 1.0L) {
    cld acc = 0.0L;
    for (int j = 35; j >= 0; --j) acc = acc * z + inv[j + 1];
    return acc;
  }
  return (std::exp(z) - 1.0L) / z;
}
cld phi2c(cld z) {
  const long double* inv = inv_factorials();
  if (std::abs(z) < 1.0L) {
    cld acc = 0.0L;
    for (int j = 35; j >= 0; --j) acc = acc * z + inv[j + 2];
    return acc;
  }
  return (std::exp(z) - 1.0L - z) / (z * z);
}

cx<double> to_cx(cld v) {
  return mk(static_cast<double>(v.real()), static_cast<double>(v.imag()));
}

// Runs f(lo, hi) over [0, n) on up to eight host threads.
template <typename F>
void parallel_ranges(long n, F&& f) {
  const int nthr = n < 4096 ? 1 : 8;
  if (nthr == 1) {
    f(0L, n);
    return;
  }
  std::vector<std::thread> th;
  for (int k = 0; k < nthr; ++k)
    th.emplace_back(f, n * k / nthr, n * (k + 1) / nthr);
  for (auto& t : th) t.join();
}

// Per-kappa tables E = e^{dt mu}, c1, c2 (eq. etd1_update / etd2_update
// weights), mu = -a |k|^2 - c - i b.k' (- i a_im |k|^2 - i c_im for complex
// coefficients).  k' is the derivative wavenumber: k, except 0 at the
// Nyquist index of its axis (so that b.grad maps real fields to real
// fields).  A kappa index i is (i0, i1, kl) of [n0][n1][nh] (the dims
// present), kl the last-axis index (half spectrum: 0..n/2; full spectrum
// of a complex state: 0..n-1).
//
// Without advection or complex coefficients the tables depend on kappa
// only through the integer |k|^2: each value that occurs (a sum of one
// square per axis) is evaluated once, in long double, and the device
// gathers the per-kappa tables (symbol_gather_kernel), so the host work
// does not grow with the number of modes.  Otherwise every kappa is
// evaluated on the host (complex long double).  Host threads: up to eight.
struct SymbolTables {
  bool per_kappa = false;                 // E, c1, c2 below, per kappa
  std::vector<cx<double>> E, c1, c2;
  std::vector<int> slot;                  // |k|^2 -> value index
  std::vector<double> vals;               // [3][nv]: E, c1, c2 per |k|^2
};

bool complex_symbols(const expdiag_ctx* h) {
  const double* bv = h->p.b;
  const int d = h->dim;
  return (bv[0] != 0.0) || (d >= 2 && bv[1] != 0.0) ||
         (d >= 3 && bv[2] != 0.0) || h->p.a_im != 0.0 || h->p.c_im != 0.0;
}

void symbol_tables(expdiag_ctx* h, SymbolTables& st) {
  const int d = h->dim;
  const long Nk = h->Nk;
  const int n0 = h->n[0], n1 = d >= 2 ? h->n[1] : 1;
  const int outer1 = d >= 3 ? n1 : 1;
  const int nl = h->n[d - 1];
  auto wn = [](int j, int n) { return j <= n / 2 ? j : j - n; };
  auto wd = [](int j, int n) { return 2 * j == n ? 0 : (j < n / 2 ? j : j - n); };
  const long double a = h->p.a, c = h->p.c, dt = h->dt;
  const long double ai = h->p.a_im, ci = h->p.c_im;
  const bool etd2 = h->scheme == EXPDIAG_ETD2;
  const bool if1 = h->scheme == EXPDIAG_IF1;
  const double* bv = h->p.b;
  if (complex_symbols(h)) {
    st.per_kappa = true;
    st.E.resize(Nk);
    st.c1.resize(Nk);
    st.c2.resize(Nk);
    auto eval = [&](long lo, long hi) {
      for (long i = lo; i < hi; ++i) {
        const int kl = static_cast<int>(i % h->nh);
        const long r = i / h->nh;
        const int i1 = d >= 3 ? static_cast<int>(r % outer1) : 0;
        const int i0 = d >= 2 ? static_cast<int>(d >= 3 ? r / outer1 : r) : 0;
        long double k2 = static_cast<long double>(wn(kl, nl)) * wn(kl, nl);
        long double bk = bv[d - 1] * static_cast<long double>(wd(kl, nl));
        if (d >= 2) {
          k2 += static_cast<long double>(wn(i0, n0)) * wn(i0, n0);
          bk += bv[0] * static_cast<long double>(wd(i0, n0));
        }
        if (d >= 3) {
          k2 += static_cast<long double>(wn(i1, n1)) * wn(i1, n1);
          bk += bv[1] * static_cast<long double>(wd(i1, n1));
        }
        const cld z = dt * cld(-a * k2 - c, -bk - ai * k2 - ci);
        // IF1 weighs N(u_n) by dt itself (eq. fully_discrete_nonlinear)
        const cld w1 = if1 ? cld(dt) : dt * phi1c(z);
        st.E[i] = to_cx(std::exp(z));
        if (etd2) {
          const cld w2 = dt * phi2c(z);
          st.c1[i] = to_cx(w1 + w2);
          st.c2[i] = to_cx(-w2);
        } else {
          st.c1[i] = to_cx(w1);
          st.c2[i] = mk(0.0, 0.0);
        }
      }
    };
    parallel_ranges(Nk, eval);
    return;
  }
  // |k|^2 = s0 + s1 + s2, one square j^2 (j = 0..n/2) per axis present
  const long h0 = d >= 2 ? n0 / 2 : 0, h1 = d >= 3 ? n1 / 2 : 0;
  const long hl = nl / 2;
  const long k2max = h0 * h0 + h1 * h1 + hl * hl;
  std::vector<char> present(k2max + 1, 0);
  for (long j0 = 0; j0 <= h0; ++j0)
    for (long j1 = 0; j1 <= h1; ++j1)
      for (long jl = 0; jl <= hl; ++jl) present[j0 * j0 + j1 * j1 + jl * jl] = 1;
  st.slot.assign(k2max + 1, -1);
  std::vector<long> vals;
  for (long v = 0; v <= k2max; ++v) {
    if (present[v]) {
      st.slot[v] = static_cast<int>(vals.size());
      vals.push_back(v);
    }
  }
  const long nv = static_cast<long>(vals.size());
  st.vals.assign(3 * nv, 0.0);
  double* tE = st.vals.data();
  double* t1 = tE + nv;
  double* t2 = t1 + nv;
  auto eval = [&](long lo, long hi) {
    for (long i = lo; i < hi; ++i) {
      const long double z = dt * (-a * static_cast<long double>(vals[i]) - c);
      const long double w1 = if1 ? dt : dt * phi1l(z);
      tE[i] = static_cast<double>(expl(z));
      if (etd2) {
        const long double w2 = dt * phi2l(z);
        t1[i] = static_cast<double>(w1 + w2);
        t2[i] = static_cast<double>(-w2);
      } else {
        t1[i] = static_cast<double>(w1);
        t2[i] = 0.0;
      }
    }
  };
  parallel_ranges(nv, eval);
}

// Per-kappa real tables from the per-|k|^2 values: kappa -> (i0, i1, kl)
// -> |k|^2 -> slot -> value (the same integer |k|^2 the host enumerated).
__global__ void symbol_gather_kernel(cx<double>* __restrict__ E,
                                     cx<double>* __restrict__ c1,
                                     cx<double>* __restrict__ c2, long Nk,
                                     int dim, int n0, int n1, int nl, int nh,
                                     const int* __restrict__ slot,
                                     const double* __restrict__ vals,
                                     int nv) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= Nk) return;
  const int kl = static_cast<int>(i % nh);
  const long r = i / nh;
  const int i1 = dim >= 3 ? static_cast<int>(r % n1) : 0;
  const int i0 = dim >= 2 ? static_cast<int>(dim >= 3 ? r / n1 : r) : 0;
  const long wl = kl <= nl / 2 ? kl : kl - nl;
  long k2 = wl * wl;
  if (dim >= 2) {
    const long w0 = i0 <= n0 / 2 ? i0 : i0 - n0;
    k2 += w0 * w0;
  }
  if (dim >= 3) {
    const long w1 = i1 <= n1 / 2 ? i1 : i1 - n1;
    k2 += w1 * w1;
  }
  const int j = slot[k2];
  E[i] = mk(vals[j], 0.0);
  c1[i] = mk(vals[nv + j], 0.0);
  c2[i] = mk(vals[2 * nv + j], 0.0);
}

int build_tables(expdiag_ctx* h) {
  const long Nk = h->Nk;
  SymbolTables sym;
  symbol_tables(h, sym);
  const int Nt = h->Nt;
  // The transform runs over N time points: Nt, or for an order-s
  // exponential BDF the N = Nt - s + 1 unknown slices s..Nt, which sit at
  // row offset o = s - 1 of a window.
  const int N = time_len(h);
  const int o = Nt - N;
  std::vector<double> gam(Nt, 1.0), igam(Nt, 1.0);
  std::vector<cx<double>> lam(Nt, mk(0.0, 0.0));
  // e^{2 pi i j/N}, j < N: every angle the time tables use
  std::vector<long double> cs(N), sn(N);
  const long double la = logl(static_cast<long double>(h->alpha));
  const long double pi = 3.141592653589793238462643383279502884L;
  const long double root = expl(la / N);
  std::vector<long double> gl(N);
  for (int l = 0; l < N; ++l) {
    const long double th = 2.0L * pi * l / N;
    cs[l] = cosl(th);
    sn[l] = sinl(th);
    gl[l] = expl(la * l / N);
    gam[l] = static_cast<double>(gl[l]);
    igam[l] = static_cast<double>(1.0L / gl[l]);
    lam[l] = mk<double>(static_cast<double>(root * cs[l]),
                        static_cast<double>(root * sn[l]));
  }
  if (h->roots != nullptr) {
    std::vector<cx<double>> rt(N);
    for (int j = 0; j < N; ++j)
      rt[j] = mk<double>(static_cast<double>(cs[j]), static_cast<double>(sn[j]));
    HIPCHK(h, hipMemcpy(h->roots, rt.data(), N * sizeof(cx<double>),
                        hipMemcpyHostToDevice));
  }
  h->cplx = complex_symbols(h);
  const TwiddleTables& tw = twiddle_tables();
  // the per-|k|^2 values and slots are staged in the handle's scratch T
  // (idle while tables are built) and gathered on the handle's stream
  const size_t slot_bytes =
      ((sym.slot.size() * sizeof(int) + 15) / 16) * 16;
  const size_t stage_bytes = slot_bytes + sym.vals.size() * sizeof(double);
  const size_t t_bytes = static_cast<size_t>(h->Nt) * Nk * sizeof(cx<double>);
  if (!sym.per_kappa && stage_bytes > t_bytes) {
    // (only grids too small for the staging area) gather on the host
    const long nv = static_cast<long>(sym.vals.size() / 3);
    sym.E.resize(Nk);
    sym.c1.resize(Nk);
    sym.c2.resize(Nk);
    const int d = h->dim, n0 = h->n[0], n1 = d >= 2 ? h->n[1] : 1;
    const int nl = h->n[d - 1];
    auto wn = [](long j, long n) { return j <= n / 2 ? j : j - n; };
    for (long i = 0; i < Nk; ++i) {
      const long kl = i % h->nh, r = i / h->nh;
      const long i1 = d >= 3 ? r % n1 : 0;
      const long i0 = d >= 2 ? (d >= 3 ? r / n1 : r) : 0;
      long k2 = wn(kl, nl) * wn(kl, nl);
      if (d >= 2) k2 += wn(i0, n0) * wn(i0, n0);
      if (d >= 3) k2 += wn(i1, n1) * wn(i1, n1);
      const int j = sym.slot[k2];
      sym.E[i] = mk(sym.vals[j], 0.0);
      sym.c1[i] = mk(sym.vals[nv + j], 0.0);
      sym.c2[i] = mk(sym.vals[2 * nv + j], 0.0);
    }
    sym.per_kappa = true;
  }
  if (sym.per_kappa) {
    HIPCHK(h, hipMemcpy(h->E, sym.E.data(), Nk * sizeof(cx<double>),
                        hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->c1, sym.c1.data(), Nk * sizeof(cx<double>),
                        hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(h->c2, sym.c2.data(), Nk * sizeof(cx<double>),
                        hipMemcpyHostToDevice));
  } else {
    char* stage = reinterpret_cast<char*>(h->T);
    HIPCHK(h, hipMemcpy(stage, sym.slot.data(), sym.slot.size() * sizeof(int),
                        hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(stage + slot_bytes, sym.vals.data(),
                        sym.vals.size() * sizeof(double),
                        hipMemcpyHostToDevice));
    const int d = h->dim;
    hipLaunchKernelGGL(symbol_gather_kernel, dim3((Nk + 255) / 256),
                       dim3(256), 0, h->stream, h->E, h->c1, h->c2, Nk, d,
                       h->n[0], d >= 2 ? h->n[1] : 1, h->n[d - 1], h->nh,
                       reinterpret_cast<const int*>(stage),
                       reinterpret_cast<const double*>(stage + slot_bytes),
                       static_cast<int>(sym.vals.size() / 3));
    HIPCHK(h, hipGetLastError());
  }
  HIPCHK(h, hipMemcpy(h->gam, gam.data(), Nt * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->igam, igam.data(), Nt * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->lam, lam.data(), Nt * sizeof(cx<double>), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->tw64, tw.d.data(), TW_N * sizeof(cx<double>), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->tw32, tw.f.data(), TW_N * sizeof(cx<float>), hipMemcpyHostToDevice));
  return 0;
}

struct Sizes {
  long Ns, Nk, nh;
};

int check_grid(const expdiag_grid* g, Sizes* sz) {
  if (g == nullptr || g->dim < 1 || g->dim > 3) return EXPDIAG_EINVAL;
  long Ns = 1;
  for (int i = 0; i < g->dim; ++i) {
    if (g->n[i] < 4 || (g->n[i] & 1)) return EXPDIAG_EINVAL;
    if (!is_pow2(g->n[i]) || g->n[i] > NMAX) return EXPDIAG_EUNSUPPORTED;
    Ns *= g->n[i];
  }
  const long nh = g->n[g->dim - 1] / 2 + 1;
  sz->Ns = Ns;
  sz->nh = nh;
  sz->Nk = Ns / g->n[g->dim - 1] * nh;
  return 0;
}

size_t footprint(const Sizes& s, int dim, int Nt, bool nonlinear,
                 bool mixed, int restart) {
  const size_t st = static_cast<size_t>(Nt) * s.Nk * sizeof(cx<double>);
  size_t b = 2 * st;                   // Uh, T
  if (nonlinear) b += st;              // Nh
  if (nonlinear && mixed && dim >= 2) b += st;  // T32, U32
  if (restart > 0) {
    b += st;                                          // T2
    b += static_cast<size_t>(restart + 1) * st;       // Krylov basis
    b += static_cast<size_t>((static_cast<long>(Nt) * s.Nk + KRY_PER_BLOCK -
                              1) / KRY_PER_BLOCK) *
         (4 * restart + 4) * sizeof(double);  // block partials
    if (nonlinear)
      b += static_cast<size_t>(Nt) * s.Ns * (sizeof(double) + sizeof(float));
  }
  b += s.Nk * 4 * sizeof(cx<double>);  // u0^, E, c1, c2
  b += TW_N * (sizeof(cx<double>) + sizeof(cx<float>));
  b += static_cast<size_t>(std::max(std::max(passb_blocks_nt(Nt, s.Nk),
                                             passb_blocks_nt(Nt - 1, s.Nk)),
                                    dft_blocks(Nt, s.Nk))) * 4 * sizeof(double);
  if (dense_ok(Nt)) b += static_cast<size_t>(Nt) * sizeof(cx<double>);
  return b;
}

template <typename P>
int dalloc(expdiag_ctx* h, P** ptr, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  if (h->arena != nullptr) {
    const size_t need = align256(bytes);
    if (h->arena_off + need > h->arena_cap)
      return fail(h, EXPDIAG_EINVAL,
                  "workspace of %zu bytes exceeded (needs more than %zu)",
                  h->arena_cap, h->arena_off + need);
    *ptr = reinterpret_cast<P*>(h->arena + h->arena_off);
    h->arena_off += need;
    h->bytes += need;
    return 0;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, EXPDIAG_ENOMEM, "hipMalloc(%zu): %s", bytes,
                hipGetErrorString(e));
  }
  *ptr = static_cast<P*>(p);
  h->bytes += bytes;
  return 0;
}

void release(expdiag_ctx* h) {
  auto fr = [](void* p) {
    if (p != nullptr) (void)hipFree(p);
  };
  if (h->gexec != nullptr) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph != nullptr) (void)hipGraphDestroy(h->graph);
  plan_free(h->plan);
  fr(h->Uh);
  fr(h->Nh);
  fr(h->T);
  fr(h->T2);
  fr(h->T32);
  fr(h->U32);
  fr(h->Uphys);
  fr(h->Uphys32);
  fr(h->u0h);
  fr(h->E);
  fr(h->c1);
  fr(h->c2);
  fr(h->gam);
  fr(h->igam);
  fr(h->lam);
  fr(h->tw64);
  fr(h->tw32);
  fr(h->roots);
  fr(h->partials);
  fr(h->red_out);
  fr(h->ctl);
  fr(h->hist);
  fr(h->V);
  fr(h->kdots);
  fr(h->kpart);
  if (h->h_ctl != nullptr) (void)hipHostFree(h->h_ctl);
  if (h->h_mirror != nullptr) (void)hipHostFree(h->h_mirror);
  if (h->h_red != nullptr) (void)hipHostFree(h->h_red);
  if (h->h_kdots != nullptr) (void)hipHostFree(h->h_kdots);
  if (h->cap_stream != nullptr) (void)hipStreamDestroy(h->cap_stream);
  for (auto& e : h->chunk_ev)
    if (e != nullptr) (void)hipEventDestroy(e);
  for (auto& e : h->events) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  h->events.clear();
}

// Snapshot of a host-mapped control block written by the device.  Read
// while later iterations run, fields may come from two different updates;
// callers use such snapshots only to size the next chunk and take final
// results after synchronising the stream.
Ctl read_mirror(const Ctl* p) {
  Ctl c;
  std::memcpy(&c, static_cast<const void*>(p), sizeof(Ctl));
  return c;
}

Ctl initial_ctl(expdiag_ctx* h, int max_iter, double tol) {
  Ctl c{};
  c.done = 0;
  c.iters = 0;
  c.max_iter = max_iter;
  c.phase = (h->mixed && h->nonlinear) ? PH_BULK : PH_FP64;
  c.tol = tol;
  c.bulk_tol = BULK_TOL;
  c.last_rel = 0.0;
  return c;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* expdiag_strerror(int code) {
  switch (code) {
    case EXPDIAG_OK:
      return "ok";
    case EXPDIAG_NOT_CONVERGED:
      return "tolerance not reached within the iteration cap";
    case EXPDIAG_EINVAL:
      return "invalid argument";
    case EXPDIAG_ENOMEM:
      return "device memory allocation failed";
    case EXPDIAG_EHIP:
      return "HIP runtime error";
    case EXPDIAG_EDIVERGED:
      return "iteration diverged (non-finite residual)";
    case EXPDIAG_EUNSUPPORTED:
      return "size not supported by the library";
    default:
      return "unknown error code";
  }
}

const char* expdiag_last_error(expdiag_t h) {
  if (h == nullptr) return g_create_err.c_str();
  return h->err.c_str();
}

size_t expdiag_footprint_bytes(const expdiag_grid* g, int Nt, int scheme,
                               int precision, int gmres_restart) {
  Sizes s{};
  if (check_grid(g, &s) != 0) return 0;
  if (scheme != EXPDIAG_ETD1 && scheme != EXPDIAG_ETD2 &&
      scheme != EXPDIAG_IF1 && bdf_order(scheme) == 0)
    return 0;
  if (bdf_order(scheme) > 0) {
    if (!bdf_ok(Nt, bdf_order(scheme))) return 0;
  } else if (!is_pow2(Nt) || Nt < 2 || Nt > 512) {
    return 0;
  }
  if (precision != EXPDIAG_FP64 && precision != EXPDIAG_MIXED) return 0;
  if (gmres_restart < 0 || gmres_restart > 64) return 0;
  // the nonlinearity is not known here: report the nonlinear footprint
  // (the exponential BDF schemes are linear only)
  return footprint(s, g->dim, Nt, bdf_order(scheme) == 0,
                   precision == EXPDIAG_MIXED, gmres_restart);
}

}  // extern "C"

namespace {

int validate_params(int Nt, double dt, double alpha, int scheme,
                    const expdiag_problem* p) {
  if (Nt < 2) return fail(nullptr, EXPDIAG_EINVAL, "Nt must be >= 2");
  const int bs = bdf_order(scheme);
  if (bs == 0 && (!is_pow2(Nt) || Nt > 512))
    return fail(nullptr, EXPDIAG_EUNSUPPORTED,
                "Nt must be a power of two <= 512");
  if (!(dt > 0.0) || !std::isfinite(dt))
    return fail(nullptr, EXPDIAG_EINVAL, "dt must be > 0");
  if (!(alpha > 0.0 && alpha < 1.0))
    return fail(nullptr, EXPDIAG_EINVAL, "alpha must lie in (0, 1)");
  if (scheme != EXPDIAG_ETD1 && scheme != EXPDIAG_ETD2 &&
      scheme != EXPDIAG_IF1 && bs == 0)
    return fail(nullptr, EXPDIAG_EINVAL, "unknown scheme %d", scheme);
  if (p->jacobian < 0 || p->jacobian > 2)
    return fail(nullptr, EXPDIAG_EINVAL, "jacobian must be 0, 1 or 2");
  if (bs > 0 && (p->n1 != 0.0 || p->n2 != 0.0 || p->n3 != 0.0))
    return fail(nullptr, EXPDIAG_EUNSUPPORTED,
                "EBDF%d is for linear problems (n1 = n2 = n3 = 0)", bs);
  if (bs > 0 && !bdf_ok(Nt, bs))
    return fail(nullptr, EXPDIAG_EUNSUPPORTED,
                "EBDF%d needs Nt - %d a power of two in 2..512, or Nt a "
                "power of two in %d..%d", bs, bs - 1, DENSE_NT_MIN,
                DENSE_NT_MAX);
  if (!(p->a >= 0.0) || !(p->c >= 0.0) || !std::isfinite(p->a) ||
      !std::isfinite(p->c) || !std::isfinite(p->n1) ||
      !std::isfinite(p->n2) || !std::isfinite(p->n3))
    return fail(nullptr, EXPDIAG_EINVAL, "a, c must be finite and >= 0");
  if (!std::isfinite(p->b[0]) || !std::isfinite(p->b[1]) ||
      !std::isfinite(p->b[2]) || !std::isfinite(p->a_im) ||
      !std::isfinite(p->c_im))
    return fail(nullptr, EXPDIAG_EINVAL,
                "advection velocity and imaginary parts must be finite");
  if (p->complex_state != 0 && p->complex_state != 1)
    return fail(nullptr, EXPDIAG_EINVAL, "complex_state must be 0 or 1");
  if ((p->a_im != 0.0 || p->c_im != 0.0) && p->complex_state == 0)
    return fail(nullptr, EXPDIAG_EINVAL,
                "complex coefficients need complex_state = 1");
  if (p->complex_state == 1 && (p->n1 != 0.0 || p->n2 != 0.0 || p->n3 != 0.0))
    return fail(nullptr, EXPDIAG_EUNSUPPORTED,
                "a complex state is for linear problems");
  if (p->precision != EXPDIAG_FP64 && p->precision != EXPDIAG_MIXED)
    return fail(nullptr, EXPDIAG_EINVAL, "unknown precision %d",
                p->precision);
  if (p->gmres_restart < 0 || p->gmres_restart > 64)
    return fail(nullptr, EXPDIAG_EINVAL, "gmres_restart must be 0..64");
  return 0;
}

// New coefficients for an existing handle of the same grid, Nt,
// nonlinearity and precision (buffers unchanged; tables rebuilt).
int reinit_params(expdiag_ctx* h, double dt, double alpha, int scheme,
                  const expdiag_problem* p) {
  RCHK(validate_params(h->Nt, dt, alpha, scheme, p));
  if ((p->complex_state == 1) != h->cstate)
    return fail(h, EXPDIAG_EINVAL, "complex_state differs from the handle's");
  const int old_scheme = h->scheme, old_tv = h->tvariant;
  const int bs = bdf_order(scheme);
  if (bs > 0)
    h->tvariant = bdf_fft_ok(h->Nt, bs) ? 0 : 1;  // by N = Nt - s + 1
  else if (bdf_order(h->scheme) > 0)
    h->tvariant = 0;
  h->scheme = scheme;
  if (passb_blocks(h) > h->max_partials) {
    // a longer transform than the handle was sized for
    h->scheme = old_scheme;
    h->tvariant = old_tv;
    return fail(h, EXPDIAG_EINVAL,
                "scheme %d needs a larger handle than this one", scheme);
  }
  h->dt = dt;
  h->alpha = alpha;
  h->p = *p;
  h->p.gmres_restart = h->restart_cap;
  return build_tables(h);
}

// Fill a handle's fields from the arguments (validated) and allocate its
// device workspace (hipMalloc, or carved from h->arena when set).  On
// failure the buffers allocated so far stay recorded in h.
int setup_handle(expdiag_ctx* h, const expdiag_grid* g, int Nt, double dt,
                 double alpha, int scheme, const expdiag_problem* p,
                 void* hip_stream) {
  Sizes s{};
  const int gc = check_grid(g, &s);
  if (gc != 0)
    return fail(nullptr, gc, "grid: dim 1..3, n a power of two, 4..4096");
  RCHK(validate_params(Nt, dt, alpha, scheme, p));
  if (p->complex_state == 1) {
    // the full spectrum: every last-axis index
    s.nh = g->n[g->dim - 1];
    s.Nk = s.Ns;
  }
  h->dim = g->dim;
  for (int i = 0; i < 3; ++i) h->n[i] = i < g->dim ? g->n[i] : 1;
  h->Nt = Nt;
  h->dt = dt;
  h->alpha = alpha;
  h->scheme = scheme;
  h->p = *p;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->Ns = s.Ns;
  h->Nk = s.Nk;
  h->nh = static_cast<int>(s.nh);
  h->nonlinear = (p->n1 != 0.0 || p->n2 != 0.0 || p->n3 != 0.0);
  h->mixed = p->precision == EXPDIAG_MIXED;
  h->cstate = p->complex_state == 1;
  h->restart_cap = p->gmres_restart;
  if (bdf_order(scheme) > 0)
    h->tvariant = bdf_fft_ok(Nt, bdf_order(scheme)) ? 0 : 1;

  const size_t st = static_cast<size_t>(Nt) * h->Nk * sizeof(cx<double>);
  int rc = 0;
  auto A = [&](auto** ptr, size_t bytes) {
    if (rc == 0) rc = dalloc(h, ptr, bytes);
  };
  A(&h->Uh, st);
  A(&h->T, st);
  if (h->nonlinear) A(&h->Nh, st);
  if (h->nonlinear && h->mixed && h->dim >= 2) {
    A(&h->T32, static_cast<size_t>(Nt) * h->Nk * sizeof(cx<float>));
    A(&h->U32, static_cast<size_t>(Nt) * h->Nk * sizeof(cx<float>));
  }
  A(&h->u0h, h->Nk * sizeof(cx<double>));
  A(&h->E, h->Nk * sizeof(cx<double>));
  A(&h->c1, h->Nk * sizeof(cx<double>));
  A(&h->c2, h->Nk * sizeof(cx<double>));
  A(&h->gam, Nt * sizeof(double));
  A(&h->igam, Nt * sizeof(double));
  A(&h->lam, Nt * sizeof(cx<double>));
  A(&h->tw64, TW_N * sizeof(cx<double>));
  A(&h->tw32, TW_N * sizeof(cx<float>));
  if (dense_ok(Nt)) {
    A(&h->roots, Nt * sizeof(cx<double>));
  }
  h->max_partials = std::max(passb_blocks_nt(time_len(h), h->Nk), 1);
  if (dense_ok(Nt))
    h->max_partials = std::max(h->max_partials, dft_blocks(Nt, h->Nk));
  A(&h->partials, static_cast<size_t>(h->max_partials) * 4 * sizeof(double));
  A(&h->red_out, 8 * sizeof(double));
  A(&h->ctl, sizeof(Ctl));
  A(&h->hist, HIST_CAP * 2 * sizeof(double));
  if (h->restart_cap > 0) {
    A(&h->T2, st);
    A(&h->V, static_cast<size_t>(h->restart_cap + 1) * st);
    h->kpart_blocks = static_cast<int>(krylov_blocks(Nt * h->Nk));
    // rows of block partials: up to 2 restart + 1 inner products per
    // Arnoldi step
    // rows of block partials: the inner products of one Arnoldi step (up
    // to 2 restart + 1 real ones; 4 restart complex ones' parts for a
    // complex state)
    A(&h->kpart, static_cast<size_t>(h->kpart_blocks) *
                     (4 * h->restart_cap + 4) * sizeof(double));
    A(&h->kdots, 8 * (h->restart_cap + 2) * sizeof(double));
    if (h->nonlinear)
      A(&h->Uphys, static_cast<size_t>(Nt) * h->Ns * sizeof(double));
    if (h->nonlinear && h->mixed)
      A(&h->Uphys32, static_cast<size_t>(Nt) * h->Ns * sizeof(float));
  }
  return rc;
}

// light: no iteration plan or graph of its own (handles driven by a batch
// or the server).
int create_impl(const expdiag_grid* g, int Nt, double dt, double alpha,
                int scheme, const expdiag_problem* p, void* hip_stream,
                expdiag_t* out, bool light) {
  g_create_err.clear();
  if (out == nullptr || p == nullptr || g == nullptr)
    return fail(nullptr, EXPDIAG_EINVAL, "null pointer argument");
  *out = nullptr;
  {
    Sizes s{};
    const int gc = check_grid(g, &s);
    if (gc != 0)
      return fail(nullptr, gc,
                  "grid: dim 1..3, n a power of two, 4..4096");
    RCHK(validate_params(Nt, dt, alpha, scheme, p));
  }
  expdiag_ctx* h = new (std::nothrow) expdiag_ctx();
  if (h == nullptr) return fail(nullptr, EXPDIAG_ENOMEM, "host allocation");
  int rc = setup_handle(h, g, Nt, dt, alpha, scheme, p, hip_stream);
  if (rc == 0) {
    if (hipHostMalloc(&h->h_ctl, sizeof(Ctl)) != hipSuccess ||
        hipHostMalloc(&h->h_mirror, sizeof(Ctl), hipHostMallocMapped) !=
            hipSuccess ||
        hipHostMalloc(&h->h_red, 8 * sizeof(double)) != hipSuccess ||
        hipHostMalloc(&h->h_kdots, 8 * (h->restart_cap + 2) *
                                       sizeof(double)) != hipSuccess)
      rc = fail(h, EXPDIAG_ENOMEM, "pinned host allocation");
  }
  if (rc == 0 &&
      hipHostGetDevicePointer(reinterpret_cast<void**>(&h->d_mirror),
                              h->h_mirror, 0) != hipSuccess)
    rc = fail(h, EXPDIAG_EHIP, "host-mapped control block");
  if (rc == 0 && hipStreamCreateWithFlags(&h->cap_stream,
                                          hipStreamNonBlocking) != hipSuccess)
    rc = fail(h, EXPDIAG_EHIP, "capture stream");
  for (auto& e : h->chunk_ev)
    if (rc == 0 &&
        hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      rc = fail(h, EXPDIAG_EHIP, "chunk events");
  if (rc == 0) rc = build_tables(h);
  if (rc == 0 && light) {
    h->use_graph = false;
    h->light = true;
  }
  if (rc == 0 && !light) {
    plan_iteration(h->plan, h, h->ctl, h->d_mirror, h->hist, h->h_mirror);
    rc = plan_upload(h, h->plan, h->cap_stream);
    if (rc == 0 && hipStreamSynchronize(h->cap_stream) != hipSuccess)
      rc = fail(h, EXPDIAG_EHIP, "plan upload");
  }
  if (rc == 0 && !light) {
    if (plan_capture(h, h->plan, h->cap_stream, h->tw64, h->tw32, &h->graph,
                     &h->gexec) != 0) {
      // plain launches of the same plan remain available
      h->use_graph = false;
      h->err.clear();
      (void)hipGetLastError();
    } else {
      h->use_graph = GRAPH_REPLAY_DEFAULT;
    }
  }
  if (rc != 0) {
    g_create_err = h->err;
    release(h);
    delete h;
    return rc;
  }
  *out = h;
  return EXPDIAG_OK;
}

}  // namespace

extern "C" {

int expdiag_create(const expdiag_grid* g, int Nt, double dt, double alpha,
                   int scheme, const expdiag_problem* p, void* hip_stream,
                   expdiag_t* out) {
  return create_impl(g, Nt, dt, alpha, scheme, p, hip_stream, out, false);
}

int expdiag_destroy(expdiag_t h) {
  if (h == nullptr) return EXPDIAG_OK;
  (void)hipStreamSynchronize(h->stream);
  release(h);
  delete h;
  return EXPDIAG_OK;
}

int expdiag_set_stream(expdiag_t h, void* hip_stream) {
  if (h == nullptr) return EXPDIAG_EINVAL;
  // work already enqueued on the old stream (table gathers, transforms)
  // finishes before the new stream may touch the same buffers
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->stream = static_cast<hipStream_t>(hip_stream);
  return EXPDIAG_OK;
}

int expdiag_set_graph(expdiag_t h, int on) {
  if (h == nullptr) return EXPDIAG_EINVAL;
  h->use_graph = on != 0 && h->gexec != nullptr;
  return EXPDIAG_OK;
}

int expdiag_set_zero_guess(expdiag_t h, int on) {
  if (h == nullptr) return EXPDIAG_EINVAL;
  h->zero_guess = on != 0;
  return EXPDIAG_OK;
}

}  // extern "C"

namespace {

// nonlinear pass A outside the iteration plan (residual / GMRES paths)
int pass_a_now(expdiag_ctx* h) {
  Plan P;
  plan_pass_a<double>(P, h, nullptr, -1);
  std::stable_sort(P.groups.begin(), P.groups.end(),
                   [](const Group& x, const Group& y) {
                     return x.stage < y.stage;
                   });
  for (auto& g : P.groups) {
    if (g.kind == K_ROW) {
      for (auto& j : g.rj)
        RCHK((launch_row1<double, ROW_FUSED, double, double>(h, j)));
    } else {
      for (auto& j : g.cj) {
        if (g.mode == 1)
          RCHK((launch_col1<double, 1, double, double>(h, g.len, j)));
        else
          RCHK((launch_col1<double, -1, double, double>(h, g.len, j)));
      }
    }
  }
  return 0;
}

// run `chunk` iterations of the handle's plan (graph replay or launches)
// IF1 with a mean Jacobian: the first shift from u_0 (after the control
// block `dctl` has been uploaded on stream `st`).
int if1_sigma_init(expdiag_ctx* h, Ctl* dctl, hipStream_t st) {
  if (h->scheme != EXPDIAG_IF1 || h->p.jacobian == 0) return 0;
  const PassBArgs a = passb_args(h);
  hipLaunchKernelGGL(if1_sigma_init_kernel<CTL_THREADS>, dim3(1),
                     dim3(CTL_THREADS), 0, st, h->u0h, h->Nk, parseval_nh(h),
                     a.inv_ns, a.jac_c[0], a.jac_c[1], a.jac_c[2], dctl);
  HIPCHK(h, hipGetLastError());
  return 0;
}

int run_iterations(expdiag_ctx* h, int chunk) {
  for (int i = 0; i < chunk; ++i) {
    if (h->use_graph && !h->prof) {
      HIPCHK(h, hipGraphLaunch(h->gexec, h->stream));
    } else {
      RCHK(plan_launch(h, h->plan, h->stream, h->tw64, h->tw32));
    }
  }
  return plan_finish(h, h->plan, h->stream);
}

// Iterations to request next: what the observed contraction predicts to
// reach the active target (flags make overshoot harmless), at least 1.
int next_chunk(const Ctl& c, double rel_prev, int it_prev) {
  constexpr int MAX_CHUNK = 64;
  const double goal = c.phase == 0 ? c.bulk_tol : c.tol;
  if (!(goal > 0.0)) return MAX_CHUNK;  // tol = 0: run to max_iter
  int next = 8;
  if (rel_prev > 0.0 && c.last_rel > 0.0 && c.iters > it_prev &&
      c.last_rel < rel_prev) {
    const double rho =
        std::pow(c.last_rel / rel_prev, 1.0 / (c.iters - it_prev));
    const double need = std::log(goal / c.last_rel) / std::log(rho);
    // (need can be huge or not finite: compare before converting)
    next = need < MAX_CHUNK ? static_cast<int>(std::ceil(need > 0 ? need : 1.0))
                            : MAX_CHUNK;
  }
  return std::max(1, std::min(next, MAX_CHUNK));
}

}  // namespace

extern "C" {

int expdiag_residual(expdiag_t h, const double* u0, const double* U,
                     double* R, double* rnorm) {
  if (h == nullptr) return EXPDIAG_EINVAL;
  if (u0 == nullptr || U == nullptr || R == nullptr)
    return fail(h, EXPDIAG_EINVAL, "null device pointer");
  if (static_cast<const void*>(U) == static_cast<const void*>(R))
    return fail(h, EXPDIAG_EINVAL, "U and R must be distinct");
  RCHK(prepare_u0(h, u0));
  RCHK(fwd_slices<ROW_R2C>(h, U, h->Uh, h->Nt));
  if (h->nonlinear) RCHK(pass_a_now(h));
  PassBArgs a = passb_args(h);
  a.Sout = h->T;
  RCHK((launch_passb1<PB_RESIDUAL, double>(h, a)));
  RCHK(launch_reduce(h, passb1_blocks(h, PB_RESIDUAL)));
  RCHK(inv_slices(h, h->T, R, h->Nt));
  if (rnorm != nullptr) {
    HIPCHK(h, hipMemcpyAsync(h->h_red, h->red_out, 4 * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    *rnorm = std::sqrt(h->h_red[0]);
  }
  return EXPDIAG_OK;
}

int expdiag_precond_apply(expdiag_t h, const double* R, double* S) {
  if (h == nullptr) return EXPDIAG_EINVAL;
  if (R == nullptr || S == nullptr)
    return fail(h, EXPDIAG_EINVAL, "null device pointer");
  RCHK(fwd_slices<ROW_R2C>(h, R, h->T, h->Nt));
  PassBArgs a = passb_args(h);
  a.Rin = h->T;
  a.Sout = h->T;
  RCHK((launch_passb1<PB_PRECOND, double>(h, a)));
  RCHK(inv_slices(h, h->T, S, h->Nt));
  return EXPDIAG_OK;
}

int expdiag_iterate(expdiag_t h, const double* u0, double* U, int max_iter,
                    double tol, int* iters, double* rel_update) {
  if (h == nullptr) return EXPDIAG_EINVAL;
  if (u0 == nullptr || U == nullptr)
    return fail(h, EXPDIAG_EINVAL, "null device pointer");
  if (max_iter < 1 || max_iter > HIST_CAP)
    return fail(h, EXPDIAG_EINVAL, "max_iter must be 1..%d", HIST_CAP);
  if (!(tol >= 0.0)) return fail(h, EXPDIAG_EINVAL, "tol must be >= 0");
  RCHK(prepare_u0(h, u0));
  RCHK(enter_guess(h, U, true, h->zero_guess));
  prof_begin(h);
  *h->h_ctl = initial_ctl(h, max_iter, tol);
  h->h_ctl->zstart = h->zero_guess && zero_start_ok(h) ? 1 : 0;
  *h->h_mirror = *h->h_ctl;
  hipLaunchKernelGGL(ctl_set_kernel, dim3(1), dim3(64), 0, h->stream, h->ctl,
                     *h->h_ctl);
  HIPCHK(h, hipGetLastError());
  RCHK(if1_sigma_init(h, h->ctl, h->stream));
  // Chunks of iterations, two in flight: while the device runs one, the
  // host sizes the next from the state the previous one left, so the
  // stream does not drain between chunks.  The first chunk is the previous
  // solve's iteration count (8 before any), the second a short (long)
  // speculative one; later ones are what the observed contraction predicts
  // beyond the iterations already enqueued.  Iterations enqueued past
  // convergence find the instance done and return at once; never more than
  // max_iter are enqueued.
  int enqueued = 0;
  double rel_prev = -1.0;
  int it_prev = 0;
  int in_flight = 0, oldest = 0;
  auto enqueue = [&](int n, int slot) -> int {
    RCHK(run_iterations(h, n));
    enqueued += n;
    HIPCHK(h, hipEventRecord(h->chunk_ev[slot], h->stream));
    ++in_flight;
    return 0;
  };
  // The exit transform is enqueued as soon as the enqueued iterations are
  // expected to suffice (so the tail of a solve has no host round trip);
  // should more iterations be needed after all, it is enqueued again.
  bool exit_queued = false;
  const bool known = h->last_iters > 0;
  RCHK(enqueue(std::min({known ? h->last_iters : 8, 64, max_iter}), 0));
  if (enqueued < max_iter)
    RCHK(enqueue(std::min(known ? 2 : 8, max_iter - enqueued), 1));
  if (known || enqueued >= max_iter) {
    RCHK(leave_bulk_state(h, h->ctl, h->stream));
    RCHK(inv_slices(h, h->Uh, U, h->Nt));
    exit_queued = true;
  }
  while (in_flight > 0) {
    HIPCHK(h, hipEventSynchronize(h->chunk_ev[oldest]));
    --in_flight;
    const Ctl c = read_mirror(h->h_mirror);
    if (c.done != 0 || c.iters >= max_iter) break;
    int add = 8;  // no contraction observed yet: keep a chunk queued
    if (rel_prev >= 0.0 && c.iters > it_prev)
      add = next_chunk(c, rel_prev, it_prev) - (enqueued - c.iters);
    rel_prev = c.last_rel;
    it_prev = c.iters;
    add = std::min(add, max_iter - enqueued);
    if (add <= 0 && in_flight == 0) add = std::min(1, max_iter - enqueued);
    if (add > 0) {
      RCHK(enqueue(add, oldest));
      exit_queued = false;
    }
    if (!exit_queued && (add <= 0 || enqueued >= max_iter)) {
      RCHK(leave_bulk_state(h, h->ctl, h->stream));
      RCHK(inv_slices(h, h->Uh, U, h->Nt));
      exit_queued = true;
    }
    oldest ^= 1;
  }
  if (!exit_queued) {
    RCHK(leave_bulk_state(h, h->ctl, h->stream));
    RCHK(inv_slices(h, h->Uh, U, h->Nt));
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  prof_resolve(h);
  const Ctl c = read_mirror(h->h_mirror);
  h->last_iters = c.iters;
  if (iters != nullptr) *iters = c.iters;
  if (rel_update != nullptr) *rel_update = c.last_rel;
  if (c.done == 2) return fail(h, EXPDIAG_EDIVERGED, "non-finite residual");
  return (c.phase == PH_FP64 && c.last_rel <= tol) ? EXPDIAG_OK
                                                   : EXPDIAG_NOT_CONVERGED;
}

int expdiag_profile_enable(expdiag_t h, int mask) {
  if (h == nullptr) return EXPDIAG_EINVAL;
  if (mask) {
    if (h->events.empty()) {
      h->events.resize(16384);
      for (auto& e : h->events) {
        HIPCHK(h, hipEventCreate(&e.a));
        HIPCHK(h, hipEventCreate(&e.b));
      }
    }
    h->ev_used = 0;
    for (int i = 0; i < NPROF; ++i) {
      h->prof_ms[i] = 0;
      h->prof_cnt[i] = 0;
      h->prof_bytes[i] = 0;
      h->prof_all[i] = 0;
    }
  }
  h->prof = mask != 0;
  h->prof_mask = mask;
  return EXPDIAG_OK;
}

int expdiag_profile_read(expdiag_t h, double* ms, long* launches,
                         double* bytes, long* timed, int nclass) {
  if (h == nullptr || ms == nullptr || nclass < 1) return EXPDIAG_EINVAL;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (size_t i = 0; i < h->ev_used; ++i) {
    float t = 0;
    HIPCHK(h, hipEventElapsedTime(&t, h->events[i].a, h->events[i].b));
    h->prof_ms[h->events[i].cls] += t;
    h->prof_cnt[h->events[i].cls] += 1;
  }
  h->ev_used = 0;
  for (int i = 0; i < nclass && i < NPROF; ++i) {
    ms[i] = h->prof_ms[i];
    if (launches != nullptr) launches[i] = h->prof_all[i];
    if (bytes != nullptr) bytes[i] = h->prof_bytes[i];
    if (timed != nullptr) timed[i] = h->prof_cnt[i];
  }
  return EXPDIAG_OK;
}

}  // extern "C"

#include "gmres.inc"
#include "batch.inc"
#include "autotune.inc"
#include "noalloc.inc"
