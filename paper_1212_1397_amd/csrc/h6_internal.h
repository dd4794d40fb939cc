// Internal declarations shared by the host plan, the solver loops and the HIP
// kernels of the helmholtz6 library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/helmholtz6.h"
#include "xform_bluestein.h"
#include "xform_rader.h"

namespace h6 {

using cplx = std::complex<double>;

// Weights of one 9-point in-plane operator acting on (centre, sum of the four
// edge neighbours, sum of the four corner neighbours).  Any operator
// alpha I + beta (D_x + D_y) + gamma D_x D_y has
//   centre = alpha - 4 beta + 4 gamma, edge = beta - 2 gamma, corner = gamma.
struct W9 {
  double2 c, e, k;
};

// Stencil weight table: [row type][plane offset -1, 0, +1], row types
// 0 = interior row, 1 = low-z closure row, 2 = high-z closure row.
struct StencilTable {
  W9 w[3][3];
};

enum KernelClass {
  KC_STENCIL = 0,
  KC_STENCIL_RESID,
  KC_XFORM_X,
  KC_XFORM_Y,
  KC_TRIDIAG,
  KC_MGS_DOTS,
  KC_MGS_UPDATE,
  KC_NORM,
  KC_AXPY,
  KC_RHS,
  KC_COUNT
};
extern const char* const kKernelClassNames[KC_COUNT];

// K extent staged per step by the dense transform kernels; the folded basis
// matrices are padded to a multiple of it.
constexpr int kDenseKChunk = 16;

// Transform along one transverse axis (Section 3.3): a sine basis for a
// Dirichlet pair, a cosine basis for a Neumann pair; M = n + 1.
struct AxisXform {
  int L = 0;        // unknowns on the axis (n for D, n + 2 for N)
  int M = 0;        // n + 1
  int neumann = 0;  // 0: DST-I pair, 1: DCT-I pair
  int fast = 0;     // 1: Rader FFT path (M = 257), 2: Bluestein FFT path (odd M <= 255), 0: dense product
  int lines = 0;    // Rader path: lines (x) / columns (y) per workgroup (autotuned)
  void* wmat = nullptr;   // dense path: folded basis matrices We, Wo of the forward, then of the inverse
  int Hm = 0, Hk = 0;     // their padded rows (multiple of 32) and columns (multiple of kDenseKChunk)
  RaderTables rader{};
  void* rader_mem = nullptr;   // one device allocation holding the tables
  BluesteinTables blue{};
  void* blue_mem = nullptr;    // one device allocation holding the Bluestein tables
};

// End rows of T_z for the z solver.  T_z is tridiag(1, -2, 1) inside; row 0
// and row n'z - 1 carry an off-diagonal of 1 or 2 and a main-diagonal term on
// Sommerfeld faces.  Dividing those two rows by their off-diagonal makes every
// off-diagonal 1 (the Thomas quantities c' and d' do not change under row
// scaling); the solver then needs only the two scaled end rows:
//   row 0:      s0 ((b0_re + i b0_im) + shift) x_0 + x_1 = s0 r_0,
//   row n'z-1:  x_{n'z-2} + sl ((bl_re + i bl_im) + shift) x_{n'z-1} = sl r_{n'z-1}.
struct ZEnds {
  double b0_re, b0_im, s0;
  double bl_re, bl_im, sl;
};

struct Timing {
  bool enabled = false;
  double ms[KC_COUNT] = {0};
  long long launches[KC_COUNT] = {0};
  double bytes[KC_COUNT] = {0};     // algorithmic HBM bytes of the timed launches
  std::vector<hipEvent_t> pool;     // recycled events
  struct Pending { hipEvent_t a, b; int cls; double bytes; };
  std::vector<Pending> pending;
};

// what a captured Arnoldi step depends on besides its index
struct GraphKey {
  void* V = nullptr;
  void* Z = nullptr;
  void* U = nullptr;                    // solution vector (whole-cycle graphs update it)
  int m = 0, flex = 0, mixed = 0, mode = 0;
  bool operator==(const GraphKey& o) const {
    return V == o.V && Z == o.Z && U == o.U && m == o.m && flex == o.flex && mixed == o.mixed &&
           mode == o.mode;
  }
};

}  // namespace h6

struct h6_plan_s {
  h6_params p{};
  int dims[3] = {0, 0, 0};          // n'x, n'y, n'z
  size_t N = 0;                     // unknowns
  int zlo_closure = 0, zhi_closure = 0;   // z face is N or S (closure row present)
  int xmirror = 0, ymirror = 0;           // x / y pair is Neumann
  h6::cplx k, kappa;
  h6::StencilTable stencil{};
  h6::AxisXform ax[2];

  // device tables
  h6::StencilTable* d_stencil = nullptr;
  double* d_lambda_x = nullptr;     // transverse eigenvalues per mode
  double* d_lambda_y = nullptr;
  h6::ZEnds zends{};                // end rows of the z tridiagonal (scaled form)
  double* d_zparams = nullptr;      // device copy for the z solver: kappa (re, im), then zends (kZParams doubles)
  void* d_cstart = nullptr;         // Thomas c' entering each z segment: [z_segments(n'z)][n'x n'y], complex
                                    // (double2, or float2 in mixed plans)

  // preconditioner workspace (complex128 vectors, or complex64 in mixed plans)
  void* w_pc[3] = {nullptr, nullptr, nullptr};   // two used

  // Krylov workspace (allocated on first solve, grown as needed)
  double2* V = nullptr;   int V_cols = 0;      // (m+1) basis vectors
  void* Z = nullptr;      int Z_cols = 0;      // FGMRES preconditioned vectors (complex64 in mixed plans)
  double2* r = nullptr;                        // residual / scratch vector
  double2* t = nullptr;                        // scratch vector
  double* partials = nullptr;                  // per-block partial sums (2 * kMaxPartials doubles)
  double2* d_scal = nullptr;                   // device scalars: reduction results, coefficients (kScal entries)
  double2* h_pinned = nullptr;                 // pinned host mirror of d_scal
  double* h_step = nullptr;    // coherent pinned host array for the Arnoldi step's Hessenberg column
  double* d_step = nullptr;    //   and |w|^2 (written by the device), and its device address
  double* h_parts = nullptr;   // coherent pinned host array of residual-norm partials (SKS), mapped:
  double* d_parts = nullptr;   //   its device address; one entry per stencil workgroup
  int parts_cap = 0;
  double2* d_gram = nullptr;  int gram_dim = 0;  // Gram matrix <q_i, q_l> of the Arnoldi basis (gram_dim^2)
  void* d_sep = nullptr;  size_t sep_bytes = 0;  // separable-source tables (helmholtz6_rhs_separable)
  hipEvent_t ev_sync = nullptr;                // host waits on scalars copied back mid-stream
  struct h6_net_s* net = nullptr;              // learned correction for FGMRES (not owned)
  int use_graphs = 0;                          // 1: capture GMRES steps as HIP graphs, 2: whole cycles
  const int* skip = nullptr;                   // while a cycle graph is captured: device stop flag that
                                               // every kernel of an Arnoldi step checks on entry
  double* d_givens = nullptr;  int givens_dim = 0;  // device least-squares state of cycle graphs
  hipStream_t gstream = nullptr;               // plan-owned stream of graph-mode solves
  hipEvent_t ev_order = nullptr;               // orders gstream after the caller's stream
  std::vector<hipGraphExec_t> step_graphs;     // one per step index (mode 1)
  hipGraphExec_t cycle_graph = nullptr;        // one restart cycle (mode 2)
  h6::GraphKey graph_key;
  int stencil_tz = 16;                         // autotuned stencil z-chunk (8, 16 or 32)
  bool spec_done = false;                      // exact spectrum bounds of A A_p^{-1} (Dirichlet)
  h6_status spec_status = H6_OK;
  double spec_lo = 0.0, spec_hi = 0.0;
  int learned_steps = 0;                       // steps of the last solve that used it

  h6::Timing timing;
  std::string last_error;
};

namespace h6 {

constexpr int kRedBlocks = 1024;   // blocks of the grid-stride reductions
constexpr int kZParams = 8;        // doubles of h6_plan_s::d_zparams
constexpr int kMaxPartials = 1 << 20;
constexpr int kScal = 4096;        // device scalar slots (double2)
constexpr int kGramMax = 16;       // Gram row entries formed by launch_update_gram
constexpr int kZSegs = 32;         // most segments per z line in the partitioned z solver
constexpr int kMaxZ = kZSegs * 17; // largest n'z of the partitioned z solver
// segments per z line: complex64 solves use 16 (32 modes per workgroup, 256-byte
// row segments) up to n'z = 272; complex128 solves and longer lines use 32 (16
// modes per workgroup, fewer registers per thread).  The segment-start table
// is built for this count.
inline int z_segments(int nz, bool f32) { return (f32 && nz <= 16 * 17) ? 16 : 32; }

// Workgroup id remap for the 8 XCDs of the chip: the hardware hands out
// consecutive workgroup ids round-robin over the XCDs (each with its own L2);
// the remap gives each XCD a contiguous range of logical ids, so neighbouring
// tiles that share cache lines or halos run under the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int nwg) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int per = nwg >> 3, rem = nwg & 7;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// kernel launchers (stream-ordered, no synchronisation)
// With F (residual form, y = F - A x): |y|^2 per workgroup into partials and,
// when fpartials is given, |F|^2 per workgroup into fpartials.
hipError_t launch_stencil(h6_plan P, const double2* x, double2* y, const double2* F,
                          double* partials, int* nparts, hipStream_t s, double* fpartials = nullptr);
// Preconditioner passes: PINV_FIRST is the forward x transform of r alone,
// PINV_REST the remaining passes (forward y, z solves, inverse y and x) on the
// plan's workspace, so a caller can enqueue the first pass before it waits on
// the host.  PINV_ALL = both.
enum { PINV_FIRST = 1, PINV_REST = 2, PINV_ALL = 3 };
hipError_t launch_pinv(h6_plan P, const double2* r, double2* z, hipStream_t s, int part = PINV_ALL);
// z = A_p^{-1} r with the work vectors ws[0], ws[1] (each N complex values in
// the plan's compute precision) instead of the plan's
hipError_t launch_pinv_ws(h6_plan P, const double2* r, double2* z, void* const ws[2], hipStream_t s);
// Fixed work space of helmholtz6_apply_Pinv_noalloc (a file-scope device
// array): its size, and its device address on the current device (looked up
// once per device).
constexpr size_t kStaticWorkBytes = size_t(128) << 20;
hipError_t static_work_address(void** out);
// U += A_p^{-1} r (the update folded into the last inverse transform)
hipError_t launch_pinv_acc(h6_plan P, const double2* r, double2* U, hipStream_t s,
                           int part = PINV_ALL);
// mixed plans only: U += A_p^{-1} r for a complex64 r
hipError_t launch_pinv_acc_f32in(h6_plan P, const float2* r, double2* U, hipStream_t s,
                                 int part = PINV_ALL);
// mixed plans only: z = A_p^{-1} r stored in complex64
hipError_t launch_pinv_f32out(h6_plan P, const double2* r, float2* z, hipStream_t s,
                              int part = PINV_ALL);
// y = A x for a complex64 x (FP64 arithmetic)
hipError_t launch_stencil_f32in(h6_plan P, const float2* x, double2* y, hipStream_t s);
// r = F - A U stored in complex64 (FP64 arithmetic and |r|^2 partials), for
// callers that only hand r to a complex64 preconditioner
// workgroups of a stencil launch on this plan (one residual-norm partial each)
int stencil_workgroups(h6_plan P);
hipError_t launch_resid_f32out(h6_plan P, const double2* U, float2* r, const double2* F,
                               double* partials, int* nparts, hipStream_t s, double* fpartials = nullptr);
// Dense (matrix-core) transforms along x / y with the axis' basis matrices
// (xform_dense.hip); acc != 0: out += result
template <typename R, typename Tin, typename Tout>
hipError_t launch_dense_x(const AxisXform& X, bool inverse, const Tin* in, Tout* out, int nlines, int acc,
                          hipStream_t s, const int* skip = nullptr);
template <typename R, typename T2>
hipError_t launch_dense_y(const AxisXform& Y, bool inverse, const T2* in, T2* out, int nx, int nz,
                          hipStream_t s, const int* skip = nullptr);
constexpr int kMaxLine = 4096;    // largest n'x, n'y (basis matrices of the dense transforms)
hipError_t launch_rhs(h6_plan P, int nsrc, const double* centres, const double* amps,
                      double sigma, double2* F, hipStream_t s);
// tab[a]: host complex128 samples, nterms x 5 derivative orders x dims[a]; synchronises s
hipError_t launch_rhs_separable(h6_plan P, int nterms, const double* coef, const double* const tab[3],
                                double2* F, hipStream_t s);
hipError_t launch_rhs_dirichlet_z(h6_plan P, int side, const double2* g, double2* F, hipStream_t s);
// face 0..5; t1 / t2: host complex128 tables (nterms x 5 x n' of the tangential axes); synchronises s
hipError_t launch_rhs_neumann(h6_plan P, int face, int nterms, const double* coef, const double* t1,
                              const double* t2, double2* F, hipStream_t s);

// Krylov helpers (double2 vectors of length P->N); reductions end in device doubles
hipError_t launch_norm2(const double2* a, size_t n, double* partials, double* out, hipStream_t s);
hipError_t launch_reduce_sum(const double* partials, int nparts, double* out, hipStream_t s);
// out[2i..2i+1] = <q_i, w> for i < m, q_i = Q + i n
// skip (all Arnoldi-step launchers): device flag; when nonzero the kernels return at once
hipError_t launch_block_dots(const double2* Q, int m, const double2* w, size_t n, double* partials,
                             double* out, hipStream_t s, const int* skip = nullptr);
// w -= sum_{i<m} c_i q_i; out[0] = |w|^2, out[1+2i..2+2i] = <q_i, w> for i < min(m, kGramMax);
// hnorm (optional, host-mapped coherent memory): a copy of out[0] for the host
hipError_t launch_update_gram(double2* w, const double2* Q, const double2* c, int m, size_t n,
                              double* partials, double* out, hipStream_t s, const int* skip = nullptr,
                              double* hnorm = nullptr);
// MGS coefficients of Arnoldi step j on the device (one workgroup), from the
// block dots <q~_i, w~> (dots, i <= j), the norm / Gram row of the last update
// pass (nrow: |q~_j|^2, <q~_i, q~_j> for i < min(j, kGramMax)) and the extra
// Gram entries i = kGramMax .. j-1 (gram2): stores nu_j, row j of the Gram
// matrix G (ld gdim), the Hessenberg column h (hcol) and the update
// coefficients c_i = nu_j h_i / nu_i (coef).  hmirror (optional, host-mapped
// coherent memory): a copy of the Hessenberg column for the host.
hipError_t launch_mgs_coef(int j, const double* dots, const double* nrow, const double* gram2,
                           double* nu, double2* G, int gdim, double2* hcol, double2* coef,
                           hipStream_t s, const int* skip = nullptr, double2* hmirror = nullptr);
// out = |a - b|^2 (device double)
hipError_t launch_diff_norm2(const double2* a, const double2* b, size_t n, double* partials, double* out,
                             hipStream_t s);
// learned correction (unet.hip): z += c(q), z complex64 when z_f32
hipError_t net_apply_add(struct h6_net_s* net, const double2* q, double kh, void* z, bool z_f32,
                         hipStream_t s);
bool net_matches(struct h6_net_s* net, const int dims[3]);
// out (+)= sum_{i < count} y_i V_i, count = min(m, *mdev) when mdev is given (device int)
hipError_t launch_multi_axpy(double2* out, const double2* V, const double2* y, int m, size_t n,
                             int accumulate, hipStream_t s, const int* mdev = nullptr);
hipError_t launch_multi_axpy_f32(double2* out, const float2* V, const double2* y, int m, size_t n,
                                 int accumulate, hipStream_t s, const int* mdev = nullptr);
// Least-squares state of a whole-cycle graph (device, one restart cycle of
// at most m steps): g (m + 1 complex), cosines (m), sines (m complex), the
// rotated Hessenberg R (m x m complex, column-major), per-step residual
// estimates (m), and int slots: stop flag, steps done.
struct GivensState {
  double2* g;
  double* cs;
  double2* sn;
  double2* R;
  double* est;
  int* stop;
  int* jdone;
};
GivensState givens_state(h6_plan P, int m);
size_t givens_bytes(int m);
// step j of the cycle: Hessenberg column (hcol, h_{i,j}, i <= j) and
// H(j+1, j) = sqrt(nrow[0]) / nu[j]; previous rotations, new rotation, g,
// estimate |g_{j+1}| / prm[1]; stop when it is <= prm[2], when j + 1 reaches
// prm[0] steps, or on breakdown.  prm: (steps allowed, ||F||, tol) doubles.
hipError_t launch_givens_step(int j, const double* nrow, const double* nu, const double2* hcol,
                              GivensState st, int m, const double* prm, hipStream_t s);
// y = R^{-1} g over the steps done, divided by nu_i (unnormalised basis), into y[0..m)
hipError_t launch_lsq_solve(int m, GivensState st, const double* nu, double2* y, hipStream_t s);
// device int slot <- 0 (a one-thread kernel; keeps memset nodes out of graphs)
hipError_t launch_clear_int(int* p, hipStream_t s);

// timing helpers
void timing_begin(h6_plan P, int cls, hipStream_t s, hipEvent_t* a);
// bytes: the algorithmic HBM traffic of the work between begin and end
void timing_end(h6_plan P, int cls, hipStream_t s, hipEvent_t a, double bytes);

// exact spectrum bounds of A A_p^{-1} (all-Dirichlet, real k), cached in the plan
h6_status spectrum_bounds(h6_plan P);
// e = c1 e + c2 t; U += e (Chebyshev step)
hipError_t launch_cheb_update(double2* e, const double2* t, double2* U, double c1, double c2, size_t n,
                              hipStream_t s);

// Queued batch (queue.hip, solve.cpp): problems of one grid shape in a
// device-side queue (longest first), lanes that take the next problem when
// theirs is done.
struct QueueEntry {            // one problem (device memory, queue order)
  const double2* F;            // caller's right-hand side and solution
  double2* U;
  const StencilTable* stencil; // the problem's own plan tables (wavenumber-dependent)
  const void* cstart;
  const double* zparams;
  double tol;
  int maxit;
  int result;                  // index of the problem in the caller's arrays
};
struct QueueResult {           // host-mapped, one per problem
  int iters;
  int status;
  double rel_resid;
};
struct QueueLane {             // device memory, one per lane
  int cur;                     // queue position of the lane's problem, -1 none
  int out;                     // problem whose U is copied out this replay, -1 none
  int pend;                    // problem finished at a cycle start, copied out next replay
  int fresh;                   // the lane took a new problem this replay
  int idle;                    // the queue was empty when the lane asked
  int skip_refill, skip_fresh; // kernel skip flags (1 = skip)
  int iters;                   // steps done on the lane's problem
  double normF;
  int* idle_mirror;            // host-mapped copy of idle
};
struct LaneRefill {
  QueueLane* lane;
  const QueueEntry* q;
  double2 *F, *U, *V0;         // the lane plan's right-hand side, solution and first basis vector
  StencilTable* stencil;       // the lane plan's tables
  void* cstart;
  double* zparams;
  size_t N;
  size_t cstart_words;         // 8-byte words of the segment-start table
  double* partials;            // kRedBlocks |F|^2 partials
};
hipError_t launch_lane_check(QueueLane* lane, const QueueEntry* q, int* head, int count, const double* rnorm2,
                             QueueResult* res, hipStream_t s);
hipError_t launch_lane_refill(const LaneRefill& a, hipStream_t s);
hipError_t launch_lane_cycle(QueueLane* lane, const QueueEntry* q, QueueResult* res, const double* rnorm2,
                             double* prm, int* stop, int* jdone, int m, hipStream_t s);
hipError_t launch_lane_count(QueueLane* lane, const int* jdone, hipStream_t s);
// sum of nparts partials into *out; skipped while *skip != 0
hipError_t launch_reduce_sum_skip(const double* partials, int nparts, double* out, const int* skip, hipStream_t s);
struct QLane {                 // one lane: a plan of its group's shape and its F / U slots
  h6_plan P = nullptr;
  double2* F = nullptr;
  double2* U = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t join = nullptr;
  int group = 0;
};
}  // namespace h6

struct h6_queue_s {
  int m = 0, count = 0;
  std::vector<h6_plan> plans;          // the problems' plans (not owned)
  std::vector<int> order;              // queue position -> problem index (groups contiguous)
  std::vector<int> goff, gcount;       // queue offset and size per group
  std::vector<h6::QLane> L;
  hipStream_t s0 = nullptr;
  hipEvent_t fork = nullptr;
  h6::QueueEntry* d_q = nullptr;
  int* d_head = nullptr;
  h6::QueueLane* d_lanes = nullptr;
  h6::QueueResult* h_res = nullptr;    // host-mapped results, one per problem
  h6::QueueResult* d_res = nullptr;
  int* h_idle = nullptr;               // host-mapped idle flags, one per lane
  int* d_idle = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string last_error;
};

namespace h6 {
h6_status queue_create(h6_plan* plans, int count, int m, int lanes, h6_queue* out, std::string& err);
h6_status queue_solve(h6_queue Q, const double2* const* F, double2* const* U, h6_solve_info* infos,
                      h6_status* statuses, std::string& err);
void queue_destroy(h6_queue Q);

void release_graphs(h6_plan P);
h6_status autotune(h6_plan P, const char* cache_path, hipStream_t s);

// solver
h6_status run_solve(h6_plan P, const double2* F, double2* U, h6_solve_info* info, hipStream_t s);

}  // namespace h6

#define H6_TRY_HIP(expr)                                                         \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess) {                                                      \
      P->last_error = std::string(#expr) + ": " + hipGetErrorString(_e);         \
      return H6_ERR_HIP;                                                         \
    }                                                                            \
  } while (0)
