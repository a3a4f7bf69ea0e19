// Handle, device workspaces and the C ABI of include/kkt_lu.h.
//
// Everything the GPU needs is uploaded once by kkt_analyze and reused by
// every refactorization and solve (the paper moves the system to the GPU once
// and keeps Krylov vectors and buffers allocated across systems, Sections 5
// and 5.1.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/kkt_lu.h"
#include "analyze.h"
#include "kernels.h"

using namespace kktlu;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct kkt_ctx {
  kkt_options opt;
  std::string err;
  bool analyzed = false;
  bool factored = false;
  Analysis an;
  double analyze_seconds = 0.0;
  std::vector<DevBuf> bufs;
  int64_t device_bytes = 0;
  // factors and maps
  int *lu_rowptr = nullptr, *lu_col = nullptr, *diag = nullptr, *lu_src = nullptr;
  double* lu_val = nullptr;
  int *lev_rows = nullptr, *ulev_rows = nullptr, *utlev_rows = nullptr, *ltlev_rows = nullptr;
  int *ut_ptr = nullptr, *ut_row = nullptr, *ut_pos = nullptr;
  int *lt_ptr = nullptr, *lt_row = nullptr, *lt_pos = nullptr;
  int *pin = nullptr, *qperm = nullptr;  // pin[i] = Q[P[i]], qperm[k] = Q[k]
  // matching and scaling (null without): pin[i] = match[Q[P[i]]] (A's row),
  // rowsc[i] = dr[pin[i]], colsc[k] = dc[Q[k]]; ascale[p] = dr_i dc_j per
  // stored entry of A and avs the scaled values (factored matrix, A's order)
  double *rowsc = nullptr, *colsc = nullptr, *ascale = nullptr, *avs = nullptr;
  // A (CSR, column view) and the current values
  int *a_rowptr = nullptr, *a_col = nullptr, *at_ptr = nullptr, *at_row = nullptr,
      *at_pos = nullptr;
  double* aval = nullptr;
  bool anorm1_valid = false;
  // dependency-driven schedules
  bool syncfree = false;
  bool light = true;  // device-coherent publication instead of acquire/release fences
  int cap = 0;        // longest LU row (LDS staging capacity)
  double *tc = nullptr, *ty = nullptr, *tz = nullptr;  // value-as-flag solve buffers (n+1)
  // multi-column solves: (n+1) x mcap buffers (grown on demand), per-column maxima
  double *mc = nullptr, *my = nullptr, *mz = nullptr;
  int mcap = 0;
  unsigned long long* colmax = nullptr;
  unsigned long long* h_colmax = nullptr;  // pinned
  SyncState* ss = nullptr;
  int *ready_ref = nullptr, *ready_a = nullptr, *ready_b = nullptr;
  ChunkSched ch_l{}, ch_u{}, ch_ut{}, ch_lt{};
  // single right-hand side: thin leading/trailing level runs solved by one
  // workgroup (index = solve mode) and the chunk schedules of the levels between
  SegSched seg_pre[4]{}, seg_post[4]{};
  ChunkSched chb[4]{};
  // dense trailing block of the refactorization: pivots tail_c0 .. n-1
  // (tail_s of them), row-major tail_S x tail_S workspace and panel scratch
  int tail_s = 0, tail_c0 = 0, tail_S = 0;
  double *tail_T = nullptr, *tail_dsc = nullptr, *tail_rhs = nullptr;
  // its task-launch factorization: task list and per-tile operation counts
  int *dlu_tasks = nullptr, *dlu_ver = nullptr;
  int dlu_ntasks = 0;
  double* red = nullptr;  // scratch of the two-stage maxima (RED_SCRATCH doubles)
  int *tail_split0 = nullptr, *tail_split2 = nullptr;
  // U solve: rows with entries in the dense block's columns, where those
  // entries start, and their terms (launch_udense_pre)
  int *u_xend = nullptr, *u_rows = nullptr;
  double* u_pre = nullptr;
  int u_nrows = 0;
  // chain-blocked single right-hand-side solves (modes 0 L, 1 U, 2 U^T, 3 L^T)
  // single-system pattern (for re-analysis) and the number of re-analyses
  std::vector<int64_t> pat_rowptr;
  std::vector<int32_t> pat_colind;
  int reanalyses = 0;
  bool in_retry = false;
  bool use_sn = false;
  // rows without dependencies in the forward solves (L; U^T), final in the gather
  uint8_t *sn_triv0 = nullptr, *sn_triv2 = nullptr;
  SnSched chs[4]{};
  int chs_levels[4] = {};
  // refactorization bands: chunks ref_cstart[band_chunk_lo[b] ..
  // + band_nchunks[b]] of ref_order (each band's chunk list ends with its end
  // offset), longest row band_cap[b]
  int *ref_order = nullptr, *ref_cstart = nullptr;
  unsigned char* ref_cmicro = nullptr;  // per chunk: a chunk of micro rows (one per lane)
  int* ref_triv = nullptr;  // rows without pivots (k_refactor_trivial)
  // A's values in factor order (fill positions zero) and the A -> factor map;
  // per L entry (i, k): (diag[k], rowptr[k + 1])
  double* luA = nullptr;
  int* a2lu = nullptr;
  int2* ref_pbnd = nullptr;
  int* ref_dlc = nullptr;  // pivots of each row before the dense trailing block
  int ref_ntriv = 0;
  // precomputed update positions of the refactorization (null: binary search)
  int* ref_moff = nullptr;
  unsigned short* ref_map = nullptr;
  int64_t ref_map_entries = 0;
  // short-row bands (launch_refactor_flat): per-row flag for the packed map
  // entries and the per-entry list bounds
  bool band_flat[REF_MAX_BANDS] = {};
  unsigned char* ref_flat = nullptr;
  int4* ref_rmeta = nullptr;  // list-kernel row metadata per order position
  long long* tl = nullptr;     // debug_timeline: 3 wall-clock values per row
  int2* ref_fl = nullptr;
  int nbands = 0;
  int band_chunk_lo[REF_MAX_BANDS] = {}, band_nchunks[REF_MAX_BANDS] = {},
      band_cap[REF_MAX_BANDS] = {};
  // statistics
  DevStats* st = nullptr;
  DevStats* h_st = nullptr;  // pinned
  // refinement workspace
  int m = 20;
  double *V = nullptr, *Z = nullptr, *w = nullptr, *r = nullptr, *xt = nullptr, *tmp = nullptr;
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *h = nullptr, *h2 = nullptr,
         *ww = nullptr, *y = nullptr, *hn = nullptr, *partial = nullptr;
  // sync-free refinement: stop-test state and workspace; fg_cols right-hand
  // sides are refined in lockstep (the Krylov vectors above hold fg_cols
  // columns each); fg_pending: a device-checked solve ran since the last report
  FgState* fs = nullptr;
  FgBufs fb{};
  int fg_cols = 1;
  bool fg_pending = false;
  // adaptive launch budget (refine_budget = -1): each solve's outcome is
  // copied to pinned host memory behind an event; a later solve reads it
  // only if the event has completed (never waits)
  FgState* h_fs = nullptr;  // pinned
  hipEvent_t ev_fs = nullptr;
  bool ev_fs_recorded = false;
  int auto_need = 0;        // iterations the last observed solve needed
  bool auto_full = false;   // next solve launches the full budget
  // block-diagonal batch (batch_count > 0): instance offsets, per-row/column
  // absolute sums, per-instance maxima (3 per instance) and etas
  int batch_count = 0;
  // shared-pattern batch (kkt_analyze_shared): inst.count instances of the
  // one analysed pattern, sharing every index structure; count = 1 otherwise
  Inst inst;
  std::vector<int64_t> row_off, nnz_off;
  int* d_row_off = nullptr;
  double *rowabs = nullptr, *colabs = nullptr, *inst_out = nullptr;
  std::vector<double> h_inst, inst_eta;
  // captured refactor + solve with device-checked refinement
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  const double *graph_b = nullptr, *graph_x = nullptr;
  // calls that replaced the factors or the matrix (kkt_info.factor_epoch)
  int64_t factor_epoch = 0;
  // report
  int warnings = 0;
  int last_iters = 0;
  double last_eta = 0.0, last_eta0 = 0.0;
};

namespace {

kkt_status fail(kkt_handle h, kkt_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

#define HIP_CHECK_VOID(call) (void)(call)

#define HIP_CHECK(h, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(h, KKT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

void free_device(kkt_handle h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
  for (auto& b : h->bufs) (void)hipFree(b.p);
  h->bufs.clear();
  h->device_bytes = 0;
  if (h->h_st) (void)hipHostFree(h->h_st);
  h->h_st = nullptr;
  if (h->h_fs) (void)hipHostFree(h->h_fs);
  h->h_fs = nullptr;
  if (h->ev_fs) (void)hipEventDestroy(h->ev_fs);
  h->ev_fs = nullptr;
  h->ev_fs_recorded = false;
  h->auto_need = 0;
  h->auto_full = false;
  if (h->h_colmax) (void)hipHostFree(h->h_colmax);
  h->h_colmax = nullptr;
  h->mc = h->my = h->mz = nullptr;
  h->mcap = 0;
  h->fs = nullptr;
  h->fb = FgBufs{};
  h->fg_cols = 1;
  h->fg_pending = false;
  h->analyzed = h->factored = false;
}

template <typename T>
kkt_status dalloc(kkt_handle h, T** out, size_t count) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    *out = nullptr;
    return fail(h, e == hipErrorOutOfMemory ? KKT_ERR_OUT_OF_MEMORY : KKT_ERR_DEVICE,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  h->bufs.push_back({p, bytes});
  h->device_bytes += (int64_t)bytes;
  *out = (T*)p;
  return KKT_OK;
}

template <typename T>
kkt_status upload(kkt_handle h, T** out, const std::vector<T>& v) {
  kkt_status st = dalloc(h, out, v.size());
  if (st != KKT_OK) return st;
  if (!v.empty()) HIP_CHECK(h, hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return KKT_OK;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

// Scale that goes with a permutation in the solves' gathers and scatters:
// the matched and scaled analysis factors Ahat = Pm Dr A Dc, so the row
// permutation (pin) carries dr and the column permutation (qperm) dc.
// length of the handle's vectors (rows of every instance of a shared-pattern
// batch)
int vlen(kkt_handle h) { return h->an.n * h->inst.count; }

const double* scale_of(kkt_handle h, const int* perm) {
  return perm == h->pin ? h->rowsc : perm == h->qperm ? h->colsc : nullptr;
}

LUView view(kkt_handle h) {
  return LUView{h->an.n, h->lu_rowptr, h->lu_col, h->diag, h->lu_src, h->lu_val};
}

// M^{-1} b through the factors: x = Q U^{-1} L^{-1} P Q^T b ('N') or the
// transposed chain ('T').  b and x may not alias h->tmp.
void apply_factors(kkt_handle h, char op, const double* b, double* x, hipStream_t s) {
  const Analysis& A = h->an;
  const int n = A.n;
  LUView lu = view(h);
  const int sweeps = h->opt.solve_jacobi_sweeps;
  if (sweeps > 0 && op == 'N') {
    // approximate triangular solves: `sweeps` Jacobi sweeps per triangle,
    // starting from the right-hand side (FGMRES takes the variable
    // preconditioner)
    launch_gather(n, h->pin, scale_of(h, h->pin), b, h->tc, s);
    const double* cur = h->tc;
    double* bufs[2] = {h->ty, h->tz};
    int k = 0;
    for (int it = 0; it < sweeps; it++, k ^= 1) {
      launch_jacobi_sweep(0, lu, h->tc, cur, bufs[k], s);
      cur = bufs[k];
    }
    // U: right-hand side cur (copied to tmp), first iterate the right-hand side
    launch_copy(n, cur, h->tmp, s);
    const double* cu = h->tmp;
    cur = h->tmp;
    for (int it = 0; it < sweeps; it++, k ^= 1) {
      launch_jacobi_sweep(1, lu, cu, cur, bufs[k], s);
      cur = bufs[k];
    }
    launch_scatter(n, h->qperm, scale_of(h, h->qperm), cur, x, s);
    return;
  }
  if (h->use_sn && h->inst.count > 1) {
    // shared-pattern batch: the instances' permuted vectors side by side
    // (stride n + 1, the spare slot per instance taking idle lanes' stores),
    // the chain-block schedule handed out per (chunk, instance)
    int* stall = &h->st->stall;
    const Inst in = h->inst;
    const int cnt = in.count;
    if (op == 'N') {
      launch_gather_sentinel_mr(n, cnt, h->pin, nullptr, b, h->tc, h->ty, h->tz, h->ss, 0x6, s,
                                h->sn_triv0, h->diag, h->lu_val, 0, in.f1);
      launch_trisolve_sn(0, 1, lu, h->chs[0], nullptr, nullptr, nullptr, h->tc, h->ty, h->ss, 1,
                         stall, s, nullptr, nullptr, in);
      launch_trisolve_sn(1, 1, lu, h->chs[1], nullptr, nullptr, nullptr, h->ty, h->tz, h->ss, 2,
                         stall, s, nullptr, nullptr, in);
      launch_scatter_mr(n, cnt, h->qperm, nullptr, h->tz, x, s);
    } else {
      launch_gather_sentinel_mr(n, cnt, h->qperm, nullptr, b, h->tc, h->ty, h->tz, h->ss, 0x6, s,
                                h->sn_triv2, h->diag, h->lu_val, 1, in.f1);
      launch_trisolve_sn(2, 1, lu, h->chs[2], h->ut_ptr, h->ut_row, h->ut_pos, h->tc, h->ty,
                         h->ss, 1, stall, s, nullptr, nullptr, in);
      launch_trisolve_sn(3, 1, lu, h->chs[3], h->lt_ptr, h->lt_row, h->lt_pos, h->ty, h->tz,
                         h->ss, 2, stall, s, nullptr, nullptr, in);
      launch_scatter_mr(n, cnt, h->pin, nullptr, h->tz, x, s);
    }
    return;
  }
  if (h->use_sn) {
    // chain-blocked sparse rows and the dense trailing block: the block comes
    // last in the forward solves (L, U^T) and first in the backward ones
    int* stall = &h->st->stall;
    const int c0 = h->tail_c0, ts = h->tail_s, S = h->tail_S;
    if (op == 'N') {
      launch_gather_sentinel(n, h->pin, scale_of(h, h->pin), b, h->tc, h->ty, h->tz, h->ss, 0x6, s, h->sn_triv0,
                             h->diag, h->lu_val, 0);
      launch_trisolve_sn(0, 1, lu, h->chs[0], nullptr, nullptr, nullptr, h->tc, h->ty, h->ss, 1,
                         stall, s);
      launch_tail_solve_mw(0, lu, h->tail_T, S, ts, c0, h->tail_split0, nullptr, nullptr, nullptr,
                           h->tc, h->tail_rhs, h->ty, stall, s);
      launch_tail_solve_mw(1, lu, h->tail_T, S, ts, c0, nullptr, nullptr, nullptr, nullptr, h->ty,
                           h->tail_rhs, h->tz, stall, s);
      launch_udense_pre(h->u_nrows, h->u_rows, h->u_xend, lu, h->tz, h->u_pre, s);
      launch_trisolve_sn(1, 1, lu, h->chs[1], nullptr, nullptr, nullptr, h->ty, h->tz, h->ss, 2,
                         stall, s, h->u_xend, h->u_pre);
      launch_scatter(n, h->qperm, scale_of(h, h->qperm), h->tz, x, s);
    } else {
      launch_gather_sentinel(n, h->qperm, scale_of(h, h->qperm), b, h->tc, h->ty, h->tz, h->ss, 0x6, s, h->sn_triv2,
                             h->diag, h->lu_val, 1);
      launch_trisolve_sn(2, 1, lu, h->chs[2], h->ut_ptr, h->ut_row, h->ut_pos, h->tc, h->ty, h->ss,
                         1, stall, s);
      launch_tail_solve_mw(2, lu, h->tail_T, S, ts, c0, h->tail_split2, h->ut_ptr, h->ut_row,
                           h->ut_pos, h->tc, h->tail_rhs, h->ty, stall, s);
      launch_tail_solve_mw(3, lu, h->tail_T, S, ts, c0, nullptr, nullptr, nullptr, nullptr, h->ty,
                           h->tail_rhs, h->tz, stall, s);
      launch_trisolve_sn(3, 1, lu, h->chs[3], h->lt_ptr, h->lt_row, h->lt_pos, h->ty, h->tz, h->ss,
                         2, stall, s);
      launch_scatter(n, h->pin, scale_of(h, h->pin), h->tz, x, s);
    }
    return;
  }
  if (h->syncfree && h->light) {
    // per triangle: thin leading levels (one workgroup), the levels between
    // (dependency-driven), thin trailing levels (one workgroup)
    auto tri = [&](int mode, const int* tp, const int* tr, const int* tq, const double* c,
                   double* y, int slot) {
      launch_trisolve_seg(mode, h->seg_pre[mode], h->lu_val, c, y, s);
      launch_trisolve_vflag(mode, lu, h->chb[mode], tp, tr, tq, c, y, h->ss, slot, &h->st->stall,
                            s);
      launch_trisolve_seg(mode, h->seg_post[mode], h->lu_val, c, y, s);
    };
    if (op == 'N') {
      launch_gather_sentinel(n, h->pin, scale_of(h, h->pin), b, h->tc, h->ty, h->tz, h->ss, 0x6, s);
      tri(0, nullptr, nullptr, nullptr, h->tc, h->ty, 1);
      tri(1, nullptr, nullptr, nullptr, h->ty, h->tz, 2);
      launch_scatter(n, h->qperm, scale_of(h, h->qperm), h->tz, x, s);
    } else {
      launch_gather_sentinel(n, h->qperm, scale_of(h, h->qperm), b, h->tc, h->ty, h->tz, h->ss, 0x6, s);
      tri(2, h->ut_ptr, h->ut_row, h->ut_pos, h->tc, h->ty, 1);
      tri(3, h->lt_ptr, h->lt_row, h->lt_pos, h->ty, h->tz, 2);
      launch_scatter(n, h->pin, scale_of(h, h->pin), h->tz, x, s);
    }
    return;
  }
  if (h->syncfree) {
    if (op == 'N') {
      launch_gather_prep(n, h->pin, scale_of(h, h->pin), b, h->tmp, h->ss, 0x6, s);
      launch_trisolve_syncfree(0, lu, h->ch_l, nullptr, nullptr, nullptr, h->tmp, h->ready_a,
                               h->ss, 1, &h->st->stall, s);
      launch_trisolve_syncfree(1, lu, h->ch_u, nullptr, nullptr, nullptr, h->tmp, h->ready_b,
                               h->ss, 2, &h->st->stall, s);
      launch_scatter(n, h->qperm, scale_of(h, h->qperm), h->tmp, x, s);
    } else {
      launch_gather_prep(n, h->qperm, scale_of(h, h->qperm), b, h->tmp, h->ss, 0x6, s);
      launch_trisolve_syncfree(2, lu, h->ch_ut, h->ut_ptr, h->ut_row, h->ut_pos, h->tmp,
                               h->ready_a, h->ss, 1, &h->st->stall, s);
      launch_trisolve_syncfree(3, lu, h->ch_lt, h->lt_ptr, h->lt_row, h->lt_pos, h->tmp,
                               h->ready_b, h->ss, 2, &h->st->stall, s);
      launch_scatter(n, h->pin, scale_of(h, h->pin), h->tmp, x, s);
    }
    return;
  }
  if (op == 'N') {
    launch_gather(n, h->pin, scale_of(h, h->pin), b, h->tmp, s);
    for (size_t l = 0; l + 1 < A.lev_ptr.size(); l++)
      launch_lsolve_rows(lu, h->lev_rows + A.lev_ptr[l], A.lev_ptr[l + 1] - A.lev_ptr[l], 0,
                         h->tmp, s);
    for (size_t l = 0; l + 1 < A.ulev_ptr.size(); l++)
      launch_usolve_rows(lu, h->ulev_rows + A.ulev_ptr[l], A.ulev_ptr[l + 1] - A.ulev_ptr[l], 0,
                         h->tmp, s);
    launch_scatter(n, h->qperm, scale_of(h, h->qperm), h->tmp, x, s);
  } else {
    launch_gather(n, h->qperm, scale_of(h, h->qperm), b, h->tmp, s);
    for (size_t l = 0; l + 1 < A.utlev_ptr.size(); l++)
      launch_utsolve_cols(lu, h->utlev_rows + A.utlev_ptr[l], A.utlev_ptr[l + 1] - A.utlev_ptr[l],
                          h->ut_ptr, h->ut_row, h->ut_pos, h->tmp, s);
    for (size_t l = 0; l + 1 < A.ltlev_ptr.size(); l++)
      launch_ltsolve_cols(lu, h->ltlev_rows + A.ltlev_ptr[l], A.ltlev_ptr[l + 1] - A.ltlev_ptr[l],
                          h->lt_ptr, h->lt_row, h->lt_pos, h->tmp, s);
    launch_scatter(n, h->pin, scale_of(h, h->pin), h->tmp, x, s);
  }
}

// (n+1) x MAX_RHS_PASS buffers of the multi-column solves (allocated by the
// analysis of a handle whose schedules have multi-column solves)
kkt_status ensure_multi(kkt_handle h, int nr) {
  if (h->mcap >= nr) return KKT_OK;
  return fail(h, KKT_ERR_STATE, "no multi-column solve workspace for this schedule");
}

// M^{-1} B for nr <= MAX_RHS_PASS columns (dependency-driven, value-as-flag)
void apply_factors_multi(kkt_handle h, char op, int nr, const double* b, double* x,
                         hipStream_t s) {
  const int n = h->an.n;
  LUView lu = view(h);
  int* stall = &h->st->stall;
  if (h->use_sn) {
    // chain-blocked sparse rows and the dense block, SN_MAX_RHS columns a pass
    const int c0 = h->tail_c0, ts = h->tail_s, S = h->tail_S;
    const size_t ld = (size_t)n + 1;
    for (int r0 = 0; r0 < nr; r0 += SN_MAX_RHS) {
      const int k = std::min(SN_MAX_RHS, nr - r0);
      const double* bb = b + (size_t)r0 * n;
      double* xx = x + (size_t)r0 * n;
      double *mc = h->mc + r0 * ld, *my = h->my + r0 * ld, *mz = h->mz + r0 * ld;
      if (op == 'N') {
        launch_gather_sentinel_mr(n, k, h->pin, scale_of(h, h->pin), bb, mc, my, mz, h->ss, 0x6, s, h->sn_triv0,
                                  h->diag, h->lu_val, 0);
        launch_trisolve_sn(0, k, lu, h->chs[0], nullptr, nullptr, nullptr, mc, my, h->ss, 1,
                           stall, s);
        launch_tail_solve(0, k, lu, h->tail_T, S, ts, c0, h->tail_split0, nullptr, nullptr,
                          nullptr, mc, h->tail_rhs, my, s);
        launch_tail_solve(1, k, lu, h->tail_T, S, ts, c0, nullptr, nullptr, nullptr, nullptr, my,
                          h->tail_rhs, mz, s);
        launch_trisolve_sn(1, k, lu, h->chs[1], nullptr, nullptr, nullptr, my, mz, h->ss, 2,
                           stall, s);
        launch_scatter_mr(n, k, h->qperm, scale_of(h, h->qperm), mz, xx, s);
      } else {
        launch_gather_sentinel_mr(n, k, h->qperm, scale_of(h, h->qperm), bb, mc, my, mz, h->ss, 0x6, s, h->sn_triv2,
                                  h->diag, h->lu_val, 1);
        launch_trisolve_sn(2, k, lu, h->chs[2], h->ut_ptr, h->ut_row, h->ut_pos, mc, my, h->ss, 1,
                           stall, s);
        launch_tail_solve(2, k, lu, h->tail_T, S, ts, c0, h->tail_split2, h->ut_ptr, h->ut_row,
                          h->ut_pos, mc, h->tail_rhs, my, s);
        launch_tail_solve(3, k, lu, h->tail_T, S, ts, c0, nullptr, nullptr, nullptr, nullptr, my,
                          h->tail_rhs, mz, s);
        launch_trisolve_sn(3, k, lu, h->chs[3], h->lt_ptr, h->lt_row, h->lt_pos, my, mz, h->ss, 2,
                           stall, s);
        launch_scatter_mr(n, k, h->pin, scale_of(h, h->pin), mz, xx, s);
      }
    }
    return;
  }
  if (op == 'N') {
    launch_gather_sentinel_mr(n, nr, h->pin, scale_of(h, h->pin), b, h->mc, h->my, h->mz, h->ss, 0x6, s);
    launch_trisolve_vflag_mr(0, nr, lu, h->ch_l, nullptr, nullptr, nullptr, h->mc, h->my, h->ss,
                             1, stall, s);
    launch_trisolve_vflag_mr(1, nr, lu, h->ch_u, nullptr, nullptr, nullptr, h->my, h->mz, h->ss,
                             2, stall, s);
    launch_scatter_mr(n, nr, h->qperm, scale_of(h, h->qperm), h->mz, x, s);
  } else {
    launch_gather_sentinel_mr(n, nr, h->qperm, scale_of(h, h->qperm), b, h->mc, h->my, h->mz, h->ss, 0x6, s);
    launch_trisolve_vflag_mr(2, nr, lu, h->ch_ut, h->ut_ptr, h->ut_row, h->ut_pos, h->mc, h->my,
                             h->ss, 1, stall, s);
    launch_trisolve_vflag_mr(3, nr, lu, h->ch_lt, h->lt_ptr, h->lt_row, h->lt_pos, h->my, h->mz,
                             h->ss, 2, stall, s);
    launch_scatter_mr(n, nr, h->pin, scale_of(h, h->pin), h->mz, x, s);
  }
}

void op_spmv(kkt_handle h, char op, const double* x, double* y, hipStream_t s) {
  if (op == 'N')
    launch_spmv(h->an.n, 'N', h->a_rowptr, h->a_col, nullptr, h->aval, x, y, s);
  else
    launch_spmv(h->an.n, 'T', h->at_ptr, h->at_row, h->at_pos, h->aval, x, y, s);
}

double eta_of(double rn, double an, double xn) {
  const double den = an * xn;
  return den == 0.0 ? (rn == 0.0 ? 0.0 : INFINITY) : rn / den;
}

// Device work of the residual check (no synchronisation: also captured into
// graphs): r = b - op(A) x with its maxima, and per-instance maxima in a batch.
void residual_launch(kkt_handle h, char op, const double* b, const double* x, double* r,
                     hipStream_t s) {
  launch_reset_stats(h->st, 2, s);
  if (op == 'N')
    launch_residual(h->an.n, 'N', h->a_rowptr, h->a_col, nullptr, h->aval, b, x, r, h->st, s,
                    h->red);
  else
    launch_residual(h->an.n, 'T', h->at_ptr, h->at_row, h->at_pos, h->aval, b, x, r, h->st, s,
                    h->red);
  if (h->batch_count > 0)
    launch_seg_stats(h->batch_count, h->d_row_off, op == 'N' ? h->rowabs : h->colabs, r, x,
                     h->inst_out, s);
}

// Read back the residual maxima (synchronises the stream); eta = the largest
// instance eta of a batch, or the system's eta.
kkt_status read_batch_eta(kkt_handle h, char op, double* eta_max);

kkt_status read_eta(kkt_handle h, char op, hipStream_t s, double* eta) {
  HIP_CHECK(h, hipMemcpyAsync(h->h_st, h->st, sizeof(DevStats), hipMemcpyDeviceToHost, s));
  HIP_CHECK(h, hipStreamSynchronize(s));
  if (h->h_st->stall)
    return fail(h, KKT_ERR_DEVICE, "a dependency wait hit its spin limit (results invalid)");
  if (h->batch_count > 0) return read_batch_eta(h, op, eta);
  const double rn = bits_to_double(h->h_st->rmax), xn = bits_to_double(h->h_st->xmax);
  const double an = bits_to_double(op == 'N' ? h->h_st->anorm : h->h_st->anorm1);
  *eta = eta_of(rn, an, xn);
  return KKT_OK;
}

kkt_status read_batch_eta(kkt_handle h, char op, double* eta_max) {
  (void)op;
  HIP_CHECK(h, hipDeviceSynchronize());
  HIP_CHECK(h, hipMemcpy(h->h_inst.data(), h->inst_out, h->h_inst.size() * sizeof(double),
                         hipMemcpyDeviceToHost));
  // maxima that keep a NaN once seen (a broken instance stays visible)
  auto nan_max = [](double a, double b) { return (a != a || b != b) ? a + b : (a > b ? a : b); };
  double mx = 0.0;
  for (int t = 0; t < h->batch_count; t++) {
    double m[3] = {0.0, 0.0, 0.0};
    for (int sl = 0; sl < SEG_SLICES; sl++)
      for (int k = 0; k < 3; k++)
        m[k] = nan_max(m[k], h->h_inst[3 * ((size_t)t * SEG_SLICES + sl) + k]);
    const double e = eta_of(m[1], m[0], m[2]);
    h->inst_eta[t] = e;
    mx = nan_max(mx, e);
  }
  if (eta_max) *eta_max = mx;
  return KKT_OK;
}

// r = b - op(A) x; returns eta (synchronises the stream)
kkt_status residual_eta(kkt_handle h, char op, const double* b, const double* x, double* r,
                        hipStream_t s, double* eta) {
  residual_launch(h, op, b, x, r, s);
  return read_eta(h, op, s, eta);
}

// Direct solve (skipped when direct_done: x already holds it) and FGMRES-CGS2
// refinement of one right-hand side.
kkt_status solve_one(kkt_handle h, char op, const double* b, double* x, hipStream_t s,
                     int* iters_out, double* eta_out, double* eta0_out, bool direct_done = false) {
  const int n = h->an.n, m = h->m;
  const kkt_options& o = h->opt;
  if (!direct_done) apply_factors(h, op, b, x, s);
  double eta;
  kkt_status st = residual_eta(h, op, b, x, h->r, s, &eta);
  if (st != KKT_OK) return st;
  *eta0_out = eta;
  int it = 0;
  bool done = eta <= o.eta_target && it >= o.min_iters;
  if (o.refine == 1) {
    // classical iterative refinement: x <- x + M^{-1} r (r from residual_eta)
    while (!done && it < o.fgmres_max_iters) {
      apply_factors(h, op, h->r, h->w, s);
      launch_add(n, h->w, x, s);
      it++;
      st = residual_eta(h, op, b, x, h->r, s, &eta);
      if (st != KKT_OK) return st;
      done = eta <= o.eta_target && it >= o.min_iters;
    }
    *iters_out = it;
    *eta_out = eta;
    return (eta <= o.eta_target) ? KKT_OK : KKT_WARN_NOT_CONVERGED;
  }
  bool at_xt = false;
  while (!done && it < o.fgmres_max_iters) {
    launch_multidot(n, 1, h->r, n, h->r, h->partial, h->ww, s);
    launch_arnoldi_start(n, m, h->r, h->ww, h->V, h->g, s);
    bool breakdown = false;
    for (int j = 0; j < m && it < o.fgmres_max_iters; j++) {
      double* vj = h->V + (long)j * n;
      double* zj = h->Z + (long)j * n;
      apply_factors(h, op, vj, zj, s);
      op_spmv(h, op, zj, h->w, s);
      launch_multidot(n, j + 1, h->V, n, h->w, h->partial, h->h, s);
      launch_multiaxpy(n, j + 1, h->V, n, h->h, h->w, s);
      launch_multidot(n, j + 1, h->V, n, h->w, h->partial, h->h2, s);
      launch_multiaxpy(n, j + 1, h->V, n, h->h2, h->w, s);
      launch_multidot(n, 1, h->w, n, h->w, h->partial, h->ww, s);
      launch_givens(j, m, h->h, h->h2, h->ww, h->H, h->cs, h->sn, h->g, h->y, h->hn, s);
      launch_scale_div(n, h->w, h->hn, h->V + (long)(j + 1) * n, s);
      launch_combine(n, j + 1, h->Z, n, h->y, x, h->xt, s);
      it++;
      st = residual_eta(h, op, b, h->xt, h->r, s, &eta);
      if (st != KKT_OK) return st;
      at_xt = true;
      double hn;
      HIP_CHECK(h, hipMemcpy(&hn, h->hn, sizeof(double), hipMemcpyDeviceToHost));
      if (eta <= o.eta_target && it >= o.min_iters) {
        done = true;
        break;
      }
      if (!(hn > 0.0)) {
        breakdown = true;
        break;
      }
    }
    // restart from the current iterate (r already holds its residual)
    if (at_xt) {
      HIP_CHECK(h, hipMemcpyAsync(x, h->xt, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
      at_xt = false;
    }
    if (breakdown) break;
  }
  if (at_xt)
    HIP_CHECK(h, hipMemcpyAsync(x, h->xt, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  *iters_out = it;
  *eta_out = eta;
  return (eta <= o.eta_target) ? KKT_OK : KKT_WARN_NOT_CONVERGED;
}

// Iterations the device-checked refinement launches per group.  Adaptive
// (refine_budget = -1): twice what the last observed solve needed plus two;
// the full budget after a solve that did not converge, after the matrix
// changed without a refactorization (kkt_update_matrix), and whenever
// refinement is part of the configuration (static pivoting, Jacobi-sweep
// solves, forced iterations).
int fg_budget(kkt_handle h) {
  const kkt_options& o = h->opt;
  int b = o.fgmres_max_iters;
  if (o.refine_budget > 0) {
    b = std::min(o.refine_budget, o.fgmres_max_iters);
  } else if (o.refine_budget < 0 && o.pivot_perturb_rel == 0.0 && o.solve_jacobi_sweeps == 0 &&
             o.min_iters == 0) {
    if (h->ev_fs_recorded && hipEventQuery(h->ev_fs) == hipSuccess) {
      h->auto_need = h->h_fs->it_max;
      if (h->h_fs->not_conv) h->auto_full = true;
      h->ev_fs_recorded = false;
    }
    if (!h->auto_full) b = std::min(o.fgmres_max_iters, 2 * h->auto_need + 2);
    h->auto_full = false;
  }
  return std::max(b, std::min(o.min_iters, o.fgmres_max_iters));
}

// Outcome of an adaptive-budget solve, copied behind an event (no wait).
void fg_observe(kkt_handle h, hipStream_t s) {
  if (h->opt.refine_budget >= 0 || !h->h_fs || !h->ev_fs) return;
  if (hipMemcpyAsync(h->h_fs, h->fs, sizeof(FgState), hipMemcpyDeviceToHost, s) == hipSuccess &&
      hipEventRecord(h->ev_fs, s) == hipSuccess)
    h->ev_fs_recorded = true;
}

// M^{-1} for g columns (column stride n)
void apply_group(kkt_handle h, char op, int g, const double* b, double* x, hipStream_t s) {
  if (g == 1)
    apply_factors(h, op, b, x, s);
  else
    apply_factors_multi(h, op, g, b, x, s);
}

// r = b - op(A) x for g columns and the device stop test after it_now
// iterations (first: the check of the direct solve); a block-diagonal batch
// is judged by its largest instance eta.
void check_group(kkt_handle h, const FgBufs& fb, char op, int g, const double* b,
                 const double* x, int it_now, int first, const FgParams& p, hipStream_t s) {
  const int n = vlen(h);
  const int batch = h->batch_count > 0 ? 1 : 0;
  if (op == 'N')
    launch_fg_resid(n, g, h->a_rowptr, h->a_col, nullptr, h->aval, b, x, h->r, fb, h->st, 0,
                    it_now, first, batch, p, s, h->inst);
  else
    launch_fg_resid(n, g, h->at_ptr, h->at_row, h->at_pos, h->aval, b, x, h->r, fb, h->st, 1,
                    it_now, first, batch, p, s, h->inst);
  if (batch) {
    launch_seg_stats(h->batch_count, h->d_row_off, op == 'N' ? h->rowabs : h->colabs, h->r, x,
                     h->inst_out, s);
    launch_fg_check_batch(h->batch_count, h->inst_out, fb, h->st, it_now, first, p, s);
  }
}

// Device-checked solve of g <= fg_cols right-hand sides (b, x column stride
// n): direct solve, stop test, then a fixed budget of refinement iterations
// (FGMRES-CGS2, or classical refinement with refine = 1) whose kernels return
// at once after the test stopped their column; the triangular solves stop
// with the whole group.  Nothing here waits for the device: the outcome is
// read by kkt_sync_report.  Stream-ordered only, so it can be captured.
// fb: the refinement's state and partial sums (the handle's, or the
// library's static scratch array for kkt_solve_noalloc).
void solve_group_async(kkt_handle h, const FgBufs& fb, char op, int g, const double* b, double* x,
                       bool first_group, int budget, hipStream_t s) {
  const int n = vlen(h), m = h->m;
  const kkt_options& o = h->opt;
  const FgParams p{o.eta_target, o.min_iters, o.fgmres_max_iters};
  const size_t gn = (size_t)g * n;
  launch_fg_begin(fb, first_group ? 1 : 0, s);
  apply_group(h, op, g, b, x, s);
  check_group(h, fb, op, g, b, x, 0, 1, p, s);
  const bool ir = o.refine == 1;
  set_launch_gate(&fb.fs->stop_all);
  for (int it = 0; it < budget; it++) {
    if (ir) {
      apply_group(h, op, g, h->r, h->w, s);
      launch_fg_add(n, g, h->w, x, fb, s);
      check_group(h, fb, op, g, b, x, it + 1, 0, p, s);
      continue;
    }
    const int j = it % m;
    if (j == 0) launch_fg_restart(n, g, m, h->r, h->xt, x, it > 0 ? 1 : 0, h->V, fb, s);
    const double* vj = h->V + j * gn;
    double* zj = h->Z + j * gn;
    apply_group(h, op, g, vj, zj, s);
    if (op == 'N')
      launch_fg_arnoldi(n, g, j, h->a_rowptr, h->a_col, nullptr, h->aval, zj, h->V, h->w, fb, s,
                        h->inst);
    else
      launch_fg_arnoldi(n, g, j, h->at_ptr, h->at_row, h->at_pos, h->aval, zj, h->V, h->w, fb,
                        s, h->inst);
    launch_fg_cgs(0, n, g, j, m, h->V, h->w, fb, s);
    launch_fg_cgs(1, n, g, j, m, h->V, h->w, fb, s);
    launch_fg_update(n, g, j, m, h->w, h->V + (j + 1) * gn, h->Z, x, h->xt, fb, s);
    check_group(h, fb, op, g, b, h->xt, it + 1, 0, p, s);
  }
  set_launch_gate(nullptr);
  launch_fg_finish(n, g, h->xt, x, ir ? 1 : 0, fb, s);
}

// All right-hand sides, device-checked, in groups of the handle's width.
// budget: iterations launched per group (fg_budget; a captured graph takes the
// full budget, since it cannot adapt between replays)
void solve_async(kkt_handle h, const FgBufs& fb, char op, int nrhs, const double* b, double* x,
                 int budget, hipStream_t s) {
  const int n = vlen(h);
  // one column at a time for approximate solves (no multi-column form) and
  // batches (their stop test is per instance of one column)
  const int gmax =
      ((op == 'N' && h->opt.solve_jacobi_sweeps > 0) || h->batch_count > 0) ? 1 : h->fg_cols;
  for (int c0 = 0; c0 < nrhs; c0 += gmax) {
    const int g = std::min(gmax, nrhs - c0);
    solve_group_async(h, fb, op, g, b + (size_t)c0 * n, x + (size_t)c0 * n, c0 == 0, budget, s);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Entry point without allocation (kkt_solve_noalloc): the refinement's
// per-call scratch -- stop-test state, reduction tickets, partial sums and
// the small least-squares arrays -- lives in this file-scope device array
// instead of the handle's workspace.  Each GPU holds its own copy until the
// process ends; its device address is looked up once per device (kkt_create,
// with that device current) and only that address is used from host code.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(2) << 20;  // 2 MiB per GPU
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch` (looked up once).
kkt_status scratch_setup(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return KKT_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return KKT_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KKT_ERR_DEVICE;
  g_scratch_ptr[dev] = p;
  return KKT_OK;
}

unsigned char* scratch_of(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (unsigned char*)g_scratch_ptr[dev];
}

// The refinement buffers for restart length m carved from the scratch array
// in 256-byte aligned pieces; false when they do not fit.
bool carve_fgbufs(unsigned char* base, int m, FgBufs* fb) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  const size_t d = sizeof(double), c = FG_MAX_COLS;
  fb->fs = (FgState*)take(sizeof(FgState));
  fb->tick1 = (unsigned int*)take(sizeof(unsigned int) * c * FG_TICK_GROUPS * FG_TICK_STRIDE);
  fb->part = (double*)take(d * c * FG_BLOCKS * 32);
  fb->hbuf = (double*)take(d * c * 32);
  fb->h2buf = (double*)take(d * c * 32);
  fb->H = (double*)take(d * c * (size_t)(m + 1) * m);
  fb->cs = (double*)take(d * c * m);
  fb->sn = (double*)take(d * c * m);
  fb->gvec = (double*)take(d * c * (m + 1));
  fb->y = (double*)take(d * c * m);
  return off <= NOALLOC_SCRATCH_BYTES;
}
}  // namespace

extern "C" {

void kkt_options_default(kkt_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->ordering = 0;
  o->pivot_tau = 1e-10;
  o->fgmres_restart = 20;
  o->fgmres_max_iters = 20;
  o->min_iters = 0;
  o->eta_target = 1e-12;
  o->tiny_pivot_rel = 1e-18;
  o->device = 0;
  o->schedule = 0;
}

kkt_status kkt_create(const kkt_options* opt, kkt_handle* out) {
  if (!out) return KKT_ERR_INVALID_ARG;
  *out = nullptr;
  kkt_options o;
  kkt_options_default(&o);
  if (opt) o = *opt;
  if (o.ordering < 0 || o.ordering > 2 || !(o.pivot_tau > 0.0 && o.pivot_tau <= 1.0) ||
      o.fgmres_restart < 1 || o.fgmres_restart > 30 || o.fgmres_max_iters < 0 ||
      o.min_iters < 0 || !(o.eta_target >= 0.0) || !(o.tiny_pivot_rel >= 0.0) || o.device < 0 ||
      o.schedule < 0 || o.schedule > 2 || o.sync_mode < 0 || o.sync_mode > 2 ||
      o.solve_entries_per_lane < 0 || o.solve_entries_per_lane > 64 ||
      (o.refactor_waves_per_block != 0 && o.refactor_waves_per_block != 1 &&
       o.refactor_waves_per_block != 2 && o.refactor_waves_per_block != 4) ||
      o.solve_thin_rows < -1 || o.solve_thin_rows > SEG_MAX_LEVEL_ROWS || o.dense_tail < -1 ||
      o.dense_tail > DENSE_TAIL_MAX || o.solve_blocks_per_cu < 0 || o.solve_blocks_per_cu > 8 ||
      o.solve_chain < -1 || o.solve_chain > SN_KMAX || o.refactor_map < -1 || o.refactor_map > 0 ||
      o.refactor_crit_height < -1 || o.refactor_waves_per_cu < 0 || o.refine < 0 || o.refine > 1 ||
      o.auto_reanalyze < 0 || o.auto_reanalyze > 1 || o.solve_jacobi_sweeps < 0 ||
      o.refactor_short_rows < -1 || o.refactor_short_rows > 0 || o.refactor_long_rows < -1 ||
      o.refactor_long_rows > 0 || o.refine_sync < 0 || o.refine_sync > 1 || o.refine_budget < -1 ||
      o.dense_lu < 0 || o.dense_lu > 1 || o.debug_spin_limit < 0 || o.debug_schedule < 0 ||
      o.matching < 0 || o.matching > 1 || o.refactor_micro_rows < -1 ||
      o.refactor_micro_rows > 0 || o.debug_schedule > 1 || o.debug_timeline < 0 ||
      o.debug_timeline > 1 || o.refactor_short_band < 0 || o.refactor_short_band > 256 ||
      !(o.pivot_perturb_rel >= 0.0 && o.pivot_perturb_rel < 1.0))
    return KKT_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o.device >= ndev) return KKT_ERR_DEVICE;
  // the device address of the no-allocation scratch array, once per device
  if (hipSetDevice(o.device) != hipSuccess || scratch_setup(o.device) != KKT_OK)
    return KKT_ERR_DEVICE;
  kkt_ctx* h = new (std::nothrow) kkt_ctx();
  if (!h) return KKT_ERR_OUT_OF_MEMORY;
  h->opt = o;
  h->m = o.fgmres_restart;
  *out = h;
  return KKT_OK;
}

kkt_status kkt_destroy(kkt_handle h) {
  if (!h) return KKT_ERR_INVALID_ARG;
  (void)hipSetDevice(h->opt.device);
  (void)hipDeviceSynchronize();
  free_device(h);
  delete h;
  return KKT_OK;
}

static kkt_status install_analysis(kkt_handle h, Analysis&& an, int st, int32_t n, int64_t nnz,
                                   const int64_t* rowptr, const int32_t* colind,
                                   const double* values0,
                                   std::chrono::steady_clock::time_point t0);

kkt_status kkt_analyze(kkt_handle h, int32_t n, int64_t nnz, const int64_t* rowptr,
                       const int32_t* colind, const double* values0, const int32_t* user_q) {
  if (!h) return KKT_ERR_INVALID_ARG;
  h->err.clear();
  if (nnz > (int64_t)INT32_MAX) return fail(h, KKT_ERR_TOO_LARGE, "nnz(A) exceeds int32");
  auto t0 = std::chrono::steady_clock::now();
  AnalyzeOptions ao;
  ao.ordering = h->opt.ordering;
  ao.tau = h->opt.pivot_tau;
  ao.matching = h->opt.matching;
  Analysis an;
  std::string msg;
  int st;
  try {
    st = analyze(n, nnz, rowptr, colind, values0, user_q, ao, an, &msg);
  } catch (const std::bad_alloc&) {
    return fail(h, KKT_ERR_OUT_OF_MEMORY, "host allocation failed in analyze");
  }
  if (st < 0) return fail(h, (kkt_status)st, msg);
  h->batch_count = 0;
  h->inst = Inst();
  h->row_off.clear();
  h->nnz_off.clear();
  // the pattern, kept for re-analysis
  h->pat_rowptr.assign(rowptr, rowptr + n + 1);
  h->pat_colind.assign(colind, colind + nnz);
  return install_analysis(h, std::move(an), st, n, nnz, rowptr, colind, values0, t0);
}

kkt_status kkt_reanalyze(kkt_handle h, const double* d_values, void* stream) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed || h->batch_count > 0 || h->pat_rowptr.empty())
    return fail(h, KKT_ERR_STATE, "kkt_reanalyze needs a single-system analysis");
  if (!d_values) return fail(h, KKT_ERR_INVALID_ARG, "d_values is NULL");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  const int32_t n = h->an.n;
  const int64_t nnz = (int64_t)h->pat_colind.size();
  std::vector<double> vals((size_t)nnz);
  HIP_CHECK(h, hipStreamSynchronize((hipStream_t)stream));
  HIP_CHECK(h, hipMemcpy(vals.data(), d_values, (size_t)nnz * sizeof(double),
                         hipMemcpyDeviceToHost));
  // the ordering depends on the pattern only: keep Q, redo the pivoting pass
  std::vector<int32_t> q(h->an.Q);
  std::vector<int64_t> rp(h->pat_rowptr);
  std::vector<int32_t> ci(h->pat_colind);
  auto t0 = std::chrono::steady_clock::now();
  AnalyzeOptions ao;
  ao.ordering = 2;
  ao.tau = h->opt.pivot_tau;
  Analysis an;
  std::string msg;
  int st;
  try {
    // with matching: the stored matching and scaling, the pivoting pass redone
    st = h->an.match.empty()
             ? analyze(n, nnz, rp.data(), ci.data(), vals.data(), q.data(), ao, an, &msg)
             : analyze_scaled(n, nnz, rp.data(), ci.data(), vals.data(), h->an.match, h->an.dr,
                              h->an.dc, q.data(), ao, an, &msg);
  } catch (const std::bad_alloc&) {
    return fail(h, KKT_ERR_OUT_OF_MEMORY, "host allocation failed in analyze");
  }
  if (st < 0) return fail(h, (kkt_status)st, msg);
  h->reanalyses++;
  return install_analysis(h, std::move(an), st, n, nnz, rp.data(), ci.data(), vals.data(), t0);
}

// Upload of an analysis (single system or block-diagonal batch) and of A's
// pattern; allocation of every workspace.
static kkt_status install_analysis(kkt_handle h, Analysis&& an, int st, int32_t n, int64_t nnz,
                                   const int64_t* rowptr, const int32_t* colind,
                                   const double* values0,
                                   std::chrono::steady_clock::time_point t0) {
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  HIP_CHECK(h, hipDeviceSynchronize());
  free_device(h);
  h->an = std::move(an);
  const Analysis& A = h->an;
  kkt_status ks;
#define UP(dst, vec)                   \
  if ((ks = upload(h, &dst, vec)) != KKT_OK) { \
    free_device(h);                    \
    return ks;                         \
  }
  UP(h->lu_rowptr, A.lu_rowptr);
  UP(h->lu_col, A.lu_col);
  UP(h->diag, A.diag);
  UP(h->lu_src, A.lu_src);
  UP(h->lev_rows, A.lev_rows);
  UP(h->ulev_rows, A.ulev_rows);
  UP(h->utlev_rows, A.utlev_rows);
  UP(h->ltlev_rows, A.ltlev_rows);
  UP(h->ut_ptr, A.ut_ptr);
  UP(h->ut_pos, A.ut_pos);
  UP(h->lt_ptr, A.lt_ptr);
  UP(h->lt_pos, A.lt_pos);
  {
    // row index of every transposed-view position
    std::vector<int32_t> rowof(A.lu_col.size());
    for (int32_t i = 0; i < n; i++)
      for (int32_t q = A.lu_rowptr[i]; q < A.lu_rowptr[i + 1]; q++) rowof[q] = i;
    std::vector<int32_t> ur(A.ut_pos.size()), lr(A.lt_pos.size());
    for (size_t t = 0; t < ur.size(); t++) ur[t] = rowof[A.ut_pos[t]];
    for (size_t t = 0; t < lr.size(); t++) lr[t] = rowof[A.lt_pos[t]];
    UP(h->ut_row, ur);
    UP(h->lt_row, lr);
    std::vector<int32_t> pin(n), q(A.Q);
    for (int32_t i = 0; i < n; i++) pin[i] = A.Q[A.P[i]];
    h->rowsc = h->colsc = h->ascale = h->avs = nullptr;
    if (!A.match.empty()) {
      // the factors are those of Ahat = Pm Dr A Dc: factor row i is A's row
      // match[Q[P[i]]] scaled by dr, factor column k is A's column Q[k]
      // scaled by dc
      std::vector<double> rsv(n), csv(n);
      for (int32_t i = 0; i < n; i++) {
        pin[i] = A.match[pin[i]];
        rsv[i] = A.dr[pin[i]];
        csv[i] = A.dc[A.Q[i]];
      }
      UP(h->rowsc, rsv);
      UP(h->colsc, csv);
      UP(h->ascale, A.ascale);
      if ((ks = dalloc(h, &h->avs, (size_t)nnz)) != KKT_OK) {
        free_device(h);
        return ks;
      }
    }
    UP(h->pin, pin);
    UP(h->qperm, q);
    // A pattern (int32 row pointers) and its column view
    std::vector<int32_t> arp(n + 1), acol(colind, colind + nnz);
    for (int32_t i = 0; i <= n; i++) arp[i] = (int32_t)rowptr[i];
    std::vector<int32_t> atp(n + 1, 0), atr(nnz), atpos(nnz);
    for (int64_t p = 0; p < nnz; p++) atp[colind[p] + 1]++;
    for (int32_t j = 0; j < n; j++) atp[j + 1] += atp[j];
    std::vector<int32_t> nx(atp.begin(), atp.end() - 1);
    for (int32_t i = 0; i < n; i++)
      for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
        int32_t t = nx[colind[p]]++;
        atr[t] = i;
        atpos[t] = (int32_t)p;
      }
    UP(h->a_rowptr, arp);
    UP(h->a_col, acol);
    UP(h->at_ptr, atp);
    UP(h->at_row, atr);
    UP(h->at_pos, atpos);
  }
  {
    // chunked level schedules of the four triangular solves: rows of one
    // level, G lanes per row with G the smallest power of two in [4, 64]
    // giving at most eight entries per lane (one load batch) for the level's
    // longest row
    auto chunks = [&](const std::vector<int32_t>& lp, const std::vector<int32_t>& rows,
                      auto len_of, ChunkSched& cs, std::vector<int32_t>& st,
                      std::vector<int32_t>& me, size_t l0 = 0, size_t l1 = SIZE_MAX) {
      st.clear();
      me.clear();
      l1 = std::min(l1, lp.size() - 1);
      for (size_t l = l0; l < l1; l++) {
        int mx = 0;
        for (int32_t t = lp[l]; t < lp[l + 1]; t++) mx = std::max(mx, (int)len_of(rows[t]));
        int lg = 2;
        const int per_lane = h->opt.solve_entries_per_lane > 0 ? h->opt.solve_entries_per_lane : 8;
        while (lg < 6 && (per_lane << lg) < mx) lg++;
        const int per = 64 >> lg;
        for (int32_t t = lp[l]; t < lp[l + 1]; t += per) {
          st.push_back(t);
          me.push_back((lg << 8) | std::min(per, lp[l + 1] - t));
        }
      }
      cs.nchunks = (int)st.size();
      cs.rows = nullptr;
    };
    std::vector<int32_t> st1, me1;
    int* dptr;
    int* dmeta;
    chunks(A.lev_ptr, A.lev_rows, [&](int i) { return A.diag[i] - A.lu_rowptr[i]; }, h->ch_l, st1,
           me1);
    UP(dptr, st1);
    UP(dmeta, me1);
    h->ch_l.start = dptr;
    h->ch_l.meta = dmeta;
    h->ch_l.rows = h->lev_rows;
    chunks(A.ulev_ptr, A.ulev_rows, [&](int i) { return A.lu_rowptr[i + 1] - A.diag[i] - 1; },
           h->ch_u, st1, me1);
    UP(dptr, st1);
    UP(dmeta, me1);
    h->ch_u.start = dptr;
    h->ch_u.meta = dmeta;
    h->ch_u.rows = h->ulev_rows;
    chunks(A.utlev_ptr, A.utlev_rows, [&](int j) { return A.ut_ptr[j + 1] - A.ut_ptr[j] - 1; },
           h->ch_ut, st1, me1);
    UP(dptr, st1);
    UP(dmeta, me1);
    h->ch_ut.start = dptr;
    h->ch_ut.meta = dmeta;
    h->ch_ut.rows = h->utlev_rows;
    chunks(A.ltlev_ptr, A.ltlev_rows, [&](int j) { return A.lt_ptr[j + 1] - A.lt_ptr[j]; },
           h->ch_lt, st1, me1);
    UP(dptr, st1);
    UP(dmeta, me1);
    h->ch_lt.start = dptr;
    h->ch_lt.meta = dmeta;
    h->ch_lt.rows = h->ltlev_rows;
    // thin runs at both ends of each schedule (modes 0 L, 1 U, 2 U^T, 3 L^T)
    const int thin = h->opt.solve_thin_rows == 0 ? 16 : h->opt.solve_thin_rows;
    const std::vector<int32_t>* tlp[4] = {&A.lev_ptr, &A.ulev_ptr, &A.utlev_ptr, &A.ltlev_ptr};
    const std::vector<int32_t>* trows[4] = {&A.lev_rows, &A.ulev_rows, &A.utlev_rows,
                                             &A.ltlev_rows};
    int* trows_dev[4] = {h->lev_rows, h->ulev_rows, h->utlev_rows, h->ltlev_rows};
    std::vector<int32_t> lu_row_of(A.lu_col.size());
    for (int32_t i = 0; i < n; i++)
      for (int32_t q = A.lu_rowptr[i]; q < A.lu_rowptr[i + 1]; q++) lu_row_of[q] = i;
    // entries of row i of the mode's triangle: (dependency row, value position)
    auto entries = [&](int mode, int i, std::vector<int32_t>& dep, std::vector<int32_t>& pos,
                       int32_t& dpos) {
      dep.clear();
      pos.clear();
      dpos = -1;
      if (mode == 0) {
        for (int32_t q = A.lu_rowptr[i]; q < A.diag[i]; q++) {
          dep.push_back(A.lu_col[q]);
          pos.push_back(q);
        }
      } else if (mode == 1) {
        dpos = A.diag[i];
        for (int32_t q = A.diag[i] + 1; q < A.lu_rowptr[i + 1]; q++) {
          dep.push_back(A.lu_col[q]);
          pos.push_back(q);
        }
      } else {
        const std::vector<int32_t>& tp = mode == 2 ? A.ut_ptr : A.lt_ptr;
        const std::vector<int32_t>& tq = mode == 2 ? A.ut_pos : A.lt_pos;
        const int32_t e = mode == 2 ? tp[i + 1] - 1 : tp[i + 1];
        if (mode == 2) dpos = tq[e];
        for (int32_t q = tp[i]; q < e; q++) {
          dep.push_back(lu_row_of[tq[q]]);
          pos.push_back(tq[q]);
        }
      }
    };
    std::vector<int32_t> slot_of(n, -1), dep, pos;
    auto seg_build = [&](int mode, size_t l0, size_t l1, SegSched& sg) -> kkt_status {
      const std::vector<int32_t>& lp = *tlp[mode];
      const std::vector<int32_t>& rows = *trows[mode];
      std::vector<int32_t> slp{0}, srow, sptr{0}, ssrc, svpos, sdpos;
      for (size_t l = l0; l < l1; l++) {
        for (int32_t t = lp[l]; t < lp[l + 1]; t++) {
          const int32_t i = rows[t];
          int32_t dp;
          entries(mode, i, dep, pos, dp);
          for (size_t k = 0; k < dep.size(); k++) {
            const int32_t j = dep[k];
            ssrc.push_back(slot_of[j] >= 0 ? -(slot_of[j] + 1) : j);
            svpos.push_back(pos[k]);
          }
          slot_of[i] = (int32_t)srow.size();
          srow.push_back(i);
          sptr.push_back((int32_t)ssrc.size());
          sdpos.push_back(dp < 0 ? 0 : dp);
        }
        slp.push_back((int32_t)srow.size());
      }
      for (int32_t i : srow) slot_of[i] = -1;
      sg.nlev = (int)(l1 - l0);
      sg.nrows = (int)srow.size();
      if (sg.nlev == 0) return KKT_OK;
      if (ssrc.empty()) {
        ssrc.push_back(0);
        svpos.push_back(0);
      }
      int *a, *b, *c, *d, *e, *f;
      kkt_status k2;
      if ((k2 = upload(h, &a, slp)) != KKT_OK || (k2 = upload(h, &b, srow)) != KKT_OK ||
          (k2 = upload(h, &c, sptr)) != KKT_OK || (k2 = upload(h, &d, ssrc)) != KKT_OK ||
          (k2 = upload(h, &e, svpos)) != KKT_OK || (k2 = upload(h, &f, sdpos)) != KKT_OK)
        return k2;
      sg.lev_ptr = a;
      sg.row = b;
      sg.ptr = c;
      sg.src = d;
      sg.vpos = e;
      sg.dpos = f;
      return KKT_OK;
    };
    auto len_fn = [&](int mode, int i) -> int {
      int32_t dp;
      entries(mode, i, dep, pos, dp);
      return (int)dep.size();
    };
    for (int mode = 0; mode < 4; mode++) {
      const std::vector<int32_t>& lp = *tlp[mode];
      const size_t nl = lp.size() - 1;
      auto width = [&](size_t l) { return lp[l + 1] - lp[l]; };
      size_t a = 0, b = nl;  // bulk levels [a, b)
      if (thin > 0) {
        int rows = 0;
        auto fits = [&](size_t l) {
          return width(l) >= 1 && width(l) <= thin && rows + width(l) <= SEG_MAX_ROWS;
        };
        while (a < nl && fits(a)) rows += width(a++);
        rows = 0;
        while (b > a && fits(b - 1)) rows += width(--b);
      }
      h->seg_pre[mode] = SegSched{};
      h->seg_post[mode] = SegSched{};
      if ((ks = seg_build(mode, 0, a, h->seg_pre[mode])) != KKT_OK ||
          (ks = seg_build(mode, b, nl, h->seg_post[mode])) != KKT_OK) {
        free_device(h);
        return ks;
      }
      chunks(lp, *trows[mode], [&](int i) { return len_fn(mode, i); }, h->chb[mode], st1, me1, a,
             b);
      if (h->chb[mode].nchunks > 0) {
        UP(dptr, st1);
        UP(dmeta, me1);
        h->chb[mode].start = dptr;
        h->chb[mode].meta = dmeta;
      }
      h->chb[mode].rows = trows_dev[mode];
    }
    const int bpc = h->opt.solve_blocks_per_cu > 0 ? h->opt.solve_blocks_per_cu : 8;
    for (ChunkSched* c : {&h->ch_l, &h->ch_u, &h->ch_ut, &h->ch_lt, &h->chb[0], &h->chb[1],
                          &h->chb[2], &h->chb[3]})
      c->blocks_per_cu = bpc;
    std::vector<int32_t> zeros(n + 1, 0);  // slot n: spare target of idle lanes
    UP(h->ready_ref, zeros);
    UP(h->ready_a, zeros);
    UP(h->ready_b, zeros);
    std::vector<SyncState> ss0(1);
    std::memset(ss0.data(), 0, sizeof(SyncState));
    UP(h->ss, ss0);
    h->cap = 0;
    for (int v : A.lev_maxlen) h->cap = std::max(h->cap, v);
    // LDS per row: value, column and pivot-row bounds of every entry (20 bytes)
    const bool fits = (size_t)((h->cap + 1) & ~1) * 20 <= 64 * 1024;
    h->syncfree = h->opt.schedule == 2 || (h->opt.schedule == 0 && fits);
    h->light = h->opt.sync_mode != 1;
    if (h->opt.schedule == 2 && !fits) {
      free_device(h);
      return fail(h, KKT_ERR_INVALID_ARG, "rows too long for the dependency-driven schedule");
    }
    // dense trailing block: density of the trailing s x s block of the factor
    // pattern for every s up to the limit (entry (i, j) lies in the blocks with
    // s >= n - min(i, j))
    h->tail_s = 0;
    if (h->syncfree && h->batch_count == 0 && h->opt.dense_tail >= 0) {
      const int smax = std::min(n, h->opt.dense_tail > 0 ? h->opt.dense_tail : 2048);
      std::vector<int64_t> cnt((size_t)smax + 1, 0);
      for (int32_t i = n - smax; i < n; i++)
        for (int32_t q = A.lu_rowptr[i]; q < A.lu_rowptr[i + 1]; q++) {
          const int32_t j = A.lu_col[q];
          if (j >= n - smax) cnt[(size_t)(n - std::min(i, j))]++;
        }
      for (int sz = 1; sz <= smax; sz++) cnt[sz] += cnt[sz - 1];
      if (h->opt.dense_tail > 0) {
        h->tail_s = smax;
      } else {
        for (int sz = 256; sz <= smax; sz += 32)
          if (2 * cnt[sz] >= (int64_t)sz * sz) h->tail_s = sz;
      }
    }
    h->tail_c0 = n - h->tail_s;
    h->tail_S = (h->tail_s + DLU_NB - 1) / DLU_NB * DLU_NB;
  }
  // rows of the short-row bands (packed update maps, launch_refactor_flat)
  std::vector<uint8_t> flat_row;
  std::vector<int32_t> order_host;  // the bands' row order (row metadata of the list kernel)
  for (bool& f : h->band_flat) f = false;
  // refactorization bands: a row's band is set by its length (LDS staging
  // size, hence rows in flight per CU) and raised to the band of any row it
  // depends on; each band is one launch.  Two bands: rows of at most 128
  // entries fed only by such rows (the short-row kernel), and the rest (at
  // 70k buses a third band for rows over 512 entries cost 0.2 ms: every
  // launch boundary waits for the last rows of the band before it, and a
  // single band for all rows cost 0.4 ms).  Within a band rows go by level of
  // the sparse phase's dependency graph (rows of the dense block do not
  // depend on each other there), and within a level by decreasing height
  // (longest chain of rows depending on them), so that a level's rows on the
  // critical chains are handed out first.
  {
    const int band_len[REF_MAX_BANDS - 1] = {
        h->opt.refactor_short_band > 0 ? h->opt.refactor_short_band : 128, 1 << 30, 1 << 30};
    const int c0 = h->tail_c0;
    std::vector<int32_t> rowof(A.lu_col.size());
    for (int32_t i = 0; i < n; i++)
      for (int32_t q = A.lu_rowptr[i]; q < A.lu_rowptr[i + 1]; q++) rowof[q] = i;
    std::vector<int32_t> height(n, 0), level(n, 0);
    int hmax = 0, lmax = 0;
    for (int32_t k = n - 1; k >= 0; k--) {
      int hk = 0;
      for (int32_t q = A.lt_ptr[k]; q < A.lt_ptr[k + 1]; q++) {
        const int32_t i = rowof[A.lt_pos[q]];
        if (k >= c0 && i >= c0) continue;
        hk = std::max(hk, height[i] + 1);
      }
      height[k] = hk;
      hmax = std::max(hmax, hk);
    }
    for (int32_t i = 0; i < n; i++) {
      int li = 0;
      for (int32_t q = A.lu_rowptr[i]; q < A.diag[i]; q++) {
        const int32_t k = A.lu_col[q];
        if (i >= c0 && k >= c0) break;
        li = std::max(li, level[k] + 1);
      }
      level[i] = li;
      lmax = std::max(lmax, li);
    }
    std::vector<int8_t> band(n, 0);
    for (int32_t i = 0; i < n; i++) {
      const int len = A.lu_rowptr[i + 1] - A.lu_rowptr[i];
      int b = 0;
      while (b < REF_MAX_BANDS - 2 && len > band_len[b]) b++;
      for (int32_t q = A.lu_rowptr[i]; q < A.diag[i]; q++) b = std::max(b, (int)band[A.lu_col[q]]);
      band[i] = (int8_t)b;
    }
    // rows without pivots in the sparse phase: copied by one parallel pass
    std::vector<uint8_t> triv(n, 0);
    std::vector<int32_t> trows;
    for (int32_t i = 0; i < n; i++) {
      const bool t = A.diag[i] == A.lu_rowptr[i] || A.lu_col[A.lu_rowptr[i]] >= c0;
      if (t) {
        triv[i] = 1;
        trows.push_back(i);
      }
    }
    h->ref_ntriv = (int)trows.size();
    if (!trows.empty()) UP(h->ref_triv, trows);
    const int hcrit = h->opt.refactor_crit_height == 0 ? 32
                      : h->opt.refactor_crit_height < 0 ? INT32_MAX
                                                        : h->opt.refactor_crit_height;
    // rows by (level, decreasing height): two stable counting sorts
    std::vector<int32_t> by_h(n), by_lh(n);
    {
      std::vector<int32_t> cnt(hmax + 2, 0);
      for (int32_t i = 0; i < n; i++) cnt[hmax - height[i] + 1]++;
      for (int v = 0; v <= hmax; v++) cnt[v + 1] += cnt[v];
      for (int32_t i = 0; i < n; i++) by_h[cnt[hmax - height[i]]++] = i;
      std::vector<int32_t> lc(lmax + 2, 0);
      for (int32_t i = 0; i < n; i++) lc[level[i] + 1]++;
      for (int v = 0; v <= lmax; v++) lc[v + 1] += lc[v];
      for (int32_t i : by_h) by_lh[lc[level[i]]++] = i;
    }
    // chunks: rows of one level (independent of each other), up to 16 per
    // ticket on wide levels; one device-scope ticket counter serializes at
    // about 10 ns per ticket, so single-row tickets would bound the wide part.
    // In a short-row band taken by the list kernel, a level's micro rows (at
    // most MICRO_ROW_LEN entries, MICRO_ROW_PIV pivots and MICRO_ROW_LIST
    // multiply-adds) come first, up to 64 to a chunk, one row per lane.
    std::vector<int32_t> order, cst;
    std::vector<unsigned char> cmic;
    const bool micro_ok = h->light && h->opt.refactor_short_rows == 0 &&
                          h->opt.refactor_map >= 0 && h->opt.refactor_micro_rows == 0;
    auto is_micro = [&](int32_t i) {
      const int32_t rs = A.lu_rowptr[i], d = A.diag[i];
      if (A.lu_rowptr[i + 1] - rs > MICRO_ROW_LEN || d - rs > MICRO_ROW_PIV) return false;
      int32_t list = 0;
      for (int32_t q = rs; q < d; q++) {
        const int32_t k = A.lu_col[q];
        list += A.lu_rowptr[k + 1] - A.diag[k] - 1;
      }
      return list <= MICRO_ROW_LIST;
    };
    order.reserve(n);
    h->nbands = 0;
    flat_row.assign(n, 0);
    for (int b = 0; b < REF_MAX_BANDS - 1; b++) {
      const int lo = (int)order.size();
      const int clo = (int)cst.size();
      int mx = 0;
      bool short_ok = true;  // rows of <= 256 entries, none of the dense block
      // rows on long chains (height >= hcrit) first: the set is closed under
      // dependencies (a row's dependency has a larger height), so this stays
      // a topological order, and those rows start before the wide levels of
      // the rest have been handed out
      for (int part = 0; part < 2; part++)
        for (int32_t i : by_lh)
          if (band[i] == b && !triv[i] && (height[i] >= hcrit) == (part == 0)) {
            order.push_back(i);
            mx = std::max(mx, A.lu_rowptr[i + 1] - A.lu_rowptr[i]);
            if (i >= c0) short_ok = false;
          }
      const int hi = (int)order.size();
      if (hi == lo) continue;
      short_ok = short_ok && mx <= 256;
      h->band_flat[h->nbands] = short_ok;
      if (short_ok)
        for (int t = lo; t < hi; t++) flat_row[order[t]] = 1;
      for (int t = lo; t < hi;) {
        int e = t;
        const bool crit = height[order[t]] >= hcrit;
        while (e < hi && level[order[e]] == level[order[t]] &&
               (height[order[e]] >= hcrit) == crit)
          e++;
        int m = t;  // [t, m): micro rows, in their order
        if (short_ok && micro_ok)
          m = (int)(std::stable_partition(order.begin() + t, order.begin() + e, is_micro) -
                    order.begin());
        for (int c = t; c < m; c += 64) {
          cst.push_back(c);
          cmic.push_back(1);
        }
        const int per = std::max(1, std::min(16, (e - m) / 8192));
        for (int c = m; c < e; c += per) {
          cst.push_back(c);
          cmic.push_back(0);
        }
        t = e;
      }
      h->band_chunk_lo[h->nbands] = clo;
      h->band_nchunks[h->nbands] = (int)cst.size() - clo;
      h->band_cap[h->nbands] = mx;
      cst.push_back(hi);  // end of the band's last chunk
      cmic.push_back(0);
      h->nbands++;
    }
    UP(h->ref_order, order);
    order_host = order;
    UP(h->ref_cstart, cst);
    h->ref_cmicro = nullptr;
    for (unsigned char c : cmic)
      if (c) {
        UP(h->ref_cmicro, cmic);
        break;
      }
  }
  // update maps of the dependency-driven refactorization: one 16-bit row
  // position per multiply-add (rows must be shorter than 65536 entries and
  // the total must fit int32 offsets)
  h->ref_moff = nullptr;
  h->ref_map = nullptr;
  h->ref_map_entries = 0;
  h->ref_fl = nullptr;
  h->ref_flat = nullptr;
  h->ref_rmeta = nullptr;
  h->tl = nullptr;
  if (h->opt.debug_timeline == 1 && h->inst.count == 1) {
    if ((ks = dalloc(h, &h->tl, (size_t)3 * n)) != KKT_OK) {
      free_device(h);
      return ks;
    }
    HIP_CHECK(h, hipMemset(h->tl, 0, (size_t)3 * n * sizeof(long long)));
  }
  if (h->syncfree && h->opt.refactor_map >= 0) {
    std::vector<int32_t> moff(A.lu_col.size(), 0);
    int64_t tot = 0;
    int maxlen = 0;
    for (int32_t i = 0; i < n; i++) {
      maxlen = std::max(maxlen, A.lu_rowptr[i + 1] - A.lu_rowptr[i]);
      for (int32_t q = A.lu_rowptr[i]; q < A.diag[i]; q++) {
        const int32_t k = A.lu_col[q];
        moff[q] = (int32_t)std::min<int64_t>(tot, INT32_MAX);
        tot += A.lu_rowptr[k + 1] - A.diag[k] - 1;
      }
    }
    if (maxlen < 65536 && tot < INT32_MAX && tot > 0) {
      UP(h->ref_moff, moff);
      if ((ks = dalloc(h, &h->ref_map, (size_t)tot)) != KKT_OK) {
        free_device(h);
        return ks;
      }
      h->ref_map_entries = tot;
      // short-row bands: per L entry (list offset of the pivot's updates, its
      // U row start minus that offset), at the diagonal (list length, 0)
      bool any_flat = false;
      if (h->light && h->opt.refactor_short_rows == 0)
        for (int b = 0; b < h->nbands; b++) any_flat = any_flat || h->band_flat[b];
      if (any_flat) {
        std::vector<int2> fl(A.lu_col.size(), make_int2(0, 0));
        for (int32_t i = 0; i < n; i++) {
          if (!flat_row[i]) continue;
          const int32_t rs = A.lu_rowptr[i], d = A.diag[i];
          int32_t len_list = 0;
          for (int32_t q = rs; q < d; q++) {
            const int32_t k = A.lu_col[q];
            const int32_t fo = moff[q] - moff[rs];
            fl[q] = make_int2(fo, A.diag[k] + 1 - fo);
            len_list = fo + (A.lu_rowptr[k + 1] - A.diag[k] - 1);
          }
          fl[d] = make_int2(len_list, 0);
        }
        UP(h->ref_fl, fl);
        UP(h->ref_flat, flat_row);
        // per position of the bands' order, for the list kernel's rows: row
        // start, length | pivots << 16, update-map offset, list length
        std::vector<int4> meta(order_host.size(), make_int4(0, 0, 0, 0));
        for (size_t r = 0; r < order_host.size(); r++) {
          const int32_t i = order_host[r];
          if (!flat_row[i]) continue;
          const int32_t rs = A.lu_rowptr[i], d = A.diag[i];
          meta[r] = make_int4(rs, (A.lu_rowptr[i + 1] - rs) | ((d - rs) << 16), moff[rs],
                              fl[d].x);
        }
        UP(h->ref_rmeta, meta);
      }
    }
  }
  if (!h->ref_fl)
    for (bool& f : h->band_flat) f = false;
  h->luA = nullptr;
  h->a2lu = nullptr;
  h->ref_pbnd = nullptr;
  h->ref_dlc = nullptr;
  if (h->syncfree) {
    std::vector<int32_t> a2lu((size_t)nnz, 0);
    const size_t fz = A.lu_col.size();
    for (size_t q = 0; q < fz; q++)
      if (A.lu_src[q] >= 0) a2lu[A.lu_src[q]] = (int32_t)q;
    std::vector<int2> pb(fz, make_int2(0, 0));
    for (int32_t i = 0; i < n; i++)
      for (int32_t q = A.lu_rowptr[i]; q < A.diag[i]; q++) {
        const int32_t k = A.lu_col[q];
        pb[q] = make_int2(A.diag[k], A.lu_rowptr[k + 1]);
      }
    UP(h->a2lu, a2lu);
    UP(h->ref_pbnd, pb);
    std::vector<int32_t> dlc(n);
    for (int32_t i = 0; i < n; i++) {
      int32_t q = A.lu_rowptr[i];
      while (q < A.diag[i] && A.lu_col[q] < h->tail_c0) q++;
      dlc[i] = q - A.lu_rowptr[i];
    }
    UP(h->ref_dlc, dlc);
    if ((ks = dalloc(h, &h->luA, fz * h->inst.count)) != KKT_OK) {
      free_device(h);
      return ks;
    }
    HIP_CHECK(h, hipMemset(h->luA, 0, fz * h->inst.count * sizeof(double)));
  }
  // chain-blocked schedules of the four solves over the rows outside the
  // dense trailing block (modes 0 L, 1 U, 2 U^T, 3 L^T)
  h->use_sn = h->syncfree && h->light && h->opt.solve_chain >= 0;
  if (h->use_sn) {
    const int c0 = h->tail_c0;
    const int kmax = h->opt.solve_chain > 0 ? std::min(h->opt.solve_chain, SN_KMAX) : SN_KMAX;
    std::vector<int32_t> rowof(A.lu_col.size());
    for (int32_t i = 0; i < n; i++)
      for (int32_t q = A.lu_rowptr[i]; q < A.lu_rowptr[i + 1]; q++) rowof[q] = i;
    for (int mode = 0; mode < 4; mode++) {
      const bool fwd = mode == 0 || mode == 2;
      // dependency list of row i (ascending dependency index), diagonal excluded
      auto lb = [&](int32_t i) -> int32_t {
        return mode == 0 ? A.lu_rowptr[i]
               : mode == 1 ? A.diag[i] + 1
               : mode == 2 ? A.ut_ptr[i]
                           : A.lt_ptr[i];
      };
      auto le = [&](int32_t i) -> int32_t {
        return mode == 0 ? A.diag[i]
               : mode == 1 ? A.lu_rowptr[i + 1]
               : mode == 2 ? A.ut_ptr[i + 1] - 1
                           : A.lt_ptr[i + 1];
      };
      auto dep = [&](int32_t q) -> int32_t {
        return mode <= 1 ? A.lu_col[q] : rowof[mode == 2 ? A.ut_pos[q] : A.lt_pos[q]];
      };
      // items: runs of consecutive rows (solve order) each depending on the
      // previous one, up to kmax rows and 64 lanes at <= 32 entries per lane
      std::vector<int32_t> item_of(c0, -1), item_first, item_len, item_lev;
      std::vector<uint8_t> triv(n, 0);
      int32_t last_row = -1;  // last row added to the current item
      auto lanes_for = [](int len) {
        int g = 1;
        while (g < 64 && g * 32 < len) g <<= 1;
        return g;
      };
      auto p2 = [](int k) {
        int p = 1;
        while (p < k) p <<= 1;
        return p;
      };
      int cur_max = 0;
      for (int32_t t = 0; t < c0; t++) {
        const int32_t i = fwd ? t : c0 - 1 - t;
        const int32_t b = lb(i), e = le(i);
        const int len = e - b;
        if (fwd && len == 0) {
          // no dependencies: final in the gather pass, not scheduled
          triv[i] = 1;
          continue;
        }
        bool ext = false;
        if (!item_first.empty() && last_row >= 0) {
          const int32_t p = fwd ? i - 1 : i + 1;
          const bool chained =
              p == last_row && len > 0 && (fwd ? dep(e - 1) == p : dep(b) == p);
          const int k = item_len.back();
          const int mx = std::max(cur_max, len);
          ext = chained && k < kmax && p2(k + 1) * lanes_for(mx) <= 64;
        }
        if (ext) {
          item_len.back()++;
          cur_max = std::max(cur_max, len);
        } else {
          item_first.push_back(i);
          item_len.push_back(1);
          cur_max = len;
        }
        item_of[i] = (int32_t)item_first.size() - 1;
        last_row = i;
      }
      if (fwd) {
        uint8_t* d = nullptr;
        UP(d, triv);
        (mode == 0 ? h->sn_triv0 : h->sn_triv2) = d;
      }
      const int nitems = (int)item_first.size();
      item_lev.assign(nitems, 0);
      int nlev = 0;
      for (int it = 0; it < nitems; it++) {
        int lv = 0;
        for (int r = 0; r < item_len[it]; r++) {
          const int32_t i = fwd ? item_first[it] + r : item_first[it] - r;
          for (int32_t q = lb(i); q < le(i); q++) {
            const int32_t j = dep(q);
            if (j >= c0 || item_of[j] < 0 || item_of[j] == it) continue;
            lv = std::max(lv, item_lev[item_of[j]] + 1);
          }
        }
        item_lev[it] = lv;
        nlev = std::max(nlev, lv + 1);
      }
      // item heights (longest chain of items depending on it): items with a
      // long chain after them are handed out first (a dependency-closed set,
      // so the order stays topological), the rest by level
      std::vector<int32_t> item_h(nitems, 0);
      for (int it = nitems - 1; it >= 0; it--)
        for (int r = 0; r < item_len[it]; r++) {
          const int32_t i = fwd ? item_first[it] + r : item_first[it] - r;
          for (int32_t q = lb(i); q < le(i); q++) {
            const int32_t j = dep(q);
            if (j >= c0 || item_of[j] < 0 || item_of[j] == it) continue;
            int32_t& hd = item_h[item_of[j]];
            hd = std::max(hd, item_h[it] + 1);
          }
        }
      const int hcrit = 2;
      // chunks in level order
      std::vector<int32_t> by_lev_ptr(nlev + 1, 0), by_lev(nitems);
      for (int it = 0; it < nitems; it++) by_lev_ptr[item_lev[it] + 1]++;
      for (int l = 0; l < nlev; l++) by_lev_ptr[l + 1] += by_lev_ptr[l];
      {
        std::vector<int32_t> fill(by_lev_ptr.begin(), by_lev_ptr.end() - 1);
        for (int it = 0; it < nitems; it++) by_lev[fill[item_lev[it]]++] = it;
      }
      std::vector<int32_t> cst, cmeta, cbase, crow, csplit;
      auto split_of = [&](int32_t i, bool chain, int32_t base) -> int32_t {
        const int32_t b = lb(i), e = le(i);
        if (!chain) return (mode == 0 || mode == 2) ? e : b;
        // internal dependencies: rows of the chunk, i.e. index >= base
        // (forward) or <= base (backward)
        int32_t q = b;
        if (fwd)
          while (q < e && dep(q) < base) q++;
        else
          while (q < e && dep(q) <= base) q++;
        return q;
      };
      for (int part = 0; part < 2; part++)
      for (int l = 0; l < nlev; l++) {
        std::vector<int32_t> singles;
        for (int32_t t = by_lev_ptr[l]; t < by_lev_ptr[l + 1]; t++) {
          const int it = by_lev[t];
          if ((item_h[it] >= hcrit) != (part == 0)) continue;
          const int k = item_len[it];
          if (k == 1) {
            singles.push_back(item_first[it]);
            continue;
          }
          int lg = 0;
          while ((1 << lg) * p2(k) < 64) lg++;
          cst.push_back((int32_t)crow.size());
          cmeta.push_back((1 << 16) | (lg << 8) | k);
          cbase.push_back(item_first[it]);
          for (int r = 0; r < k; r++) {
            const int32_t i = fwd ? item_first[it] + r : item_first[it] - r;
            crow.push_back(i);
            csplit.push_back(split_of(i, true, item_first[it]));
          }
        }
        if (singles.empty()) continue;
        // the level's single rows by length, so that each chunk's lane groups
        // (2^lg lanes per row, at most per_lane entries per lane, 64 >> lg
        // rows) fit its own longest row rather than the level's
        const int per_lane =
            h->opt.solve_entries_per_lane > 0 ? h->opt.solve_entries_per_lane : 8;
        auto lg_for = [&](int32_t i) {
          int lg = 0;
          while (lg < 6 && (per_lane << lg) < le(i) - lb(i)) lg++;
          return lg;
        };
        std::stable_sort(singles.begin(), singles.end(), [&](int32_t x, int32_t y) {
          return le(x) - lb(x) < le(y) - lb(y);
        });
        for (size_t a = 0; a < singles.size();) {
          int lg = lg_for(singles[a]);
          size_t k = 0;
          for (;;) {
            k = std::min<size_t>((size_t)(64 >> lg), singles.size() - a);
            const int lg2 = lg_for(singles[a + k - 1]);
            if (lg2 <= lg) break;
            lg = lg2;
          }
          cst.push_back((int32_t)crow.size());
          cmeta.push_back((lg << 8) | (int)k);
          cbase.push_back(0);
          for (size_t r = 0; r < k; r++) {
            crow.push_back(singles[a + r]);
            csplit.push_back(split_of(singles[a + r], false, 0));
          }
          a += k;
        }
      }
      SnSched& sn = h->chs[mode];
      sn = SnSched{};
      sn.nchunks = (int)cst.size();
      sn.blocks_per_cu = h->opt.solve_blocks_per_cu > 0 ? h->opt.solve_blocks_per_cu : 8;
      h->chs_levels[mode] = nlev;
      if (sn.nchunks > 0) {
        int *a1, *a2, *a3, *a4, *a5;
        UP(a1, cst);
        UP(a2, cmeta);
        UP(a3, cbase);
        UP(a4, crow);
        UP(a5, csplit);
        sn.start = a1;
        sn.meta = a2;
        sn.base = a3;
        sn.rows = a4;
        sn.split = a5;
      }
    }
    // U solve: the rows before the dense block with entries in its columns,
    // and where those entries start (their terms are summed in one pass once
    // the block is solved)
    h->u_xend = nullptr;
    h->u_rows = nullptr;
    h->u_pre = nullptr;
    h->u_nrows = 0;
    if (h->tail_s > 0) {
      std::vector<int32_t> xend(n + 1, 0), urows;
      for (int32_t i = 0; i < c0; i++) {
        int32_t q = A.diag[i] + 1;
        const int32_t e = A.lu_rowptr[i + 1];
        while (q < e && A.lu_col[q] < c0) q++;
        xend[i] = q;
        if (q < e) urows.push_back(i);
      }
      for (int32_t i = c0; i <= n; i++) xend[i] = i < n ? A.lu_rowptr[i + 1] : 0;
      if (!urows.empty()) {
        UP(h->u_xend, xend);
        UP(h->u_rows, urows);
        h->u_nrows = (int)urows.size();
        if ((ks = dalloc(h, &h->u_pre, (size_t)n + 1)) != KKT_OK) {
          free_device(h);
          return ks;
        }
        HIP_CHECK(h, hipMemset(h->u_pre, 0, ((size_t)n + 1) * sizeof(double)));
      }
    }
    // external/internal boundary of the dense block's rows (modes 0 and 2)
    if (h->tail_s > 0) {
      std::vector<int32_t> s0(h->tail_s), s2(h->tail_s);
      for (int t = 0; t < h->tail_s; t++) {
        const int32_t i = c0 + t;
        int32_t q = A.lu_rowptr[i];
        while (q < A.diag[i] && A.lu_col[q] < c0) q++;
        s0[t] = q;
        q = A.ut_ptr[i];
        while (q < A.ut_ptr[i + 1] - 1 && rowof[A.ut_pos[q]] < c0) q++;
        s2[t] = q;
      }
      UP(h->tail_split0, s0);
      UP(h->tail_split2, s2);
    }
  }
#undef UP
  const size_t f = A.lu_col.size();
  const int m = h->m;
  // right-hand sides refined in lockstep: up to FG_MAX_COLS where the
  // schedule has multi-column solves, as many as keep the Krylov vectors
  // ((2m + 4) per column) within 2 GiB
  // a shared-pattern batch holds every instance's values and vectors
  const size_t cnt = (size_t)h->inst.count;
  int gc = 1;
  if (h->syncfree && h->light && cnt == 1) {
    gc = FG_MAX_COLS;
    while (gc > 1 && (size_t)gc * (2 * m + 4) * (size_t)n * sizeof(double) > (size_t(2) << 30))
      gc >>= 1;
  }
  h->fg_cols = gc;
  const size_t gn = (size_t)gc * n * cnt;
  if ((ks = dalloc(h, &h->lu_val, f * cnt)) != KKT_OK ||
      (ks = dalloc(h, &h->aval, (size_t)nnz * cnt)) != KKT_OK ||
      (ks = dalloc(h, &h->st, 1)) != KKT_OK ||
      (ks = dalloc(h, &h->V, (size_t)(m + 1) * gn)) != KKT_OK ||
      (ks = dalloc(h, &h->Z, (size_t)m * gn)) != KKT_OK || (ks = dalloc(h, &h->w, gn)) != KKT_OK ||
      (ks = dalloc(h, &h->r, gn)) != KKT_OK || (ks = dalloc(h, &h->xt, gn)) != KKT_OK ||
      (ks = dalloc(h, &h->fs, 1)) != KKT_OK ||
      (ks = dalloc(h, &h->fb.part, (size_t)FG_MAX_COLS * FG_BLOCKS * 32)) != KKT_OK ||
      (ks = dalloc(h, &h->fb.tick1, (size_t)FG_MAX_COLS * FG_TICK_GROUPS * FG_TICK_STRIDE)) !=
          KKT_OK ||
      (ks = dalloc(h, &h->fb.hbuf, (size_t)FG_MAX_COLS * 32)) != KKT_OK ||
      (ks = dalloc(h, &h->fb.h2buf, (size_t)FG_MAX_COLS * 32)) != KKT_OK ||
      (ks = dalloc(h, &h->fb.H, (size_t)FG_MAX_COLS * (m + 1) * m)) != KKT_OK ||
      (ks = dalloc(h, &h->fb.cs, (size_t)FG_MAX_COLS * m)) != KKT_OK ||
      (ks = dalloc(h, &h->fb.sn, (size_t)FG_MAX_COLS * m)) != KKT_OK ||
      (ks = dalloc(h, &h->fb.gvec, (size_t)FG_MAX_COLS * (m + 1))) != KKT_OK ||
      (ks = dalloc(h, &h->fb.y, (size_t)FG_MAX_COLS * m)) != KKT_OK ||
      (ks = dalloc(h, &h->tmp, ((size_t)n + 1) * cnt)) != KKT_OK ||
      (ks = dalloc(h, &h->tc, ((size_t)n + 1) * cnt)) != KKT_OK ||
      (ks = dalloc(h, &h->ty, ((size_t)n + 1) * cnt)) != KKT_OK ||
      (ks = dalloc(h, &h->tz, ((size_t)n + 1) * cnt)) != KKT_OK ||
      (ks = dalloc(h, &h->H, (size_t)(m + 1) * m)) != KKT_OK ||
      (ks = dalloc(h, &h->cs, m + 1)) != KKT_OK || (ks = dalloc(h, &h->sn, m + 1)) != KKT_OK ||
      (ks = dalloc(h, &h->g, m + 1)) != KKT_OK || (ks = dalloc(h, &h->h, m + 1)) != KKT_OK ||
      (ks = dalloc(h, &h->h2, m + 1)) != KKT_OK || (ks = dalloc(h, &h->ww, 1)) != KKT_OK ||
      (ks = dalloc(h, &h->y, m + 1)) != KKT_OK || (ks = dalloc(h, &h->hn, 1)) != KKT_OK ||
      (ks = dalloc(h, &h->partial, 256 * 32)) != KKT_OK ||
      (ks = dalloc(h, &h->red, RED_SCRATCH)) != KKT_OK) {
    free_device(h);
    return ks;
  }
  if (h->tail_s > 0 &&
      ((ks = dalloc(h, &h->tail_T, (size_t)h->tail_S * h->tail_S)) != KKT_OK ||
       (ks = dalloc(h, &h->tail_dsc, (size_t)DLU_NB * DLU_NB *
                                         (h->opt.dense_lu == 1 ? h->tail_S / DLU_NB : 1))) != KKT_OK ||
       (ks = dalloc(h, &h->tail_rhs, (size_t)h->tail_S * 8)) != KKT_OK)) {
    free_device(h);
    return ks;
  }
  h->dlu_tasks = h->dlu_ver = nullptr;
  h->dlu_ntasks = 0;
  if (h->tail_s > 0 && h->opt.dense_lu == 1) {
    const int nt = h->tail_S / DLU_NB;
    const std::vector<int> tasks = dense_lu_tasks(nt);
    if ((ks = upload(h, &h->dlu_tasks, tasks)) != KKT_OK ||
        (ks = dalloc(h, &h->dlu_ver, (size_t)nt * nt)) != KKT_OK) {
      free_device(h);
      return ks;
    }
    h->dlu_ntasks = (int)tasks.size();
  }
  if (h->batch_count > 0) {
    std::vector<int32_t> ro(h->row_off.begin(), h->row_off.end());
    if ((ks = upload(h, &h->d_row_off, ro)) != KKT_OK ||
        (ks = dalloc(h, &h->rowabs, (size_t)n * cnt)) != KKT_OK ||
        (ks = dalloc(h, &h->colabs, (size_t)n * cnt)) != KKT_OK ||
        (ks = dalloc(h, &h->inst_out, (size_t)3 * SEG_SLICES * h->batch_count)) != KKT_OK) {
      free_device(h);
      return ks;
    }
    h->h_inst.assign((size_t)3 * SEG_SLICES * h->batch_count, 0.0);
    h->inst_eta.assign(h->batch_count, 0.0);
  }
  // the pivoting pass's factors are the current factors until the first
  // refactor (every instance of a shared-pattern batch starts from them)
  for (size_t t = 0; t < cnt; t++) {
    HIP_CHECK(h, hipMemcpy(h->lu_val + t * f, A.lu_val0.data(), f * sizeof(double),
                           hipMemcpyHostToDevice));
    HIP_CHECK(h, hipMemcpy(h->aval + t * (size_t)nnz, values0, (size_t)nnz * sizeof(double),
                           hipMemcpyHostToDevice));
  }
  HIP_CHECK(h, hipHostMalloc((void**)&h->h_st, sizeof(DevStats), hipHostMallocDefault));
  HIP_CHECK(h, hipHostMalloc((void**)&h->h_fs, sizeof(FgState), hipHostMallocDefault));
  HIP_CHECK(h, hipEventCreateWithFlags(&h->ev_fs, hipEventDisableTiming));
  HIP_CHECK(h, hipHostMalloc((void**)&h->h_colmax, sizeof(unsigned long long) * 2 * MAX_RHS_PASS,
                             hipHostMallocDefault));
  if ((ks = dalloc(h, &h->colmax, 2 * MAX_RHS_PASS)) != KKT_OK) {
    free_device(h);
    return ks;
  }
  h->fb.fs = h->fs;
  HIP_CHECK(h, hipMemset(h->fs, 0, sizeof(FgState)));
  // Krylov vectors start finite: a column that stopped early still passes
  // its (unused) basis vector through the group's triangular solves
  HIP_CHECK(h, hipMemset(h->V, 0, (size_t)(m + 1) * gn * sizeof(double)));
  HIP_CHECK(h, hipMemset(h->Z, 0, (size_t)m * gn * sizeof(double)));
  HIP_CHECK(h, hipMemset(h->r, 0, gn * sizeof(double)));
  if (h->syncfree && h->light) {
    // multi-column solve buffers, (n+1) x MAX_RHS_PASS each
    const size_t cnt = (size_t)(n + 1) * MAX_RHS_PASS;
    if ((ks = dalloc(h, &h->mc, cnt)) != KKT_OK || (ks = dalloc(h, &h->my, cnt)) != KKT_OK ||
        (ks = dalloc(h, &h->mz, cnt)) != KKT_OK) {
      free_device(h);
      return ks;
    }
    h->mcap = MAX_RHS_PASS;
  }
  HIP_CHECK(h, hipMemcpy(&h->st->spin_limit, &h->opt.debug_spin_limit, sizeof(int),
                         hipMemcpyHostToDevice));
  if (!set_debug_schedule(h->opt.debug_schedule))
    return fail(h, KKT_ERR_DEVICE, "cannot set the debug schedule flag");
  launch_reset_stats(h->st, 1 | 2 | 8, nullptr);
  launch_copy_anorm(n, h->a_rowptr, h->a_col, h->aval, h->aval, h->st, nullptr, nullptr,
                    h->rowabs, nullptr, nullptr, nullptr, 1, h->ascale, h->avs, h->inst);
  launch_pivot_stats(view(h), h->st, h->opt.tiny_pivot_rel, h->red, nullptr, h->inst);
  if (h->ref_map) launch_build_refmap(view(h), h->ref_moff, h->ref_map, h->ref_flat, nullptr);
  // the dense block's copy of the pivoting pass's factors (the solves read it)
  if (h->tail_s > 0)
    launch_tail_scatter(view(h), h->tail_c0, h->tail_s, h->tail_S, h->tail_T, nullptr);
  HIP_CHECK(h, hipGetLastError());
  HIP_CHECK(h, hipDeviceSynchronize());
  h->anorm1_valid = false;
  h->analyzed = true;
  h->factored = true;
  h->factor_epoch++;
  h->warnings = st > 0 ? (1 << st) : 0;
  h->analyze_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return (kkt_status)st;
}

kkt_status kkt_analyze_batch(kkt_handle h, int32_t npat, const int32_t* n, const int64_t* nnz,
                             const int64_t* const* rowptr, const int32_t* const* colind,
                             const double* const* values0, int32_t count,
                             const int32_t* inst_pattern) {
  if (!h) return KKT_ERR_INVALID_ARG;
  h->err.clear();
  if (h->opt.matching != 0)
    return fail(h, KKT_ERR_INVALID_ARG, "matching is supported for single-system analyses only");
  auto t0 = std::chrono::steady_clock::now();
  AnalyzeOptions ao;
  ao.ordering = h->opt.ordering == 2 ? 0 : h->opt.ordering;
  ao.tau = h->opt.pivot_tau;
  Analysis an;
  std::vector<int64_t> row_off, nnz_off;
  std::string msg;
  int st;
  try {
    st = analyze_batch(npat, n, nnz, rowptr, colind, values0, count, inst_pattern, ao, an, row_off,
                       nnz_off, &msg);
  } catch (const std::bad_alloc&) {
    return fail(h, KKT_ERR_OUT_OF_MEMORY, "host allocation failed in analyze_batch");
  }
  if (st < 0) return fail(h, (kkt_status)st, msg);
  // the block-diagonal A: instance patterns concatenated with row/column offsets
  const int32_t N = an.n;
  const int64_t NNZ = an.nnz;
  std::vector<int64_t> rp(N + 1);
  std::vector<int32_t> ci(NNZ);
  std::vector<double> v0(NNZ);
  for (int32_t t = 0; t < count; t++) {
    const int32_t p = inst_pattern[t];
    const int32_t ro = (int32_t)row_off[t];
    const int64_t no = nnz_off[t];
    for (int32_t i = 0; i < n[p]; i++) rp[ro + i] = no + rowptr[p][i];
    for (int64_t q = 0; q < nnz[p]; q++) {
      ci[no + q] = ro + colind[p][q];
      v0[no + q] = values0[p][q];
    }
  }
  rp[N] = NNZ;
  h->batch_count = count;
  h->inst = Inst();
  h->row_off = row_off;
  h->nnz_off = nnz_off;
  return install_analysis(h, std::move(an), st, N, NNZ, rp.data(), ci.data(), v0.data(), t0);
}

kkt_status kkt_analyze_shared(kkt_handle h, int32_t n, int64_t nnz, const int64_t* rowptr,
                              const int32_t* colind, const double* values0, int32_t count) {
  if (!h) return KKT_ERR_INVALID_ARG;
  h->err.clear();
  if (count < 1 || n < 1 || !rowptr || !colind || !values0)
    return fail(h, KKT_ERR_INVALID_ARG, "bad count, size or pointer");
  const kkt_options& o = h->opt;
  if (o.matching != 0 || o.schedule == 1 || o.sync_mode == 1 || o.refactor_short_rows != 0 ||
      o.refactor_long_rows != 0 || o.refactor_map != 0 || o.solve_chain < 0 ||
      o.solve_jacobi_sweeps != 0 || o.refine_sync != 0)
    return fail(h, KKT_ERR_INVALID_ARG,
                "shared-pattern batches run the default dependency-driven kernels only");
  const int64_t lim = INT32_MAX;
  if ((int64_t)n * count + count > lim || nnz * count > lim)
    return fail(h, KKT_ERR_TOO_LARGE, "the batch exceeds the int32 index range");
  auto t0 = std::chrono::steady_clock::now();
  AnalyzeOptions ao;
  ao.ordering = o.ordering == 2 ? 0 : o.ordering;
  ao.tau = o.pivot_tau;
  Analysis an;
  std::string msg;
  int st;
  try {
    st = analyze(n, nnz, rowptr, colind, values0, nullptr, ao, an, &msg);
  } catch (const std::bad_alloc&) {
    return fail(h, KKT_ERR_OUT_OF_MEMORY, "host allocation failed in analyze");
  }
  if (st < 0) return fail(h, (kkt_status)st, msg);
  if ((int64_t)an.lu_col.size() * count > lim)
    return fail(h, KKT_ERR_TOO_LARGE, "the batch's factors exceed the int32 index range");
  h->batch_count = count;
  h->inst = Inst();
  h->inst.count = count;
  h->inst.n1 = n;
  h->inst.a1 = (int)nnz;
  h->inst.f1 = (int)an.lu_col.size();
  h->row_off.assign((size_t)count + 1, 0);
  h->nnz_off.assign((size_t)count + 1, 0);
  for (int32_t t = 0; t <= count; t++) {
    h->row_off[t] = (int64_t)t * n;
    h->nnz_off[t] = (int64_t)t * nnz;
  }
  h->pat_rowptr.clear();
  h->pat_colind.clear();
  kkt_status ks = install_analysis(h, std::move(an), st, n, nnz, rowptr, colind, values0, t0);
  if (ks < 0) return ks;
  bool kernels_ok = h->syncfree && h->light && h->use_sn && h->tail_s == 0 && h->ref_fl;
  for (int b = 0; kernels_ok && b < h->nbands; b++)
    kernels_ok = h->band_flat[b] || (h->ref_map && h->luA && h->ref_pbnd && h->ref_dlc &&
                                     (size_t)h->band_cap[b] * 8 <= 64 * 1024);
  if (!kernels_ok) {
    free_device(h);
    h->inst = Inst();
    h->batch_count = 0;
    return fail(h, KKT_ERR_INVALID_ARG,
                "this pattern does not take the dependency-driven kernels a shared-pattern batch "
                "needs");
  }
  return ks;
}

kkt_status kkt_batch_layout(kkt_handle h, int64_t* row_offset, int64_t* nnz_offset) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed || h->batch_count == 0) return fail(h, KKT_ERR_STATE, "no batch analysis");
  if (row_offset) std::memcpy(row_offset, h->row_off.data(), h->row_off.size() * sizeof(int64_t));
  if (nnz_offset) std::memcpy(nnz_offset, h->nnz_off.data(), h->nnz_off.size() * sizeof(int64_t));
  return KKT_OK;
}

kkt_status kkt_batch_eta(kkt_handle h, double* eta) {
  if (!h || !eta) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed || h->batch_count == 0) return fail(h, KKT_ERR_STATE, "no batch analysis");
  // per-instance maxima of the last residual check (the final iterate)
  kkt_status ks = read_batch_eta(h, 'N', nullptr);
  if (ks != KKT_OK) return ks;
  std::memcpy(eta, h->inst_eta.data(), h->inst_eta.size() * sizeof(double));
  return KKT_OK;
}

// The refactorization's launches (stream-ordered only, capturable).
static kkt_status refactor_launch(kkt_handle h, const double* d_values, hipStream_t s) {
  const Analysis& A = h->an;
  LUView lu = view(h);
  // values of the factored matrix in A's order: A's own, or the matched and
  // scaled ones (written by the copy pass)
  const double* fa = h->avs ? h->avs : h->aval;
  launch_reset_stats(h->st, 1, s);
  const Inst in = h->inst;  // instances of a shared-pattern batch
  if (h->syncfree) {
    launch_copy_anorm(A.n, h->a_rowptr, h->a_col, d_values, h->aval, h->st, s, h->ss, h->rowabs,
                      h->a2lu, h->luA, nullptr, 1, h->ascale, h->avs, in);
    if (h->light) launch_fill_sentinel(h->lu_val, (long long)A.lu_col.size() * in.count, s);
    launch_refactor_trivial(lu, h->ref_triv, h->ref_ntriv, fa, h->ready_ref, h->ss, s,
                            h->luA, h->tail_c0, h->st, h->opt.pivot_perturb_rel, in);
    for (int b = 0; b < h->nbands; b++)
      if (h->band_flat[b]) {
        if (!launch_refactor_flat(lu, h->ref_cstart + h->band_chunk_lo[b], h->band_nchunks[b], b,
                                  h->band_cap[b], h->ss, &h->st->stall,
                                  h->ref_rmeta, h->ref_map, h->luA, h->ref_fl,
                                  h->ref_cmicro ? h->ref_cmicro + h->band_chunk_lo[b] : nullptr,
                                  h->opt.refactor_waves_per_cu, h->st, h->opt.pivot_perturb_rel,
                                  s, h->ref_order, h->tl, in))
          return fail(h, KKT_ERR_DEVICE, "short-row refactorization not launchable");
      } else if (h->light && h->ref_map && h->luA && h->ref_pbnd && h->ref_dlc &&
                 h->opt.refactor_long_rows == 0 && (size_t)h->band_cap[b] * 8 <= 64 * 1024) {
        if (!launch_refactor_wg(lu, h->ref_order, h->ref_cstart + h->band_chunk_lo[b],
                                h->band_nchunks[b], b, h->band_cap[b], h->ss, &h->st->stall,
                                h->tail_c0, h->ref_dlc, h->ref_moff, h->ref_map, h->luA,
                                h->ref_pbnd, h->opt.refactor_waves_per_cu, h->st,
                                h->opt.pivot_perturb_rel, s, h->tl, in))
          return fail(h, KKT_ERR_DEVICE, "long-row refactorization not launchable");
      } else if (!launch_refactor_syncfree(lu, h->ref_order, h->ref_cstart + h->band_chunk_lo[b],
                                    h->band_nchunks[b], b, h->band_cap[b], fa, h->ready_ref,
                                    h->ss, &h->st->stall, h->light,
                                    h->opt.refactor_waves_per_block, h->tail_c0, h->ref_moff,
                                    h->ref_map, h->luA, h->ref_pbnd,
                                    h->opt.refactor_waves_per_cu, h->st, h->opt.pivot_perturb_rel,
                                    s))
        return fail(h, KKT_ERR_DEVICE, "dependency-driven refactorization not launchable");
    if (h->tail_s > 0) {
      launch_tail_scatter(lu, h->tail_c0, h->tail_s, h->tail_S, h->tail_T, s);
      if (h->dlu_tasks) {
        launch_dlu_reset(h->dlu_ver, h->tail_S / DLU_NB, h->ss, s);
        if (!launch_dense_lu_tasks(h->tail_T, h->tail_S, h->tail_s, h->dlu_tasks, h->dlu_ntasks,
                                   h->dlu_ver, h->tail_dsc, h->ss, &h->st->stall, h->st,
                                   h->opt.pivot_perturb_rel, s))
          return fail(h, KKT_ERR_DEVICE, "dense-block task launch not launchable");
      } else
      launch_dense_lu(h->tail_T, h->tail_S, h->tail_s, h->tail_dsc, h->st,
                      h->opt.pivot_perturb_rel, s);
      launch_tail_gather(lu, h->tail_c0, h->tail_T, h->tail_S, s);
    }
  } else {
    launch_copy_anorm(A.n, h->a_rowptr, h->a_col, d_values, h->aval, h->st, s, nullptr,
                      h->rowabs, nullptr, nullptr, nullptr, 1, h->ascale, h->avs);
    for (size_t l = 0; l + 1 < A.lev_ptr.size(); l++)
      launch_refactor_rows(lu, h->lev_rows + A.lev_ptr[l], A.lev_ptr[l + 1] - A.lev_ptr[l],
                           A.lev_maxlen[l], fa, h->st, h->opt.pivot_perturb_rel, s);
  }
  launch_pivot_stats(lu, h->st, h->opt.tiny_pivot_rel, h->red, s, in);
  return KKT_OK;
}

kkt_status kkt_refactor(kkt_handle h, const double* d_values, void* stream) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "kkt_refactor before kkt_analyze");
  if (!d_values) return fail(h, KKT_ERR_INVALID_ARG, "d_values is NULL");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  kkt_status ks = refactor_launch(h, d_values, (hipStream_t)stream);
  if (ks != KKT_OK) return ks;
  HIP_CHECK(h, hipGetLastError());
  h->anorm1_valid = false;
  h->factored = true;
  h->factor_epoch++;
  return KKT_OK;
}

kkt_status kkt_graph_capture(kkt_handle h, const double* d_values, const double* d_b, double* d_x,
                             void* stream) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "kkt_graph_capture before kkt_analyze");
  if (!d_values || !d_b || !d_x || !stream)
    return fail(h, KKT_ERR_INVALID_ARG, "null pointer or the legacy default stream");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  HIP_CHECK(h, hipDeviceSynchronize());
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
  hipStream_t s = (hipStream_t)stream;
  HIP_CHECK(h, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  kkt_status ks = refactor_launch(h, d_values, s);
  if (ks == KKT_OK) {
    const kkt_options& o = h->opt;
    const int full = std::max(o.refine_budget > 0 ? std::min(o.refine_budget, o.fgmres_max_iters)
                                                  : o.fgmres_max_iters,
                              std::min(o.min_iters, o.fgmres_max_iters));
    solve_async(h, h->fb, 'N', 1, d_b, d_x, full, s);
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (ks != KKT_OK) {
    if (g) (void)hipGraphDestroy(g);
    return ks;
  }
  if (e != hipSuccess)
    return fail(h, KKT_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  h->graph = g;
  HIP_CHECK(h, hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0));
  h->graph_b = d_b;
  h->graph_x = d_x;
  return KKT_OK;
}

kkt_status kkt_graph_launch(kkt_handle h, void* stream) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->graph_exec) return fail(h, KKT_ERR_STATE, "no captured graph");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  HIP_CHECK(h, hipGraphLaunch(h->graph_exec, (hipStream_t)stream));
  h->anorm1_valid = false;
  h->factored = true;
  h->factor_epoch++;
  h->fg_pending = true;
  return KKT_OK;
}

kkt_status kkt_update_matrix(kkt_handle h, const double* d_values, void* stream) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "kkt_update_matrix before kkt_analyze");
  if (!d_values) return fail(h, KKT_ERR_INVALID_ARG, "d_values is NULL");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  hipStream_t s = (hipStream_t)stream;
  // keep the pivot statistics of the current factors, recompute ||A||_inf
  launch_reset_stats(h->st, 4, s);
  launch_copy_anorm(h->an.n, h->a_rowptr, h->a_col, d_values, h->aval, h->st, s, nullptr,
                    h->rowabs, nullptr, nullptr, nullptr, 0, nullptr, nullptr, h->inst);
  HIP_CHECK(h, hipGetLastError());
  h->anorm1_valid = false;
  h->factor_epoch++;
  h->auto_full = true;  // the factors are now those of another matrix
  return KKT_OK;
}

kkt_status kkt_solve(kkt_handle h, char op, int32_t nrhs, const double* d_b, double* d_x,
                     void* stream) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->factored) return fail(h, KKT_ERR_STATE, "kkt_solve before kkt_analyze");
  if ((op != 'N' && op != 'T') || nrhs < 0 || (nrhs > 0 && (!d_b || !d_x)))
    return fail(h, KKT_ERR_INVALID_ARG, "bad op, nrhs or pointer");
  const int n = vlen(h);
  if (nrhs > 0 && d_b < d_x + (size_t)nrhs * n && d_x < d_b + (size_t)nrhs * n)
    return fail(h, KKT_ERR_INVALID_ARG, "d_b and d_x overlap");
  if (h->inst.count > 1 && (nrhs > 1 || h->opt.refine_sync != 0))
    return fail(h, KKT_ERR_INVALID_ARG,
                "a shared-pattern batch solves one right-hand side per instance, with the stop "
                "test on the device (refine_sync = 0)");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  hipStream_t s = (hipStream_t)stream;
  if (op == 'T' && !h->anorm1_valid) {
    launch_anorm1(h->an.n, h->at_ptr, h->at_pos, h->aval, h->st, s, h->colabs, h->inst);
    h->anorm1_valid = true;
  }
  if (h->opt.refine_sync == 0) {
    // stop test on the device, fixed launch budget, no host synchronisation
    if (nrhs == 0) {
      h->fg_pending = false;
      h->last_iters = 0;
      h->last_eta = h->last_eta0 = 0.0;
      return KKT_OK;
    }
    solve_async(h, h->fb, op, nrhs, d_b, d_x, fg_budget(h), s);
    fg_observe(h, s);
    HIP_CHECK(h, hipGetLastError());
    h->fg_pending = true;
    if (h->opt.auto_reanalyze == 1 && !h->in_retry && h->batch_count == 0 &&
        !h->pat_rowptr.empty()) {
      // the re-analysis decision needs the outcome on the host
      FgState fsh;
      HIP_CHECK(h, hipMemcpyAsync(&fsh, h->fs, sizeof fsh, hipMemcpyDeviceToHost, s));
      HIP_CHECK(h, hipStreamSynchronize(s));
      if (fsh.not_conv) {
        kkt_status ks = kkt_reanalyze(h, h->aval, stream);
        if (ks < 0) return ks;
        h->in_retry = true;
        ks = kkt_solve(h, op, nrhs, d_b, d_x, stream);
        h->in_retry = false;
        h->warnings |= 1 << KKT_WARN_REANALYZED;
        return ks;
      }
    }
    return KKT_OK;
  }
  kkt_status worst = KKT_OK;
  int itmax = 0;
  double emax = 0.0, e0max = 0.0;
  auto account = [&](kkt_status st, int it, double eta, double eta0) {
    if (st > 0) worst = st;
    itmax = std::max(itmax, it);
    if (!(eta <= emax)) emax = eta;
    if (!(eta0 <= e0max)) e0max = eta0;
  };
  if (h->syncfree && h->light && nrhs > 1 && h->batch_count == 0) {
    // all columns of a pass through one dependency-driven launch per
    // triangle, one read-back of every column's eta, refinement only where
    // a column misses the target
    for (int c0 = 0; c0 < nrhs; c0 += MAX_RHS_PASS) {
      const int nr = std::min(MAX_RHS_PASS, nrhs - c0);
      const double* b = d_b + (size_t)c0 * n;
      double* x = d_x + (size_t)c0 * n;
      kkt_status ks = ensure_multi(h, nr);
      if (ks != KKT_OK) return ks;
      apply_factors_multi(h, op, nr, b, x, s);
      if (op == 'N')
        launch_residual_mr(n, nr, h->a_rowptr, h->a_col, nullptr, h->aval, b, x, h->colmax, s);
      else
        launch_residual_mr(n, nr, h->at_ptr, h->at_row, h->at_pos, h->aval, b, x, h->colmax, s);
      HIP_CHECK(h, hipMemcpyAsync(h->h_colmax, h->colmax, sizeof(unsigned long long) * 2 * nr,
                                  hipMemcpyDeviceToHost, s));
      HIP_CHECK(h, hipMemcpyAsync(h->h_st, h->st, sizeof(DevStats), hipMemcpyDeviceToHost, s));
      HIP_CHECK(h, hipStreamSynchronize(s));
      if (h->h_st->stall)
        return fail(h, KKT_ERR_DEVICE, "a dependency wait hit its spin limit (results invalid)");
      const double an = bits_to_double(op == 'N' ? h->h_st->anorm : h->h_st->anorm1);
      for (int c = 0; c < nr; c++) {
        const double rn = bits_to_double(h->h_colmax[2 * c]);
        const double den = an * bits_to_double(h->h_colmax[2 * c + 1]);
        const double eta0 = den == 0.0 ? (rn == 0.0 ? 0.0 : INFINITY) : rn / den;
        if (eta0 <= h->opt.eta_target && h->opt.min_iters == 0) {
          account(KKT_OK, 0, eta0, eta0);
          continue;
        }
        int it;
        double eta, e0;
        kkt_status st = solve_one(h, op, b + (size_t)c * n, x + (size_t)c * n, s, &it, &eta, &e0,
                                  true);
        if (st < 0) return st;
        account(st, it, eta, eta0);
      }
    }
  } else {
    for (int c = 0; c < nrhs; c++) {
      int it;
      double eta, eta0;
      kkt_status st =
          solve_one(h, op, d_b + (size_t)c * n, d_x + (size_t)c * n, s, &it, &eta, &eta0);
      if (st < 0) return st;
      account(st, it, eta, eta0);
    }
  }
  HIP_CHECK(h, hipGetLastError());
  h->last_iters = itmax;
  h->last_eta = emax;
  h->last_eta0 = e0max;
  h->fg_pending = false;
  if (worst > 0) h->warnings |= 1 << worst;
  if (worst == KKT_WARN_NOT_CONVERGED && h->opt.auto_reanalyze == 1 && !h->in_retry &&
      h->batch_count == 0 && !h->pat_rowptr.empty()) {
    // the stored pivot sequence no longer suits the matrix: redo the pivoting
    // pass on the current values (the factors of that pass become current)
    // and solve once more
    kkt_status ks = kkt_reanalyze(h, h->aval, stream);
    if (ks < 0) return ks;
    h->in_retry = true;
    ks = kkt_solve(h, op, nrhs, d_b, d_x, stream);
    h->in_retry = false;
    h->warnings |= 1 << KKT_WARN_REANALYZED;
    return ks;
  }
  return worst;
}

kkt_status kkt_grad_values(kkt_handle h, int32_t nrhs, const double* d_lambda, const double* d_x,
                           double* d_grad, void* stream) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "kkt_grad_values before kkt_analyze");
  if (nrhs <= 0 || !d_lambda || !d_x || !d_grad)
    return fail(h, KKT_ERR_INVALID_ARG, "bad nrhs or pointer");
  if (h->inst.count > 1)
    return fail(h, KKT_ERR_STATE, "kkt_grad_values is for single systems and block-diagonal batches");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  hipStream_t s = (hipStream_t)stream;
  launch_grad_sddmm(h->an.n, nrhs, h->a_rowptr, h->a_col, d_lambda, d_x, d_grad, s);
  HIP_CHECK(h, hipGetLastError());
  return KKT_OK;
}

kkt_status kkt_solve_noalloc(kkt_handle h, char op, int32_t nrhs, const double* d_b, double* d_x,
                             void* stream) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->factored) return fail(h, KKT_ERR_STATE, "kkt_solve_noalloc before kkt_analyze");
  if ((op != 'N' && op != 'T') || nrhs < 0 || (nrhs > 0 && (!d_b || !d_x)))
    return fail(h, KKT_ERR_INVALID_ARG, "bad op, nrhs or pointer");
  if (h->inst.count > 1)
    return fail(h, KKT_ERR_STATE, "kkt_solve_noalloc is for single systems and block-diagonal batches");
  const int n = h->an.n;
  if (nrhs > 0 && d_b < d_x + (size_t)nrhs * n && d_x < d_b + (size_t)nrhs * n)
    return fail(h, KKT_ERR_INVALID_ARG, "d_b and d_x overlap");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  unsigned char* base = scratch_of(h->opt.device);
  if (!base) return fail(h, KKT_ERR_STATE, "no scratch array address for this device");
  FgBufs fb{};
  if (!carve_fgbufs(base, h->m, &fb))
    return fail(h, KKT_ERR_INVALID_ARG,
                "the refinement state for this restart length exceeds the 2 MiB scratch array");
  hipStream_t s = (hipStream_t)stream;
  if (op == 'T' && !h->anorm1_valid) {
    launch_anorm1(h->an.n, h->at_ptr, h->at_pos, h->aval, h->st, s, h->colabs, h->inst);
    h->anorm1_valid = true;
  }
  if (nrhs == 0) {
    h->fg_pending = false;
    h->last_iters = 0;
    h->last_eta = h->last_eta0 = 0.0;
    return KKT_OK;
  }
  solve_async(h, fb, op, nrhs, d_b, d_x, fg_budget(h), s);
  // the outcome into the handle's own state, where kkt_sync_report reads it
  HIP_CHECK(h, hipMemcpyAsync(h->fs, fb.fs, sizeof(FgState), hipMemcpyDeviceToDevice, s));
  fg_observe(h, s);
  HIP_CHECK(h, hipGetLastError());
  h->fg_pending = true;
  return KKT_OK;
}

kkt_status kkt_sync_report(kkt_handle h, kkt_report* out) {
  if (!h || !out) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "no analysis");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  HIP_CHECK(h, hipDeviceSynchronize());
  DevStats d;
  HIP_CHECK(h, hipMemcpy(&d, h->st, sizeof d, hipMemcpyDeviceToHost));
  if (d.stall) return fail(h, KKT_ERR_DEVICE, "a dependency wait hit its spin limit (results invalid)");
  if (h->fg_pending) {
    // outcome of the device-checked solves (kkt_solve, graph replays)
    FgState fsh;
    HIP_CHECK(h, hipMemcpy(&fsh, h->fs, sizeof fsh, hipMemcpyDeviceToHost));
    h->last_iters = fsh.it_max;
    h->last_eta = bits_to_double(fsh.eta_max);
    h->last_eta0 = bits_to_double(fsh.eta0_max);
    if (fsh.not_conv) h->warnings |= 1 << KKT_WARN_NOT_CONVERGED;
    h->fg_pending = false;
  }
  int warn = h->warnings;
  if (d.tiny) warn |= 1 << KKT_WARN_TINY_PIVOT;
  if (d.perturbed) warn |= 1 << KKT_WARN_PERTURBED_PIVOT;
  out->warnings = warn;
  out->iters = h->last_iters;
  out->eta = h->last_eta;
  out->eta0 = h->last_eta0;
  out->min_pivot = bits_to_double(d.min_piv);
  out->max_pivot = bits_to_double(d.max_piv);
  out->anorm_inf = bits_to_double(d.anorm);
  out->growth = eta_of(bits_to_double(d.umax), bits_to_double(d.anorm_f), 1.0);
  h->warnings = 0;
  // the report is filled either way
  if (d.nonfinite_in)
    return fail(h, KKT_ERR_NONFINITE, "the refactorized values hold a NaN or an infinity");
  return KKT_OK;
}

kkt_status kkt_get_info(kkt_handle h, kkt_info* out) {
  if (!h || !out) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "no analysis");
  const Analysis& A = h->an;
  const int32_t cnt = h->inst.count;  // a shared-pattern batch: totals over its instances
  out->n = A.n * cnt;
  out->nnz = A.nnz * cnt;
  out->nnz_l = A.nnz_l * cnt;
  out->nnz_u = A.nnz_u * cnt;
  out->levels = (int32_t)A.lev_ptr.size() - 1;
  out->levels_u = (int32_t)A.ulev_ptr.size() - 1;
  out->analyze_status = A.warn_singular ? KKT_WARN_NUMERICALLY_SINGULAR : KKT_OK;
  out->device_bytes = h->device_bytes;
  out->analyze_seconds = h->analyze_seconds;
  out->dense_tail = h->tail_s;
  out->factor_epoch = h->factor_epoch;
  out->levels_sparse = 0;
  for (int32_t l = 0; l + 1 < (int32_t)A.lev_ptr.size(); l++)
    for (int32_t k = A.lev_ptr[l]; k < A.lev_ptr[l + 1]; k++)
      if (A.lev_rows[k] < h->tail_c0) {
        out->levels_sparse = l + 1;
        break;
      }
  out->solve_block_levels[0] = h->use_sn ? h->chs_levels[0] : 0;
  out->solve_block_levels[1] = h->use_sn ? h->chs_levels[1] : 0;
  return KKT_OK;
}

kkt_status kkt_debug_timeline(kkt_handle h, int64_t* out) {
  if (!h || !out) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed || !h->tl)
    return fail(h, KKT_ERR_STATE, "no timeline (create the handle with debug_timeline = 1)");
  HIP_CHECK(h, hipSetDevice(h->opt.device));
  HIP_CHECK(h, hipDeviceSynchronize());
  const int32_t n = h->an.n;
  std::vector<long long> raw((size_t)3 * n);
  HIP_CHECK(h, hipMemcpy(raw.data(), h->tl, raw.size() * sizeof(long long),
                         hipMemcpyDeviceToHost));
  int khz = 0;
  HIP_CHECK(h, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->opt.device));
  if (khz <= 0) return fail(h, KKT_ERR_DEVICE, "no wall-clock rate");
  const long long mask = (1ll << 62) - 1;
  long long t0 = -1;
  for (int32_t i = 0; i < n; i++)
    if (raw[3 * (size_t)i + 2] != 0 && (t0 < 0 || raw[3 * (size_t)i] < t0)) t0 = raw[3 * (size_t)i];
  const double ns = 1e6 / khz;  // nanoseconds per tick
  for (int32_t i = 0; i < n; i++) {
    const long long e = raw[3 * (size_t)i + 2];
    int64_t* o = out + 4 * (size_t)i;
    if (e == 0) {
      o[0] = o[1] = o[2] = -1;
      o[3] = 0;
      continue;
    }
    o[0] = (int64_t)((raw[3 * (size_t)i] - t0) * ns);
    o[1] = (int64_t)((raw[3 * (size_t)i + 1] - t0) * ns);
    o[2] = (int64_t)(((e & mask) - t0) * ns);
    o[3] = (int64_t)((unsigned long long)e >> 62);
  }
  return KKT_OK;
}

kkt_status kkt_get_scaling(kkt_handle h, int32_t* match, double* dr, double* dc) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "no analysis");
  const Analysis& A = h->an;
  if (A.match.empty()) return fail(h, KKT_ERR_STATE, "the analysis did not match and scale");
  if (match) std::memcpy(match, A.match.data(), A.match.size() * sizeof(int32_t));
  if (dr) std::memcpy(dr, A.dr.data(), A.dr.size() * sizeof(double));
  if (dc) std::memcpy(dc, A.dc.data(), A.dc.size() * sizeof(double));
  return KKT_OK;
}

// (a shared-pattern batch answers in block-diagonal form: instance t's
// rows and columns offset by t n, its factor entries by t nnz(L+U))
kkt_status kkt_get_perm(kkt_handle h, int32_t* p, int32_t* q) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "no analysis");
  const int32_t n = h->an.n;
  for (int32_t t = 0; t < h->inst.count; t++)
    for (int32_t i = 0; i < n; i++) {
      if (p) p[(size_t)t * n + i] = h->an.P[i] + t * n;
      if (q) q[(size_t)t * n + i] = h->an.Q[i] + t * n;
    }
  return KKT_OK;
}

kkt_status kkt_get_lu(kkt_handle h, int64_t* rowptr, int32_t* colind, double* values) {
  if (!h) return KKT_ERR_INVALID_ARG;
  if (!h->analyzed) return fail(h, KKT_ERR_STATE, "no analysis");
  const Analysis& A = h->an;
  const int32_t n = A.n;
  const size_t f = A.lu_col.size();
  const int32_t cnt = h->inst.count;
  for (int32_t t = 0; t < cnt; t++) {
    if (rowptr)
      for (int32_t i = 0; i < n + (t == cnt - 1 ? 1 : 0); i++)
        rowptr[(size_t)t * n + i] = (int64_t)t * (int64_t)f + A.lu_rowptr[i];
    if (colind)
      for (size_t q = 0; q < f; q++) colind[t * f + q] = A.lu_col[q] + t * n;
  }
  if (values) {
    HIP_CHECK(h, hipSetDevice(h->opt.device));
    HIP_CHECK(h, hipDeviceSynchronize());
    HIP_CHECK(h, hipMemcpy(values, h->lu_val, f * cnt * sizeof(double), hipMemcpyDeviceToHost));
  }
  return KKT_OK;
}

const char* kkt_last_error(kkt_handle h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"

struct kkt_host_analysis {
  Analysis an;
};

extern "C" {

kkt_status kkt_analysis_create(const kkt_options* opt, int32_t n, int64_t nnz,
                               const int64_t* rowptr, const int32_t* colind,
                               const double* values0, const int32_t* user_q, kkt_analysis* out,
                               char* msg, int32_t msg_len) {
  if (!out) return KKT_ERR_INVALID_ARG;
  *out = nullptr;
  kkt_options o;
  kkt_options_default(&o);
  if (opt) o = *opt;
  AnalyzeOptions ao;
  ao.ordering = o.ordering;
  ao.tau = o.pivot_tau;
  ao.matching = o.matching;
  kkt_host_analysis* a = new (std::nothrow) kkt_host_analysis();
  if (!a) return KKT_ERR_OUT_OF_MEMORY;
  std::string m;
  int st;
  try {
    st = analyze(n, nnz, rowptr, colind, values0, user_q, ao, a->an, &m);
  } catch (const std::bad_alloc&) {
    st = KKT_ERR_OUT_OF_MEMORY;
    m = "host allocation failed";
  }
  if (st < 0) {
    delete a;
    if (msg && msg_len > 0) {
      std::strncpy(msg, m.c_str(), (size_t)msg_len - 1);
      msg[msg_len - 1] = 0;
    }
    return (kkt_status)st;
  }
  *out = a;
  return (kkt_status)st;
}

kkt_status kkt_analysis_info(kkt_analysis a, kkt_info* out) {
  if (!a || !out) return KKT_ERR_INVALID_ARG;
  const Analysis& A = a->an;
  std::memset(out, 0, sizeof(*out));
  out->n = A.n;
  out->nnz = A.nnz;
  out->nnz_l = A.nnz_l;
  out->nnz_u = A.nnz_u;
  out->levels = (int32_t)A.lev_ptr.size() - 1;
  out->levels_u = (int32_t)A.ulev_ptr.size() - 1;
  out->analyze_status = A.warn_singular ? KKT_WARN_NUMERICALLY_SINGULAR : KKT_OK;
  out->levels_sparse = out->levels;  // the dense block is chosen on the device handle
  return KKT_OK;
}

kkt_status kkt_analysis_scaling(kkt_analysis a, int32_t* match, double* dr, double* dc) {
  if (!a) return KKT_ERR_INVALID_ARG;
  const Analysis& A = a->an;
  if (A.match.empty()) return KKT_ERR_STATE;
  if (match) std::memcpy(match, A.match.data(), A.match.size() * sizeof(int32_t));
  if (dr) std::memcpy(dr, A.dr.data(), A.dr.size() * sizeof(double));
  if (dc) std::memcpy(dc, A.dc.data(), A.dc.size() * sizeof(double));
  return KKT_OK;
}

kkt_status kkt_analysis_perm(kkt_analysis a, int32_t* p, int32_t* q) {
  if (!a) return KKT_ERR_INVALID_ARG;
  if (p) std::memcpy(p, a->an.P.data(), a->an.P.size() * sizeof(int32_t));
  if (q) std::memcpy(q, a->an.Q.data(), a->an.Q.size() * sizeof(int32_t));
  return KKT_OK;
}

kkt_status kkt_analysis_lu(kkt_analysis a, int64_t* rowptr, int32_t* colind, double* values) {
  if (!a) return KKT_ERR_INVALID_ARG;
  const Analysis& A = a->an;
  if (rowptr)
    for (size_t i = 0; i < A.lu_rowptr.size(); i++) rowptr[i] = A.lu_rowptr[i];
  if (colind) std::memcpy(colind, A.lu_col.data(), A.lu_col.size() * sizeof(int32_t));
  if (values) std::memcpy(values, A.lu_val0.data(), A.lu_val0.size() * sizeof(double));
  return KKT_OK;
}

kkt_status kkt_analysis_levels(kkt_analysis a, int32_t* level_ptr, int32_t* rows) {
  if (!a) return KKT_ERR_INVALID_ARG;
  const Analysis& A = a->an;
  if (level_ptr) std::memcpy(level_ptr, A.lev_ptr.data(), A.lev_ptr.size() * sizeof(int32_t));
  if (rows) std::memcpy(rows, A.lev_rows.data(), A.lev_rows.size() * sizeof(int32_t));
  return KKT_OK;
}

void kkt_analysis_destroy(kkt_analysis a) { delete a; }

}  // extern "C"
