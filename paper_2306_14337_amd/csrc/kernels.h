// Device kernels of the refactor/solve path and their host-side launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace kktlu {

// Instances of one pattern that share every index structure (a shared-pattern
// batch): instance t's rows are t n1 .. t n1 + n1 - 1 of the batch vectors, its
// A values start at t a1 and its factor values at t f1; count = 1 otherwise.
struct Inst {
  int count = 1;
  int n1 = 0;
  int a1 = 0, f1 = 0;  // the batch's totals stay below 2^31 (checked at analysis)
};


// Refactorization statistics accumulated on the device (reset per refactor).
struct DevStats {
  unsigned long long min_piv;  // bits of min |u_kk| (non-negative doubles order like uint64)
  unsigned long long max_piv;  // bits of max |u_kk|
  unsigned long long anorm;    // bits of ||A||_inf
  unsigned long long anorm1;   // bits of ||A||_1
  unsigned long long rmax;     // bits of ||r||_inf (scratch of the residual kernel)
  unsigned long long xmax;     // bits of ||x||_inf
  unsigned long long umax;     // bits of max |u_ij| over U (growth numerator)
  unsigned long long anorm_f;  // bits of ||A||_inf of the factored matrix (the matched and
                               // scaled one when the analysis matched; else = anorm)
  int tiny;                    // a tiny or non-finite pivot was seen
  int stall;                   // a dependency wait hit its spin limit (sticky)
  int spin_limit;              // host-set debug limit on every wait (0 = none); follows stall
  int perturbed;               // a pivot was raised to the perturbation threshold
  int nonfinite_in;            // the last refactorization's values held a NaN or an infinity
};

// Sync-free refinement: the stop test of every right-hand side runs on the
// device and the host launches a fixed budget of iterations whose kernels
// return at once for a stopped column.  Right-hand sides are refined in
// groups of at most FG_MAX_COLS columns in lockstep (one triangular-solve
// launch per group and step).
constexpr int FG_MAX_COLS = 8;
constexpr int FG_BLOCKS = 512;  // workgroups per column of a refinement pass
constexpr int FG_RESID_BLOCKS = 4096;  // workgroups per column of the residual pass
constexpr int SEG_SLICES = 16;  // partial per-instance maxima of a batch (launch_seg_stats)
struct FgCol {
  int stop;       // this column's remaining iterations do nothing
  int it;         // iterations done
  int breakdown;  // an Arnoldi step produced w = 0
  int conv;       // eta <= target at the last check
  double eta, eta0, hn, beta;
  unsigned int ticket;  // last-workgroup counter of the fused reductions
  int pad[7];
};
struct FgState {
  FgCol col[FG_MAX_COLS];
  int stop_all;  // every column of the group stopped: gates the triangular solves
  int nstopped;
  // summary over the right-hand sides of the last solve
  int it_max;
  int not_conv;
  unsigned long long eta_max, eta0_max;  // bit patterns (order of non-negative doubles)
};
struct FgParams {
  double eta_target;
  int min_iters;
  int max_iters;
};
// Device workspace of the sync-free refinement: partial sums (FG_MAX_COLS x
// FG_BLOCKS x 32), the two Gram-Schmidt coefficient vectors (32 per column),
// and per column the Hessenberg matrix ((m+1) x m), rotations (m each), g
// (m+1) and y (m).
// Residual pass tickets: FG_TICK_GROUPS first-level counters per column,
// each on its own 128-byte line (FG_TICK_STRIDE unsigned ints apart).
constexpr int FG_TICK_GROUPS = 16;
constexpr int FG_TICK_STRIDE = 32;
struct FgBufs {
  FgState* fs;
  unsigned int* tick1;  // FG_MAX_COLS x FG_TICK_GROUPS x FG_TICK_STRIDE
  double* part;
  double* hbuf;
  double* h2buf;
  double* H;
  double* cs;
  double* sn;
  double* gvec;
  double* y;
};

// Launch gate: while set (non-null), the solve-path kernels launched by this
// host thread (gathers, scatters, triangular solves, dense-block solves,
// per-instance statistics) take the device word as an argument and return at
// once when it is non-zero.  Set around the launches of a sync-free
// refinement so that its triangular solves stop with the group.
void set_launch_gate(const int* gate);
// Adversarial ticket schedule of the persistent kernels (debug; process-wide
// on the current device).  False if the device symbol could not be written.
bool set_debug_schedule(int on);

void launch_fg_begin(const FgBufs& fb, int reset_summary, hipStream_t s);
// r = b - op(A) x for ncols columns (column stride n) and the stop test after
// it_now iterations (first: the check after the direct solve; batch: r only,
// the test follows in launch_fg_check_batch after the per-instance maxima).
// (ptr, idx, pos) as for launch_residual; use_anorm1 selects ||A||_1 (op T).
void launch_fg_resid(int n, int ncols, const int* ptr, const int* idx, const int* pos,
                     const double* aval, const double* b, const double* x, double* r,
                     const FgBufs& fb, const DevStats* st, int use_anorm1, int it_now, int first,
                     int batch, const FgParams& p, hipStream_t s, Inst in = Inst());
void launch_fg_check_batch(int count, const double* inst, const FgBufs& fb, const DevStats* st,
                           int it_now, int first, const FgParams& p, hipStream_t s);
// start of an Arnoldi cycle: x = xt if copy, beta = ||r||, g, v0 = r / beta
void launch_fg_restart(int n, int ncols, int m, const double* r, const double* xt, double* x,
                       int copy, double* v0, const FgBufs& fb, hipStream_t s);
// step j: w = op(A) z_j, h = V^T w; basis vector q of column c at V + (q * ncols + c) * n
void launch_fg_arnoldi(int n, int ncols, int j, const int* ptr, const int* idx, const int* pos,
                       const double* aval, const double* Zj, const double* V, double* w,
                       const FgBufs& fb, hipStream_t s, Inst in = Inst());
// pass 0: w -= V h, h2 = V^T w; pass 1: w -= V h2, ||w||, Givens update, y
void launch_fg_cgs(int pass, int n, int ncols, int j, int m, const double* V, double* w,
                   const FgBufs& fb, hipStream_t s);
// v_{j+1} = w / ||w||, xt = x + Z y (Z's vector q of column c at Z + (q * ncols + c) * n)
void launch_fg_update(int n, int ncols, int j, int m, const double* w, double* vnext,
                      const double* Z, const double* x, double* xt, const FgBufs& fb,
                      hipStream_t s);
void launch_fg_add(int n, int ncols, const double* d, double* x, const FgBufs& fb, hipStream_t s);
// x = xt for FGMRES columns that iterated (ir = 0); summary of the group
void launch_fg_finish(int n, int ncols, const double* xt, double* x, int ir, const FgBufs& fb,
                      hipStream_t s);

// Refactorization rows are split into at most this many bands by row length.
constexpr int REF_MAX_BANDS = 4;

// Scheduling state of the dependency-driven kernels, kept on the device so
// that a captured launch sequence replays correctly: the kernel that precedes
// a dependency-driven phase zeroes its ticket counter and advances its epoch;
// a row is finished in the current phase when ready[row] == epoch.
// Slots: 0 refactorization, 1 first triangular solve, 2 second one.
// The refactorization bands (one launch each) hand out their chunks through
// TICKET_STREAMS interleaved counters: chunk c belongs to stream c % S and a
// workgroup b fetches from stream b % S only (S = min(TICKET_STREAMS, grid)),
// so one device-scope counter no longer serializes every fetch.  Each counter
// sits on its own 128-byte line.
constexpr int TICKET_STREAMS = 8;
constexpr int TICKET_STRIDE = 32;

struct SyncState {
  unsigned int ticket[4];
  int epoch[4];
  // refactorization band b, stream s: band_stream[b][s * TICKET_STRIDE]
  // (reset with slot 0)
  alignas(128) unsigned int band_stream[REF_MAX_BANDS][TICKET_STREAMS * TICKET_STRIDE];
  // chain-blocked solves of slot k, stream s: slot_stream[k][s * TICKET_STRIDE]
  alignas(128) unsigned int slot_stream[4][TICKET_STREAMS * TICKET_STRIDE];
  // dense trailing block's task launch (reset by launch_dlu_reset)
  alignas(128) unsigned int dlu_stream[TICKET_STREAMS * TICKET_STRIDE];
};

// Work chunks of a triangular-solve schedule: chunk c covers rows
// rows[start[c] .. start[c] + count) of one level, each row handled by a
// group of G = 1 << lg lanes; meta[c] = (lg << 8) | count.
struct ChunkSched {
  int nchunks;
  const int* start;
  const int* meta;
  const int* rows;
  int blocks_per_cu = 8;  // persistent grid: 256-thread workgroups per CU
};

// A run of thin levels (few rows each) of a triangular-solve schedule,
// solved by one workgroup level by level with barriers (no cross-CU
// dependency traffic).  Rows are in level order; entry q of segment row j
// (ptr[j] <= q < ptr[j+1]) multiplies val[vpos[q]] with y[src[q]] if
// src[q] >= 0 (a row outside the segment, final before the launch) or with
// the segment's own row -src[q]-1 (kept in LDS); dpos[j] is the diagonal's
// position (U and U^T modes).
struct SegSched {
  int nlev = 0, nrows = 0;
  const int* lev_ptr = nullptr;  // nlev+1, into rows
  const int* row = nullptr;      // nrows: global row index
  const int* ptr = nullptr;      // nrows+1
  const int* src = nullptr;
  const int* vpos = nullptr;
  const int* dpos = nullptr;
};
// rows of one level a segment kernel handles at most, and segment capacity
// (its results stay in LDS: 128 KiB)
constexpr int SEG_MAX_LEVEL_ROWS = 256;
constexpr int SEG_MAX_ROWS = 16384;

// Chain-blocked schedule of a triangular solve (k_trisolve_sn): chunk c has
// rows rows[start[c] .. start[c] + k) (slots), meta[c] = (chain << 16) |
// (lg << 8) | k with G = 1 << lg lanes per row; a chain chunk's rows are
// consecutive in the solve order starting at row base[c], each depending on
// earlier rows of the chunk only through its internal entries; split[slot]
// separates a row's external entries from its internal ones.
constexpr int SN_KMAX = 32;
struct SnSched {
  int nchunks = 0;
  const int* start = nullptr;
  const int* meta = nullptr;
  const int* base = nullptr;
  const int* rows = nullptr;
  const int* split = nullptr;
  int blocks_per_cu = 8;
};
// largest dense trailing block (its solve keeps the block's vector in LDS)
constexpr int DENSE_TAIL_MAX = 2048;

struct LUView {
  int n;
  const int* rowptr;  // n+1
  const int* col;     // f
  const int* diag;    // n
  const int* src;     // f: A position or -1
  double* val;        // f
};

// level-synchronous refactorization of the rows rows[0..nrows) (all their
// dependencies finished in earlier launches).  maxlen = longest row.
// perturb_rel > 0: a final pivot with |u_ii| < perturb_rel ||A||_inf (from
// st->anorm) becomes copysign(perturb_rel ||A||_inf, u_ii) and st->perturbed
// is raised (static pivoting); the same in every refactorization kernel.
void launch_refactor_rows(const LUView& lu, const int* rows, int nrows, int maxlen,
                          const double* aval, DevStats* st, double perturb_rel, hipStream_t s);
// Dependency-driven refactorization of all rows in one launch: waves take
// rows in topological order (order[]) through a ticket counter and wait on
// per-row ready flags.  cap = LDS staging capacity per row (>= longest row).
// Returns false if the configuration cannot be launched.
// Every wait is bounded: past the spin limit a wave sets *stall, and waves
// that see *stall stop waiting, so the grid always drains.
// light: device-coherent data accesses, every factor value its own ready flag
// (lu.val must hold the sentinel on entry: launch_fill_sentinel), instead of
// ready flags with acquire/release fences.
// wpb_pref: waves (rows in flight) per workgroup, 0 = chosen from the LDS need.
// c0: first row/column of the dense trailing block (n = none): rows i >= c0
// apply only the pivots k < c0 (the block is finished by launch_dense_lu).
// Band b: the rows order[cstart[0] .. cstart[nchunks]) (topological order;
// every dependency outside them finished by an earlier launch), taken by the
// waves in chunks order[cstart[c] .. cstart[c+1]) of rows of one level (one
// ticket per chunk: the counters' atomic rate would otherwise bound the wide
// levels), cap >= their longest row, the band's ticket streams
// ss->band_stream[b].
// moff/map (both or neither): precomputed update positions (launch_build_refmap)
// replacing the per-entry binary search.  max_waves_per_cu > 0 caps the
// persistent grid below the occupancy limit.
// luA (nullable): A's values already scattered into factor order (fill
// positions zero), replacing the gather through lu.src; pbnd (nullable): per
// L entry (i, k) the pair (diag[k], rowptr[k + 1]).
bool launch_refactor_syncfree(const LUView& lu, const int* order, const int* cstart,
                              int nchunks, int band, int cap, const double* aval, int* ready,
                              SyncState* ss, int* stall, bool light, int wpb_pref, int c0,
                              const int* moff, const unsigned short* map, const double* luA,
                              const int2* pbnd, int max_waves_per_cu, DevStats* st,
                              double perturb_rel, hipStream_t s);
// map[moff[q] + u] = position in row i of U(k, >k)'s u-th column, for every L
// entry q = (i, k) (moff: offsets indexed by factor position, host-computed)
// flat (nullable, one byte per row): rows of the short-row kernel get packed
// entries (pivot index << 8) | position (their rows have at most 256 entries)
void launch_build_refmap(const LUView& lu, const int* moff, unsigned short* map,
                         const unsigned char* flat, hipStream_t s);

// Any band: one workgroup of several waves per row, the pivot steps taken by
// the waves in turn (each has its next pivot row in flight while the others
// apply theirs).  Device-coherent value-as-flag publication, update maps, A in
// factor order (luA) and pivot-row bounds (pbnd) required; dlc[i] = pivots of
// row i before the dense trailing block (c0); cap >= the band's longest row.
bool launch_refactor_wg(const LUView& lu, const int* order, const int* cstart, int nchunks,
                        int band, int cap, SyncState* ss, int* stall, int c0, const int* dlc,
                        const int* moff, const unsigned short* map, const double* luA,
                        const int2* pbnd, int max_waves_per_cu, DevStats* st, double perturb_rel,
                        hipStream_t s, long long* tl = nullptr, Inst in = Inst());

// A short-row band: one wave per row, every row of the band at most 256
// entries, no row of the dense block.  fl[q] for the
// row's L entries q = (offset of pivot q's first multiply-add in the row's
// list, U row start of pivot q minus that offset), at the diagonal q =
// (length of the list, 0); map holds packed entries (launch_build_refmap with
// flat).  rmeta: per position of the bands' row order, (row start, length |
// pivots << 16, update-map offset, list length); cstart holds positions in
// that order.  Device-coherent value-as-flag publication only.  cmicro (may be
// null): per chunk, non-zero for a chunk of micro rows (one level, at most 64
// rows of at most MICRO_LEN entries, MICRO_PIV pivots and MICRO_LIST
// multiply-adds), taken one row per lane.
constexpr int MICRO_ROW_LEN = 8, MICRO_ROW_PIV = 4, MICRO_ROW_LIST = 4;
bool launch_refactor_flat(const LUView& lu, const int* cstart, int nchunks, int band, int cap,
                          SyncState* ss, int* stall, const int4* rmeta,
                          const unsigned short* map, const double* luA, const int2* fl,
                          const unsigned char* cmicro, int max_waves_per_cu, DevStats* st,
                          double perturb_rel, hipStream_t s, const int* order = nullptr,
                          long long* tl = nullptr, Inst in = Inst());
// tl (debug): per-row timeline of the two band kernels, 3 wall-clock values per
// row (start, last poll that found an input missing, end | kind << 62); order
// (the bands' row order) is read only when tl is set

// Dense trailing block: rows and columns c0 .. c0+s-1 of the factors in pivot
// order, held row-major in T (S x S, S = s rounded up to DLU_NB; the padding
// is an identity block).  scatter: T := the block's LU-pattern entries (zero
// elsewhere); dense_lu: in-place LU without pivoting, every entry updated by
// fma(-l_ik, u_kj, a_ij) in ascending k, l_ik = a_ik / u_kk (the order of the
// sparse refactorization, so the results agree bit for bit); gather: the
// pattern entries back into the factors.  dsc: DLU_NB^2 doubles of scratch.
constexpr int DLU_NB = 32;
void launch_tail_scatter(const LUView& lu, int c0, int s, int S, double* T, hipStream_t st);
void launch_dense_lu(double* T, int S, int s, double* dsc, DevStats* stats, double perturb_rel,
                     hipStream_t st);
// The same LU as one dependency-driven launch over DLU_NB x DLU_NB tiles (nt =
// S / DLU_NB per side): tasks (dense_lu_tasks) do one panel workgroup's work
// (diagonal tile with one column and one row tile) or apply one panel's
// update to a tile; ver[nt * nt] counts the operations finished on each tile
// and is what the tasks wait for.  Dk: nt DLU_NB^2 doubles for the factored
// diagonal tiles, installed in T by a second launch.  Bitwise the same values
// as launch_dense_lu.  launch_dlu_reset zeroes ver and the task tickets
// (stream-ordered before).
std::vector<int> dense_lu_tasks(int nt);
void launch_dlu_reset(int* ver, int nt, SyncState* ss, hipStream_t st);
bool launch_dense_lu_tasks(double* T, int S, int s, const int* tasks, int ntasks, int* ver,
                           double* Dk, SyncState* ss, int* stall, DevStats* stats,
                           double perturb_rel, hipStream_t st);
void launch_tail_gather(const LUView& lu, int c0, const double* T, int S, hipStream_t st);
// Dependency-driven triangular solve of one right-hand side in place on y.
// mode 0: unit L rows, 1: U rows, 2: U^T columns (tptr/trow/tpos view of U),
// 3: unit L^T columns (view of strict L).  slot: SyncState slot (1 or 2).
void launch_trisolve_syncfree(int mode, const LUView& lu, const ChunkSched& cs, const int* tptr,
                              const int* trow, const int* tpos, double* y, int* ready,
                              SyncState* ss, int slot, int* stall, hipStream_t s);
// Value-as-flag triangular solve: reads right-hand side c, writes y, which
// must hold the sentinel on entry (launch_gather_sentinel); c, y: n+1 entries.
void launch_trisolve_vflag(int mode, const LUView& lu, const ChunkSched& cs, const int* tptr,
                           const int* trow, const int* tpos, const double* c, double* y,
                           SyncState* ss, int slot, int* stall, hipStream_t s);
// One workgroup solves a thin segment (mode as launch_trisolve_syncfree):
// y[row] = (c[row] - sum) (/ u_ii); plain loads and stores, so the segment
// must not overlap a dependency-driven launch on the same vector.
void launch_trisolve_seg(int mode, const SegSched& sg, const double* val, const double* c,
                         double* y, hipStream_t s);
// Chain-blocked value-as-flag solve (modes as launch_trisolve_syncfree) of
// nr <= SN_MAX_RHS right-hand sides; c, y column-major with leading dimension
// n + 1, y holding the sentinel wherever it is not yet final.
constexpr int SN_MAX_RHS = 8;
// Mode 1, one right-hand side: xend/pre (nullable, both or neither) exclude
// each row's entries in the dense block's columns from the external terms and
// add pre[i] instead (launch_udense_pre).
void launch_trisolve_sn(int mode, int nr, const LUView& lu, const SnSched& sn, const int* tptr,
                        const int* trow, const int* tpos, const double* c, double* y,
                        SyncState* ss, int slot, int* stall, hipStream_t s,
                        const int* xend = nullptr, const double* pre = nullptr,
                        Inst in = Inst());
// pre[i] = sum over q in [xend[i], rowptr[i + 1]) of val[q] * y[col[q]] for
// the nu rows urows (the U rows' terms in the dense block's columns)
void launch_udense_pre(int nu, const int* urows, const int* xend, const LUView& lu, const double* y,
                       double* pre, hipStream_t st);
// Dense trailing block of a solve (rows c0 .. c0 + s - 1, T as left by
// launch_dense_lu or launch_tail_scatter), nr columns (ld n + 1): modes 0
// and 2 first form rhs = c - external terms (split[t]: end of row c0 + t's
// entries outside the block), then every mode solves its dense triangle into
// y[c0 ..].  For modes 1 and 3 the block comes first and rhs is c + c0.
// rhs_buf: 8 S doubles.
void launch_tail_solve(int mode, int nr, const LUView& lu, const double* T, int S, int s, int c0,
                       const int* split, const int* tptr, const int* trow, const int* tpos,
                       const double* c, double* rhs_buf, double* y, hipStream_t st);
// One right-hand side, the dense block's rows solved by S / 32 workgroups (one
// per 32-row block) that take the other blocks' values from y as they appear:
// y + c0 must hold the sentinel at every position not yet final (or its final
// value).  Same modes and arguments as launch_tail_solve.
void launch_tail_solve_mw(int mode, const LUView& lu, const double* T, int S, int s, int c0,
                          const int* split, const int* tptr, const int* trow, const int* tpos,
                          const double* c, double* rhs_buf, double* y, int* stall,
                          hipStream_t st);
// Right-hand sides per multi-column pass.
constexpr int MAX_RHS_PASS = 32;
// The same for nr <= MAX_RHS_PASS columns at once; c, y column-major with
// leading dimension n + 1.
void launch_trisolve_vflag_mr(int mode, int nr, const LUView& lu, const ChunkSched& cs,
                              const int* tptr, const int* trow, const int* tpos, const double* c,
                              double* y, SyncState* ss, int slot, int* stall, hipStream_t s);
// c[r][i] = x[r][perm[i]] (x: ld n; c, y, z: ld n + 1), y, z := sentinel,
// except y on rows with triv[i] != 0 (no dependencies in the first triangle):
// y = c, or c / val[diag[i]] if div
void launch_gather_sentinel_mr(int n, int nr, const int* perm, const double* scale, const double* x,
                               double* c,
                               double* y, double* z, SyncState* ss, int mask, hipStream_t s,
                               const unsigned char* triv = nullptr, const int* diag = nullptr,
                               const double* val = nullptr, int div = 0, long long f1 = 0);
// x[r][perm[i]] = z[r][i]
void launch_scatter_mr(int n, int nr, const int* perm, const double* scale, const double* z, double* x,
                       hipStream_t s);
// per-column max |B - op(A) X| and max |X| into colmax[2r], colmax[2r+1]
// (uint64 bit patterns of non-negative doubles); zeroes colmax first
void launch_residual_mr(int n, int nr, const int* ptr, const int* idx, const int* pos,
                        const double* aval, const double* B, const double* X,
                        unsigned long long* colmax, hipStream_t s);
// c[i] = x[perm[i]]; y, z := sentinel (y on trivial rows as in the _mr form);
// plus the sync_prep of mask
void launch_gather_sentinel(int n, const int* perm, const double* scale, const double* x, double* c,
                            double* y,
                            double* z, SyncState* ss, int mask, hipStream_t s,
                            const unsigned char* triv = nullptr, const int* diag = nullptr,
                            const double* val = nullptr, int div = 0);
// p[0 .. count) := the value-as-flag sentinel (before a device-coherent
// refactorization: its rows' values are their own ready flags)
void launch_fill_sentinel(double* p, long long count, hipStream_t s);
// factor rows without pivots: val = staged A row, ready = current epoch
void launch_refactor_trivial(const LUView& lu, const int* rows, int nrows, const double* aval,
                             int* ready, const SyncState* ss, hipStream_t s, const double* luA,
                             int c0, DevStats* st, double perturb_rel, Inst in = Inst());
// zero the tickets and advance the epochs of the slots in mask (bit k = slot k)
void launch_sync_prep(SyncState* ss, int mask, hipStream_t s);
// y[i] = x[perm[i]] and, if ss != nullptr, the sync_prep of mask (fused)
void launch_gather_prep(int n, const int* perm, const double* scale, const double* x, double* y,
                        SyncState* ss,
                        int mask, hipStream_t s);

// pivot statistics (min/max |u_kk|, tiny test against tiny_rel * ||A||_inf,
// max |u_ij| over U); red: RED_SCRATCH doubles for the per-workgroup partials
void launch_pivot_stats(const LUView& lu, DevStats* st, double tiny_rel, double* red,
                        hipStream_t s, Inst in = Inst());

// A copy + ||A||_inf (and, if ss != nullptr, the sync_prep of slot 0; if
// rowabs != nullptr, every row's absolute sum; if luA != nullptr, the values
// also scattered into factor order: luA[a2lu[p]] = A[p]).  red (nullable,
// RED_SCRATCH doubles): scratch of a two-stage maximum over a larger grid.
constexpr int RED_SCRATCH = 2 * 4096;
// fnorm: also set anorm_f, the norm of the factored matrix (= ||A||_inf, or
// of the matched and scaled matrix when ascale is given: then avs and luA get
// a_p * ascale[p]); kkt_update_matrix leaves anorm_f alone (fnorm = 0).
void launch_copy_anorm(int n, const int* arow, const int* acol, const double* src, double* dst,
                       DevStats* st, hipStream_t s, SyncState* ss = nullptr,
                       double* rowabs = nullptr, const int* a2lu = nullptr,
                       double* luA = nullptr, double* red = nullptr, int fnorm = 1,
                       const double* ascale = nullptr, double* avs = nullptr, Inst in = Inst());
// ||A||_1 through the column view (and every column's absolute sum)
void launch_anorm1(int n, const int* cptr, const int* cpos, const double* aval, DevStats* st,
                   hipStream_t s, double* colabs = nullptr, Inst in = Inst());
// per-instance maxima of a block-diagonal batch, SEG_SLICES partial results
// per instance: out[3 (t SEG_SLICES + s) + 0..2] = max matabs, max |r|, max |x|
// over slice s of rows [row_off[t], row_off[t+1]) (out holds
// 3 SEG_SLICES count doubles)
void launch_seg_stats(int count, const int* row_off, const double* matabs, const double* r,
                      const double* x, double* out, hipStream_t s);
void launch_reset_stats(DevStats* st, int what, hipStream_t s);

// triangular solves on one right-hand side, in place on y
void launch_lsolve_rows(const LUView& lu, const int* rows, int nrows, int maxlen, double* y,
                        hipStream_t s);
void launch_usolve_rows(const LUView& lu, const int* rows, int nrows, int maxlen, double* y,
                        hipStream_t s);
// transposed: columns via (ptr, row, pos) views
void launch_utsolve_cols(const LUView& lu, const int* cols, int ncols, const int* tptr,
                         const int* trow, const int* tpos, double* y, hipStream_t s);
void launch_ltsolve_cols(const LUView& lu, const int* cols, int ncols, const int* tptr,
                         const int* trow, const int* tpos, double* y, hipStream_t s);

// y[i] = x[perm[i]]  /  y[perm[i]] = x[i]
// gathers and scatters carry an optional per-position scale (nullptr = none):
// y[i] = x[perm[i]] * scale[i]; scatter y[perm[i]] = x[i] * scale[i]
void launch_gather(int n, const int* perm, const double* scale, const double* x, double* y,
                   hipStream_t s);
void launch_scatter(int n, const int* perm, const double* scale, const double* x, double* y,
                    hipStream_t s);

// r = b - op(A) x and the maxima ||r||_inf, ||x||_inf into st; red as in
// launch_copy_anorm
void launch_residual(int n, char op, const int* ptr, const int* idx, const int* pos,
                     const double* aval, const double* b, const double* x, double* r, DevStats* st,
                     hipStream_t s, double* red = nullptr);
// y = op(A) x
void launch_spmv(int n, char op, const int* ptr, const int* idx, const int* pos, const double* aval,
                 const double* x, double* y, hipStream_t s);

// h[i] = sum_t V[i*ld + t] * w[t], i < m  (two-stage deterministic reduction)
void launch_multidot(int n, int m, const double* V, long ld, const double* w, double* partial,
                     double* h, hipStream_t s);
// w -= sum_i h[i] V[i]
void launch_multiaxpy(int n, int m, const double* V, long ld, const double* h, double* w,
                      hipStream_t s);
// out[t] = base[t] + sum_i y[i] Z[i]
void launch_combine(int n, int m, const double* Z, long ld, const double* y, const double* base,
                    double* out, hipStream_t s);
// x += d
void launch_add(int n, const double* d, double* x, hipStream_t s);
// one Jacobi sweep of the unit-L (mode 0) or U (mode 1) solve with right-hand
// side c: yout = c - strict part * yin (then / diagonal for U); all rows at once
void launch_jacobi_sweep(int mode, const LUView& lu, const double* c, const double* yin,
                         double* yout, hipStream_t s);
// y = x * (1 / *scal)  (scal on the device)
void launch_scale_div(int n, const double* x, const double* scal, double* y, hipStream_t s);
// Givens / small least-squares update of column j of the Hessenberg matrix
// (FGMRES bookkeeping, one thread): column = h + h2 (the two CGS passes) and
// ||w|| = sqrt(*ww); H column-major (m+1) x m; writes y (j+1 entries) and
// *hn_out = ||w||.
void launch_givens(int j, int m, const double* h, const double* h2, const double* ww, double* H,
                   double* cs, double* sn, double* g, double* y, double* hn_out, hipStream_t s);
// g = [beta, 0, ...], v0 = r / beta (beta = sqrt(dot) computed on device)
void launch_arnoldi_start(int n, int m, const double* r, const double* rr, double* v0, double* g,
                          hipStream_t s);

// adjoint: grad[p] = -sum_r lam[r][i] x[r][j] over the stored entries p = (i, j)
// (lam, x column-major n x nrhs)
void launch_grad_sddmm(int n, int nrhs, const int* arow_ptr, const int* acol, const double* lam,
                       const double* x, double* grad, hipStream_t s);
// y = x (n entries)
void launch_copy(int n, const double* x, double* y, hipStream_t s);

}  // namespace kktlu
