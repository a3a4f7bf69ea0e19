// HIP kernels for gfx950 (CDNA4, wave64): fixed-pattern sparse LU
// refactorization, triangular solves, residuals and FGMRES-CGS2 pieces.
//
// Arithmetic policy of the refactorization: the updates of each entry are
// applied in ascending pivot-step order as fma(-l, u, a) and l = a / u_kk is
// the IEEE-rounded quotient, which is exactly the sequence of operations of a
// left-looking column factorization; the factors therefore agree bit for bit
// with any implementation that follows the same definition.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace kktlu {

namespace {

// Launch gate of the solve-path kernels (set_launch_gate): every workgroup
// reads the gate word first and returns when it is non-zero, uniformly, before
// any barrier, ticket or store.  The word is written by an earlier kernel on
// the same stream, so a plain load sees it.
#define KKT_GATE(g)                   \
  do {                                \
    if ((g) != nullptr && *(g) != 0) return; \
  } while (0)

thread_local const int* t_gate = nullptr;

constexpr int WAVE = 64;
// k_refactor_wg: waves per row and register buffers per wave (pivot steps in
// flight per row = their product).  Measured at 70k buses (refactorization
// ms): 1 x 2 3.20, 1 x 3 3.21, 2 x 1 3.28, 4 x 1 3.66, 8 x 1 4.16: more rows
// in flight beat more waves per row.
#ifndef KKTLU_WG_WPR
#define KKTLU_WG_WPR 1
#endif
#ifndef KKTLU_WG_DEPTH
#define KKTLU_WG_DEPTH 2
#endif
// k_dlu_update tile edge (70k buses, refactorization ms: 64 2.95, 32 2.87)
#ifndef KKTLU_DLU_TILE
#define KKTLU_DLU_TILE 32
#endif
// k_dlu_panel: pivots between the barriers that let the row-panel wave follow
// the diagonal block's wave (1056-row block, one dense LU in microseconds:
// 1 540, 2 539, 4 541, 8 555, 16 594)
#ifndef KKTLU_DLU_CHUNK
#define KKTLU_DLU_CHUNK 4
#endif
constexpr int RG_TRIV = 8;  // lanes per row of k_refactor_trivial

__device__ __forceinline__ void wave_sync() {
  // LDS operations of one wavefront complete in issue order; this keeps the
  // compiler from moving LDS accesses across the step boundary.
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ unsigned long long dbits(double v) {
  return (unsigned long long)__double_as_longlong(v);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

// first position p in [lo, hi) with a[p] >= key
// Static pivoting: a pivot below the threshold (finite, |d| < thr) takes the
// threshold's magnitude with its own sign; thr <= 0 disables it.
__device__ __forceinline__ double perturb_pivot(double d, double thr) {
  return (thr > 0.0 && fabs(d) < thr) ? copysign(thr, d) : d;
}

__device__ __forceinline__ int lower_bound_i(const int* a, int lo, int hi, int key) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Refactorization, up-looking row form (cf. the paper's Algorithm
// "alg:ginkgo-lu", read with alpha = a_id / u_dd).  Row i of P A' is staged in
// LDS straight from A through the value map (fill entries start at zero);
// for each L entry k of row i in ascending order: l_ik = a_ik / u_kk, then
// a_ij -= l_ik * u_kj for every j in U(k, >k), located in row i by binary
// search over the staged column list.  One wavefront per row; WPB rows per
// workgroup.
// ---------------------------------------------------------------------------
template <int CAP, int WPB>
__global__ __launch_bounds__(WPB* WAVE) void k_refactor_rows_lds(
    const int* __restrict__ rows, int nrows, const int* __restrict__ rowptr,
    const int* __restrict__ col, const int* __restrict__ diag, const int* __restrict__ src,
    const double* __restrict__ aval, double* __restrict__ val, DevStats* st, double prel) {
  __shared__ int s_col[WPB][CAP];
  __shared__ double s_val[WPB][CAP];
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int r = blockIdx.x * WPB + wave;
  if (r >= nrows) return;  // only wavefront-level synchronisation below
  const int i = rows[r];
  const int rs = rowptr[i], len = rowptr[i + 1] - rs, dl = diag[i] - rs;
  int* sc = s_col[wave];
  double* sv = s_val[wave];
  for (int t = lane; t < len; t += WAVE) {
    sc[t] = col[rs + t];
    const int s = src[rs + t];
    sv[t] = s >= 0 ? aval[s] : 0.0;
  }
  wave_sync();
  for (int t = 0; t < dl; t++) {
    const int k = sc[t];
    const int dk = diag[k];
    const int ke = rowptr[k + 1];
    const double lik = sv[t] / val[dk];
    for (int q = dk + 1 + lane; q < ke; q += WAVE) {
      const int j = col[q];
      const double u = val[q];
      const int p = lower_bound_i(sc, t + 1, len, j);
      // the fill pattern guarantees j is in row i; the test keeps a corrupt
      // pattern from writing outside this row
      if (p < len && sc[p] == j) sv[p] = __builtin_fma(-lik, u, sv[p]);
    }
    wave_sync();
    if (lane == 0) sv[t] = lik;
    wave_sync();
  }
  if (prel > 0.0) {
    const double thr = prel * __longlong_as_double((long long)st->anorm_f);
    const double d = sv[dl];
    if (fabs(d) < thr) {
      if (lane == 0) sv[dl] = perturb_pivot(d, thr);
      st->perturbed = 1;
    }
    wave_sync();
  }
  for (int t = lane; t < len; t += WAVE) val[rs + t] = sv[t];
}

// Same computation with the row kept in global memory (rows longer than the
// LDS staging capacity).  One wavefront per workgroup.
__global__ __launch_bounds__(WAVE) void k_refactor_rows_global(
    const int* __restrict__ rows, int nrows, const int* __restrict__ rowptr,
    const int* __restrict__ col, const int* __restrict__ diag, const int* __restrict__ src,
    const double* __restrict__ aval, double* val, DevStats* st, double prel) {
  const int lane = threadIdx.x;
  const int r = blockIdx.x;
  if (r >= nrows) return;
  const int i = rows[r];
  const int rs = rowptr[i], re = rowptr[i + 1], dpos = diag[i];
  for (int q = rs + lane; q < re; q += WAVE) {
    const int s = src[q];
    val[q] = s >= 0 ? aval[s] : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  for (int t = rs; t < dpos; t++) {
    const int k = col[t];
    const int dk = diag[k];
    const int ke = rowptr[k + 1];
    const double lik = val[t] / val[dk];
    for (int q = dk + 1 + lane; q < ke; q += WAVE) {
      const int j = col[q];
      const double u = val[q];
      const int p = lower_bound_i(col, t + 1, re, j);
      if (p < re && col[p] == j) val[p] = __builtin_fma(-lik, u, val[p]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) val[t] = lik;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
  if (prel > 0.0) {
    const double thr = prel * __longlong_as_double((long long)st->anorm_f);
    const double d = val[dpos];
    if (fabs(d) < thr) {
      if (lane == 0) val[dpos] = perturb_pivot(d, thr);
      st->perturbed = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Dependency-driven ("sync-free") variants.  Waves fetch work in topological
// order through a ticket counter; a wave only ever waits for rows with smaller
// tickets, which were fetched by waves that are already running, so the
// oldest unfinished row always has its inputs and the grid drains.  A
// finished row is published with a device-scope release (its values, then
// ready[row] = epoch); a consumer observes the flag with device-scope loads
// and issues one device-scope acquire for a whole batch of ready inputs (the
// eight XCDs have separate L2 caches).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ld_flag(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Value-as-flag protocols: a value not yet produced holds a signaling-NaN bit
// pattern that no arithmetic result carries (results are quiet NaNs at
// worst); consumers poll the value itself with device-coherent loads.
constexpr unsigned long long SENTINEL = 0x7FF0DEAD5EED0001ull;

__device__ __forceinline__ bool is_sentinel(double v) {
  return (unsigned long long)__double_as_longlong(v) == SENTINEL;
}

// Inputs enter the value-as-flag arrays through this: any NaN becomes the
// canonical quiet NaN, so no input can carry the sentinel's bit pattern.
__device__ __forceinline__ double canon_nan(double v) {
  return v != v ? __longlong_as_double(0x7FF8000000000000ll) : v;
}

__global__ void k_fill_sentinel(double* __restrict__ p, long long count) {
  const double sent = __longlong_as_double((long long)SENTINEL);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x)
    p[e] = sent;
}

// 2^20 polling rounds (each a device-scope load plus a short sleep, about a
// microsecond): far longer than any legitimate wait of one factorization or
// solve, short enough that a broken schedule drains in about a second
constexpr int SPIN_LIMIT = 1 << 20;

// Broadcast of a lane-0 value through a scalar register.  Unlike a shuffle,
// the result is provably wave-uniform, so loops whose exit depends on it stay
// uniform loops (a shuffle-broadcast exit condition lets the compiler treat
// the loop as divergent and split lane 0's flag store out of it).
__device__ __forceinline__ unsigned int bcast0(unsigned int v) {
  return (unsigned int)__builtin_amdgcn_readfirstlane((int)v);
}

// Next chunk of a launch whose chunks are handed out through nstreams
// interleaved ticket counters (chunk c in stream c % nstreams, workgroup b
// fetching from stream b % nstreams; every stream has a workgroup since
// nstreams <= grid).  Deadlock freedom as with one counter: let u be the
// lowest unfinished chunk.  Its inputs lie in lower chunks, all finished.  If
// u was fetched, its wave completes it; if not, every fetched chunk of its
// stream is lower, hence finished, so that stream's waves are free and one
// of them fetches u next.  Returns a value >= nchunks once the stream is
// exhausted.
//
// Adversarial schedule (debug, g_debug_schedule != 0): workgroup b fetches
// from stream nstreams - 1 - b % nstreams instead (a different workgroup,
// hence XCD, for every chunk; each stream still has as many workgroups), and
// it pauses a pseudo-random 0-7 x 128 cycles after each fetch, so chunks start
// and publish in another order.  Results must not change.
__device__ int g_debug_schedule = 0;

__device__ __forceinline__ int next_chunk(unsigned int* streams, int nstreams, int lane) {
  const int dbg = g_debug_schedule;
  const int b = (int)(blockIdx.x % (unsigned int)nstreams);
  const int s = dbg ? nstreams - 1 - b : b;
  const unsigned int m =
      bcast0(atomicAdd(streams + s * TICKET_STRIDE, lane == 0 ? 1u : 0u));
  if (dbg) {
    const unsigned int h = (m * 2654435761u) ^ (blockIdx.x * 40503u);
    for (unsigned int k = 0; k < ((h >> 13) & 7u); k++) __builtin_amdgcn_s_sleep(2);
  }
  return (int)m * nstreams + s;
}

// One more round of waiting allowed?  False once the limit is hit here (the
// wave raises *stall) or anywhere else (another wave raised it).
// The stall flag is polled every 64th round only; between rounds the wave
// pauses 64 cycles.  (A pause growing with the wait, meant to keep far-ahead
// waves off the memory system, measured slower: it delays the waves at the
// dependency front by up to the pause length.)
// stall[1] (DevStats::spin_limit) > 0 is a host-set debug limit on a wave's
// polls, read on its second poll and with every stall-flag check.
__device__ __forceinline__ bool keep_waiting(int* spins, int* stall) {
  if ((*spins & 63) == 63 || *spins == 1) {
    if ((*spins & 63) == 63 && ld_flag(stall)) return false;
    const int lim = stall[1];
    if (lim > 0 && *spins >= lim) {
      st_flag(stall, 1);
      return false;
    }
  }
  if (++*spins > SPIN_LIMIT) {
    st_flag(stall, 1);
    return false;
  }
  __builtin_amdgcn_s_sleep(1);
  return true;
}

// Device-coherent ("light") publication: data written with device-scope
// stores (write-through to the level shared by all XCDs) and read with
// device-scope loads, so neither an L2 writeback nor an L2 invalidate is
// needed; the producer only waits for its stores to complete before raising
// the flag.
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stores_done() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);  // every outstanding memory operation complete
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Up-looking refactorization, as k_refactor_rows_lds, in one launch.  The L
// entries of a row are consumed in ascending order; before entry t the wave
// checks (one lane per entry) how many of the next 64 inputs are finished and
// takes one acquire fence for all of them.
//
// No branch in the work loop depends on the lane index: the ticket atomic is
// issued by every lane (only lane 0 adds 1) and every lane stores the same
// flag value.  A lane-0-only region at the loop boundary lets the compiler
// split the loop so that lanes 1..63 iterate without lane 0 on a stale
// ticket, which never terminates.
// Rows of the refactorization without pivots (no L entries before the dense
// block): their factor row is the staged A row.  8 lanes per row; the ready
// flag carries the epoch of the current refactorization (a later launch reads
// both, so plain stores suffice).
__global__ __launch_bounds__(256) void k_refactor_trivial(int nrows, const int* __restrict__ rows,
                                                          const int* __restrict__ rowptr,
                                                          const int* __restrict__ src,
                                                          const double* __restrict__ aval,
                                                          double* __restrict__ val0, int* ready,
                                                          const SyncState* ss,
                                                          const double* __restrict__ luA0,
                                                          const int* __restrict__ diag, int c0,
                                                          DevStats* st, double prel, Inst in) {
  const int lane = threadIdx.x % WAVE, g = lane / RG_TRIV, gl = lane % RG_TRIV;
  const int epoch = ss->epoch[0];
  const double thr = prel > 0.0 ? prel * __longlong_as_double((long long)st->anorm_f) : 0.0;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  const int total = nrows * in.count;  // the rows of every instance
  for (int r0 = wid * (WAVE / RG_TRIV); r0 < total; r0 += nw * (WAVE / RG_TRIV)) {
    const int rg = r0 + g;
    if (rg >= total) continue;
    const int ti = rg / nrows;
    const int i = rows[rg - ti * nrows];
    double* val = val0 + ti * in.f1;
    const double* luA = luA0 ? luA0 + ti * in.f1 : nullptr;
    const int dq = i < c0 ? diag[i] : -1;  // pivots of the dense block: there
    for (int q = rowptr[i] + gl; q < rowptr[i + 1]; q += RG_TRIV) {
      double v;
      if (luA) {
        v = luA[q];
      } else {
        const int sq = src[q];
        v = sq >= 0 ? aval[sq + ti * in.a1] : 0.0;
      }
      if (q == dq && fabs(v) < thr) {
        v = perturb_pivot(v, thr);
        st->perturbed = 1;
      }
      val[q] = v;
    }
    if (gl == 0) ready[i] = epoch;
  }
}

// Update maps of the refactorization, built once per analysis: for the L
// entry q = (i, k), map[moff[q] + u] = position (from the row start) of the
// column of U(k, >k)'s u-th entry in row i; rows flagged in flat (rows of at
// most 256 entries) carry (q - row start) << 8 in the high byte as well.
// Wave per row, lanes over U(k).
__global__ __launch_bounds__(256) void k_build_refmap(int n, const int* __restrict__ rowptr,
                                                      const int* __restrict__ col,
                                                      const int* __restrict__ diag,
                                                      const int* __restrict__ moff,
                                                      unsigned short* __restrict__ map,
                                                      const unsigned char* __restrict__ flat) {
  const int lane = threadIdx.x % WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  for (int i = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE; i < n; i += nw) {
    const int rs = rowptr[i], re = rowptr[i + 1];
    const bool packed = flat != nullptr && flat[i] != 0;
    for (int q = rs; q < diag[i]; q++) {
      const int k = col[q], ub = diag[k] + 1, ue = rowptr[k + 1];
      const int mo = moff[q];
      const int hi = packed ? (q - rs) << 8 : 0;
      for (int u = ub + lane; u < ue; u += WAVE) {
        const int p = lower_bound_i(col, q + 1, re, col[u]);
        map[mo + (u - ub)] = (unsigned short)(hi | (p - rs));
      }
    }
  }
}

// MAPPED: the target position of every update comes from a precomputed map
// (map[moff[q] + u] = position in row i of the u-th entry of U(k, >k) for
// the L entry q = (i, k)) instead of a binary search over the staged columns.
template <int WPB, bool LIGHT, bool MAPPED>
__global__ __launch_bounds__(WPB* WAVE) void k_refactor_syncfree(
    const int* __restrict__ order, const int* __restrict__ cstart, int nchunks,
    unsigned int* tickets, int nstreams, const int* __restrict__ rowptr,
    const int* __restrict__ col, const int* __restrict__ diag, const int* __restrict__ src,
    const double* __restrict__ aval, double* val, int* ready, SyncState* ss, int* stall, int cap,
    int c0, const int* __restrict__ moff, const unsigned short* __restrict__ map,
    const double* __restrict__ luA, const int2* __restrict__ pbnd, DevStats* st, double prel) {
  extern __shared__ double smem_d[];
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  // LDS per wave: values (cap doubles), pivot-row bounds (cap int2), columns (cap ints)
  double* sv = smem_d + (size_t)wave * cap;
  int2* sk = reinterpret_cast<int2*>(smem_d + (size_t)WPB * cap) + (size_t)wave * cap;
  int* sc = reinterpret_cast<int*>(smem_d + (size_t)WPB * cap * 2) + (size_t)wave * cap;
  const int epoch = ss->epoch[0];
  const double thr = prel > 0.0 ? prel * __longlong_as_double((long long)st->anorm_f) : 0.0;
  for (;;) {
    const int tk = next_chunk(tickets, nstreams, lane);
    if (tk >= nchunks) break;
    const int r_end = cstart[tk + 1];
    for (int r = cstart[tk]; r < r_end; r++) {
    const int i = order[r];
    wave_sync();  // the previous row of this chunk is done with the staging area
    const int rs = rowptr[i], len = rowptr[i + 1] - rs;
    int dl = diag[i] - rs;
    // the row's columns and A values (luA: already in factor order, else
    // gathered through src), and the bounds (diagonal position, row end) of
    // every pivot row it needs (pbnd: precomputed per L entry), all loaded
    // in parallel up front
    for (int t = lane; t < len; t += WAVE) {
      sc[t] = col[rs + t];
      if (luA) {
        sv[t] = luA[rs + t];
      } else {
        const int s = src[rs + t];
        sv[t] = s >= 0 ? aval[s] : 0.0;
      }
    }
    for (int t = lane; t < dl; t += WAVE) {
      if (pbnd) {
        sk[t] = pbnd[rs + t];
      } else {
        const int k = col[rs + t];
        sk[t] = make_int2(diag[k], rowptr[k + 1]);
      }
    }
    wave_sync();
    // rows of the dense trailing block take only the pivots before it here
    if (i >= c0) dl = lower_bound_i(sc, 0, dl, c0);
    int ready_upto = 0, spins = 0;
    // software pipeline: the pivot and the first 64 entries of the next ready
    // pivot row are in flight while the current one is applied
    double ukk = 0.0, u0 = 0.0;
    int j0 = -1, mo = 0;
    bool have = false;
    for (int t = 0; t < dl; t++) {
      if (t >= ready_upto) {
        for (;;) {
          // LIGHT: a pivot row is final once its diagonal value is (the
          // values themselves are the flags; every entry is checked on use)
          const int q = t + lane;
          const bool ok = q >= dl || (LIGHT ? !is_sentinel(ld_coh(val + sk[q].x))
                                            : ld_flag(ready + sc[q]) == epoch);
          const unsigned long long bad = __ballot(!ok);
          const int first_bad = bad ? __ffsll((long long)bad) - 1 : WAVE;
          if (first_bad > 0) {
            ready_upto = t + first_bad;
            break;
          }
          // entry t itself is missing
          bool go = true;
          if (LIGHT) {
            // poll the pivot's diagonal together with the first 64 entries
            // of its U row: once none of them reads as the sentinel they are
            // the values of this pivot step, so the step starts without a
            // re-check or a reload (on a chain of rows each waiting for the
            // one before, this wait is the critical path)
            const int2 kw = sk[t];
            const int q = kw.x + 1 + lane;
            if (MAPPED) mo = moff[rs + t];
            j0 = -1;
            if (q < kw.y) j0 = MAPPED ? (int)map[mo + lane] : col[q];
            for (;;) {
              ukk = ld_coh(val + kw.x);
              u0 = q < kw.y ? ld_coh(val + q) : 0.0;
              const bool miss = is_sentinel(ukk) || (q < kw.y && is_sentinel(u0));
              if (__ballot(miss) == 0) break;
              go = bcast0(keep_waiting(&spins, stall) ? 1u : 0u) != 0u;
              if (!go) break;
            }
            if (go) {
              ready_upto = t + 1;
              have = true;
              break;
            }
          } else {
            const int kt = sc[t];
            while (go && bcast0((unsigned int)ld_flag(ready + kt)) != (unsigned int)epoch)
              go = bcast0(keep_waiting(&spins, stall) ? 1u : 0u) != 0u;
          }
          if (!go) {
            ready_upto = dl;
            break;
          }
        }
        if (!LIGHT) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      const int2 kk = sk[t];
      // j0: first-chunk entry's column (binary search) or target position (map)
      if (!have) {
        ukk = LIGHT ? ld_coh(val + kk.x) : val[kk.x];
        const int q = kk.x + 1 + lane;
        j0 = -1;
        if (MAPPED) mo = moff[rs + t];
        if (q < kk.y) {
          j0 = MAPPED ? (int)map[mo + lane] : col[q];
          u0 = LIGHT ? ld_coh(val + q) : val[q];
        }
      }
      double ukk_n = 0.0, u0_n = 0.0;
      int j0_n = -1, mo_n = 0;
      const bool have_n = t + 1 < dl && t + 1 < ready_upto;
      if (have_n) {
        const int2 kn = sk[t + 1];
        ukk_n = LIGHT ? ld_coh(val + kn.x) : val[kn.x];
        const int q = kn.x + 1 + lane;
        if (MAPPED) mo_n = moff[rs + t + 1];
        if (q < kn.y) {
          j0_n = MAPPED ? (int)map[mo_n + lane] : col[q];
          u0_n = LIGHT ? ld_coh(val + q) : val[q];
        }
      }
      const double lik = sv[t] / ukk;
      // LIGHT: an entry of the pivot row may still be in flight although its
      // diagonal has landed
      if (LIGHT && j0 >= 0)
        while (is_sentinel(u0) && keep_waiting(&spins, stall)) u0 = ld_coh(val + kk.x + 1 + lane);
      if (MAPPED) {
        if (j0 >= 0) sv[j0] = __builtin_fma(-lik, u0, sv[j0]);
        // remaining chunks: four loads of each kind in flight per lane
        const int ub = kk.x + 1;
        for (int q0 = ub + WAVE + lane; q0 < kk.y; q0 += 4 * WAVE) {
          double u[4];
          int p[4];
#pragma unroll
          for (int z = 0; z < 4; z++) {
            const int q = q0 + z * WAVE;
            p[z] = -1;
            u[z] = 0.0;
            if (q < kk.y) {
              p[z] = map[mo + (q - ub)];
              u[z] = LIGHT ? ld_coh(val + q) : val[q];
            }
          }
#pragma unroll
          for (int z = 0; z < 4; z++) {
            if (LIGHT && p[z] >= 0)
              while (is_sentinel(u[z]) && keep_waiting(&spins, stall))
                u[z] = ld_coh(val + q0 + z * WAVE);
            if (p[z] >= 0) sv[p[z]] = __builtin_fma(-lik, u[z], sv[p[z]]);
          }
        }
      } else {
        if (j0 >= 0) {
          const int p = lower_bound_i(sc, t + 1, len, j0);
          if (p < len && sc[p] == j0) sv[p] = __builtin_fma(-lik, u0, sv[p]);
        }
        for (int q = kk.x + 1 + WAVE + lane; q < kk.y; q += WAVE) {
          const int j = col[q];
          double u = LIGHT ? ld_coh(val + q) : val[q];
          if (LIGHT)
            while (is_sentinel(u) && keep_waiting(&spins, stall)) u = ld_coh(val + q);
          const int p = lower_bound_i(sc, t + 1, len, j);
          if (p < len && sc[p] == j) sv[p] = __builtin_fma(-lik, u, sv[p]);
        }
      }
      wave_sync();
      sv[t] = lik;  // every lane writes the same value
      wave_sync();
      ukk = ukk_n;
      u0 = u0_n;
      j0 = j0_n;
      mo = mo_n;
      have = have_n;
    }
    // static pivoting of this row's pivot (rows of the dense block: there)
    if (thr > 0.0 && i < c0) {
      const int dr = diag[i] - rs;
      const double d = sv[dr];
      if (fabs(d) < thr) {
        wave_sync();
        sv[dr] = perturb_pivot(d, thr);  // every lane writes the same value
        st->perturbed = 1;
      }
      wave_sync();
    }
    // LIGHT: each value is its own flag (the factor started filled with the
    // sentinel), so no completion wait and no flag; otherwise values, a
    // device-scope release, then the flag
    for (int t = lane; t < len; t += WAVE) {
      if (LIGHT)
        st_coh(val + rs + t, sv[t]);
      else
        val[rs + t] = sv[t];
    }
    if (!LIGHT) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      st_flag(ready + i, epoch);  // every lane, same address and value
    }
    }
  }
}

// Triangular solve of one right-hand side, dependency driven.  A wave takes
// one chunk (rows of one level, G lanes per row); every lane waits for the
// inputs of its own entries, the wave takes one acquire fence, the groups
// reduce their dot products and publish their rows.
//   MODE 0  L rows:   y_i -= sum_{q < diag_i} val_q y_{col_q}
//   MODE 1  U rows:   y_i = (y_i - sum_{q > diag_i} val_q y_{col_q}) / u_ii
//   MODE 2  U^T cols: y_j = (y_j - sum_t val_{pos_t} y_{row_t}) / u_jj
//   MODE 3  L^T cols: y_j -= sum_t val_{pos_t} y_{row_t}
// As in the refactorization, no lane-indexed branch guards a store: every
// lane of a group writes its row's (identical) result and flag, and lanes
// without a row write to the spare slot n of y and ready (n + 1 entries).
template <int MODE>
__global__ __launch_bounds__(256) void k_trisolve_syncfree(const int* __restrict__ gate, 
    int n, int nchunks, const int* __restrict__ ch_start, const int* __restrict__ ch_meta,
    const int* __restrict__ rows, const int* __restrict__ rowptr, const int* __restrict__ col,
    const int* __restrict__ diag, const int* __restrict__ tptr, const int* __restrict__ trow,
    const int* __restrict__ tpos, const double* __restrict__ val, double* y, int* ready,
    SyncState* ss, int slot, int* stall) {
  KKT_GATE(gate);
  const int lane = threadIdx.x % WAVE;
  const int epoch = ss->epoch[slot];
  unsigned int* ticket = &ss->ticket[slot];
  for (;;) {
    const unsigned int tk = bcast0(atomicAdd(ticket, lane == 0 ? 1u : 0u));
    if (tk >= (unsigned int)nchunks) break;
    const int meta = ch_meta[tk];
    const int lg = meta >> 8, cnt = meta & 0xff;
    const int G = 1 << lg;
    const int grp = lane >> lg, gl = lane & (G - 1);
    const bool active = grp < cnt;
    const int i = active ? rows[ch_start[tk] + grp] : n;
    int b = 0, e = 0, dpos = 0;
    if (active) {
      if (MODE == 0) {
        b = rowptr[i];
        e = diag[i];
      } else if (MODE == 1) {
        dpos = diag[i];
        b = dpos + 1;
        e = rowptr[i + 1];
      } else if (MODE == 2) {
        b = tptr[i];
        e = tptr[i + 1] - 1;
        dpos = tpos[e];
      } else {
        b = tptr[i];
        e = tptr[i + 1];
      }
    }
    int spins = 0;
    for (int q = b + gl; q < e; q += G) {
      const int k = MODE <= 1 ? col[q] : trow[q];
      while (ld_flag(ready + k) != epoch && keep_waiting(&spins, stall)) {
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double s = 0.0;
    for (int q = b + gl; q < e; q += G) {
      if (MODE <= 1)
        s += val[q] * y[col[q]];
      else
        s += val[tpos[q]] * y[trow[q]];
    }
    // butterfly: every lane of the group ends with the same sum
    for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
    const double yi = y[i];
    y[i] = (MODE == 0 || MODE == 3) ? yi - s : (yi - s) / val[dpos];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    st_flag(ready + i, epoch);
  }
}

// Value-as-flag triangular solve: the output vector starts filled with a
// signaling-NaN bit pattern that no arithmetic result can carry (results are
// quiet NaNs at worst), so a consumer spins on the value itself with
// device-scope loads and the producer publishes with one device-scope store:
// one round trip per dependency and no fences.  Input c and output y are
// separate arrays (n + 1 entries; slot n takes idle lanes' writes).

template <int MODE>
__global__ __launch_bounds__(256) void k_trisolve_vflag(const int* __restrict__ gate, 
    int n, int nchunks, const int* __restrict__ ch_start, const int* __restrict__ ch_meta,
    const int* __restrict__ rows, const int* __restrict__ rowptr, const int* __restrict__ col,
    const int* __restrict__ diag, const int* __restrict__ tptr, const int* __restrict__ trow,
    const int* __restrict__ tpos, const double* __restrict__ val, const double* __restrict__ c,
    double* y, SyncState* ss, int slot, int* stall) {
  KKT_GATE(gate);
  const int lane = threadIdx.x % WAVE;
  unsigned int* ticket = &ss->ticket[slot];
  for (;;) {
    const unsigned int tk = bcast0(atomicAdd(ticket, lane == 0 ? 1u : 0u));
    if (tk >= (unsigned int)nchunks) break;
    const int meta = ch_meta[tk];
    const int lg = meta >> 8, cnt = meta & 0xff;
    const int G = 1 << lg;
    const int grp = lane >> lg, gl = lane & (G - 1);
    const bool active = grp < cnt;
    const int i = active ? rows[ch_start[tk] + grp] : n;
    int b = 0, e = 0, dpos = 0;
    if (active) {
      if (MODE == 0) {
        b = rowptr[i];
        e = diag[i];
      } else if (MODE == 1) {
        dpos = diag[i];
        b = dpos + 1;
        e = rowptr[i + 1];
      } else if (MODE == 2) {
        b = tptr[i];
        e = tptr[i + 1] - 1;
        dpos = tpos[e];
      } else {
        b = tptr[i];
        e = tptr[i + 1];
      }
    }
    int spins = 0;
    double s = 0.0;
    // batches of VB entries per lane: all VB dependency loads are in flight
    // together, then each is checked (and re-polled only if not yet written);
    // the per-lane summation order stays ascending
    constexpr int VB = 8;
    for (int q0 = b + gl; q0 < e; q0 += VB * G) {
      int k[VB];
      double v[VB], yk[VB];
#pragma unroll
      for (int u = 0; u < VB; u++) {
        const int q = q0 + u * G;
        k[u] = n;
        v[u] = 0.0;
        if (q < e) {
          k[u] = MODE <= 1 ? col[q] : trow[q];
          v[u] = MODE <= 1 ? val[q] : val[tpos[q]];
        }
      }
#pragma unroll
      for (int u = 0; u < VB; u++) yk[u] = q0 + u * G < e ? ld_coh(y + k[u]) : 0.0;
#pragma unroll
      for (int u = 0; u < VB; u++) {
        while (is_sentinel(yk[u]) && keep_waiting(&spins, stall)) yk[u] = ld_coh(y + k[u]);
        if (q0 + u * G < e) s += v[u] * yk[u];
      }
    }
    for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
    const double ci = c[i];
    st_coh(y + i, (MODE == 0 || MODE == 3) ? ci - s : (ci - s) / val[dpos]);
  }
}

__device__ __forceinline__ void sync_prep(SyncState* ss, int mask) {
  for (int k = 0; k < 4; k++)
    if (mask & (1 << k)) {
      ss->ticket[k] = 0u;
      ss->epoch[k] = ss->epoch[k] + 1;
      for (int t = 0; t < TICKET_STREAMS; t++) ss->slot_stream[k][t * TICKET_STRIDE] = 0u;
      if (k == 0)
        for (int b = 0; b < REF_MAX_BANDS; b++)
          for (int t = 0; t < TICKET_STREAMS; t++) ss->band_stream[b][t * TICKET_STRIDE] = 0u;
    }
}

__global__ void k_sync_prep(SyncState* ss, int mask) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sync_prep(ss, mask);
}

// ---------------------------------------------------------------------------
// Thin segment of a triangular solve on one workgroup.  The top of the
// elimination tree is a long run of levels with a handful of rows each; across
// CUs every level costs a device-scope round trip, inside one workgroup it
// costs two barriers.  Per level the 16 waves are split over the level's rows
// (waves per row = 16 / rows), each wave reduces its share of a row's dot
// product, and one thread per row finishes it; segment results stay in LDS.
// The matrix entries (and the solution values from outside the segment) of
// level l + 1 are loaded while level l is computed.
// ---------------------------------------------------------------------------
constexpr int SEG_THREADS = 1024;
constexpr int SEG_WAVES = SEG_THREADS / WAVE;
constexpr int SEG_PF = 4;  // prefetched entries per lane and level

// Work of one level for the calling thread.  Levels of up to 16 rows: waves
// per row ng = 16 / rows, thread t < rows finishes row t from the waves'
// partial sums.  Wider levels (up to SEG_MAX_LEVEL_ROWS rows): G = 1024 / P
// lanes per row (P = rows rounded up to a power of two), the group's first
// lane finishes the row from a shuffle reduction.  The finishing thread also
// prefetches its row index, right-hand side and (U, U^T) diagonal.
struct SegWork {
  int q0, stride, e;  // entries q0, q0 + stride, ... < e
  int slot, ri;       // finisher: segment slot and row index (slot < 0: none)
  double rc, rd;
};

__device__ __forceinline__ int seg_group(int nr) {
  int p = 32;
  while (p < nr) p <<= 1;
  return SEG_THREADS / p;
}

template <int MODE>
__device__ __forceinline__ void seg_fetch(int lev, int nlev, const int* __restrict__ lev_ptr,
                                          const int* __restrict__ row,
                                          const int* __restrict__ ptr,
                                          const int* __restrict__ src,
                                          const int* __restrict__ vpos,
                                          const int* __restrict__ dpos,
                                          const double* __restrict__ val,
                                          const double* __restrict__ c,
                                          const double* __restrict__ y, int* fs, double* fv,
                                          double* fy, SegWork& wk) {
  const int t = threadIdx.x, w = t / WAVE, lane = t % WAVE;
  wk.q0 = 0;
  wk.stride = 1;
  wk.e = 0;
  wk.slot = -1;
  wk.ri = 0;
  wk.rc = 0.0;
  wk.rd = 1.0;
#pragma unroll
  for (int k = 0; k < SEG_PF; k++) {
    fs[k] = 0;
    fv[k] = 0.0;
    fy[k] = 0.0;
  }
  if (lev >= nlev) return;
  const int r0 = lev_ptr[lev], nr = lev_ptr[lev + 1] - r0;
  int j = -1;
  if (nr <= 16) {
    if (t < nr) wk.slot = r0 + t;
    const int ng = SEG_WAVES / nr;
    const int rr = w / ng, g = w % ng;
    if (rr < nr) {
      j = r0 + rr;
      wk.q0 = g * WAVE + lane;
      wk.stride = ng * WAVE;
    }
  } else {
    const int G = seg_group(nr);
    const int rr = t / G, gl = t % G;
    if (rr < nr) {
      j = r0 + rr;
      wk.q0 = gl;
      wk.stride = G;
      if (gl == 0) wk.slot = j;
    }
  }
  if (wk.slot >= 0) {
    wk.ri = row[wk.slot];
    wk.rc = c[wk.ri];
    if (MODE == 1 || MODE == 2) wk.rd = val[dpos[wk.slot]];
  }
  if (j < 0) return;
  wk.q0 += ptr[j];
  wk.e = ptr[j + 1];
#pragma unroll
  for (int k = 0; k < SEG_PF; k++) {
    const int q = wk.q0 + k * wk.stride;
    if (q < wk.e) {
      const int sq = src[q];
      fs[k] = sq;
      fv[k] = val[vpos[q]];
      if (sq >= 0) fy[k] = y[sq];
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(SEG_THREADS) void k_trisolve_seg(const int* __restrict__ gate, 
    int nlev, const int* __restrict__ lev_ptr, const int* __restrict__ row,
    const int* __restrict__ ptr, const int* __restrict__ src, const int* __restrict__ vpos,
    const int* __restrict__ dpos, const double* __restrict__ val, const double* __restrict__ c,
    double* __restrict__ y) {
  KKT_GATE(gate);
  __shared__ double ly[SEG_MAX_ROWS];
  __shared__ double part[SEG_WAVES];
  const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  int cs[SEG_PF];
  double cv[SEG_PF], cy[SEG_PF];
  SegWork cw;
  seg_fetch<MODE>(0, nlev, lev_ptr, row, ptr, src, vpos, dpos, val, c, y, cs, cv, cy, cw);
  for (int l = 0; l < nlev; l++) {
    int ns[SEG_PF];
    double nv[SEG_PF], ny[SEG_PF];
    SegWork nw;
    seg_fetch<MODE>(l + 1, nlev, lev_ptr, row, ptr, src, vpos, dpos, val, c, y, ns, nv, ny, nw);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < SEG_PF; k++) s += cv[k] * (cs[k] >= 0 ? cy[k] : ly[-cs[k] - 1]);
    for (int q = cw.q0 + SEG_PF * cw.stride; q < cw.e; q += cw.stride) {
      const int sq = src[q];
      s += val[vpos[q]] * (sq >= 0 ? y[sq] : ly[-sq - 1]);
    }
    const int nr = lev_ptr[l + 1] - lev_ptr[l];
    double tot;
    if (nr <= 16) {
      s = wave_sum(s);
      if (lane == 0) part[w] = s;
      __syncthreads();
      const int ng = SEG_WAVES / nr;
      tot = 0.0;
      if (cw.slot >= 0)
        for (int g = 0; g < ng; g++) tot += part[(int)threadIdx.x * ng + g];
    } else {
      const int G = seg_group(nr);
      for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
      tot = s;
    }
    if (cw.slot >= 0) {
      double yi = cw.rc - tot;
      if (MODE == 1 || MODE == 2) yi /= cw.rd;
      ly[cw.slot] = yi;
      y[cw.ri] = yi;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SEG_PF; k++) {
      cs[k] = ns[k];
      cv[k] = nv[k];
      cy[k] = ny[k];
    }
    cw = nw;
  }
}

// ---------------------------------------------------------------------------
// Dense trailing block.  The last rows of the pivot order couple to nearly
// every later pivot (the top separators of the elimination tree), so their
// block of the factors is dense and its row-by-row dependency chain is as
// long as the block.  It is finished as a dense right-looking LU in panels of
// DLU_NB pivots: one launch factors the panel (diagonal block, the column
// panel below it, the row panel right of it), one launch applies the panel's
// rank-DLU_NB update to the trailing matrix.  Every entry still receives
// fma(-l_ik, u_kj, a_ij) for k in ascending order, and an update whose l or u
// lies outside the sparse pattern is an exact zero update, so the values are
// those of the sparse refactorization bit for bit.  FP64 runs at the same
// peak rate on the vector ALUs as on the matrix cores of this chip, so the
// tile update uses vector FMAs, which keep that order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// wave per row r of T: zero the row (unit diagonal on padding rows), then the
// pattern entries of factor row c0 + r in columns >= c0
__global__ __launch_bounds__(256) void k_tail_scatter(int c0, int s, int S,
                                                      const int* __restrict__ rowptr,
                                                      const int* __restrict__ col,
                                                      const double* __restrict__ val, double* T) {
  const int lane = threadIdx.x % WAVE;
  const int r = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (r >= S) return;
  double* Tr = T + (size_t)r * S;
  for (int c = lane; c < S; c += WAVE) Tr[c] = (r >= s && c == r) ? 1.0 : 0.0;
  if (r >= s) return;
  stores_done();  // the zeros land before the values at the same addresses
  const int i = c0 + r;
  for (int q = rowptr[i] + lane; q < rowptr[i + 1]; q += WAVE) {
    const int j = col[q];
    if (j >= c0) Tr[j - c0] = val[q];
  }
}

__global__ __launch_bounds__(256) void k_tail_gather(int c0, int s, int S,
                                                     const int* __restrict__ rowptr,
                                                     const int* __restrict__ col,
                                                     const double* __restrict__ T, double* val) {
  const int lane = threadIdx.x % WAVE;
  const int r = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (r >= s) return;
  const double* Tr = T + (size_t)r * S;
  const int i = c0 + r;
  for (int q = rowptr[i] + lane; q < rowptr[i + 1]; q += WAVE) {
    const int j = col[q];
    if (j >= c0) val[q] = Tr[j - c0];
  }
}

// Panel k0 (m = S - k0 - NB rows and columns beyond the diagonal block),
// workgroup b of cdiv(m, NB), two waves:
//  * wave 0 holds the diagonal block's rows in lanes 0 .. NB-1 and the column
//    panel's rows k0 + NB + NB b + (lane - NB) in lanes NB .. 2NB-1, and runs
//    the right-looking elimination on all of them at once: pivot row k's
//    entries are broadcast with readlane, every lane below it divides by u_kk
//    and applies the row; the panel rows ride along at no extra cost.  The
//    multipliers of column k go to LDS (Lt[k][t]) as they are made.
//  * wave 1 solves NB columns of the row panel (thread per column) with those
//    multipliers, CH pivots behind wave 0 (a barrier every CH pivots).
// Every workgroup factors the diagonal block redundantly (no grid-wide
// wait); the diagonal block in T stays untouched (other workgroups may still
// be reading it): workgroup 0 leaves its factored form in dsc, which the
// following k_dlu_update copies into T.  The arithmetic per entry is the
// plain one (l = a / u_kk, a = fma(-l, u, a) in ascending k), so the factors
// are those of the sparse refactorization bit for bit.
template <int NB, int CH>
__global__ __launch_bounds__(128) void k_dlu_panel(double* T, int S, int k0, int m, double* dsc,
                                                   int s, DevStats* st, double prel) {
  static_assert(2 * NB == WAVE && NB % CH == 0, "rows of the panel fill one wave");
  __shared__ double Lt[NB][NB];      // Lt[k][t] = l_tk (t > k)
  __shared__ double Ur[NB][NB + 1];  // U rows of the diagonal block
  const int tid = threadIdx.x, lane = tid % WAVE, b = blockIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid / WAVE);
  if (w == 0) {
    const double thr = prel > 0.0 ? prel * __longlong_as_double((long long)st->anorm_f) : 0.0;
    const int q = NB * b + lane - NB;  // column-panel row, counted from k0 + NB
    const bool act = lane < NB || q < m;
    const size_t row = lane < NB ? (size_t)(k0 + lane) : (size_t)(k0 + NB + q);
    double r[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) r[j] = 0.0;
    if (act)
#pragma unroll
      for (int j = 0; j < NB; j++) r[j] = T[row * S + k0 + j];
#pragma unroll
    for (int k = 0; k < NB; k++) {
      // static pivoting of pivot k0 + k (real rows only) before its use
      if (lane == k && k0 + k < s && fabs(r[k]) < thr) {
        if (b == 0) st->perturbed = 1;
        r[k] = perturb_pivot(r[k], thr);
      }
      const double ukk = readlane_d(r[k], k);
      if (lane > k) {
        const double l = r[k] / ukk;
#pragma unroll
        for (int j = k + 1; j < NB; j++) r[j] = __builtin_fma(-l, readlane_d(r[j], k), r[j]);
        r[k] = l;
        if (lane < NB) Lt[k][lane] = l;
      }
      if (k % CH == CH - 1) __syncthreads();
    }
    if (lane < NB) {
#pragma unroll
      for (int j = 0; j < NB; j++)
        if (j >= lane) Ur[lane][j] = r[j];
    } else if (act) {
#pragma unroll
      for (int j = 0; j < NB; j++) T[row * S + k0 + j] = r[j];
    }
  } else {
    const int jc = NB * b + lane;  // row-panel column, counted from k0 + NB
    const bool act = lane < NB && jc < m;
    double c[NB];
#pragma unroll
    for (int t = 0; t < NB; t++) c[t] = 0.0;
    if (act)
#pragma unroll
      for (int t = 0; t < NB; t++) c[t] = T[(size_t)(k0 + t) * S + k0 + NB + jc];
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (k % CH == 0) __syncthreads();
#pragma unroll
      for (int t = k + 1; t < NB; t++) c[t] = __builtin_fma(-Lt[k][t], c[k], c[t]);
      // finish each stretch before the next barrier: left to itself the
      // compiler sinks these FMAs into the guarded stores below and holds
      // every multiplier loaded from LDS in registers until then
      if (k % CH == CH - 1)
#pragma unroll
        for (int t = 0; t < NB; t++) asm volatile("" : "+v"(c[t]));
    }
    if (act)
#pragma unroll
      for (int t = 0; t < NB; t++) T[(size_t)(k0 + t) * S + k0 + NB + jc] = c[t];
  }
  __syncthreads();
  if (b == 0)
    for (int e = tid; e < NB * NB; e += blockDim.x) {
      const int t = e / NB, j = e % NB;
      dsc[e] = j < t ? Lt[j][t] : Ur[t][j];
    }
}

// Trailing update of panel k0 on TS x TS tiles (TS / 16 x TS / 16 entries per
// thread, rows ty + 16 a, columns tx + 16 b): a_ij = fma(-l_ik, u_kj, a_ij)
// for the panel's k in ascending order.  Tile (0, 0) also installs the
// factored diagonal block of the panel from dsc.
template <int NB, int TS>
__global__ __launch_bounds__(256) void k_dlu_update(double* T, int S, int k0,
                                                    const double* __restrict__ dsc) {
  constexpr int RA = TS / 16;
  __shared__ double Ls[TS][NB + 1];
  __shared__ double Us[NB][TS];
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int e = tid; e < NB * NB; e += 256)
      T[(size_t)(k0 + e / NB) * S + k0 + e % NB] = dsc[e];
  const int base = k0 + NB;
  const int r0 = base + blockIdx.y * TS, q0 = base + blockIdx.x * TS;
  if (r0 >= S || q0 >= S) return;
  for (int e = tid; e < TS * NB; e += 256) {
    const int ii = e / NB, k = e % NB;
    Ls[ii][k] = r0 + ii < S ? T[(size_t)(r0 + ii) * S + k0 + k] : 0.0;
  }
  for (int e = tid; e < NB * TS; e += 256) {
    const int k = e / TS, jj = e % TS;
    Us[k][jj] = q0 + jj < S ? T[(size_t)(k0 + k) * S + q0 + jj] : 0.0;
  }
  __syncthreads();
  const int tx = tid % 16, ty = tid / 16;
  double acc[RA][RA];
#pragma unroll
  for (int a = 0; a < RA; a++)
#pragma unroll
    for (int c = 0; c < RA; c++) {
      const int r = r0 + ty + 16 * a, q = q0 + tx + 16 * c;
      acc[a][c] = (r < S && q < S) ? T[(size_t)r * S + q] : 0.0;
    }
#pragma unroll 4
  for (int k = 0; k < NB; k++) {
    double lv[RA], uv[RA];
#pragma unroll
    for (int a = 0; a < RA; a++) lv[a] = Ls[ty + 16 * a][k];
#pragma unroll
    for (int c = 0; c < RA; c++) uv[c] = Us[k][tx + 16 * c];
#pragma unroll
    for (int a = 0; a < RA; a++)
#pragma unroll
      for (int c = 0; c < RA; c++) acc[a][c] = __builtin_fma(-lv[a], uv[c], acc[a][c]);
  }
#pragma unroll
  for (int a = 0; a < RA; a++)
#pragma unroll
    for (int c = 0; c < RA; c++) {
      const int r = r0 + ty + 16 * a, q = q0 + tx + 16 * c;
      if (r < S && q < S) T[(size_t)r * S + q] = acc[a][c];
    }
}

// Dense trailing block as one dependency-driven launch.  The block is cut
// into NB x NB tiles; a task is one of
//   P(k, i)   the panel work of workgroup b = i - k - 1 of k_dlu_panel at
//             panel k: factor diagonal tile (k, k) (redundantly, as there),
//             finish column tile (i, k) in the same wave and row tile (k, i)
//             in a second wave; i = nt: the diagonal tile alone (last panel)
//   G(i,j,k)  tile (i, j) -= L(i, k) U(k, j)             (2 x 2 entries per thread)
// with exactly the arithmetic of k_dlu_panel / k_dlu_update, so the values
// are the same bit for bit.  ver[i * nt + j] counts the operations finished
// on tile (i, j): the G updates of steps 0 .. min(i, j) - 1, then its own P
// step.  A task waits for its inputs' counts (device-coherent flags; tile
// data moves with device-coherent loads and stores, so no cache maintenance
// is needed between XCDs) and hands out through eight ticket streams in an
// order where every task's inputs come earlier, which keeps the persistent
// grid deadlock-free as in the sparse refactorization.  Panel k + 1 is listed
// right after the updates of its own tiles, ahead of the rest of step k's
// update (look-ahead of one panel), so the diagonal chain does not wait for
// the bulk of the trailing matrix.  The factored diagonal tiles go to Dk
// (P(k, k + 1) writes tile k's); k_dlu_install copies them into T after the
// launch, as no task reads a diagonal tile after its own panel.
// Task code: type << 21 | i << 14 | j << 7 | k (type 0 P, 1 G).
template <int NB>
struct DluPanelLds {
  struct {
    double Lt[NB][NB];      // Lt[k][t] = l_tk (t > k)
    double Ur[NB][NB + 1];  // U rows of the diagonal tile
  } fac;
};

template <int NB, int CH>
__device__ __forceinline__ void dlu_panel_task(double* T, int S, int k0, int q0, double* D,
                                               int s, DevStats* st, double thr, bool owner,
                                               DluPanelLds<NB>& sh) {
  const int tid = threadIdx.x, lane = tid % WAVE;
  const int w = __builtin_amdgcn_readfirstlane(tid / WAVE);
  if (w == 0) {
    // lanes 0 .. NB-1: rows of the diagonal tile; NB .. 2NB-1: column tile
    const bool act = lane < NB || q0 >= 0;
    const size_t row = lane < NB ? (size_t)(k0 + lane) : (size_t)(q0 + lane - NB);
    double r[NB];
#pragma unroll
    for (int j = 0; j < NB; j++) r[j] = 0.0;
    if (act)
#pragma unroll
      for (int j = 0; j < NB; j++) r[j] = ld_coh(T + row * S + k0 + j);
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (lane == k && k0 + k < s && fabs(r[k]) < thr) {
        if (owner) st->perturbed = 1;
        r[k] = perturb_pivot(r[k], thr);
      }
      const double ukk = readlane_d(r[k], k);
      if (lane > k) {
        const double l = r[k] / ukk;
#pragma unroll
        for (int j = k + 1; j < NB; j++) r[j] = __builtin_fma(-l, readlane_d(r[j], k), r[j]);
        r[k] = l;
        if (lane < NB) sh.fac.Lt[k][lane] = l;
      }
      if (k % CH == CH - 1) __syncthreads();
    }
    if (lane < NB) {
#pragma unroll
      for (int j = 0; j < NB; j++)
        if (j >= lane) sh.fac.Ur[lane][j] = r[j];
    } else if (act) {
#pragma unroll
      for (int j = 0; j < NB; j++) st_coh(T + row * S + k0 + j, r[j]);
    }
  } else if (w == 1) {
    // row tile, thread per column
    const bool act = lane < NB && q0 >= 0;
    double c[NB];
#pragma unroll
    for (int t = 0; t < NB; t++) c[t] = 0.0;
    if (act)
#pragma unroll
      for (int t = 0; t < NB; t++) c[t] = ld_coh(T + (size_t)(k0 + t) * S + q0 + lane);
#pragma unroll
    for (int k = 0; k < NB; k++) {
      if (k % CH == 0) __syncthreads();
#pragma unroll
      for (int t = k + 1; t < NB; t++) c[t] = __builtin_fma(-sh.fac.Lt[k][t], c[k], c[t]);
      if (k % CH == CH - 1)
#pragma unroll
        for (int t = 0; t < NB; t++) asm volatile("" : "+v"(c[t]));
    }
    if (act)
#pragma unroll
      for (int t = 0; t < NB; t++) st_coh(T + (size_t)(k0 + t) * S + q0 + lane, c[t]);
  } else {
    for (int k = 0; k < NB; k += CH) __syncthreads();
  }
  __syncthreads();
  if (owner)
    for (int e = tid; e < NB * NB; e += blockDim.x) {
      const int t = e / NB, j = e % NB;
      D[e] = j < t ? sh.fac.Lt[j][t] : sh.fac.Ur[t][j];
    }
}

template <int NB, int CH>
__global__ __launch_bounds__(256) void k_dlu_tasks(double* T, int S, int s, int nt,
                                                   const int* __restrict__ tasks, int ntasks,
                                                   int* ver, double* Dk, SyncState* ss,
                                                   int nstreams, int* stall, DevStats* st,
                                                   double prel) {
  __shared__ union {
    DluPanelLds<NB> p;
    struct {
      double A[NB][NB + 1];
      double Bt[NB][NB];
    } g;
  } sh;
  __shared__ int task_s, ok_s;
  const int tid = threadIdx.x, lane = tid % WAVE;
  const double thr = prel > 0.0 ? prel * __longlong_as_double((long long)st->anorm_f) : 0.0;
  for (;;) {
    if (tid < WAVE) {
      const int c = next_chunk(ss->dlu_stream, nstreams, lane);
      if (lane == 0) task_s = c < ntasks ? tasks[c] : -1;
    }
    __syncthreads();
    const int code = task_s;
    if (code < 0) break;
    const int type = code >> 21, i = (code >> 14) & 127, j = (code >> 7) & 127, k = code & 127;
    // inputs: (tile index, count it must reach)
    if (tid == 0) {
      int dep[3], want[3], nd = 0;
      if (type == 0) {
        dep[nd] = k * nt + k, want[nd++] = k;
        if (i < nt) {
          dep[nd] = i * nt + k, want[nd++] = k;
          dep[nd] = k * nt + i, want[nd++] = k;
        }
      } else {
        dep[nd] = i * nt + j, want[nd++] = k;
        dep[nd] = i * nt + k, want[nd++] = k + 1;
        dep[nd] = k * nt + j, want[nd++] = k + 1;
      }
      int spins = 0, ok = 1;
      for (int d = 0; d < nd && ok; d++)
        while (ld_flag(ver + dep[d]) < want[d])
          if (!keep_waiting(&spins, stall)) {
            ok = 0;
            break;
          }
      ok_s = ok;
    }
    __syncthreads();
    if (!ok_s) break;
    if (type == 0) {
      dlu_panel_task<NB, CH>(T, S, k * NB, i < nt ? i * NB : -1, Dk + (size_t)k * NB * NB, s, st,
                             thr, i == k + 1, sh.p);
      stores_done();
      __syncthreads();  // every store of the task complete
      if (tid == 0 && i < nt) {
        st_flag(ver + i * nt + k, k + 1);
        st_flag(ver + k * nt + i, k + 1);
      }
    } else {
      // A := L(i, k), Bt := U(k, j); 2 x 2 entries per thread: rows ty + 16 a,
      // columns tx + 16 c
      const int k0 = k * NB, r0 = i * NB, q0 = j * NB;
      for (int e = tid; e < NB * NB; e += blockDim.x) {
        sh.g.A[e / NB][e % NB] = ld_coh(T + (size_t)(r0 + e / NB) * S + k0 + e % NB);
        sh.g.Bt[e / NB][e % NB] = ld_coh(T + (size_t)(k0 + e / NB) * S + q0 + e % NB);
      }
      __syncthreads();
      const int tx = tid % 16, ty = tid / 16;
      double acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 2; c++)
          acc[a][c] = ld_coh(T + (size_t)(r0 + ty + 16 * a) * S + q0 + tx + 16 * c);
#pragma unroll 4
      for (int kk = 0; kk < NB; kk++) {
        double lv[2], uv[2];
#pragma unroll
        for (int a = 0; a < 2; a++) lv[a] = sh.g.A[ty + 16 * a][kk];
#pragma unroll
        for (int c = 0; c < 2; c++) uv[c] = sh.g.Bt[kk][tx + 16 * c];
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
          for (int c = 0; c < 2; c++) acc[a][c] = __builtin_fma(-lv[a], uv[c], acc[a][c]);
      }
#pragma unroll
      for (int a = 0; a < 2; a++)
#pragma unroll
        for (int c = 0; c < 2; c++)
          st_coh(T + (size_t)(r0 + ty + 16 * a) * S + q0 + tx + 16 * c, acc[a][c]);
      stores_done();
      __syncthreads();  // every store of the task complete
      if (tid == 0) st_flag(ver + i * nt + j, k + 1);
    }
  }
}

// The factored diagonal tiles (Dk, tile k at Dk + k NB^2) into T.
template <int NB>
__global__ __launch_bounds__(256) void k_dlu_install(double* T, int S, const double* __restrict__ Dk) {
  const int k = blockIdx.x;
  const double* D = Dk + (size_t)k * NB * NB;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x)
    T[(size_t)(k * NB + e / NB) * S + k * NB + e % NB] = D[e];
}

__global__ void k_dlu_reset(int* ver, int count, SyncState* ss) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x)
    ver[e] = 0;
  if (blockIdx.x == 0 && threadIdx.x < TICKET_STREAMS)
    ss->dlu_stream[threadIdx.x * TICKET_STRIDE] = 0u;
}

// ---------------------------------------------------------------------------
// Chain-blocked triangular solve (value-as-flag publication).  Consecutive
// rows of the solve order in which each row depends on the one before form a
// chain block of up to SN_KMAX rows, solved by one wave: the external terms
// of all rows first (their inputs come from earlier blocks, waited for as in
// k_trisolve_vflag), then the block's own triangle in registers and LDS, so a
// chain of k rows costs one cross-CU hop instead of k.  Rows without a chain
// are grouped per level as in k_trisolve_vflag.  Entries of a slot's row:
//   MODE 0  L row i:    external [rowptr_i, split), internal [split, diag_i)
//   MODE 1  U row i:    internal (diag_i, split), external [split, rowptr_i+1)
//   MODE 2  U^T col i:  external [tptr_i, split), internal [split, tptr_i+1 - 1)
//   MODE 3  L^T col i:  internal [tptr_i, split), external [split, tptr_i+1)
// Internal entry with dependency row j sits in triangle column
// j - base (modes 0, 2) or base - j (modes 1, 3).
// ---------------------------------------------------------------------------
// NR >= nr right-hand sides (column r at c + r * ld, y + r * ld; ld = n + 1
// for several, unused for one): every lane keeps nr sums.  Instances of a
// shared-pattern batch (in.count > 1, one right-hand side each): ticket =
// chunk x instances + instance; instance t's factor values start at t in.f1,
// its c and y at t (n + 1).
template <int MODE, int NR, bool SH>
__global__ __launch_bounds__(256) void k_trisolve_sn(const int* __restrict__ gate, 
    int n, int nr, int ld, int nchunks, const int* __restrict__ ch_start,
    const int* __restrict__ ch_meta, const int* __restrict__ ch_base, const int* __restrict__ rows,
    const int* __restrict__ split, const int* __restrict__ rowptr, const int* __restrict__ col,
    const int* __restrict__ diag, const int* __restrict__ tptr, const int* __restrict__ trow,
    const int* __restrict__ tpos, const double* __restrict__ val0, const double* __restrict__ c0,
    double* y0, SyncState* ss, int slot, int nstreams, int* stall, const int* __restrict__ xend,
    const double* __restrict__ pre, Inst in) {
  KKT_GATE(gate);
  if constexpr (!SH) in = Inst();  // one instance: the decode below folds away
  // the block's strictly lower triangle, packed by rows: entry (g, h), h < g,
  // at g (g - 1) / 2 + h (half the LDS of a square, so all eight workgroups
  // per CU fit)
  constexpr int TRI = SN_KMAX * (SN_KMAX - 1) / 2;
  __shared__ double tri_all[256 / WAVE][TRI];
  const int lane = threadIdx.x % WAVE;
  double* tri = tri_all[threadIdx.x / WAVE];
  for (;;) {
    const int tk0 = next_chunk(ss->slot_stream[slot], nstreams, lane);
    if (tk0 >= nchunks * in.count) break;
    const int tk = tk0 / in.count, inst = tk0 - tk * in.count;
    const double* val = val0 + (size_t)inst * in.f1;
    const double* c = c0 + (size_t)inst * (n + 1);
    double* y = y0 + (size_t)inst * (n + 1);
    const int meta = ch_meta[tk];
    const int k = meta & 0xff, lg = (meta >> 8) & 0xf;
    const bool chain = (meta >> 16) != 0;
    const int G = 1 << lg;
    const int grp = lane >> lg, gl = lane & (G - 1);
    const bool active = grp < k;
    const int s0 = ch_start[tk];
    const int i = active ? rows[s0 + grp] : n;
    const int sp = active ? split[s0 + grp] : 0;
    int eb = 0, ee = 0, ib = 0, ie = 0, dpos = 0;
    if (active) {
      if (MODE == 0) {
        eb = rowptr[i];
        ee = sp;
        ib = sp;
        ie = diag[i];
      } else if (MODE == 1) {
        dpos = diag[i];
        ib = dpos + 1;
        ie = sp;
        eb = sp;
        // xend: the entries in the dense block's columns were summed into
        // pre[i] by a bulk pass (their inputs are final before this launch)
        ee = xend ? xend[i] : rowptr[i + 1];
      } else if (MODE == 2) {
        eb = tptr[i];
        ee = sp;
        ib = sp;
        ie = tptr[i + 1] - 1;
        dpos = tpos[ie];
      } else {
        ib = tptr[i];
        ie = sp;
        eb = sp;
        ee = tptr[i + 1];
      }
    }
    double ci[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) ci[r] = r < nr ? c[(size_t)r * ld + i] : 0.0;
    const double dv = (MODE == 1 || MODE == 2) && active ? val[dpos] : 1.0;
    // inverted once, off the critical path: the chain block's row-by-row
    // steps below multiply instead of dividing (one more rounding per entry
    // of y, far inside the solve's accuracy)
    const double dvi = 1.0 / dv;
    if (chain) {
      // the block's own triangle into LDS (issued before the waits below)
      const int b = ch_base[tk];
      for (int e = lane; e < k * (k - 1) / 2; e += WAVE) tri[e] = 0.0;
      wave_sync();
      for (int q = ib + gl; q < ie; q += G) {
        const int j = MODE <= 1 ? col[q] : trow[q];
        const double v = MODE <= 1 ? val[q] : val[tpos[q]];
        const int sg = (MODE == 0 || MODE == 2) ? j - b : b - j;
        if (sg >= 0 && sg < grp) tri[grp * (grp - 1) / 2 + sg] = v;
      }
    }
    int spins = 0;
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) s[r] = 0.0;
    constexpr int VB = NR == 1 ? 8 : (NR <= 4 ? 2 : 1);
    // batches of VB entries per lane; the next batch's column indices and
    // values load while this batch's y values are polled (one memory round
    // trip per batch on the path after a late input, not two)
    int kn[VB];
    double vn[VB];
    auto load_batch = [&](int q0) {
#pragma unroll
      for (int u = 0; u < VB; u++) {
        const int q = q0 + u * G;
        kn[u] = n;
        vn[u] = 0.0;
        if (q < ee) {
          kn[u] = MODE <= 1 ? col[q] : trow[q];
          vn[u] = MODE <= 1 ? val[q] : val[tpos[q]];
        }
      }
    };
    load_batch(eb + gl);
    for (int q0 = eb + gl; q0 < ee; q0 += VB * G) {
      int kk[VB];
      double v[VB], yk[VB][NR];
#pragma unroll
      for (int u = 0; u < VB; u++) {
        kk[u] = kn[u];
        v[u] = vn[u];
      }
#pragma unroll
      for (int u = 0; u < VB; u++)
#pragma unroll
        for (int r = 0; r < NR; r++)
          yk[u][r] = (q0 + u * G < ee && r < nr) ? ld_coh(y + (size_t)r * ld + kk[u]) : 0.0;
      if (q0 + VB * G < ee) load_batch(q0 + VB * G);
#pragma unroll
      for (int u = 0; u < VB; u++)
#pragma unroll
        for (int r = 0; r < NR; r++) {
          while (is_sentinel(yk[u][r]) && keep_waiting(&spins, stall))
            yk[u][r] = ld_coh(y + (size_t)r * ld + kk[u]);
          if (q0 + u * G < ee) s[r] += v[u] * yk[u][r];
        }
    }
#pragma unroll
    for (int r = 0; r < NR; r++)
      for (int off = G >> 1; off > 0; off >>= 1) s[r] += __shfl_xor(s[r], off, WAVE);
    if (MODE == 1 && NR == 1 && pre && active) s[0] += pre[i];
    if (chain) {
      wave_sync();
      // row sg is final at step sg: its values go to every lane, the later
      // rows take their terms with them
      for (int sg = 0; sg < k; sg++) {
        const double tv = (grp > sg && active) ? tri[grp * (grp - 1) / 2 + sg] : 0.0;
#pragma unroll
        for (int r = 0; r < NR; r++) {
          double yv = ci[r] - s[r];
          if (MODE == 1 || MODE == 2) yv *= dvi;
          const double ys = readlane_d(yv, sg << lg);
          s[r] += tv * ys;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
      double yv = ci[r] - s[r];
      if (MODE == 1 || MODE == 2) yv *= dvi;
      if (r < nr) st_coh(y + (size_t)r * ld + i, yv);
    }
  }
}

// U solve, rows before the dense trailing block: pre[i] = sum of the row's
// entries in the block's columns (positions xend[i] .. rowptr[i + 1]) times
// the solution values there, final once the block is solved.  8 lanes per
// row, rows listed in urows.
__global__ __launch_bounds__(256) void k_udense_pre(const int* __restrict__ gate, int nu, const int* __restrict__ urows,
                                                    const int* __restrict__ xend,
                                                    const int* __restrict__ rowptr,
                                                    const int* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ y,
                                                    double* __restrict__ pre) {
  KKT_GATE(gate);
  constexpr int RL = 8;
  const int lane = threadIdx.x % WAVE, g = lane / RL, gl = lane % RL;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  for (int r0 = wid * (WAVE / RL); r0 < nu; r0 += nw * (WAVE / RL)) {
    const int t = r0 + g;
    double acc = 0.0;
    int i = 0;
    if (t < nu) {
      i = urows[t];
      const int e = rowptr[i + 1];
      // four gathers of each lane in flight (rows just before the block
      // have hundreds of such entries)
      for (int q0 = xend[i] + gl; q0 < e; q0 += 4 * RL) {
        double v[4], yv[4];
#pragma unroll
        for (int z = 0; z < 4; z++) {
          const int q = q0 + z * RL;
          v[z] = 0.0;
          yv[z] = 0.0;
          if (q < e) {
            v[z] = val[q];
            yv[z] = y[col[q]];
          }
        }
#pragma unroll
        for (int z = 0; z < 4; z++) acc += v[z] * yv[z];
      }
    }
    for (int off = RL >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, WAVE);
    if (t < nu && gl == 0) pre[i] = acc;
  }
}

// External terms of the dense trailing block's rows (modes 0 and 2; their
// inputs are final): rhs[t] = c[c0 + t] - sum over the entries before split[t]
// of row (MODE 0) / column (MODE 2) c0 + t; rhs[t] = 0 on padding rows.
template <int MODE>
__global__ __launch_bounds__(256) void k_tail_ext(const int* __restrict__ gate, int c0, int s, int S, int nr, int ld,
                                                  const int* __restrict__ split,
                                                  const int* __restrict__ rowptr,
                                                  const int* __restrict__ col,
                                                  const int* __restrict__ tptr,
                                                  const int* __restrict__ trow,
                                                  const int* __restrict__ tpos,
                                                  const double* __restrict__ val,
                                                  const double* __restrict__ c,
                                                  const double* __restrict__ y, double* rhs) {
  KKT_GATE(gate);
  const int lane = threadIdx.x % WAVE;
  const int t = blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  const int r = blockIdx.y;
  if (t >= S || r >= nr) return;
  if (t >= s) {
    if (lane == 0) rhs[(size_t)r * S + t] = 0.0;
    return;
  }
  const int i = c0 + t;
  const double* yr = y + (size_t)r * ld;
  const int b = MODE == 0 ? rowptr[i] : tptr[i];
  double acc = 0.0;
  for (int q = b + lane; q < split[t]; q += WAVE)
    acc += MODE == 0 ? val[q] * yr[col[q]] : val[tpos[q]] * yr[trow[q]];
  acc = wave_sum(acc);
  if (lane == 0) rhs[(size_t)r * S + t] = c[(size_t)r * ld + i] - acc;
}

// Dense triangular solve on the trailing block by one workgroup, blocks of
// TB = 32 rows: for each block, wave r (r < nr) solves column r's diagonal
// triangle with the block's matrix rows in registers (broadcast by readlane),
// then every thread takes the block's terms out of one remaining row for all
// columns.  x (nr columns of S) lives in LDS.
//   MODE 0: L (unit lower), forward      MODE 1: U (upper), backward
//   MODE 2: U^T (lower), forward         MODE 3: L^T (unit upper), backward
// M[r][q] is T[r][q] (modes 0, 1) or T[q][r] (modes 2, 3).  rhs: column r at
// rhs + r * rld; y: column r at y + r * ld.
constexpr int TB = 32;
constexpr int TAIL_NR = 8;  // columns per dense-block solve launch
template <int MODE, int NRT>
__global__ __launch_bounds__(1024) void k_tail_trsv(const int* __restrict__ gate, const double* __restrict__ T, int S, int s,
                                                    int c0, int nr, const double* __restrict__ rhs,
                                                    int rld, double* y, int ld) {
  KKT_GATE(gate);
  extern __shared__ double xs[];
  constexpr bool fwd = MODE == 0 || MODE == 2;
  constexpr bool trans = MODE == 2 || MODE == 3;
  auto M = [&](int r, int q) -> double {
    return trans ? T[(size_t)q * S + r] : T[(size_t)r * S + q];
  };
  for (int cr = 0; cr < nr; cr++)
    for (int t = threadIdx.x; t < S; t += blockDim.x)
      xs[(size_t)cr * S + t] = t < s ? rhs[(size_t)cr * rld + t] : 0.0;
  __syncthreads();
  const int nb = S / TB;
  const int wv = threadIdx.x / WAVE;
  __shared__ double ms[TB][TB + 1];  // the block's diagonal triangle
  for (int bb = 0; bb < nb; bb++) {
    const int b0 = (fwd ? bb : nb - 1 - bb) * TB;
    // remaining rows: after the block (forward) or before it (backward)
    const int lo = fwd ? b0 + TB : 0, hi = fwd ? S : b0;
    // nothing here depends on x: one diagonal-block value per thread first,
    // then all TB matrix values of this thread's first remaining row, so the
    // latter are still in flight while the block is solved
    // (unconditional loads at clamped addresses, so that the compiler can
    // count them and wait for the diagonal value alone)
    const int dr = (threadIdx.x / TB) % TB, dq = threadIdx.x % TB;
    const double dv = M(b0 + dr, b0 + dq);
    const int row0 = lo + threadIdx.x;
    const int rowc = row0 < S ? row0 : S - 1;
    double mv[TB];
#pragma unroll
    for (int q = 0; q < TB; q++) mv[q] = M(rowc, b0 + q);
    if (threadIdx.x < TB * TB) ms[dr][dq] = dv;
    __syncthreads();
    if (wv < nr) {
      double* x = xs + (size_t)wv * S;
      const int r = threadIdx.x % WAVE;
      const int rr = r % TB;
      double xr = r < TB ? x[b0 + r] : 0.0;
#pragma unroll
      for (int st = 0; st < TB; st++) {
        const int q = fwd ? st : TB - 1 - st;
        const double mq = ms[rr][q];
        if (MODE == 1 || MODE == 2) xr = r == q ? xr / mq : xr;
        const double xq = readlane_d(xr, q);
        const bool later = fwd ? r > q : r < q;
        const double nx = __builtin_fma(-mq, xq, xr);
        xr = later ? nx : xr;
      }
      if (r < TB) x[b0 + r] = xr;
    }
    __syncthreads();
    for (int row = row0; row < hi; row += blockDim.x) {
      // NRT == 1: the single column needs no guard (nr == 1)
      double acc[NRT];
#pragma unroll
      for (int cr = 0; cr < NRT; cr++)
        acc[cr] = (NRT == 1 || cr < nr) ? xs[(size_t)cr * S + row] : 0.0;
      if (row != row0) {
#pragma unroll
        for (int q = 0; q < TB; q++) mv[q] = M(row, b0 + q);
      }
#pragma unroll
      for (int q = 0; q < TB; q++) {
#pragma unroll
        for (int cr = 0; cr < NRT; cr++)
          if (NRT == 1 || cr < nr)
            acc[cr] = __builtin_fma(-mv[q], xs[(size_t)cr * S + b0 + q], acc[cr]);
      }
#pragma unroll
      for (int cr = 0; cr < NRT; cr++)
        if (NRT == 1 || cr < nr) xs[(size_t)cr * S + row] = acc[cr];
    }
    __syncthreads();
  }
  for (int cr = 0; cr < nr; cr++)
    for (int t = threadIdx.x; t < s; t += blockDim.x)
      y[(size_t)cr * ld + c0 + t] = xs[(size_t)cr * S + t];
}

// Dense triangular solve on the trailing block, one right-hand side, by
// S / TB workgroups: workgroup g takes block row b (b = g forward, nb-1-g
// backward) of TB rows.  Its threads (row r = tid / 8, column lane tid % 8)
// accumulate the terms of every block the rows depend on as soon as that
// block's solution values appear in y (they hold the sentinel until then),
// with the matrix values of the next block already in flight; then wave 0
// solves the block's diagonal triangle (rows in lanes, readlane broadcasts)
// and publishes its values with device-coherent stores.  Modes and M as in
// k_tail_trsv; rhs[t] (t < s) is the right-hand side of block row t, y + c0
// the output (rows t >= s are the identity padding, x = 0, not stored).
template <int MODE>
__global__ __launch_bounds__(256) void k_tail_mw(const int* __restrict__ gate, const double* __restrict__ T, int S, int s,
                                                 int c0, const double* __restrict__ rhs,
                                                 double* y, int* stall) {
  KKT_GATE(gate);
  constexpr bool fwd = MODE == 0 || MODE == 2;
  constexpr bool trans = MODE == 2 || MODE == 3;
  auto M = [&](int r, int q) -> double {
    return trans ? T[(size_t)q * S + r] : T[(size_t)r * S + q];
  };
  const int nb = S / TB;
  const int g = blockIdx.x;
  const int b = fwd ? g : nb - 1 - g;
  const int tid = threadIdx.x, r = tid >> 3, cl = tid & 7;
  const int row = b * TB + r;
  __shared__ double sacc[TB];
  int spins = 0;
  double* yb = y + c0;
  double acc = 0.0;
  // wave 0 finishes the block: its rows of the diagonal block and its
  // right-hand side are loaded now (inputs of earlier launches), off the
  // critical path that runs through the dependency polls below
  const int lr = tid, rr = lr % TB, rw = b * TB + rr;
  double md[TB], rh = 0.0, dinv = 1.0;
  if (tid < WAVE) {
#pragma unroll
    for (int q = 0; q < TB; q++) md[q] = M(rw, b * TB + q);
    rh = (lr < TB && rw < s) ? rhs[rw] : 0.0;
    if (MODE == 1 || MODE == 2) {
      // the row's own diagonal entry, inverted once here: the triangle's
      // chain below then multiplies instead of dividing (one more rounding
      // per entry of x, far inside the solve's accuracy)
      double d = 1.0;
#pragma unroll
      for (int q = 0; q < TB; q++) d = rr == q ? md[q] : d;
      dinv = 1.0 / d;
    }
  }
  // dependency blocks in solve order: 0 .. b-1 (forward), nb-1 .. b+1 (backward)
  const int ndep = fwd ? b : nb - 1 - b;
  double m[4], mn[4];
  auto load_m = [&](double* dst, int j) {
    const int bd = fwd ? j : nb - 1 - j;
#pragma unroll
    for (int u = 0; u < 4; u++) dst[u] = M(row, bd * TB + cl * 4 + u);
  };
  if (ndep > 0) load_m(m, 0);
  for (int j = 0; j < ndep; j++) {
    if (j + 1 < ndep) load_m(mn, j + 1);
    const int bd = fwd ? j : nb - 1 - j;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int t = bd * TB + cl * 4 + u;
      double xv = 0.0;
      if (t < s) {
        xv = ld_coh(yb + t);
        while (is_sentinel(xv) && keep_waiting(&spins, stall)) xv = ld_coh(yb + t);
      }
      acc = __builtin_fma(m[u], xv, acc);
    }
#pragma unroll
    for (int u = 0; u < 4; u++) m[u] = mn[u];
  }
  // the 8 column lanes of a row are consecutive lanes of one wave
  for (int off = 4; off > 0; off >>= 1) acc += __shfl_xor(acc, off, WAVE);
  if (cl == 0) sacc[r] = acc;
  __syncthreads();
  if (tid < WAVE) {
    double xr = (lr < TB && rw < s) ? rh - sacc[rr] : 0.0;
#pragma unroll
    for (int st = 0; st < TB; st++) {
      const int q = fwd ? st : TB - 1 - st;
      if (MODE == 1 || MODE == 2) xr = lr == q ? xr * dinv : xr;
      const double xq = readlane_d(xr, q);
      const bool later = fwd ? lr > q : lr < q;
      const double nx = __builtin_fma(-md[q], xq, xr);
      xr = later ? nx : xr;
    }
    if (lr < TB && rw < s) st_coh(yb + rw, xr);
  }
}

// Several right-hand sides in one launch (nr <= NR, column-major with leading
// dimension ld = n + 1): each entry's NR dependency loads are in flight
// together; the dependency depth is paid once for all columns.
template <int MODE, int NR>
__global__ __launch_bounds__(256) void k_trisolve_vflag_mr(const int* __restrict__ gate, 
    int n, int nr, int ld, int nchunks, const int* __restrict__ ch_start,
    const int* __restrict__ ch_meta, const int* __restrict__ rows, const int* __restrict__ rowptr,
    const int* __restrict__ col, const int* __restrict__ diag, const int* __restrict__ tptr,
    const int* __restrict__ trow, const int* __restrict__ tpos, const double* __restrict__ val,
    const double* __restrict__ c, double* y, SyncState* ss, int slot, int* stall) {
  KKT_GATE(gate);
  const int lane = threadIdx.x % WAVE;
  unsigned int* ticket = &ss->ticket[slot];
  for (;;) {
    const unsigned int tk = bcast0(atomicAdd(ticket, lane == 0 ? 1u : 0u));
    if (tk >= (unsigned int)nchunks) break;
    const int meta = ch_meta[tk];
    const int lg = meta >> 8, cnt = meta & 0xff;
    const int G = 1 << lg;
    const int grp = lane >> lg, gl = lane & (G - 1);
    const bool active = grp < cnt;
    const int i = active ? rows[ch_start[tk] + grp] : n;
    int b = 0, e = 0, dpos = 0;
    if (active) {
      if (MODE == 0) {
        b = rowptr[i];
        e = diag[i];
      } else if (MODE == 1) {
        dpos = diag[i];
        b = dpos + 1;
        e = rowptr[i + 1];
      } else if (MODE == 2) {
        b = tptr[i];
        e = tptr[i + 1] - 1;
        dpos = tpos[e];
      } else {
        b = tptr[i];
        e = tptr[i + 1];
      }
    }
    int spins = 0;
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) acc[r] = 0.0;
    for (int q = b + gl; q < e; q += G) {
      const int k = MODE <= 1 ? col[q] : trow[q];
      const double v = MODE <= 1 ? val[q] : val[tpos[q]];
      double yk[NR];
#pragma unroll
      for (int r = 0; r < NR; r++) yk[r] = r < nr ? ld_coh(y + (size_t)r * ld + k) : 0.0;
#pragma unroll
      for (int r = 0; r < NR; r++) {
        while (is_sentinel(yk[r]) && keep_waiting(&spins, stall))
          yk[r] = ld_coh(y + (size_t)r * ld + k);
        acc[r] += v * yk[r];
      }
    }
#pragma unroll
    for (int r = 0; r < NR; r++) {
      double s = acc[r];
      for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
      if (r < nr) {
        const double ci = c[(size_t)r * ld + i];
        st_coh(y + (size_t)r * ld + i,
               (MODE == 0 || MODE == 3) ? ci - s : (ci - s) / val[dpos]);
      }
    }
  }
}

// multi-column gather: c[r][i] = x[r][perm[i]] (x: ld n, c/y/z: ld n + 1),
// y and z set to the sentinel; plus the sync_prep of mask
__global__ void k_gather_sentinel_mr(const int* __restrict__ gate, int n, int nr, const int* __restrict__ perm,
                                     const double* __restrict__ scale, const double* __restrict__ x, double* __restrict__ c,
                                     double* __restrict__ y, double* __restrict__ z,
                                     SyncState* ss, int mask,
                                     const unsigned char* __restrict__ triv,
                                     const int* __restrict__ diag,
                                     const double* __restrict__ val, int div);

// c[i] = x[perm[i]], and the two solve outputs y, z set to the sentinel
// Rows without dependencies in the first triangle (triv[i] != 0) get their
// final value here: y = c, or y = c / u_ii when div is set (a U^T first).
__global__ void k_gather_sentinel(const int* __restrict__ gate, int n, const int* __restrict__ perm,
                                  const double* __restrict__ scale, const double* __restrict__ x, double* __restrict__ c,
                                  double* __restrict__ y, double* __restrict__ z, SyncState* ss,
                                  int mask, const unsigned char* __restrict__ triv,
                                  const int* __restrict__ diag, const double* __restrict__ val,
                                  int div) {
  KKT_GATE(gate);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double ci = canon_nan(scale ? x[perm[i]] * scale[i] : x[perm[i]]);
    c[i] = ci;
    const double sent = __longlong_as_double((long long)SENTINEL);
    y[i] = (triv && triv[i]) ? (div ? ci / val[diag[i]] : ci) : sent;
    z[i] = sent;
  }
  if (ss && i == 0) sync_prep(ss, mask);
}

__global__ void k_gather_sentinel_mr(const int* __restrict__ gate, int n, int nr, const int* __restrict__ perm,
                                     const double* __restrict__ scale, const double* __restrict__ x, double* __restrict__ c,
                                     double* __restrict__ y, double* __restrict__ z,
                                     SyncState* ss, int mask,
                                     const unsigned char* __restrict__ triv,
                                     const int* __restrict__ diag,
                                     const double* __restrict__ val, int div, long long f1) {
  KKT_GATE(gate);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i < n && r < nr) {
    const size_t o = (size_t)r * (n + 1) + i;
    const double xi = x[(size_t)r * n + perm[i]];
    const double ci = canon_nan(scale ? xi * scale[i] : xi);
    c[o] = ci;
    const double sent = __longlong_as_double((long long)SENTINEL);
    // column r's factors at r f1 (the instances of a shared-pattern batch;
    // f1 = 0 for right-hand sides of one system)
    y[o] = (triv && triv[i]) ? (div ? ci / val[r * f1 + diag[i]] : ci) : sent;
    z[o] = sent;
  }
  if (ss && i == 0 && r == 0) sync_prep(ss, mask);
}

// x[r][perm[i]] = z[r][i] (z: ld n + 1, x: ld n)
__global__ void k_scatter_mr(const int* __restrict__ gate, int n, int nr, const int* __restrict__ perm,
                             const double* __restrict__ scale, const double* __restrict__ z,
                             double* __restrict__ x) {
  KKT_GATE(gate);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i < n && r < nr) {
    const double zi = z[(size_t)r * (n + 1) + i];
    x[(size_t)r * n + perm[i]] = scale ? zi * scale[i] : zi;
  }
}

__global__ void k_gather_prep(const int* __restrict__ gate, int n, const int* __restrict__ perm,
                              const double* __restrict__ scale, const double* __restrict__ x,
                              double* __restrict__ y, SyncState* ss, int mask) {
  KKT_GATE(gate);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = canon_nan(scale ? x[perm[i]] * scale[i] : x[perm[i]]);
  if (ss && i == 0) sync_prep(ss, mask);
}

__global__ void k_reset_stats(DevStats* st, int what) {
  if (threadIdx.x == 0) {
    if (what & 1) {
      st->min_piv = dbits(__builtin_huge_val());
      st->max_piv = 0ull;
      st->anorm = 0ull;
      st->anorm1 = 0ull;
      st->umax = 0ull;
      st->anorm_f = 0ull;
      st->tiny = 0;
      st->perturbed = 0;
      st->nonfinite_in = 0;
    }
    if (what & 2) {
      st->rmax = 0ull;
      st->xmax = 0ull;
    }
    if (what & 4) {
      st->anorm = 0ull;
      st->anorm1 = 0ull;
    }
    if (what & 8) st->stall = 0;
  }
}

// ---------------------------------------------------------------------------
// Passes over A (copy + norms, residual, SpMV).  KKT rows are short (about 8
// entries), so 8 lanes share a row and a wave covers 8 rows; rows are
// grid-strided and every wave issues one atomic for its reductions (one
// atomic per row on a single address serialises the whole pass).
// ---------------------------------------------------------------------------
constexpr int RG = 8;  // lanes per row

// instance of batch row r in a shared-pattern batch (0 otherwise)
__device__ __forceinline__ int inst_of(int r, const Inst& in) {
  return in.count > 1 ? r / in.n1 : 0;
}

// max that propagates NaN (fmax would drop it and hide a broken solution)
__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

__device__ __forceinline__ double group_sum(double v) {
  for (int off = RG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ __forceinline__ double wave_nanmax(double v) {
  for (int off = WAVE / 2; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

// max over a 256-thread workgroup (NaN-propagating), valid in thread 0; the
// caller then issues one atomic per workgroup: same-address atomics
// serialize, so one per wave over a large grid costs more than the pass
__device__ __forceinline__ double block_nanmax(double v, double* red) {
  v = wave_nanmax(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();  // red may still be read by a previous call
  if (threadIdx.x % WAVE == 0) red[w] = v;
  __syncthreads();
  double m = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x / WAVE); q++) m = nanmax(m, red[q]);
  return m;
}

// Pivot health after a refactorization: min / max |u_kk|, the tiny or
// non-finite pivot test against tiny_rel * ||A||_inf, and max |u_ij| over
// every stored U entry (the growth figure's numerator, NaN-propagating).
// 8 lanes per row; lane 0 of a row group also takes the diagonal.
__global__ __launch_bounds__(256) void k_pivot_stats(int n, const int* __restrict__ rowptr,
                                                     const int* __restrict__ diag,
                                                     const double* __restrict__ val0, DevStats* st,
                                                     double tiny_rel, double* __restrict__ red,
                                                     Inst in) {
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  const double anorm = __longlong_as_double((long long)st->anorm_f);
  double mn = __builtin_huge_val(), mx = 0.0, um = 0.0;
  int tiny = 0;
  // four row groups per round, their first loads all in flight before any is
  // used; lane 0 of a row's group holds its diagonal (the U part's first entry)
  constexpr int U = 4;
  const int stride = nw * (WAVE / RG);
  for (int r0 = wid * (WAVE / RG); r0 < n; r0 += U * stride) {
    int d[U], e[U];
    const double* vr[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int ig = r0 + u * stride + g;
      d[u] = 0;
      e[u] = 0;
      vr[u] = val0;
      if (ig < n) {
        const int ti = inst_of(ig, in);
        const int i = ig - ti * in.n1;
        vr[u] = val0 + ti * in.f1;
        d[u] = diag[i];
        e[u] = rowptr[i + 1];
      }
    }
    double a0[U];
#pragma unroll
    for (int u = 0; u < U; u++) a0[u] = d[u] + gl < e[u] ? fabs(vr[u][d[u] + gl]) : 0.0;
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (d[u] + gl < e[u]) {
        um = nanmax(um, a0[u]);
        if (gl == 0) {
          mn = fmin(mn, a0[u]);
          mx = fmax(mx, a0[u]);
          tiny |= !(a0[u] >= tiny_rel * anorm) || isinf(a0[u]);
        }
      }
      // long U parts (the rows next to and inside the dense block hold up to
      // a thousand entries): eight loads in flight per lane
      for (int t = d[u] + gl + RG; t < e[u]; t += 8 * RG) {
        double q[8];
#pragma unroll
        for (int v = 0; v < 8; v++) q[v] = t + v * RG < e[u] ? fabs(vr[u][t + v * RG]) : 0.0;
#pragma unroll
        for (int v = 0; v < 8; v++) um = nanmax(um, q[v]);
      }
    }
  }
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off, WAVE));
    mx = fmax(mx, __shfl_xor(mx, off, WAVE));
    tiny |= __shfl_xor(tiny, off, WAVE);
  }
  __shared__ double rmn[4], rmx[4], rum[4];
  __shared__ int rt[4];
  um = block_nanmax(um, rum);
  const int w = threadIdx.x / WAVE;
  if (threadIdx.x % WAVE == 0) {
    rmn[w] = mn;
    rmx[w] = mx;
    rt[w] = tiny;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x / WAVE); q++) {
      mn = fmin(mn, rmn[q]);
      mx = fmax(mx, rmx[q]);
      tiny |= rt[q];
    }
    // the workgroup's partial results; k_pivot_stats_final folds them in
    // (same-address atomics from every workgroup cost more than the pass)
    double* o = red + 4 * blockIdx.x;
    o[0] = mn;
    o[1] = mx;
    o[2] = um;
    o[3] = tiny ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_pivot_stats_final(int nb, const double* __restrict__ red,
                                                           DevStats* st) {
  double mn = __builtin_huge_val(), mx = 0.0, um = 0.0;
  int tiny = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    mn = fmin(mn, red[4 * b]);
    mx = fmax(mx, red[4 * b + 1]);
    um = nanmax(um, red[4 * b + 2]);
    tiny |= red[4 * b + 3] != 0.0;
  }
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, off, WAVE));
    mx = fmax(mx, __shfl_xor(mx, off, WAVE));
    tiny |= __shfl_xor(tiny, off, WAVE);
  }
  __shared__ double rmn[4], rmx[4], rum[4];
  __shared__ int rt[4];
  um = block_nanmax(um, rum);
  const int w = threadIdx.x / WAVE;
  if (threadIdx.x % WAVE == 0) {
    rmn[w] = mn;
    rmx[w] = mx;
    rt[w] = tiny;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x / WAVE); q++) {
      mn = fmin(mn, rmn[q]);
      mx = fmax(mx, rmx[q]);
      tiny |= rt[q];
    }
    atomicMin(&st->min_piv, dbits(mn));
    atomicMax(&st->max_piv, dbits(mx));
    // NaN bit patterns exceed every finite or infinite one as uint64
    atomicMax(&st->umax, um != um ? 0x7FF8000000000000ull : dbits(um));
    if (tiny) atomicOr(&st->tiny, 1);
  }
}

// Per-instance maxima of a block-diagonal batch, SEG_SLICES partial results
// per instance: block (s, t) reduces slice s of rows [row_off[t],
// row_off[t+1]) to out[3 (t SEG_SLICES + s)] = max matabs (the instance's
// matrix norm), + 1 = max |r|, + 2 = max |x|.
__global__ __launch_bounds__(256) void k_seg_stats(const int* __restrict__ gate,
                                                   const int* __restrict__ row_off,
                                                   const double* __restrict__ matabs,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ out) {
  KKT_GATE(gate);
  __shared__ double red[3][256 / WAVE];
  const int t = blockIdx.y, sl = blockIdx.x;
  const int a0 = row_off[t], len = row_off[t + 1] - a0;
  const int a = a0 + (int)((long long)len * sl / SEG_SLICES);
  const int b = a0 + (int)((long long)len * (sl + 1) / SEG_SLICES);
  double m0 = 0.0, m1 = 0.0, m2 = 0.0;
  for (int i = a + threadIdx.x; i < b; i += blockDim.x) {
    m0 = nanmax(m0, matabs[i]);
    m1 = nanmax(m1, fabs(r[i]));
    m2 = nanmax(m2, fabs(x[i]));
  }
  m0 = wave_nanmax(m0);
  m1 = wave_nanmax(m1);
  m2 = wave_nanmax(m2);
  const int w = threadIdx.x / WAVE;
  if (threadIdx.x % WAVE == 0) {
    red[0][w] = m0;
    red[1][w] = m1;
    red[2][w] = m2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double m = 0.0;
    for (int q = 0; q < 256 / WAVE; q++) m = nanmax(m, red[threadIdx.x][q]);
    out[3 * ((size_t)t * SEG_SLICES + sl) + threadIdx.x] = m;
  }
}

// copy of A's values and ||A||_inf (and, if rowabs != nullptr, every row's
// absolute sum for per-instance norms)
// A's values copied (dst), their row sums of |a| (rowabs) and ||A||_inf.
// luA: the values scattered into factor order through a2lu.  fnorm: also
// the factored matrix's norm (anorm_f; red_out then holds two maxima per
// workgroup).  ascale (with avs): the factored matrix is the matched and
// scaled one, a_p * ascale[p] (exact powers of two) goes to avs and luA, and
// its row sums give anorm_f.
template <bool SH>
__global__ __launch_bounds__(256) void k_copy_anorm(int n, const int* __restrict__ arow,
                                                    const double* __restrict__ src, double* dst,
                                                    DevStats* st, SyncState* ss,
                                                    double* __restrict__ rowabs,
                                                    const int* __restrict__ a2lu,
                                                    double* __restrict__ luA,
                                                    double* __restrict__ red_out, int fnorm,
                                                    const double* __restrict__ ascale,
                                                    double* __restrict__ avs, Inst in) {
  if constexpr (!SH) in = Inst();  // one instance: the decode below folds away
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  if (ss && blockIdx.x == 0 && threadIdx.x == 0) sync_prep(ss, 1);
  double m = 0.0, mf = 0.0;
  // four row groups per round, their loads all in flight before any is used
  constexpr int U = 4;
  const int stride = nw * (WAVE / RG);
  for (int r0 = wid * (WAVE / RG); r0 < n; r0 += U * stride) {
    // rows of the pattern's CSR: local entries p, A position p + ao, factor
    // positions a2lu[p] + fo (instance offsets of a shared-pattern batch)
    int ii[U], p0[U], pe[U], ao[U], fo[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      ii[u] = r0 + u * stride + g;
      p0[u] = 0;
      pe[u] = 0;
      ao[u] = 0;
      fo[u] = 0;
      if (ii[u] < n) {
        const int t = inst_of(ii[u], in);
        const int il = ii[u] - t * in.n1;
        ao[u] = t * in.a1;
        fo[u] = t * in.f1;
        p0[u] = arow[il] + gl;
        pe[u] = arow[il + 1];
      }
    }
    double v0[U];
    int q0[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      v0[u] = 0.0;
      q0[u] = 0;
      if (p0[u] < pe[u]) {
        v0[u] = src[p0[u] + ao[u]];
        if (luA) q0[u] = a2lu[p0[u]] + fo[u];
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      double s = 0.0, sf = 0.0;
      if (p0[u] < pe[u]) {
        dst[p0[u] + ao[u]] = v0[u];
        const double w = canon_nan(ascale ? v0[u] * ascale[p0[u]] : v0[u]);
        if (ascale) avs[p0[u]] = w;
        if (luA) luA[q0[u]] = w;
        s = fabs(v0[u]);
        sf = fabs(w);
      }
      for (int p = p0[u] + RG; p < pe[u]; p += RG) {
        const double v = src[p + ao[u]];
        dst[p + ao[u]] = v;
        const double w = canon_nan(ascale ? v * ascale[p] : v);
        if (ascale) avs[p] = w;
        if (luA) luA[a2lu[p] + fo[u]] = w;
        s += fabs(v);
        sf += fabs(w);
      }
      s = group_sum(s);
      sf = group_sum(sf);
      const int i = ii[u];
      if (i < n) {
        m = nanmax(m, s);
        mf = nanmax(mf, sf);
        if (rowabs && gl == 0) rowabs[i] = s;
      }
    }
  }
  __shared__ double red[2][4];
  m = block_nanmax(m, red[0]);
  mf = block_nanmax(mf, red[1]);
  if (threadIdx.x == 0) {
    // a NaN or an infinity among the values makes its row's sum non-finite
    if (!(m <= __DBL_MAX__)) st->nonfinite_in = 1;
    if (red_out) {  // reduced by k_red_max
      if (fnorm) {
        red_out[2 * blockIdx.x] = m;
        red_out[2 * blockIdx.x + 1] = mf;
      } else {
        red_out[blockIdx.x] = m;
      }
    } else {
      atomicMax(&st->anorm, dbits(m));
      if (fnorm) atomicMax(&st->anorm_f, dbits(mf));
    }
  }
}

// ||A||_1 through the column view
__global__ __launch_bounds__(256) void k_anorm1(int n, const int* __restrict__ cptr,
                                                const int* __restrict__ cpos,
                                                const double* __restrict__ aval, DevStats* st,
                                                double* __restrict__ colabs, Inst in) {
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  double m = 0.0;
  for (int r0 = wid * (WAVE / RG); r0 < n; r0 += nw * (WAVE / RG)) {
    const int j = r0 + g;
    double s = 0.0;
    if (j < n) {
      const int t = inst_of(j, in);
      const int jl = j - t * in.n1;
      const double* av = aval + t * in.a1;
      for (int q = cptr[jl] + gl; q < cptr[jl + 1]; q += RG) s += fabs(av[cpos[q]]);
    }
    s = group_sum(s);
    if (j < n) {
      m = nanmax(m, s);
      if (colabs && gl == 0) colabs[j] = s;
    }
  }
  __shared__ double red[4];
  m = block_nanmax(m, red);
  if (threadIdx.x == 0) atomicMax(&st->anorm1, dbits(m));
}

// ---------------------------------------------------------------------------
// Triangular solves, one wavefront per row (level-synchronous launches).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lsolve_rows(const int* __restrict__ gate, const int* __restrict__ rows, int nrows,
                                                     const int* __restrict__ rowptr,
                                                     const int* __restrict__ col,
                                                     const int* __restrict__ diag,
                                                     const double* __restrict__ val, double* y) {
  KKT_GATE(gate);
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE, lane = threadIdx.x % WAVE;
  if (wave >= nrows) return;
  const int i = rows[wave];
  double s = 0.0;
  for (int q = rowptr[i] + lane; q < diag[i]; q += WAVE) s += val[q] * y[col[q]];
  s = wave_sum(s);
  if (lane == 0) y[i] -= s;
}

__global__ __launch_bounds__(256) void k_usolve_rows(const int* __restrict__ gate, const int* __restrict__ rows, int nrows,
                                                     const int* __restrict__ rowptr,
                                                     const int* __restrict__ col,
                                                     const int* __restrict__ diag,
                                                     const double* __restrict__ val, double* y) {
  KKT_GATE(gate);
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE, lane = threadIdx.x % WAVE;
  if (wave >= nrows) return;
  const int i = rows[wave];
  const int d = diag[i];
  double s = 0.0;
  for (int q = d + 1 + lane; q < rowptr[i + 1]; q += WAVE) s += val[q] * y[col[q]];
  s = wave_sum(s);
  if (lane == 0) y[i] = (y[i] - s) / val[d];
}

// U^T t = s: column j of U (rows i <= j, diagonal last)
__global__ __launch_bounds__(256) void k_utsolve_cols(const int* __restrict__ gate, const int* __restrict__ cols, int ncols,
                                                      const int* __restrict__ tptr,
                                                      const int* __restrict__ trow,
                                                      const int* __restrict__ tpos,
                                                      const double* __restrict__ val, double* y) {
  KKT_GATE(gate);
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE, lane = threadIdx.x % WAVE;
  if (wave >= ncols) return;
  const int j = cols[wave];
  const int te = tptr[j + 1] - 1;  // diagonal
  double s = 0.0;
  for (int t = tptr[j] + lane; t < te; t += WAVE) s += val[tpos[t]] * y[trow[t]];
  s = wave_sum(s);
  if (lane == 0) y[j] = (y[j] - s) / val[tpos[te]];
}

// L^T w = t: column j of strict L (rows i > j)
__global__ __launch_bounds__(256) void k_ltsolve_cols(const int* __restrict__ gate, const int* __restrict__ cols, int ncols,
                                                      const int* __restrict__ tptr,
                                                      const int* __restrict__ trow,
                                                      const int* __restrict__ tpos,
                                                      const double* __restrict__ val, double* y) {
  KKT_GATE(gate);
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE, lane = threadIdx.x % WAVE;
  if (wave >= ncols) return;
  const int j = cols[wave];
  double s = 0.0;
  for (int t = tptr[j] + lane; t < tptr[j + 1]; t += WAVE) s += val[tpos[t]] * y[trow[t]];
  s = wave_sum(s);
  if (lane == 0) y[j] -= s;
}

// y[i] = x[perm[i]] (times scale[i]); scatter: y[perm[i]] = x[i] (times scale[i])
__global__ void k_gather(const int* __restrict__ gate, int n, const int* __restrict__ perm,
                         const double* __restrict__ scale, const double* __restrict__ x,
                         double* __restrict__ y) {
  KKT_GATE(gate);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = canon_nan(scale ? x[perm[i]] * scale[i] : x[perm[i]]);
}
__global__ void k_scatter(const int* __restrict__ gate, int n, const int* __restrict__ perm,
                          const double* __restrict__ scale, const double* __restrict__ x,
                          double* __restrict__ y) {
  KKT_GATE(gate);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[perm[i]] = scale ? x[i] * scale[i] : x[i];
}

// r = b - op(A) x, max |r|, max |x| (8 lanes per row of op(A), one atomic
// per wave); for op 'T' the (ptr, idx, pos) triple is A's column view.
__global__ __launch_bounds__(256) void k_residual(int n, const int* __restrict__ ptr,
                                                  const int* __restrict__ idx,
                                                  const int* __restrict__ pos,
                                                  const double* __restrict__ aval,
                                                  const double* __restrict__ b,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ r, DevStats* st,
                                                  double* __restrict__ red_out) {
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  double rm = 0.0, xm = 0.0;
  // four row groups per round, their first entries' loads all in flight
  // before any is used (a wave otherwise waits one gather per round)
  constexpr int U = 4;
  const int stride = nw * (WAVE / RG);
  for (int r0 = wid * (WAVE / RG); r0 < n; r0 += U * stride) {
    int ii[U], t0[U], te[U];
    double s[U], av[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      ii[u] = r0 + u * stride + g;
      t0[u] = 0;
      te[u] = 0;
      if (ii[u] < n) {
        t0[u] = ptr[ii[u]] + gl;
        te[u] = ptr[ii[u] + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      av[u] = 0.0;
      xv[u] = 0.0;
      if (t0[u] < te[u]) {
        av[u] = aval[pos ? pos[t0[u]] : t0[u]];
        xv[u] = x[idx[t0[u]]];
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      s[u] = av[u] * xv[u];
      for (int t = t0[u] + RG; t < te[u]; t += RG) s[u] += aval[pos ? pos[t] : t] * x[idx[t]];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const double su = group_sum(s[u]);
      const int i = ii[u];
      if (i < n) {
        const double ri = b[i] - su;
        if (r && gl == 0) r[i] = ri;
        rm = nanmax(rm, fabs(ri));
        xm = nanmax(xm, fabs(x[i]));
      }
    }
  }
  __shared__ double red[2][4];
  rm = block_nanmax(rm, red[0]);
  xm = block_nanmax(xm, red[1]);
  if (threadIdx.x == 0) {
    if (red_out) {  // reduced by k_red_max
      red_out[2 * blockIdx.x] = rm;
      red_out[2 * blockIdx.x + 1] = xm;
    } else {
      atomicMax(&st->rmax, dbits(rm));
      atomicMax(&st->xmax, dbits(xm));
    }
  }
}

// Second stage of a maximum over a large grid: the first stage left one
// (NaN-propagating) maximum per workgroup and quantity in red (nq
// quantities interleaved, nb workgroups); one workgroup stores the maxima's
// bit patterns into out[0 .. nq) (uint64 order = order of non-negative
// doubles).  Same-address atomics from thousands of workgroups would
// serialize.
__global__ __launch_bounds__(1024) void k_red_max(const double* __restrict__ red, int nb, int nq,
                                                  unsigned long long* out0,
                                                  unsigned long long* out1) {
  __shared__ double sh[2][1024 / WAVE];
  double m[2] = {0.0, 0.0};
  // every load of a thread in flight before any is used
  const int nv = nb * nq;
#pragma unroll 8
  for (int e = threadIdx.x; e < nv; e += blockDim.x) {
    const double v = red[e];
    if (e % nq == 0)
      m[0] = nanmax(m[0], v);
    else
      m[1] = nanmax(m[1], v);
  }
  const int w = threadIdx.x / WAVE;
  for (int qi = 0; qi < 2; qi++) {
    const double v = wave_nanmax(m[qi]);
    if (threadIdx.x % WAVE == 0) sh[qi][w] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int qi = 0; qi < nq; qi++) {
      double t = 0.0;
      for (int q = 0; q < (int)(blockDim.x / WAVE); q++) t = nanmax(t, sh[qi][q]);
      *(qi == 0 ? out0 : out1) = dbits(t);
    }
  }
}

// Column r = blockIdx.y of R = B - op(A) X (all ld n): per-column maxima
// colmax[2r] = max |r|, colmax[2r+1] = max |x| (uint64 bit patterns).
__global__ __launch_bounds__(256) void k_residual_mr(int n, const int* __restrict__ ptr,
                                                     const int* __restrict__ idx,
                                                     const int* __restrict__ pos,
                                                     const double* __restrict__ aval,
                                                     const double* __restrict__ B,
                                                     const double* __restrict__ X,
                                                     unsigned long long* colmax) {
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  const double* b = B + (size_t)blockIdx.y * n;
  const double* x = X + (size_t)blockIdx.y * n;
  double rm = 0.0, xm = 0.0;
  for (int r0 = wid * (WAVE / RG); r0 < n; r0 += nw * (WAVE / RG)) {
    const int i = r0 + g;
    double s = 0.0;
    if (i < n)
      for (int t = ptr[i] + gl; t < ptr[i + 1]; t += RG) s += aval[pos ? pos[t] : t] * x[idx[t]];
    s = group_sum(s);
    if (i < n) {
      rm = nanmax(rm, fabs(b[i] - s));
      xm = nanmax(xm, fabs(x[i]));
    }
  }
  __shared__ double red[2][4];
  rm = block_nanmax(rm, red[0]);
  xm = block_nanmax(xm, red[1]);
  if (threadIdx.x == 0) {
    atomicMax(colmax + 2 * blockIdx.y, dbits(rm));
    atomicMax(colmax + 2 * blockIdx.y + 1, dbits(xm));
  }
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

__global__ __launch_bounds__(256) void k_spmv(int n, const int* __restrict__ ptr,
                                              const int* __restrict__ idx,
                                              const int* __restrict__ pos,
                                              const double* __restrict__ aval,
                                              const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  for (int r0 = wid * (WAVE / RG); r0 < n; r0 += nw * (WAVE / RG)) {
    const int i = r0 + g;
    double s = 0.0;
    if (i < n)
      for (int t = ptr[i] + gl; t < ptr[i + 1]; t += RG) s += aval[pos ? pos[t] : t] * x[idx[t]];
    s = group_sum(s);
    if (i < n && gl == 0) y[i] = s;
  }
}

// One Jacobi sweep of a triangular solve (approximate triangular solves,
// the future-work direction of Section 6): every row at once from the
// previous iterate, 8 lanes per row.
//   MODE 0  unit L:  yout_i = c_i - sum_{k<i} l_ik yin_k
//   MODE 1  U:       yout_i = (c_i - sum_{k>i} u_ik yin_k) / u_ii
template <int MODE>
__global__ __launch_bounds__(256) void k_jacobi_sweep(const int* __restrict__ gate, int n, const int* __restrict__ rowptr,
                                                      const int* __restrict__ col,
                                                      const int* __restrict__ diag,
                                                      const double* __restrict__ val,
                                                      const double* __restrict__ c,
                                                      const double* __restrict__ yin,
                                                      double* __restrict__ yout) {
  KKT_GATE(gate);
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  for (int r0 = wid * (WAVE / RG); r0 < n; r0 += nw * (WAVE / RG)) {
    const int i = r0 + g;
    double s = 0.0;
    int dq = 0;
    if (i < n) {
      dq = diag[i];
      const int b = MODE == 0 ? rowptr[i] : dq + 1, e = MODE == 0 ? dq : rowptr[i + 1];
      for (int q = b + gl; q < e; q += RG) s += val[q] * yin[col[q]];
    }
    s = group_sum(s);
    if (i < n && gl == 0) yout[i] = MODE == 0 ? c[i] - s : (c[i] - s) / val[dq];
  }
}

// ---------------------------------------------------------------------------
// FGMRES-CGS2 pieces
// ---------------------------------------------------------------------------
constexpr int MD_BLOCK = 256;
constexpr int MD_MAXM = 32;
constexpr int MD_GRID = 256;

__global__ __launch_bounds__(MD_BLOCK) void k_multidot_partial(int n, int m,
                                                               const double* __restrict__ V,
                                                               long ld,
                                                               const double* __restrict__ w,
                                                               double* __restrict__ partial) {
  __shared__ double red[MD_BLOCK / WAVE][MD_MAXM];
  double acc[MD_MAXM];
  for (int i = 0; i < m; i++) acc[i] = 0.0;
  for (int t = blockIdx.x * MD_BLOCK + threadIdx.x; t < n; t += gridDim.x * MD_BLOCK) {
    const double wt = w[t];
    for (int i = 0; i < m; i++) acc[i] += V[(long)i * ld + t] * wt;
  }
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  for (int i = 0; i < m; i++) {
    const double s = wave_sum(acc[i]);
    if (lane == 0) red[wave][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < m) {
    double s = 0.0;
    for (int q = 0; q < MD_BLOCK / WAVE; q++) s += red[q][threadIdx.x];
    partial[blockIdx.x * MD_MAXM + threadIdx.x] = s;
  }
}

__global__ void k_multidot_final(int m, int nblocks, const double* __restrict__ partial,
                                 double* __restrict__ h) {
  const int i = threadIdx.x;
  if (i < m) {
    double s = 0.0;
    for (int b = 0; b < nblocks; b++) s += partial[b * MD_MAXM + i];
    h[i] = s;
  }
}

__global__ void k_multiaxpy(int n, int m, const double* __restrict__ V, long ld,
                            const double* __restrict__ h, double* __restrict__ w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s = w[t];
  for (int i = 0; i < m; i++) s -= h[i] * V[(long)i * ld + t];
  w[t] = s;
}

__global__ void k_combine(int n, int m, const double* __restrict__ Z, long ld,
                          const double* __restrict__ y, const double* __restrict__ base,
                          double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s = base[t];
  for (int i = 0; i < m; i++) s += y[i] * Z[(long)i * ld + t];
  out[t] = s;
}

__global__ void k_scale_div(int n, const double* __restrict__ x, const double* __restrict__ scal,
                            double* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double d = scal[0];
  y[t] = d > 0.0 ? x[t] / d : 0.0;
}

// x += d (classical refinement step)
__global__ void k_add(const int* __restrict__ gate, int n, const double* __restrict__ d, double* __restrict__ x) {
  KKT_GATE(gate);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] += d[t];
}

// Column j of the Hessenberg matrix from the two CGS passes (h + h2) and
// ww = ||w||^2: store it, apply the earlier rotations, build rotation j,
// update g and back-substitute y (j+1 entries).  *hn_out = ||w||.
__global__ void k_givens(int j, int m, const double* __restrict__ h, const double* __restrict__ h2,
                         const double* __restrict__ ww, double* H, double* cs, double* sn,
                         double* g, double* y, double* hn_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* Hj = H + (long)j * (m + 1);
  for (int i = 0; i <= j; i++) Hj[i] = h[i] + h2[i];
  const double hn = sqrt(ww[0]);
  hn_out[0] = hn;
  Hj[j + 1] = hn;
  for (int i = 0; i < j; i++) {
    const double a = Hj[i], b = Hj[i + 1];
    Hj[i] = cs[i] * a + sn[i] * b;
    Hj[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double den = hypot(Hj[j], Hj[j + 1]);
  cs[j] = den > 0.0 ? Hj[j] / den : 1.0;
  sn[j] = den > 0.0 ? Hj[j + 1] / den : 0.0;
  Hj[j] = den;
  Hj[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  for (int i = j; i >= 0; i--) {
    double s = g[i];
    for (int t = i + 1; t <= j; t++) s -= H[(long)t * (m + 1) + i] * y[t];
    y[i] = s / H[(long)i * (m + 1) + i];
  }
}

// rr = ||r||^2 on the device: g = (sqrt(rr), 0, ...), v0 = r / sqrt(rr)
__global__ void k_arnoldi_start(int n, int m, const double* __restrict__ r,
                                const double* __restrict__ rr, double* __restrict__ v0,
                                double* __restrict__ g) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const double beta = sqrt(rr[0]);
  if (t < n) v0[t] = beta > 0.0 ? r[t] / beta : 0.0;
  if (t <= m) g[t] = t == 0 ? beta : 0.0;
}

// ---------------------------------------------------------------------------
// Adjoint on the pattern
// ---------------------------------------------------------------------------
// grad[p] = -sum_r lam[r][i] * x[r][j] for every stored p = (i, j); lam, x
// column-major n x nrhs.  Eight lanes per row, one stored entry each; the
// right-hand sides are summed in ascending order.
__global__ __launch_bounds__(256) void k_grad_sddmm(int n, int nrhs, const int* __restrict__ arow,
                                                    const int* __restrict__ acol,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ grad) {
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  for (int i = wid * (WAVE / RG) + g; i - g < n; i += nw * (WAVE / RG)) {
    if (i >= n) continue;
    for (int p = arow[i] + gl; p < arow[i + 1]; p += RG) {
      const int j = acol[p];
      double s = 0.0;
      for (int r = 0; r < nrhs; r++) s += lam[(size_t)r * n + i] * x[(size_t)r * n + j];
      grad[p] = -s;
    }
  }
}

// y = x (gated: part of the solve path)
__global__ void k_copy(const int* __restrict__ gate, int n, const double* __restrict__ x,
                       double* __restrict__ y) {
  KKT_GATE(gate);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = x[t];
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// grid of the grid-strided row passes: 32 rows per 256-thread block, capped
// so that each wave loops over several row groups (one atomic per wave)
// grids of the row passes: enough waves to stream A at full bandwidth, few
// enough workgroups that their one atomic each stays cheap
inline int rows_grid(int n) { return std::max(1, std::min(cdiv(n, 32), 1024)); }


// Micro rows of a short-row band: at most MICRO_LEN entries, MICRO_PIV
// pivots and MICRO_LIST multiply-adds.  One lane takes the whole row (a chunk
// of such rows is one level of the dependency graph, so its rows do not wait
// for each other): the row's values sit in the wave's LDS area, entry k of
// lane l at sa[k * WAVE + l]; the pivot diagonals and every U entry of the
// list are requested in one round, entries still reading as the sentinel are
// polled again, then the arithmetic runs pivot after pivot in ascending order
// with the same quotient and fma(-l, u, a) as the wave-per-row code.  List
// entry e belongs to the last pivot t whose list offset fl.x is at most e, so
// the U addresses do not wait for the map.
constexpr int MICRO_LEN = MICRO_ROW_LEN, MICRO_PIV = MICRO_ROW_PIV, MICRO_LIST = MICRO_ROW_LIST;

// Row timeline (debug_timeline): tl[3 i] = the row's start (staged), tl[3 i +
// 1] = the last poll that still found one of its inputs missing (the start if
// none did), tl[3 i + 2] = after its stores completed, with the kernel kind in
// bits 62-63 (1 micro row, 2 list kernel, 3 long-row kernel); wall-clock
// ticks.
__device__ __forceinline__ void tl_record(long long* tl, int i, long long t0, long long t1,
                                          long long kind) {
  stores_done();
  tl[3 * (size_t)i] = t0;
  tl[3 * (size_t)i + 1] = t1;
  tl[3 * (size_t)i + 2] = (long long)wall_clock64() | (kind << 62);
}

// doubles of LDS per wave of k_refactor_flat (cap even)
__host__ __device__ constexpr int flat_area(int cap) {
  return 2 * cap > MICRO_LEN * WAVE ? 2 * cap : MICRO_LEN * WAVE;
}

template <bool TL>
__device__ __forceinline__ void refactor_micro_row(int4 mt, int i, int lane, double* sa,
                                                   double* val, int* stall,
                                                   const unsigned short* __restrict__ map,
                                                   const double* __restrict__ luA,
                                                   const int2* __restrict__ fl, DevStats* st,
                                                   double thr, long long* tl) {
  const long long tl0 = TL ? (long long)wall_clock64() : 0;
  // row start, length, pivots, update-map offset, list length
  const int rs = mt.x, len = mt.y & 0xffff, dl = mt.y >> 16, mb = mt.z, nl = mt.w;
  for (int k = 0; k < len; k++) sa[k * WAVE + lane] = luA[rs + k];
  double d[MICRO_PIV], u[MICRO_LIST];
  unsigned int mm[MICRO_LIST];  // packed map entries: pivot << 8 | target position
  {
    // fx[t]: list offset of pivot t (MICRO_LIST past the row's pivots), fy[t]:
    // its U row start minus that offset
    int fx[MICRO_PIV], fy[MICRO_PIV];
#pragma unroll
    for (int t = 0; t < MICRO_PIV; t++) {
      fx[t] = MICRO_LIST;
      fy[t] = 0;
      d[t] = 1.0;
      if (t < dl) {
        const int2 f = fl[rs + t];
        fx[t] = f.x;
        fy[t] = f.y;
        d[t] = ld_coh(val + (f.x + f.y - 1));
      }
    }
#pragma unroll
    for (int e = 0; e < MICRO_LIST; e++) {
      mm[e] = 0;
      u[e] = 0.0;
      if (e < nl) {
        int y = fy[0];
#pragma unroll
        for (int q = 1; q < MICRO_PIV; q++)
          if (fx[q] <= e) y = fy[q];
        mm[e] = map[mb + e];
        u[e] = ld_coh(val + (e + y));
      }
    }
  }
  // pivot rows not finished when first read: poll the missing values (their
  // addresses are recomputed from fl)
  int spins = 0;
  long long tl1 = tl0;
  for (;;) {
    bool miss = false;
#pragma unroll
    for (int t = 0; t < MICRO_PIV; t++) miss = miss || (t < dl && is_sentinel(d[t]));
#pragma unroll
    for (int e = 0; e < MICRO_LIST; e++) miss = miss || (e < nl && is_sentinel(u[e]));
    if (!miss || !keep_waiting(&spins, stall)) break;
    if constexpr (TL) tl1 = (long long)wall_clock64();
#pragma unroll
    for (int t = 0; t < MICRO_PIV; t++)
      if (t < dl && is_sentinel(d[t])) {
        const int2 f = fl[rs + t];
        d[t] = ld_coh(val + (f.x + f.y - 1));
      }
#pragma unroll
    for (int e = 0; e < MICRO_LIST; e++)
      if (e < nl && is_sentinel(u[e])) u[e] = ld_coh(val + (e + fl[rs + (int)(mm[e] >> 8)].y));
  }
#pragma unroll
  for (int t = 0; t < MICRO_PIV; t++) {
    if (t < dl) {
      const double l = sa[t * WAVE + lane] / d[t];
#pragma unroll
      for (int e = 0; e < MICRO_LIST; e++)
        if (e < nl && (int)(mm[e] >> 8) == t) {
          double* w = sa + (int)(mm[e] & 255u) * WAVE + lane;
          *w = __builtin_fma(-l, u[e], *w);
        }
      sa[t * WAVE + lane] = l;
    }
  }
  if (thr > 0.0) {
    double* w = sa + dl * WAVE + lane;
    if (fabs(*w) < thr) {
      *w = perturb_pivot(*w, thr);
      st->perturbed = 1;
    }
  }
  for (int k = 0; k < len; k++) st_coh(val + rs + k, sa[k * WAVE + lane]);
  if constexpr (TL) tl_record(tl, i, tl0, tl1, 1);
}

// Rows of a short-row band (at most 256 entries each; no row of the dense
// block).  One wave per row, as
// k_refactor_syncfree, but the row's multiply-adds form one list, pivot after
// pivot, each pivot row's U entries in order: for the row's L entries q,
// fl[q] = (offset of pivot q's first list entry, U row start of pivot q minus
// that offset), and at the diagonal fl = (list length, 0); the packed map
// gives every list entry as (pivot index << 8) | target position.  Up to 256
// list entries (four per lane) of pivots already seen finished are loaded at
// once, so a row costs a few memory round trips rather than one or two per
// pivot; the arithmetic still runs pivot after pivot in ascending order with
// the same fma(-l, u, a) and quotient as every other refactorization code.
// Publication: device-coherent stores of the values into a factor array that
// holds the sentinel; a pivot row is finished once its diagonal is, and each
// of its other entries is re-polled while it still reads as the sentinel.
// Chunks flagged in cmicro hold micro rows, one per lane (refactor_micro_row).
// Per row few dependent memory round trips: the chunk's row metadata (rmeta,
// per order position: row start, length | pivots << 16, map offset, list
// length) comes in one load for all its rows; the staging of values and list
// bounds is the second; the first list window goes out together with the
// pivot-diagonal poll (entries of pivots not finished yet read as the sentinel
// and are polled again before use), its U addresses found from the staged list
// bounds rather than from the map.
template <int WPB, bool TL, bool SH>
__global__ __launch_bounds__(WPB* WAVE) void k_refactor_flat(
    const int* __restrict__ cstart, int nchunks, unsigned int* tickets, int nstreams,
    double* val0, int* stall, int cap, const int4* __restrict__ rmeta,
    const unsigned short* __restrict__ map, const double* __restrict__ luA0,
    const int2* __restrict__ fl, const unsigned char* __restrict__ cmicro, DevStats* st,
    double prel, const int* __restrict__ order, long long* tl, Inst in) {
  if constexpr (!SH) in = Inst();  // one instance: the decode below folds away
  extern __shared__ double smem_d[];
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  // LDS per wave, one area of flat_area(cap) doubles: values (cap doubles),
  // list bounds per L entry (cap int2); or, for a chunk of micro rows, their
  // values (MICRO_LEN x WAVE doubles)
  double* sv = smem_d + (size_t)wave * flat_area(cap);
  int2* sf = reinterpret_cast<int2*>(sv + cap);
  const double thr = prel > 0.0 ? prel * __longlong_as_double((long long)st->anorm_f) : 0.0;
  for (;;) {
    const int tk = next_chunk(tickets, nstreams, lane);
    if (tk >= nchunks * in.count) break;
    // ticket = chunk x instances + instance (every instance of a chunk before
    // the next chunk: a topological order for each instance)
    const int ch = tk / in.count, inst = tk - ch * in.count;
    double* val = val0 + (size_t)inst * in.f1;
    const double* luA = luA0 + (size_t)inst * in.f1;
    const int cs = cstart[ch], ce = cstart[ch + 1];
    // the chunk's rows (at most 64), one per lane
    const int4 mt = cs + lane < ce ? rmeta[cs + lane] : make_int4(0, 0, 0, 0);
    if (cmicro != nullptr && bcast0(cmicro[ch]) != 0u) {
      wave_sync();  // the last row of a previous chunk is done with the area
      if (cs + lane < ce)
        refactor_micro_row<TL>(mt, TL ? order[cs + lane] : 0, lane, sv, val, stall, map, luA, fl, st,
                           thr, tl);
      continue;
    }
    for (int r = cs; r < ce; r++) {
      const int k = r - cs;
      const int rs = __builtin_amdgcn_readlane(mt.x, k);
      const int ld = __builtin_amdgcn_readlane(mt.y, k);
      const int len = ld & 0xffff, dl = ld >> 16;
      const int mb = __builtin_amdgcn_readlane(mt.z, k);
      const int nl = __builtin_amdgcn_readlane(mt.w, k);
      wave_sync();  // the previous row of this chunk is done with the staging area
      for (int t = lane; t < len; t += WAVE) sv[t] = luA[rs + t];
      for (int t = lane; t <= dl; t += WAVE) sf[t] = fl[rs + t];
      wave_sync();
      const long long tl0 = TL ? (long long)wall_clock64() : 0;
      long long tl1 = tl0;
      int ready_upto = 0, t0 = 0, spins = 0;
      double dv = 0.0;  // lane q: diagonal of pivot t0 + q
      double u[4];
      int tp[4];  // packed map entry of the loaded list entry, -1 if none
      // list window [wbeg, wend): entry e's pivot is the last t with
      // sf[t].x <= e (pivots without U entries share their successor's
      // offset), so its U value sits at e + sf[t].y
      int wbeg = 0, wend = min(4 * WAVE, nl);
      auto load_window = [&]() {
#pragma unroll
        for (int z = 0; z < 4; z++) {
          const int e = wbeg + lane + z * WAVE;
          tp[z] = -1;
          u[z] = 0.0;
          if (e < wend) {
            tp[z] = (int)map[mb + e];
            int lo = 0, hi = dl - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (sf[mid].x <= e)
                lo = mid;
              else
                hi = mid - 1;
            }
            u[z] = ld_coh(val + (e + sf[lo].y));
          }
        }
      };
      load_window();  // in flight with the first pivot poll below
      for (int t = 0; t < dl; t++) {
        if (t >= ready_upto) {
          for (;;) {
            // one pivot diagonal per lane; the values double as the batch of
            // pivots for the quotients below
            const int q = t + lane;
            bool ok = true;
            if (q < dl) {
              const int2 f = sf[q];
              dv = ld_coh(val + (f.x + f.y - 1));
              ok = !is_sentinel(dv);
            }
            const unsigned long long bad = __ballot(!ok);
            const int first_bad = bad ? __ffsll((long long)bad) - 1 : WAVE;
            if (first_bad > 0) {
              // never past the row's last pivot: sf[ready_upto] bounds the
              // list windows below
              ready_upto = min(dl, t + first_bad);
              t0 = t;
              break;
            }
            // pivot t itself is missing: poll its diagonal (a single request
            // per wave) until it is set, then re-check the batch
            const int2 f = sf[t];
            const int dpt = f.x + f.y - 1;
            bool go = true;
            while (go && bcast0(is_sentinel(ld_coh(val + dpt)) ? 1u : 0u) != 0u)
              go = bcast0(keep_waiting(&spins, stall) ? 1u : 0u) != 0u;
            if constexpr (TL) tl1 = (long long)wall_clock64();
            if (!go) {  // stalled: drain
              ready_upto = dl;
              t0 = t;
              break;
            }
          }
        }
        const double ukk = readlane_d(dv, (t - t0) & (WAVE - 1));
        const double lik = sv[t] / ukk;
        const int oe = sf[t + 1].x;
        const int dt = sf[t].y;
        for (;;) {
#pragma unroll
          for (int z = 0; z < 4; z++) {
            if ((tp[z] >> 8) == t) {
              if (TL && is_sentinel(u[z])) tl1 = (long long)wall_clock64();
              while (is_sentinel(u[z]) && keep_waiting(&spins, stall))
                u[z] = ld_coh(val + (wbeg + lane + z * WAVE + dt));
              const int p = tp[z] & 255;
              sv[p] = __builtin_fma(-lik, u[z], sv[p]);
            }
          }
          if (oe <= wend) break;
          // next window of the list (pivot t's entries continue past this
          // one; a window that cannot advance means inconsistent list
          // bounds: report a stall rather than loop)
          wbeg = wend;
          wend = min(wbeg + 4 * WAVE, nl);
          if (wend <= wbeg) {
            st_flag(stall, 1);
            break;
          }
          load_window();
        }
        wave_sync();
        sv[t] = lik;  // every lane writes the same value
        wave_sync();
      }
      // static pivoting of this row's pivot
      if (thr > 0.0) {
        const double d = sv[dl];
        if (fabs(d) < thr) {
          wave_sync();
          sv[dl] = perturb_pivot(d, thr);  // every lane writes the same value
          st->perturbed = 1;
        }
        wave_sync();
      }
      for (int t = lane; t < len; t += WAVE) st_coh(val + rs + t, sv[t]);
      if constexpr (TL) {
        long long t1 = tl1;  // the latest wait of any lane
        for (int off = WAVE / 2; off > 0; off >>= 1) {
          const long long o = __shfl_xor(t1, off, WAVE);
          t1 = o > t1 ? o : t1;
        }
        if (lane == 0) tl_record(tl, order[r], tl0, t1, 2);
      }
    }
  }
}


// Rows of a band by workgroups: one workgroup of WPR waves per row (default
// one).  The row's pivot steps stay one at a time in ascending order (a
// workgroup barrier between two steps), but wave w owns the steps t = w,
// w + WPR, ...: right
// after a step it loads the pivot, the first R * 64 U entries and their
// target positions of the step WPR * DEPTH later (DEPTH register buffers per
// wave), so while the other waves apply theirs those loads are in flight, and
// a step costs about one pass over LDS rather than a memory round trip.
// Values that still read as the sentinel are polled again before use (the
// pivot row was not finished yet).  Only the row's values live in LDS (8 bytes
// per entry, so many long rows fit on a CU at once); each wave keeps the
// pivot-row bounds and update-map offsets of its next 64 steps in registers,
// one step per lane.  dlc[i]: pivots of row i in this phase (those before the
// dense trailing block).
template <int WPR, int DEPTH, bool TL, bool SH>
__global__ __launch_bounds__(WPR* WAVE) void k_refactor_wg(
    const int* __restrict__ order, const int* __restrict__ cstart, int nchunks,
    unsigned int* tickets, int nstreams, const int* __restrict__ rowptr,
    const int* __restrict__ dlc, double* val0, int* stall, const int* __restrict__ moff,
    const unsigned short* __restrict__ map, const double* __restrict__ luA0,
    const int2* __restrict__ pbnd, const int* __restrict__ diag, int c0, DevStats* st,
    double prel, long long* tl, Inst in) {
  if constexpr (!SH) in = Inst();  // one instance: the decode below folds away
  constexpr int R = 4;  // prefetched chunks of 64 U entries per pivot step
  constexpr int NT = WPR * WAVE;
  constexpr int AHEAD = WPR * DEPTH;
  extern __shared__ double smem_d[];
  __shared__ int s_tk;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
  const int lane = threadIdx.x % WAVE;
  double* sv = smem_d;  // the row's values
  const double thr = prel > 0.0 ? prel * __longlong_as_double((long long)st->anorm_f) : 0.0;
  struct Step {
    double ukk;
    double u[R];
    int p[R];
    int2 kk;  // pivot row: diagonal position, row end
    int mo;   // update-map offset
  };
  for (;;) {
    if (wave == 0) {
      const int tk = next_chunk(tickets, nstreams, lane);
      s_tk = tk;  // every lane of wave 0 writes the same value
    }
    __syncthreads();
    const int tk = __builtin_amdgcn_readfirstlane(s_tk);
    __syncthreads();  // read by every wave before the next fetch overwrites it
    if (tk >= nchunks * in.count) break;
    const int ch = tk / in.count, inst = tk - ch * in.count;
    double* val = val0 + (size_t)inst * in.f1;
    const double* luA = luA0 + (size_t)inst * in.f1;
    const int r_end = cstart[ch + 1];
    for (int r = cstart[ch]; r < r_end; r++) {
      const int i = order[r];
      const int rs = rowptr[i], len = rowptr[i + 1] - rs;
      const int dl = dlc[i];
      int spins = 0;
      long long tl0 = 0, tl1 = 0;
      for (int t = threadIdx.x; t < len; t += NT) sv[t] = luA[rs + t];
      // this wave's steps w + WPR * (64 * ib + lane): pivot-row bounds, map offsets
      int ib = -1, ib_mo = 0;
      int2 ib_kk = make_int2(0, 0);
      auto load = [&](Step& b, int t) {
        const int own = (t - wave) / WPR;
        if ((own >> 6) != ib) {
          ib = own >> 6;
          const int tq = wave + WPR * ((ib << 6) + lane);
          ib_kk = tq < dl ? pbnd[rs + tq] : make_int2(0, 0);
          ib_mo = tq < dl ? moff[rs + tq] : 0;
        }
        const int l = own & (WAVE - 1);
        b.kk = make_int2(__builtin_amdgcn_readlane(ib_kk.x, l),
                         __builtin_amdgcn_readlane(ib_kk.y, l));
        b.mo = __builtin_amdgcn_readlane(ib_mo, l);
        const int ub = b.kk.x + 1;
        b.ukk = ld_coh(val + b.kk.x);
#pragma unroll
        for (int z = 0; z < R; z++) {
          const int q = ub + lane + z * WAVE;
          b.p[z] = -1;
          b.u[z] = 0.0;
          if (q < b.kk.y) {
            b.p[z] = map[b.mo + (q - ub)];
            b.u[z] = ld_coh(val + q);
          }
        }
      };
      auto step = [&](Step& b, int t) {
        const int ub = b.kk.x + 1;
        // values loaded before the pivot row was finished: poll them again
        for (;;) {
          bool miss = is_sentinel(b.ukk);
#pragma unroll
          for (int z = 0; z < R; z++) miss = miss || (b.p[z] >= 0 && is_sentinel(b.u[z]));
          if (__ballot(miss) == 0) break;
          if constexpr (TL) tl1 = (long long)wall_clock64();
          if (bcast0(keep_waiting(&spins, stall) ? 1u : 0u) == 0u) break;
          if (is_sentinel(b.ukk)) b.ukk = ld_coh(val + b.kk.x);
#pragma unroll
          for (int z = 0; z < R; z++)
            if (b.p[z] >= 0 && is_sentinel(b.u[z])) b.u[z] = ld_coh(val + ub + lane + z * WAVE);
        }
        const double lik = sv[t] / b.ukk;
#pragma unroll
        for (int z = 0; z < R; z++)
          if (b.p[z] >= 0) sv[b.p[z]] = __builtin_fma(-lik, b.u[z], sv[b.p[z]]);
        // the rest of a longer U row: four loads of each kind in flight per lane
        for (int q0 = ub + R * WAVE + lane; q0 < b.kk.y; q0 += 4 * WAVE) {
          double v[4];
          int pq[4];
#pragma unroll
          for (int z = 0; z < 4; z++) {
            const int q = q0 + z * WAVE;
            pq[z] = -1;
            v[z] = 0.0;
            if (q < b.kk.y) {
              pq[z] = map[b.mo + (q - ub)];
              v[z] = ld_coh(val + q);
            }
          }
#pragma unroll
          for (int z = 0; z < 4; z++) {
            if (pq[z] >= 0)
              while (is_sentinel(v[z]) && keep_waiting(&spins, stall))
                v[z] = ld_coh(val + q0 + z * WAVE);
            if (pq[z] >= 0) sv[pq[z]] = __builtin_fma(-lik, v[z], sv[pq[z]]);
          }
        }
        wave_sync();
        sv[t] = lik;  // every lane writes the same value
        wave_sync();
      };
      Step buf[DEPTH];
#pragma unroll
      for (int d = 0; d < DEPTH; d++)
        if (wave + d * WPR < dl) load(buf[d], wave + d * WPR);
      __syncthreads();  // the row's values are staged
      if constexpr (TL) tl0 = tl1 = (long long)wall_clock64();
      for (int tb = 0; tb < dl; tb += AHEAD) {
#pragma unroll
        for (int d = 0; d < DEPTH; d++) {
          for (int w = 0; w < WPR; w++) {
            const int t = tb + d * WPR + w;
            if (t >= dl) break;
            if (w == wave) {
              step(buf[d], t);
              if (t + AHEAD < dl) load(buf[d], t + AHEAD);
            }
            __syncthreads();
          }
        }
      }
      // static pivoting of this row's pivot (rows of the dense block: there)
      if (thr > 0.0 && i < c0) {
        const int dr = diag[i] - rs;
        const double d = sv[dr];
        __syncthreads();
        if (fabs(d) < thr) {
          sv[dr] = perturb_pivot(d, thr);  // every thread writes the same value
          st->perturbed = 1;
        }
        __syncthreads();
      }
      for (int t = threadIdx.x; t < len; t += NT) st_coh(val + rs + t, sv[t]);
      if (TL && threadIdx.x == 0) tl_record(tl, i, tl0, tl1, 3);
      __syncthreads();  // the staging area is reused by the next row
    }
  }
}

// ---------------------------------------------------------------------------
// Sync-free refinement.  The stop test of every right-hand side runs on the
// device: each residual pass finishes its maxima in the workgroup that
// arrives last, which computes eta and raises the column's stop flag, and
// every later refinement kernel of that column returns at once.  The host
// therefore launches a fixed budget of iterations and never waits.  One
// Arnoldi step (operator product, both classical Gram-Schmidt passes, Givens
// update) is three fused passes whose dot products finish the same way, then
// one pass forms the next basis vector and the candidate solution.  Sums over
// workgroups are taken in a fixed order, so results do not depend on timing.
// ---------------------------------------------------------------------------
constexpr int FG_T = 256;  // threads per workgroup of the refinement passes
constexpr int FG_Q = 32;   // basis vectors a dot-product pass handles at most

__device__ __forceinline__ double eta_dev(double rn, double an, double xn) {
  const double den = an * xn;
  return den == 0.0 ? (rn == 0.0 ? 0.0 : __builtin_huge_val()) : rn / den;
}

__device__ __forceinline__ double bits_dev(unsigned long long b) {
  return __longlong_as_double((long long)b);
}

// The workgroup that arrives last at a fused reduction.  Every workgroup has
// stored its partial results with device-coherent stores; each thread waits
// for its stores, then thread 0 takes a ticket.  The workgroup holding ticket
// nb - 1 reads every partial with device-coherent loads and resets the
// counter for the next launch (launches on one stream never overlap).
__device__ bool fg_last_block(unsigned int* ticket, unsigned int nb) {
  __shared__ int last;
  stores_done();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int t =
        __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == nb - 1u) ? 1 : 0;
    if (last) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return last != 0;
}

// fg_last_block over two levels: workgroup b counts in at counter
// b % FG_TICK_GROUPS of tick1 (each on its own line, the group's workgroups
// share an XCD), the last of each group at ticket.  A thousand workgroups at
// one address serialise at the point of coherence (about 60 us at 1024);
// here each counter takes at most nb / FG_TICK_GROUPS of them.
__device__ bool fg_last_block2(unsigned int* ticket, unsigned int* tick1, unsigned int nb) {
  __shared__ int last;
  stores_done();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int G = (unsigned int)FG_TICK_GROUPS;
    const unsigned int g = blockIdx.x % G;
    const unsigned int ng = (nb - g + G - 1) / G;  // workgroups of group g
    unsigned int* t1 = tick1 + g * FG_TICK_STRIDE;
    last = 0;
    const unsigned int a =
        __hip_atomic_fetch_add(t1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a == ng - 1u) {
      __hip_atomic_store(t1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned int ngr = nb < G ? nb : G;
      const unsigned int t =
          __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (t == ngr - 1u) {
        last = 1;
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  __syncthreads();
  return last != 0;
}

// Workgroup sum (fixed order), valid in thread 0.
__device__ __forceinline__ double fg_block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();  // red may still be read by a previous call
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < FG_T / WAVE; q++) s += red[q];
  return s;
}

// Last workgroup: out[q] = sum over b < nb of pc[b * FG_Q + q] for q < nq, in
// a fixed order (eight slices of the workgroups, then the slices in order).
// Sum of the partials p[b * stride] for b = b0, b0 + step, ... below nb, added
// in that order, with eight device-coherent loads in flight at a time.
__device__ __forceinline__ double coh_sum(const double* p, int b0, int nb, int step, int stride) {
  double s = 0.0;
  for (int b = b0; b < nb; b += 8 * step) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const int bb = b + k * step;
      v[k] = bb < nb ? ld_coh(p + (size_t)bb * stride) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; k++)
      if (b + k * step < nb) s += v[k];
  }
  return s;
}

// As coh_sum, the NaN-propagating maximum.
__device__ __forceinline__ double coh_max(const double* p, int b0, int nb, int step, int stride) {
  double s = 0.0;
  for (int b = b0; b < nb; b += 8 * step) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const int bb = b + k * step;
      v[k] = bb < nb ? ld_coh(p + (size_t)bb * stride) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; k++) s = nanmax(s, v[k]);
  }
  return s;
}

__device__ void fg_reduce_q(const double* pc, int nb, int nq, double* out) {
  __shared__ double red[FG_T];
  const int q = threadIdx.x % FG_Q, k = threadIdx.x / FG_Q;
  double s = 0.0;
  if (q < nq) s = coh_sum(pc + q, k, nb, FG_T / FG_Q, FG_Q);
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < nq) {
    double t = 0.0;
    for (int kk = 0; kk < FG_T / FG_Q; kk++) t += red[kk * FG_Q + threadIdx.x];
    out[threadIdx.x] = t;
  }
}

// Stop test of column c after `it_now` iterations (0: the direct solve).
__device__ void fg_decide(FgState* fs, int c, int ncols, double eta, int it_now, int first,
                          const FgParams& p, int stalled) {
  FgCol* col = &fs->col[c];
  col->eta = eta;
  if (first) col->eta0 = eta;
  col->it = it_now;
  const int conv = eta <= p.eta_target ? 1 : 0;  // false for NaN
  col->conv = conv;
  const bool stop =
      (conv && it_now >= p.min_iters) || col->breakdown || it_now >= p.max_iters || stalled;
  if (stop && !col->stop) {
    col->stop = 1;
    if (atomicAdd(&fs->nstopped, 1) + 1 == ncols) fs->stop_all = 1;
  }
}

__global__ void k_fg_begin(FgState* fs, unsigned int* tick1, int reset_summary) {
  const int t = threadIdx.x;
  // first-level residual tickets (a stalled earlier pass may have left counts)
  for (int e = t; e < FG_MAX_COLS * FG_TICK_GROUPS; e += blockDim.x) tick1[e * FG_TICK_STRIDE] = 0u;
  if (t < FG_MAX_COLS) {
    FgCol* col = &fs->col[t];
    col->stop = 0;
    col->it = 0;
    col->breakdown = 0;
    col->conv = 0;
    col->eta = col->eta0 = col->hn = col->beta = 0.0;
    col->ticket = 0u;
  }
  if (t == 0) {
    fs->stop_all = 0;
    fs->nstopped = 0;
    if (reset_summary) {
      fs->it_max = 0;
      fs->not_conv = 0;
      fs->eta_max = 0ull;
      fs->eta0_max = 0ull;
    }
  }
}

// r = b - op(A) x for column c = blockIdx.y (all vectors column stride n), then
// the stop test from max |r|, max |x| and ||A|| (BATCH: r only; the
// per-instance test follows in k_fg_check_batch).  first: the check after the
// direct solve (runs even for a stopped column and records eta0).
template <bool BATCH>
__global__ __launch_bounds__(FG_T) void k_fg_resid(
    int n, const int* __restrict__ ptr, const int* __restrict__ idx, const int* __restrict__ pos,
    const double* __restrict__ aval, const double* __restrict__ b, const double* __restrict__ x,
    double* __restrict__ r, double* __restrict__ part, FgState* fs, unsigned int* tick1,
    const DevStats* st, int use_anorm1, int ncols, int it_now, int first, FgParams p, Inst in) {
  const int c = blockIdx.y;
  FgCol* col = &fs->col[c];
  if (!first && ld_flag(&col->stop)) return;
  const double* bc = b + (size_t)c * n;
  const double* xc = x + (size_t)c * n;
  double* rc = r + (size_t)c * n;
  const int lane = threadIdx.x % WAVE, g = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  double rm = 0.0, xm = 0.0;
  constexpr int U = 4;  // row groups per round, first loads all in flight
  const int stride = nw * (WAVE / RG);
  for (int r0 = wid * (WAVE / RG); r0 < n; r0 += U * stride) {
    int ii[U], t0[U], te[U];
    double sacc[U], av[U], xv[U];
    // a shared-pattern batch: the pattern's local entries, A values at
    // + ao, the instance's x at + xo
    int ao[U], xo[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      ii[u] = r0 + u * stride + g;
      t0[u] = 0;
      te[u] = 0;
      ao[u] = 0;
      xo[u] = 0;
      if (ii[u] < n) {
        const int ti = inst_of(ii[u], in);
        const int il = ii[u] - ti * in.n1;
        ao[u] = ti * in.a1;
        xo[u] = ti * in.n1;
        t0[u] = ptr[il] + gl;
        te[u] = ptr[il + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      av[u] = 0.0;
      xv[u] = 0.0;
      if (t0[u] < te[u]) {
        av[u] = aval[(pos ? pos[t0[u]] : t0[u]) + ao[u]];
        xv[u] = xc[idx[t0[u]] + xo[u]];
      }
    }
    // the rows' further entries, the U rows' loads in flight together (each
    // lane's sum still runs over its entries in order)
    int tt[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      sacc[u] = av[u] * xv[u];
      tt[u] = t0[u] + RG;
    }
    for (;;) {
      bool more = false;
#pragma unroll
      for (int u = 0; u < U; u++) {
        av[u] = 0.0;
        xv[u] = 0.0;
        if (tt[u] < te[u]) {
          av[u] = aval[(pos ? pos[tt[u]] : tt[u]) + ao[u]];
          xv[u] = xc[idx[tt[u]] + xo[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++)
        if (tt[u] < te[u]) {
          sacc[u] += av[u] * xv[u];
          tt[u] += RG;
          more = true;
        }
      if (!more) break;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const double su = group_sum(sacc[u]);
      const int i = ii[u];
      if (i < n) {
        const double ri = bc[i] - su;
        if (gl == 0) rc[i] = ri;
        rm = nanmax(rm, fabs(ri));
        xm = nanmax(xm, fabs(xc[i]));
      }
    }
  }
  if (BATCH) return;
  __shared__ double red[2][FG_T / WAVE];
  rm = block_nanmax(rm, red[0]);
  xm = block_nanmax(xm, red[1]);
  double* pc = part + (size_t)c * gridDim.x * 2;
  if (threadIdx.x == 0) {
    st_coh(pc + 2 * blockIdx.x, rm);
    st_coh(pc + 2 * blockIdx.x + 1, xm);
  }
  if (!fg_last_block2(&col->ticket, tick1 + (size_t)c * FG_TICK_GROUPS * FG_TICK_STRIDE, gridDim.x))
    return;
  double a = coh_max(pc, threadIdx.x, gridDim.x, FG_T, 2);
  double bm = coh_max(pc + 1, threadIdx.x, gridDim.x, FG_T, 2);
  a = block_nanmax(a, red[0]);
  bm = block_nanmax(bm, red[1]);
  if (threadIdx.x == 0) {
    const double an = bits_dev(use_anorm1 ? st->anorm1 : st->anorm);
    fg_decide(fs, c, ncols, eta_dev(a, an, bm), it_now, first, p, ld_flag(&st->stall));
  }
}

// Stop test of a block-diagonal batch (one column): eta = the largest
// instance eta from the per-instance maxima (anorm, max |r|, max |x|).
__global__ __launch_bounds__(FG_T) void k_fg_check_batch(int count, const double* __restrict__ inst,
                                                          FgState* fs, const DevStats* st,
                                                          int it_now, int first, FgParams p) {
  if (!first && ld_flag(&fs->col[0].stop)) return;
  __shared__ double red[FG_T / WAVE];
  double e = 0.0;
  for (int t = threadIdx.x; t < count; t += FG_T) {
    double m[3] = {0.0, 0.0, 0.0};
    for (int sl = 0; sl < SEG_SLICES; sl++)
      for (int k = 0; k < 3; k++) m[k] = nanmax(m[k], inst[3 * ((size_t)t * SEG_SLICES + sl) + k]);
    e = nanmax(e, eta_dev(m[1], m[0], m[2]));
  }
  e = block_nanmax(e, red);
  if (threadIdx.x == 0) fg_decide(fs, 0, 1, e, it_now, first, p, ld_flag(&st->stall));
}

// Start of an Arnoldi cycle: x = xt (copy: the cycle continues from the last
// candidate, whose residual r holds), beta = ||r||, g = (beta, 0, ...).
__global__ __launch_bounds__(FG_T) void k_fg_restart(int n, int m, const double* __restrict__ r,
                                                     const double* __restrict__ xt,
                                                     double* __restrict__ x, int copy,
                                                     double* __restrict__ part,
                                                     double* __restrict__ gvec, FgState* fs) {
  const int c = blockIdx.y;
  FgCol* col = &fs->col[c];
  if (ld_flag(&col->stop)) return;
  const size_t o = (size_t)c * n;
  double acc = 0.0;
  for (int t = blockIdx.x * FG_T + threadIdx.x; t < n; t += gridDim.x * FG_T) {
    if (copy) x[o + t] = xt[o + t];
    const double v = r[o + t];
    acc += v * v;
  }
  __shared__ double red[FG_T / WAVE];
  const double sb = fg_block_sum(acc, red);
  double* pc = part + (size_t)c * gridDim.x;
  if (threadIdx.x == 0) st_coh(pc + blockIdx.x, sb);
  if (!fg_last_block(&col->ticket, gridDim.x)) return;
  double a = coh_sum(pc, threadIdx.x, gridDim.x, FG_T, 1);
  a = fg_block_sum(a, red);
  if (threadIdx.x == 0) {
    const double beta = sqrt(a);
    col->beta = beta;
    double* gc = gvec + (size_t)c * (m + 1);
    gc[0] = beta;
    for (int i = 1; i <= m; i++) gc[i] = 0.0;
  }
}

// v0 = r / beta
__global__ __launch_bounds__(FG_T) void k_fg_v0(int n, const double* __restrict__ r,
                                                double* __restrict__ v0, const FgState* fs) {
  const int c = blockIdx.y;
  if (ld_flag(&fs->col[c].stop)) return;
  const double beta = fs->col[c].beta;
  const size_t o = (size_t)c * n;
  for (int t = blockIdx.x * FG_T + threadIdx.x; t < n; t += gridDim.x * FG_T)
    v0[o + t] = beta > 0.0 ? r[o + t] / beta : 0.0;
}

// Arnoldi step j, first pass: w = op(A) z_j and h[q] = v_q . w for q <= j.
// The 8 lanes of a row all hold w_i after the group sum; lane gl takes the
// basis vectors q = gl, gl + 8, gl + 16, gl + 24.  Basis vector q of column
// c starts at V + (q * g + c) * n.
__global__ __launch_bounds__(FG_T) void k_fg_arnoldi(
    int n, int g, int j, const int* __restrict__ ptr, const int* __restrict__ idx,
    const int* __restrict__ pos, const double* __restrict__ aval, const double* __restrict__ Zj,
    const double* __restrict__ V, double* __restrict__ w, double* __restrict__ part,
    double* __restrict__ hbuf, FgState* fs, Inst in) {
  const int c = blockIdx.y;
  FgCol* col = &fs->col[c];
  if (ld_flag(&col->stop)) return;
  const double* zc = Zj + (size_t)c * n;
  double* wc = w + (size_t)c * n;
  const double* vc = V + (size_t)c * n;
  const size_t vs = (size_t)g * n;
  const int lane = threadIdx.x % WAVE, grp = lane / RG, gl = lane % RG;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int nw = gridDim.x * blockDim.x / WAVE;
  double acc[FG_Q / RG] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = wid * (WAVE / RG); i0 < n; i0 += nw * (WAVE / RG)) {
    const int i = i0 + grp;
    double sacc = 0.0;
    if (i < n) {
      // a shared-pattern batch: the pattern's local entries, the instance's
      // A values and z
      const int ti = inst_of(i, in);
      const int il = i - ti * in.n1;
      const double* av = aval + ti * in.a1;
      const double* zt = zc + ti * in.n1;
      for (int t = ptr[il] + gl; t < ptr[il + 1]; t += RG) sacc += av[pos ? pos[t] : t] * zt[idx[t]];
    }
    const double wi = group_sum(sacc);
    if (i < n) {
      if (gl == 0) wc[i] = wi;
#pragma unroll
      for (int k = 0; k < FG_Q / RG; k++) {
        const int q = gl + RG * k;
        if (q <= j) acc[k] += vc[q * vs + i] * wi;
      }
    }
  }
  // lanes with the same gl (one per row group of the wave) hold the same q
#pragma unroll
  for (int k = 0; k < FG_Q / RG; k++)
    for (int off = RG; off < WAVE; off <<= 1) acc[k] += __shfl_xor(acc[k], off, WAVE);
  __shared__ double red[FG_T / WAVE][FG_Q];
  const int wv = threadIdx.x / WAVE;
  if (lane < RG)
#pragma unroll
    for (int k = 0; k < FG_Q / RG; k++) red[wv][lane + RG * k] = acc[k];
  __syncthreads();
  double* pc = part + (size_t)c * gridDim.x * FG_Q;
  if ((int)threadIdx.x <= j) {
    double s = 0.0;
    for (int q = 0; q < FG_T / WAVE; q++) s += red[q][threadIdx.x];
    st_coh(pc + (size_t)blockIdx.x * FG_Q + threadIdx.x, s);
  }
  if (!fg_last_block(&col->ticket, gridDim.x)) return;
  fg_reduce_q(pc, gridDim.x, j + 1, hbuf + c * FG_Q);
}

// Gram-Schmidt passes of step j.  MODE 0: w -= V h (h from the first pass),
// then h2[q] = v_q . w.  MODE 1: w -= V h2, then ||w||^2, and the last
// workgroup updates the least-squares problem: Hessenberg column j = h + h2,
// ||w|| below it, the earlier rotations applied, rotation j built, g rotated
// and y solved (j + 1 entries).  H is column-major (m + 1) x m per column.
template <int MODE>
__global__ __launch_bounds__(FG_T) void k_fg_cgs(
    int n, int g, int j, int m, const double* __restrict__ V, double* __restrict__ w,
    double* __restrict__ part, const double* __restrict__ hb, double* __restrict__ h2b,
    double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
    double* __restrict__ gvec, double* __restrict__ yv, FgState* fs) {
  const int c = blockIdx.y;
  FgCol* col = &fs->col[c];
  if (ld_flag(&col->stop)) return;
  const double* vc = V + (size_t)c * n;
  const size_t vs = (size_t)g * n;
  double* wc = w + (size_t)c * n;
  const double* hin = (MODE == 0 ? hb : h2b) + c * FG_Q;
  double hc[FG_Q];
#pragma unroll
  for (int q = 0; q < FG_Q; q++) hc[q] = q <= j ? hin[q] : 0.0;
  double acc[MODE == 0 ? FG_Q : 1];
#pragma unroll
  for (int q = 0; q < (MODE == 0 ? FG_Q : 1); q++) acc[q] = 0.0;
  for (int t = blockIdx.x * FG_T + threadIdx.x; t < n; t += gridDim.x * FG_T) {
    double wt = wc[t];
#pragma unroll
    for (int q = 0; q < FG_Q; q++)
      if (q <= j) wt -= hc[q] * vc[q * vs + t];
    wc[t] = wt;
    if (MODE == 0) {
#pragma unroll
      for (int q = 0; q < FG_Q; q++)
        if (q <= j) acc[q] += vc[q * vs + t] * wt;
    } else {
      acc[0] += wt * wt;
    }
  }
  if (MODE == 0) {
    __shared__ double red[FG_T / WAVE][FG_Q];
    const int wv = threadIdx.x / WAVE;
#pragma unroll
    for (int q = 0; q < FG_Q; q++)
      if (q <= j) {
        const double sq = wave_sum(acc[q]);
        if (threadIdx.x % WAVE == 0) red[wv][q] = sq;
      }
    __syncthreads();
    double* pc = part + (size_t)c * gridDim.x * FG_Q;
    if ((int)threadIdx.x <= j) {
      double s = 0.0;
      for (int q = 0; q < FG_T / WAVE; q++) s += red[q][threadIdx.x];
      st_coh(pc + (size_t)blockIdx.x * FG_Q + threadIdx.x, s);
    }
    if (!fg_last_block(&col->ticket, gridDim.x)) return;
    fg_reduce_q(pc, gridDim.x, j + 1, h2b + c * FG_Q);
  } else {
    __shared__ double red[FG_T / WAVE];
    const double sb = fg_block_sum(acc[0], red);
    double* pc = part + (size_t)c * gridDim.x;
    if (threadIdx.x == 0) st_coh(pc + blockIdx.x, sb);
    if (!fg_last_block(&col->ticket, gridDim.x)) return;
    double a = coh_sum(pc, threadIdx.x, gridDim.x, FG_T, 1);
    a = fg_block_sum(a, red);
    if (threadIdx.x != 0) return;
    double* Hc = H + (size_t)c * (m + 1) * m;
    double* csc = cs + (size_t)c * m;
    double* snc = sn + (size_t)c * m;
    double* gc = gvec + (size_t)c * (m + 1);
    double* yc = yv + (size_t)c * m;
    double* Hj = Hc + (size_t)j * (m + 1);
    for (int i = 0; i <= j; i++) Hj[i] = hb[c * FG_Q + i] + h2b[c * FG_Q + i];
    const double hn = sqrt(a);
    col->hn = hn;
    if (!(hn > 0.0)) col->breakdown = 1;
    Hj[j + 1] = hn;
    for (int i = 0; i < j; i++) {
      const double p0 = Hj[i], p1 = Hj[i + 1];
      Hj[i] = csc[i] * p0 + snc[i] * p1;
      Hj[i + 1] = -snc[i] * p0 + csc[i] * p1;
    }
    const double den = hypot(Hj[j], Hj[j + 1]);
    csc[j] = den > 0.0 ? Hj[j] / den : 1.0;
    snc[j] = den > 0.0 ? Hj[j + 1] / den : 0.0;
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    gc[j + 1] = -snc[j] * gc[j];
    gc[j] = csc[j] * gc[j];
    for (int i = j; i >= 0; i--) {
      double s = gc[i];
      for (int t = i + 1; t <= j; t++) s -= Hc[(size_t)t * (m + 1) + i] * yc[t];
      yc[i] = s / Hc[(size_t)i * (m + 1) + i];
    }
  }
}

// v_{j+1} = w / ||w|| (0 after a breakdown) and the candidate xt = x + Z y.
__global__ __launch_bounds__(FG_T) void k_fg_update(int n, int g, int j, int m,
                                                    const double* __restrict__ w,
                                                    double* __restrict__ vnext,
                                                    const double* __restrict__ Z,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ xt,
                                                    const double* __restrict__ yv,
                                                    const FgState* fs) {
  const int c = blockIdx.y;
  if (ld_flag(&fs->col[c].stop)) return;
  const double hn = fs->col[c].hn;
  double yc[FG_Q];
#pragma unroll
  for (int q = 0; q < FG_Q; q++) yc[q] = q <= j ? yv[(size_t)c * m + q] : 0.0;
  const size_t o = (size_t)c * n, zs = (size_t)g * n;
  for (int t = blockIdx.x * FG_T + threadIdx.x; t < n; t += gridDim.x * FG_T) {
    vnext[o + t] = hn > 0.0 ? w[o + t] / hn : 0.0;
    double s = x[o + t];
#pragma unroll
    for (int q = 0; q < FG_Q; q++)
      if (q <= j) s += yc[q] * Z[q * zs + o + t];
    xt[o + t] = s;
  }
}

// classical refinement step x += d for a running column
__global__ __launch_bounds__(FG_T) void k_fg_add(int n, const double* __restrict__ d,
                                                 double* __restrict__ x, const FgState* fs) {
  const int c = blockIdx.y;
  if (ld_flag(&fs->col[c].stop)) return;
  const size_t o = (size_t)c * n;
  for (int t = blockIdx.x * FG_T + threadIdx.x; t < n; t += gridDim.x * FG_T) x[o + t] += d[o + t];
}

// End of a group: FGMRES columns that iterated take the last candidate; every
// column folds its iterations and etas into the solve's summary.
__global__ __launch_bounds__(FG_T) void k_fg_finish(int n, const double* __restrict__ xt,
                                                    double* __restrict__ x, int ir, FgState* fs) {
  const int c = blockIdx.y;
  const FgCol* col = &fs->col[c];
  const int it = col->it;
  const size_t o = (size_t)c * n;
  if (!ir && it > 0)
    for (int t = blockIdx.x * FG_T + threadIdx.x; t < n; t += gridDim.x * FG_T) x[o + t] = xt[o + t];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicMax(&fs->it_max, it);
    if (!col->conv) atomicOr(&fs->not_conv, 1);
    atomicMax(&fs->eta_max, dbits(col->eta));
    atomicMax(&fs->eta0_max, dbits(col->eta0));
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void set_launch_gate(const int* gate) { t_gate = gate; }

bool set_debug_schedule(int on) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_debug_schedule), &on, sizeof(int)) == hipSuccess;
}

namespace {
// refinement passes: elementwise grids (four elements per thread at least)
// and row grids (eight lanes per row, four row groups per round)
int fg_grid(int n) { return std::max(1, std::min(FG_BLOCKS, cdiv(n, FG_T * 4))); }
// (the Arnoldi pass keeps FG_Q partial sums per workgroup and column: at most
// FG_BLOCKS workgroups fill the partial buffer of FG_BLOCKS x 32 per column)
int fg_rows_grid(int n) {
  static_assert(FG_Q <= 32, "Arnoldi partials exceed their buffer");
  return std::max(1, std::min(FG_BLOCKS, cdiv(n, (FG_T / WAVE) * (WAVE / RG) * 4)));
}
// the residual pass keeps two partial maxima per workgroup and column, so the
// same buffer holds FG_RESID_BLOCKS workgroups of them
int fg_resid_grid(int n) {
  static_assert(2 * FG_RESID_BLOCKS <= 32 * FG_BLOCKS, "residual partials exceed their buffer");
  return std::max(1, std::min(FG_RESID_BLOCKS, cdiv(n, (FG_T / WAVE) * (WAVE / RG) * 4)));
}
}  // namespace

void launch_fg_begin(const FgBufs& fb, int reset_summary, hipStream_t s) {
  hipLaunchKernelGGL(k_fg_begin, dim3(1), dim3(64), 0, s, fb.fs, fb.tick1, reset_summary);
}

void launch_fg_resid(int n, int ncols, const int* ptr, const int* idx, const int* pos,
                     const double* aval, const double* b, const double* x, double* r,
                     const FgBufs& fb, const DevStats* st, int use_anorm1, int it_now, int first,
                     int batch, const FgParams& p, hipStream_t s, Inst in) {
  // a single system's pass ends in the last-workgroup ticket: 1024 workgroups
  // there (70k buses, solve ms: 4096 1.24, 1024 1.23, 256 1.33); a batch pass
  // has no ticket and keeps the full grid
  const dim3 grid(batch ? fg_resid_grid(n) : std::min(1024, fg_resid_grid(n)), ncols);
  if (batch)
    hipLaunchKernelGGL(k_fg_resid<true>, grid, dim3(FG_T), 0, s, n, ptr, idx, pos, aval, b, x, r,
                       fb.part, fb.fs, fb.tick1, st, use_anorm1, ncols, it_now, first, p, in);
  else
    hipLaunchKernelGGL(k_fg_resid<false>, grid, dim3(FG_T), 0, s, n, ptr, idx, pos, aval, b, x, r,
                       fb.part, fb.fs, fb.tick1, st, use_anorm1, ncols, it_now, first, p, in);
}

void launch_fg_check_batch(int count, const double* inst, const FgBufs& fb, const DevStats* st,
                           int it_now, int first, const FgParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_fg_check_batch, dim3(1), dim3(FG_T), 0, s, count, inst, fb.fs, st, it_now,
                     first, p);
}

void launch_fg_restart(int n, int ncols, int m, const double* r, const double* xt, double* x,
                       int copy, double* v0, const FgBufs& fb, hipStream_t s) {
  const dim3 grid(fg_grid(n), ncols);
  hipLaunchKernelGGL(k_fg_restart, grid, dim3(FG_T), 0, s, n, m, r, xt, x, copy, fb.part, fb.gvec,
                     fb.fs);
  hipLaunchKernelGGL(k_fg_v0, grid, dim3(FG_T), 0, s, n, r, v0, (const FgState*)fb.fs);
}

void launch_fg_arnoldi(int n, int ncols, int j, const int* ptr, const int* idx, const int* pos,
                       const double* aval, const double* Zj, const double* V, double* w,
                       const FgBufs& fb, hipStream_t s, Inst in) {
  hipLaunchKernelGGL(k_fg_arnoldi, dim3(fg_rows_grid(n), ncols), dim3(FG_T), 0, s, n, ncols, j,
                     ptr, idx, pos, aval, Zj, V, w, fb.part, fb.hbuf, fb.fs, in);
}

void launch_fg_cgs(int pass, int n, int ncols, int j, int m, const double* V, double* w,
                   const FgBufs& fb, hipStream_t s) {
  const dim3 grid(fg_grid(n), ncols);
  if (pass == 0)
    hipLaunchKernelGGL(k_fg_cgs<0>, grid, dim3(FG_T), 0, s, n, ncols, j, m, V, w, fb.part,
                       (const double*)fb.hbuf, fb.h2buf, fb.H, fb.cs, fb.sn, fb.gvec, fb.y, fb.fs);
  else
    hipLaunchKernelGGL(k_fg_cgs<1>, grid, dim3(FG_T), 0, s, n, ncols, j, m, V, w, fb.part,
                       (const double*)fb.hbuf, fb.h2buf, fb.H, fb.cs, fb.sn, fb.gvec, fb.y, fb.fs);
}

void launch_fg_update(int n, int ncols, int j, int m, const double* w, double* vnext,
                      const double* Z, const double* x, double* xt, const FgBufs& fb,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_fg_update, dim3(fg_grid(n), ncols), dim3(FG_T), 0, s, n, ncols, j, m, w,
                     vnext, Z, x, xt, (const double*)fb.y, (const FgState*)fb.fs);
}

void launch_fg_add(int n, int ncols, const double* d, double* x, const FgBufs& fb, hipStream_t s) {
  hipLaunchKernelGGL(k_fg_add, dim3(fg_grid(n), ncols), dim3(FG_T), 0, s, n, d, x,
                     (const FgState*)fb.fs);
}

void launch_fg_finish(int n, int ncols, const double* xt, double* x, int ir, const FgBufs& fb,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_fg_finish, dim3(fg_grid(n), ncols), dim3(FG_T), 0, s, n, xt, x, ir, fb.fs);
}

void launch_refactor_rows(const LUView& lu, const int* rows, int nrows, int maxlen,
                          const double* aval, DevStats* st, double prel, hipStream_t s) {
  if (nrows <= 0) return;
  if (maxlen <= 128) {
    constexpr int W = 4;
    hipLaunchKernelGGL((k_refactor_rows_lds<128, W>), dim3(cdiv(nrows, W)), dim3(W * WAVE), 0, s,
                       rows, nrows, lu.rowptr, lu.col, lu.diag, lu.src, aval, lu.val, st, prel);
  } else if (maxlen <= 1024) {
    constexpr int W = 2;
    hipLaunchKernelGGL((k_refactor_rows_lds<1024, W>), dim3(cdiv(nrows, W)), dim3(W * WAVE), 0, s,
                       rows, nrows, lu.rowptr, lu.col, lu.diag, lu.src, aval, lu.val, st, prel);
  } else if (maxlen <= 4096) {
    hipLaunchKernelGGL((k_refactor_rows_lds<4096, 1>), dim3(nrows), dim3(WAVE), 0, s, rows, nrows,
                       lu.rowptr, lu.col, lu.diag, lu.src, aval, lu.val, st, prel);
  } else {
    hipLaunchKernelGGL(k_refactor_rows_global, dim3(nrows), dim3(WAVE), 0, s, rows, nrows,
                       lu.rowptr, lu.col, lu.diag, lu.src, aval, lu.val, st, prel);
  }
}

void launch_pivot_stats(const LUView& lu, DevStats* st, double tiny_rel, double* red,
                        hipStream_t s, Inst in) {
  // 70k buses, us: 2048 workgroups 35 + 6 (final pass), 1024 43 + 4; one
  // pass ending in same-address atomics from all 1024 workgroups: 69
  const int total = lu.n * in.count, nb = std::max(1, std::min(cdiv(total, 32), 2048));
  static_assert(4 * 2048 <= RED_SCRATCH, "pivot statistics partials exceed their buffer");
  hipLaunchKernelGGL(k_pivot_stats, dim3(nb), dim3(256), 0, s, total, lu.rowptr, lu.diag, lu.val,
                     st, tiny_rel, red, in);
  hipLaunchKernelGGL(k_pivot_stats_final, dim3(1), dim3(256), 0, s, nb, (const double*)red, st);
}

// Row passes with a two-stage maximum (red != nullptr): a larger grid keeps
// more loads in flight without same-address atomics at its end (at 70k buses
// the residual pass drops from 88 to 61 + 6 us; the A copy, bound by its
// scattered stores, gains nothing and keeps the single pass).
constexpr int RED_BLOCKS = 4096;
inline int rows_grid_red(int n) { return std::max(1, std::min(cdiv(n, 32), RED_BLOCKS)); }

void launch_copy_anorm(int n, const int* arow, const int*, const double* src, double* dst,
                       DevStats* st, hipStream_t s, SyncState* ss, double* rowabs,
                       const int* a2lu, double* luA, double* red, int fnorm,
                       const double* ascale, double* avs, Inst in) {
  const int total = n * in.count;
  const int nb = red ? rows_grid_red(total) : rows_grid(total);
  hipLaunchKernelGGL(in.count > 1 ? k_copy_anorm<true> : k_copy_anorm<false>, dim3(nb), dim3(256),
                     0, s, total, arow, src, dst, st, ss, rowabs, a2lu, luA, red, fnorm, ascale,
                     avs, in);
  if (red)
    hipLaunchKernelGGL(k_red_max, dim3(1), dim3(1024), 0, s, (const double*)red, nb,
                       fnorm ? 2 : 1, &st->anorm, fnorm ? &st->anorm_f : &st->anorm);
}

void launch_seg_stats(int count, const int* row_off, const double* matabs, const double* r,
                      const double* x, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_stats, dim3(SEG_SLICES, count), dim3(256), 0, s, t_gate, row_off, matabs,
                     r, x, out);
}

void launch_fill_sentinel(double* p, long long count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_sentinel, dim3((unsigned)std::min<long long>(4096, (count + 255) / 256)),
                     dim3(256), 0, s, p, count);
}

void launch_refactor_trivial(const LUView& lu, const int* rows, int nrows, const double* aval,
                             int* ready, const SyncState* ss, hipStream_t s, const double* luA,
                             int c0, DevStats* st, double perturb_rel, Inst in) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_refactor_trivial,
                     dim3(std::max(1, std::min(cdiv((long)nrows * in.count, 32), 2048))),
                     dim3(256), 0, s, nrows, rows, lu.rowptr, lu.src, aval, lu.val, ready, ss,
                     luA, lu.diag, c0, st, perturb_rel, in);
}

void launch_build_refmap(const LUView& lu, const int* moff, unsigned short* map,
                         const unsigned char* flat, hipStream_t s) {
  hipLaunchKernelGGL(k_build_refmap, dim3(std::max(1, std::min(cdiv(lu.n, 4), 4096))), dim3(256),
                     0, s, lu.n, lu.rowptr, lu.col, lu.diag, moff, map, flat);
}

bool launch_refactor_wg(const LUView& lu, const int* order, const int* cstart, int nchunks,
                        int band, int cap, SyncState* ss, int* stall, int c0, const int* dlc,
                        const int* moff, const unsigned short* map, const double* luA,
                        const int2* pbnd, int max_waves_per_cu, DevStats* st, double perturb_rel,
                        hipStream_t s, long long* tl, Inst in) {
  if (nchunks <= 0) return true;
  if (band < 0 || band >= REF_MAX_BANDS || !dlc || !moff || !map || !luA || !pbnd) return false;
  constexpr int WPR = KKTLU_WG_WPR, DEPTH = KKTLU_WG_DEPTH;
  const size_t shm = (size_t)std::max(cap, 1) * sizeof(double);
  if (shm > 64 * 1024) return false;
  static int ncu = 0;
  if (ncu == 0) {
    int d = 0;
    (void)hipGetDevice(&d);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d);
    if (ncu <= 0) ncu = 256;
  }
  // the timeline is recorded by its own instantiation (no cost otherwise),
  // for single systems and block-diagonal batches
  if (in.count > 1) tl = nullptr;
  auto kern = in.count > 1 ? k_refactor_wg<WPR, DEPTH, false, true>
               : tl          ? k_refactor_wg<WPR, DEPTH, true, false>
                             : k_refactor_wg<WPR, DEPTH, false, false>;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, WPR * WAVE, shm) != hipSuccess ||
      nb <= 0)
    nb = 1;
  if (max_waves_per_cu > 0) nb = std::max(1, std::min(nb, max_waves_per_cu / WPR));
  const int grid = std::max(1, (int)std::min<long>(nb * ncu, (long)nchunks * in.count));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WPR * WAVE), shm, s, order, cstart, nchunks,
                     ss->band_stream[band], std::min(TICKET_STREAMS, grid), lu.rowptr, dlc, lu.val,
                     stall, moff, map, luA, pbnd, lu.diag, c0, st, perturb_rel, tl, in);
  return true;
}

bool launch_refactor_flat(const LUView& lu, const int* cstart, int nchunks, int band, int cap,
                          SyncState* ss, int* stall, const int4* rmeta,
                          const unsigned short* map, const double* luA, const int2* fl,
                          const unsigned char* cmicro, int max_waves_per_cu, DevStats* st,
                          double perturb_rel, hipStream_t s, const int* order, long long* tl,
                          Inst in) {
  if (nchunks <= 0) return true;
  if (band < 0 || band >= REF_MAX_BANDS || cap > 256 || !rmeta || !map || !luA || !fl)
    return false;
  cap = (cap + 1) & ~1;
  constexpr int WPB = 4;
  const size_t shm = (size_t)flat_area(cap) * sizeof(double) * WPB;
  static int ncu = 0;
  if (ncu == 0) {
    int d = 0;
    (void)hipGetDevice(&d);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d);
    if (ncu <= 0) ncu = 256;
  }
  if (in.count > 1) tl = nullptr;
  auto kern = in.count > 1 ? k_refactor_flat<WPB, false, true>
               : tl          ? k_refactor_flat<WPB, true, false>
                             : k_refactor_flat<WPB, false, false>;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, WPB * WAVE, shm) != hipSuccess ||
      nb <= 0)
    nb = 1;
  if (max_waves_per_cu > 0) nb = std::max(1, std::min(nb, max_waves_per_cu / WPB));
  const int grid = std::max(1, std::min(nb * ncu, cdiv((long)nchunks * in.count, WPB)));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WPB * WAVE), shm, s, cstart, nchunks,
                     ss->band_stream[band], std::min(TICKET_STREAMS, grid), lu.val, stall, cap,
                     rmeta, map, luA, fl, cmicro, st, perturb_rel, order, tl, in);
  return true;
}

bool launch_refactor_syncfree(const LUView& lu, const int* order, const int* cstart,
                              int nchunks, int band, int cap, const double* aval, int* ready,
                              SyncState* ss, int* stall, bool light, int wpb_pref, int c0,
                              const int* moff, const unsigned short* map, const double* luA,
                              const int2* pbnd, int max_waves_per_cu, DevStats* st,
                              double perturb_rel, hipStream_t s) {
  if (nchunks <= 0) return true;
  if (band < 0 || band >= REF_MAX_BANDS) return false;
  cap = (cap + 1) & ~1;
  const size_t per_wave = (size_t)cap * (sizeof(double) + sizeof(int2) + sizeof(int));
  if (per_wave > 64 * 1024) return false;
  static int ncu = 0;
  if (ncu == 0) {
    int d = 0;
    (void)hipGetDevice(&d);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d);
    if (ncu <= 0) ncu = 256;
  }
  auto go = [&](auto kernel, int wpb) {
    const size_t shm = per_wave * wpb;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, wpb * WAVE, shm) != hipSuccess ||
        nb <= 0)
      nb = 1;
    if (max_waves_per_cu > 0) nb = std::max(1, std::min(nb, max_waves_per_cu / wpb));
    const int grid = std::max(1, std::min(nb * ncu, cdiv(nchunks, wpb)));
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(wpb * WAVE), shm, s, order, cstart, nchunks,
                       ss->band_stream[band], std::min(TICKET_STREAMS, grid), lu.rowptr, lu.col,
                       lu.diag, lu.src, aval, lu.val,
                       ready, ss, stall, cap, c0, moff, map, luA, pbnd, st, perturb_rel);
  };
  // waves per block: the preference if its LDS fits in 64 KiB, else the
  // largest of 4, 2, 1 that fits (4 only for rows short enough for 32 KiB)
  int wpb = 1;
  if (wpb_pref > 0) {
    wpb = wpb_pref;
    while (wpb > 1 && per_wave * wpb > 64 * 1024) wpb >>= 1;
  } else if (per_wave * 4 <= 32 * 1024) {
    wpb = 4;
  } else if (per_wave * 2 <= 64 * 1024) {
    wpb = 2;
  }
  const bool mapped = moff != nullptr && map != nullptr;
#define RF_GO(W, L)                                   \
  do {                                                \
    if (mapped)                                       \
      go(k_refactor_syncfree<W, L, true>, W);         \
    else                                              \
      go(k_refactor_syncfree<W, L, false>, W);        \
  } while (0)
  if (light) {
    if (wpb == 4)
      RF_GO(4, true);
    else if (wpb == 2)
      RF_GO(2, true);
    else
      RF_GO(1, true);
  } else {
    if (wpb == 4)
      RF_GO(4, false);
    else if (wpb == 2)
      RF_GO(2, false);
    else
      RF_GO(1, false);
  }
#undef RF_GO
  return true;
}

void launch_trisolve_syncfree(int mode, const LUView& lu, const ChunkSched& cs, const int* tptr,
                              const int* trow, const int* tpos, double* y, int* ready,
                              SyncState* ss, int slot, int* stall, hipStream_t s) {
  if (cs.nchunks <= 0) return;
  static int ncu = 0;
  if (ncu == 0) {
    int d = 0;
    (void)hipGetDevice(&d);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d);
    if (ncu <= 0) ncu = 256;
  }
  const int grid = std::max(1, std::min(ncu * cs.blocks_per_cu, cdiv(cs.nchunks, 4)));
#define TS_LAUNCH(M)                                                                            \
  hipLaunchKernelGGL(k_trisolve_syncfree<M>, dim3(grid), dim3(256), 0, s, t_gate, lu.n, cs.nchunks,       \
                     cs.start, \
                     cs.meta, cs.rows, lu.rowptr, lu.col, lu.diag, tptr, trow, tpos, lu.val, y, \
                     ready, ss, slot, stall)
  switch (mode) {
    case 0: TS_LAUNCH(0); break;
    case 1: TS_LAUNCH(1); break;
    case 2: TS_LAUNCH(2); break;
    default: TS_LAUNCH(3); break;
  }
#undef TS_LAUNCH
}

void launch_trisolve_vflag(int mode, const LUView& lu, const ChunkSched& cs, const int* tptr,
                           const int* trow, const int* tpos, const double* c, double* y,
                           SyncState* ss, int slot, int* stall, hipStream_t s) {
  if (cs.nchunks <= 0) return;
  static int ncu = 0;
  if (ncu == 0) {
    int d = 0;
    (void)hipGetDevice(&d);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d);
    if (ncu <= 0) ncu = 256;
  }
  const int grid = std::max(1, std::min(ncu * cs.blocks_per_cu, cdiv(cs.nchunks, 4)));
#define TV_LAUNCH(M)                                                                          \
  hipLaunchKernelGGL(k_trisolve_vflag<M>, dim3(grid), dim3(256), 0, s, t_gate, lu.n, cs.nchunks,      \
                     cs.start, cs.meta, cs.rows, lu.rowptr, lu.col, lu.diag, tptr, trow, tpos, \
                     lu.val, c, y, ss, slot, stall)
  switch (mode) {
    case 0: TV_LAUNCH(0); break;
    case 1: TV_LAUNCH(1); break;
    case 2: TV_LAUNCH(2); break;
    default: TV_LAUNCH(3); break;
  }
#undef TV_LAUNCH
}

void launch_trisolve_vflag_mr(int mode, int nr, const LUView& lu, const ChunkSched& cs,
                              const int* tptr, const int* trow, const int* tpos, const double* c,
                              double* y, SyncState* ss, int slot, int* stall, hipStream_t s) {
  if (cs.nchunks <= 0 || nr <= 0) return;
  static int ncu = 0;
  if (ncu == 0) {
    int d = 0;
    (void)hipGetDevice(&d);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d);
    if (ncu <= 0) ncu = 256;
  }
  const int grid = std::max(1, std::min(ncu * cs.blocks_per_cu, cdiv(cs.nchunks, 4)));
  const int ld = lu.n + 1;
#define TM_LAUNCH(M, R)                                                                        \
  hipLaunchKernelGGL((k_trisolve_vflag_mr<M, R>), dim3(grid), dim3(256), 0, s, t_gate, lu.n, nr, ld,   \
                     cs.nchunks, cs.start, cs.meta, cs.rows, lu.rowptr, lu.col, lu.diag, tptr, \
                     trow, tpos, lu.val, c, y, ss, slot, stall)
#define TM_MODES(R)                 \
  switch (mode) {                   \
    case 0: TM_LAUNCH(0, R); break; \
    case 1: TM_LAUNCH(1, R); break; \
    case 2: TM_LAUNCH(2, R); break; \
    default: TM_LAUNCH(3, R); break; \
  }
  if (nr <= 4) {
    TM_MODES(4)
  } else if (nr <= 8) {
    TM_MODES(8)
  } else {
    TM_MODES(MAX_RHS_PASS)
  }
#undef TM_MODES
#undef TM_LAUNCH
}

void launch_tail_scatter(const LUView& lu, int c0, int s, int S, double* T, hipStream_t st) {
  if (s <= 0) return;
  hipLaunchKernelGGL(k_tail_scatter, dim3(cdiv(S, 4)), dim3(256), 0, st, c0, s, S, lu.rowptr,
                     lu.col, lu.val, T);
}

std::vector<int> dense_lu_tasks(int nt) {
  std::vector<int> t;
  auto code = [](int type, int i, int j, int k) { return type << 21 | i << 14 | j << 7 | k; };
  auto panel = [&](int k) {
    for (int i = k + 1; i < std::max(nt, k + 2); i++) t.push_back(code(0, i, 0, k));
  };
  panel(0);
  for (int k = 0; k + 1 < nt; k++) {
    const int n1 = k + 1;
    // the next panel's tiles, then that panel, then the rest of step k
    t.push_back(code(1, n1, n1, k));
    for (int r = n1 + 1; r < nt; r++) {
      t.push_back(code(1, r, n1, k));
      t.push_back(code(1, n1, r, k));
    }
    panel(n1);
    for (int i = n1 + 1; i < nt; i++)
      for (int j = n1 + 1; j < nt; j++) t.push_back(code(1, i, j, k));
  }
  return t;
}

void launch_dlu_reset(int* ver, int nt, SyncState* ss, hipStream_t st) {
  hipLaunchKernelGGL(k_dlu_reset, dim3(std::max(1, cdiv(nt * nt, 256))), dim3(256), 0, st, ver,
                     nt * nt, ss);
}

bool launch_dense_lu_tasks(double* T, int S, int s, const int* tasks, int ntasks, int* ver,
                           double* Dk, SyncState* ss, int* stall, DevStats* stats, double prel,
                           hipStream_t st) {
  if (S <= 0 || S % DLU_NB != 0 || S / DLU_NB > 64) return false;
  auto kern = k_dlu_tasks<DLU_NB, KKTLU_DLU_CHUNK>;
  static int ncu = 0, occ = 0;
  if (ncu == 0) {
    int d = 0;
    (void)hipGetDevice(&d);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d);
    if (ncu <= 0) ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern),
                                                     256, 0) != hipSuccess ||
        occ <= 0)
      occ = 1;
  }
  // every workgroup resident (each ticket stream needs a running workgroup)
  const int nt = S / DLU_NB;
  const int grid = std::max(1, std::min(ncu * occ, ntasks));
  const int nstreams = std::min(TICKET_STREAMS, grid);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, T, S, s, nt, tasks, ntasks, ver, Dk, ss,
                     nstreams, stall, stats, prel);
  hipLaunchKernelGGL(k_dlu_install<DLU_NB>, dim3(nt), dim3(256), 0, st, T, S, (const double*)Dk);
  return true;
}

void launch_tail_gather(const LUView& lu, int c0, const double* T, int S, hipStream_t st) {
  const int s = lu.n - c0;
  if (s <= 0) return;
  hipLaunchKernelGGL(k_tail_gather, dim3(cdiv(s, 4)), dim3(256), 0, st, c0, s, S, lu.rowptr,
                     lu.col, T, lu.val);
}

void launch_dense_lu(double* T, int S, int s, double* dsc, DevStats* stats, double prel,
                     hipStream_t st) {
  for (int k0 = 0; k0 < S; k0 += DLU_NB) {
    const int rest = S - k0 - DLU_NB;
    hipLaunchKernelGGL((k_dlu_panel<DLU_NB, KKTLU_DLU_CHUNK>), dim3(std::max(1, cdiv(rest, DLU_NB))),
                       dim3(2 * WAVE), 0, st, T, S, k0, rest, dsc, s, stats, prel);
    const int nt = std::max(1, cdiv(rest, KKTLU_DLU_TILE));
    hipLaunchKernelGGL((k_dlu_update<DLU_NB, KKTLU_DLU_TILE>), dim3(nt, nt), dim3(256), 0, st, T, S,
                       k0, (const double*)dsc);
  }
}

void launch_trisolve_sn(int mode, int nr, const LUView& lu, const SnSched& sn, const int* tptr,
                        const int* trow, const int* tpos, const double* c, double* y,
                        SyncState* ss, int slot, int* stall, hipStream_t s, const int* xend,
                        const double* pre, Inst in) {
  if (mode != 1 || nr != 1 || in.count > 1) {
    xend = nullptr;
    pre = nullptr;
  }
  if (sn.nchunks <= 0 || nr <= 0) return;
  static int ncu = 0;
  if (ncu == 0) {
    int d = 0;
    (void)hipGetDevice(&d);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d);
    if (ncu <= 0) ncu = 256;
  }
  // every workgroup resident at once (the ticket streams need a running
  // workgroup each): at most the occupancy limit per CU
  static int occ[4][4] = {};
  const bool sh = in.count > 1;
  const int ri = sh ? 3 : (nr == 1 ? 0 : (nr <= 4 ? 1 : 2));
  int& nb = occ[mode & 3][ri];
  if (nb == 0) {
    auto probe = [&](const void* k) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, 0) != hipSuccess || nb <= 0)
        nb = 1;
    };
#define SN_OCC(M, R, S) probe(reinterpret_cast<const void*>(&k_trisolve_sn<M, R, S>))
#define SN_OCC_R(M)                  \
  if (ri == 3) SN_OCC(M, 1, true);   \
  else if (ri == 0) SN_OCC(M, 1, false); \
  else if (ri == 1) SN_OCC(M, 4, false); \
  else SN_OCC(M, SN_MAX_RHS, false)
    switch (mode) {
      case 0: SN_OCC_R(0); break;
      case 1: SN_OCC_R(1); break;
      case 2: SN_OCC_R(2); break;
      default: SN_OCC_R(3); break;
    }
#undef SN_OCC_R
#undef SN_OCC
  }
  if (in.count > 1 && nr != 1) return;  // instances carry one right-hand side each
  const int grid = std::max(
      1, std::min(ncu * std::min(sn.blocks_per_cu, nb), cdiv((long)sn.nchunks * in.count, 4)));
  const int nstreams = std::min(TICKET_STREAMS, grid);
  const int ld = lu.n + 1;
#define SN_LAUNCH(M, R, S)                                                                      \
  hipLaunchKernelGGL((k_trisolve_sn<M, R, S>), dim3(grid), dim3(256), 0, s, t_gate, lu.n, nr, ld,       \
                     sn.nchunks, sn.start, sn.meta, sn.base, sn.rows, sn.split, lu.rowptr,       \
                     lu.col, lu.diag, tptr, trow, tpos, lu.val, c, y, ss, slot, nstreams, stall, \
                     xend, pre, in)
#define SN_MODES_S(R, S)               \
  switch (mode) {                      \
    case 0: SN_LAUNCH(0, R, S); break; \
    case 1: SN_LAUNCH(1, R, S); break; \
    case 2: SN_LAUNCH(2, R, S); break; \
    default: SN_LAUNCH(3, R, S); break; \
  }
#define SN_MODES(R) SN_MODES_S(R, false)
  if (sh) {
    SN_MODES_S(1, true)
  } else if (nr == 1) {
    SN_MODES(1)
  } else if (nr <= 4) {
    SN_MODES(4)
  } else {
    SN_MODES(SN_MAX_RHS)
  }
#undef SN_MODES
#undef SN_MODES_S
#undef SN_LAUNCH
}

void launch_tail_solve(int mode, int nr, const LUView& lu, const double* T, int S, int s, int c0,
                       const int* split, const int* tptr, const int* trow, const int* tpos,
                       const double* c, double* rhs_buf, double* y, hipStream_t st) {
  if (s <= 0 || S > DENSE_TAIL_MAX || nr <= 0) return;
  const int ld = lu.n + 1;
  for (int r0 = 0; r0 < nr; r0 += TAIL_NR) {
    const int k = std::min(TAIL_NR, nr - r0);
    const double* cr = c + (size_t)r0 * ld;
    double* yr = y + (size_t)r0 * ld;
    const double* rhs = cr + c0;
    int rld = ld;
    if (mode == 0 || mode == 2) {
      if (mode == 0)
        hipLaunchKernelGGL(k_tail_ext<0>, dim3(cdiv(S, 4), k), dim3(256), 0, st, t_gate, c0, s, S, k, ld,
                           split, lu.rowptr, lu.col, tptr, trow, tpos, lu.val, cr, yr, rhs_buf);
      else
        hipLaunchKernelGGL(k_tail_ext<2>, dim3(cdiv(S, 4), k), dim3(256), 0, st, t_gate, c0, s, S, k, ld,
                           split, lu.rowptr, lu.col, tptr, trow, tpos, lu.val, cr, yr, rhs_buf);
      rhs = rhs_buf;
      rld = S;
    }
    const size_t shm = (size_t)k * S * sizeof(double);
    static bool attr_set = false;
    const int mx = TAIL_NR * DENSE_TAIL_MAX * (int)sizeof(double);
#define TT_ATTR(M, R)                                                                   \
  (void)hipFuncSetAttribute((const void*)k_tail_trsv<M, R>,                             \
                            hipFuncAttributeMaxDynamicSharedMemorySize, mx)
    if (!attr_set) {
      TT_ATTR(0, 1); TT_ATTR(1, 1); TT_ATTR(2, 1); TT_ATTR(3, 1);
      TT_ATTR(0, TAIL_NR); TT_ATTR(1, TAIL_NR); TT_ATTR(2, TAIL_NR); TT_ATTR(3, TAIL_NR);
      attr_set = true;
    }
#undef TT_ATTR
#define TT_LAUNCH(M, R)                                                                          \
  hipLaunchKernelGGL((k_tail_trsv<M, R>), dim3(1), dim3(1024), shm, st, t_gate, T, S, s, c0, k, rhs, rld, \
                     yr, ld)
#define TT_MODES(R)                 \
  switch (mode) {                   \
    case 0: TT_LAUNCH(0, R); break; \
    case 1: TT_LAUNCH(1, R); break; \
    case 2: TT_LAUNCH(2, R); break; \
    default: TT_LAUNCH(3, R); break; \
  }
    if (k == 1) {
      TT_MODES(1)
    } else {
      TT_MODES(TAIL_NR)
    }
#undef TT_MODES
#undef TT_LAUNCH
  }
}

void launch_udense_pre(int nu, const int* urows, const int* xend, const LUView& lu, const double* y,
                       double* pre, hipStream_t st) {
  if (nu <= 0) return;
  hipLaunchKernelGGL(k_udense_pre, dim3(std::max(1, std::min(cdiv(nu, 32), 2048))), dim3(256), 0,
                     st, t_gate, nu, urows, xend, lu.rowptr, lu.col, lu.val, y, pre);
}

void launch_tail_solve_mw(int mode, const LUView& lu, const double* T, int S, int s, int c0,
                          const int* split, const int* tptr, const int* trow, const int* tpos,
                          const double* c, double* rhs_buf, double* y, int* stall,
                          hipStream_t st) {
  if (s <= 0 || S > DENSE_TAIL_MAX || S % TB != 0) return;
  const int ld = lu.n + 1;
  const double* rhs = c + c0;
  if (mode == 0 || mode == 2) {
    if (mode == 0)
      hipLaunchKernelGGL(k_tail_ext<0>, dim3(cdiv(S, 4), 1), dim3(256), 0, st, t_gate, c0, s, S, 1, ld,
                         split, lu.rowptr, lu.col, tptr, trow, tpos, lu.val, c, y, rhs_buf);
    else
      hipLaunchKernelGGL(k_tail_ext<2>, dim3(cdiv(S, 4), 1), dim3(256), 0, st, t_gate, c0, s, S, 1, ld,
                         split, lu.rowptr, lu.col, tptr, trow, tpos, lu.val, c, y, rhs_buf);
    rhs = rhs_buf;
  }
  const int nb = S / TB;
  switch (mode) {
    case 0:
      hipLaunchKernelGGL(k_tail_mw<0>, dim3(nb), dim3(256), 0, st, t_gate, T, S, s, c0, rhs, y, stall);
      break;
    case 1:
      hipLaunchKernelGGL(k_tail_mw<1>, dim3(nb), dim3(256), 0, st, t_gate, T, S, s, c0, rhs, y, stall);
      break;
    case 2:
      hipLaunchKernelGGL(k_tail_mw<2>, dim3(nb), dim3(256), 0, st, t_gate, T, S, s, c0, rhs, y, stall);
      break;
    default:
      hipLaunchKernelGGL(k_tail_mw<3>, dim3(nb), dim3(256), 0, st, t_gate, T, S, s, c0, rhs, y, stall);
      break;
  }
}

void launch_trisolve_seg(int mode, const SegSched& sg, const double* val, const double* c,
                         double* y, hipStream_t s) {
  if (sg.nlev <= 0) return;
#define SG_LAUNCH(M)                                                                             \
  hipLaunchKernelGGL(k_trisolve_seg<M>, dim3(1), dim3(SEG_THREADS), 0, s, t_gate, sg.nlev, sg.lev_ptr, \
                     sg.row, sg.ptr, sg.src, sg.vpos, sg.dpos, val, c, y)
  switch (mode) {
    case 0: SG_LAUNCH(0); break;
    case 1: SG_LAUNCH(1); break;
    case 2: SG_LAUNCH(2); break;
    default: SG_LAUNCH(3); break;
  }
#undef SG_LAUNCH
}

void launch_gather_sentinel_mr(int n, int nr, const int* perm, const double* scale, const double* x, double* c,
                               double* y, double* z, SyncState* ss, int mask, hipStream_t s,
                               const unsigned char* triv, const int* diag, const double* val,
                               int div, long long f1) {
  hipLaunchKernelGGL(k_gather_sentinel_mr, dim3(cdiv(n, 256), nr), dim3(256), 0, s, t_gate, n, nr, perm, scale,
                     x, c, y, z, ss, mask, triv, diag, val, div, f1);
}

void launch_scatter_mr(int n, int nr, const int* perm, const double* scale, const double* z, double* x,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_mr, dim3(cdiv(n, 256), nr), dim3(256), 0, s, t_gate, n, nr, perm, scale, z, x);
}

void launch_residual_mr(int n, int nr, const int* ptr, const int* idx, const int* pos,
                        const double* aval, const double* B, const double* X,
                        unsigned long long* colmax, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, colmax, 2 * nr);
  hipLaunchKernelGGL(k_residual_mr, dim3(std::max(1, rows_grid(n) / 4), nr), dim3(256), 0, s, n,
                     ptr, idx, pos, aval, B, X, colmax);
}

void launch_gather_sentinel(int n, const int* perm, const double* scale, const double* x, double* c, double* y,
                            double* z, SyncState* ss, int mask, hipStream_t s,
                            const unsigned char* triv, const int* diag, const double* val,
                            int div) {
  hipLaunchKernelGGL(k_gather_sentinel, dim3(cdiv(n, 256)), dim3(256), 0, s, t_gate, n, perm, scale, x, c, y, z,
                     ss, mask, triv, diag, val, div);
}

void launch_sync_prep(SyncState* ss, int mask, hipStream_t s) {
  hipLaunchKernelGGL(k_sync_prep, dim3(1), dim3(64), 0, s, ss, mask);
}

void launch_gather_prep(int n, const int* perm, const double* scale, const double* x, double* y, SyncState* ss,
                        int mask, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_prep, dim3(cdiv(n, 256)), dim3(256), 0, s, t_gate, n, perm, scale, x, y, ss, mask);
}

void launch_anorm1(int n, const int* cptr, const int* cpos, const double* aval, DevStats* st,
                   hipStream_t s, double* colabs, Inst in) {
  const int total = n * in.count;
  hipLaunchKernelGGL(k_anorm1, dim3(rows_grid(total)), dim3(256), 0, s, total, cptr, cpos,
                     aval, st, colabs, in);
}

void launch_reset_stats(DevStats* st, int what, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_stats, dim3(1), dim3(64), 0, s, st, what);
}

void launch_lsolve_rows(const LUView& lu, const int* rows, int nrows, int, double* y,
                        hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_lsolve_rows, dim3(cdiv((long)nrows * WAVE, 256)), dim3(256), 0, s, t_gate, rows,
                     nrows, lu.rowptr, lu.col, lu.diag, lu.val, y);
}

void launch_usolve_rows(const LUView& lu, const int* rows, int nrows, int, double* y,
                        hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_usolve_rows, dim3(cdiv((long)nrows * WAVE, 256)), dim3(256), 0, s, t_gate, rows,
                     nrows, lu.rowptr, lu.col, lu.diag, lu.val, y);
}

void launch_utsolve_cols(const LUView& lu, const int* cols, int ncols, const int* tptr,
                         const int* trow, const int* tpos, double* y, hipStream_t s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_utsolve_cols, dim3(cdiv((long)ncols * WAVE, 256)), dim3(256), 0, s, t_gate, cols,
                     ncols, tptr, trow, tpos, lu.val, y);
}

void launch_ltsolve_cols(const LUView& lu, const int* cols, int ncols, const int* tptr,
                         const int* trow, const int* tpos, double* y, hipStream_t s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_ltsolve_cols, dim3(cdiv((long)ncols * WAVE, 256)), dim3(256), 0, s, t_gate, cols,
                     ncols, tptr, trow, tpos, lu.val, y);
}

void launch_gather(int n, const int* perm, const double* scale, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(cdiv(n, 256)), dim3(256), 0, s, t_gate, n, perm, scale, x, y);
}
void launch_scatter(int n, const int* perm, const double* scale, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(cdiv(n, 256)), dim3(256), 0, s, t_gate, n, perm, scale, x, y);
}

void launch_residual(int n, char, const int* ptr, const int* idx, const int* pos,
                     const double* aval, const double* b, const double* x, double* r, DevStats* st,
                     hipStream_t s, double* red) {
  const int nb = red ? rows_grid_red(n) : rows_grid(n);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, s, n, ptr, idx, pos, aval, b, x, r, st,
                     red);
  if (red)
    hipLaunchKernelGGL(k_red_max, dim3(1), dim3(1024), 0, s, (const double*)red, nb, 2, &st->rmax,
                       &st->xmax);
}

void launch_spmv(int n, char, const int* ptr, const int* idx, const int* pos, const double* aval,
                 const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(rows_grid(n)), dim3(256), 0, s, n, ptr, idx, pos,
                     aval, x, y);
}

void launch_multidot(int n, int m, const double* V, long ld, const double* w, double* partial,
                     double* h, hipStream_t s) {
  const int grid = std::min(MD_GRID, cdiv(n, MD_BLOCK));
  hipLaunchKernelGGL(k_multidot_partial, dim3(grid), dim3(MD_BLOCK), 0, s, n, m, V, ld, w,
                     partial);
  hipLaunchKernelGGL(k_multidot_final, dim3(1), dim3(64), 0, s, m, grid, partial, h);
}

void launch_multiaxpy(int n, int m, const double* V, long ld, const double* h, double* w,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_multiaxpy, dim3(cdiv(n, 256)), dim3(256), 0, s, n, m, V, ld, h, w);
}

void launch_combine(int n, int m, const double* Z, long ld, const double* y, const double* base,
                    double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(cdiv(n, 256)), dim3(256), 0, s, n, m, Z, ld, y, base, out);
}

void launch_jacobi_sweep(int mode, const LUView& lu, const double* c, const double* yin,
                         double* yout, hipStream_t s) {
  if (mode == 0)
    hipLaunchKernelGGL(k_jacobi_sweep<0>, dim3(rows_grid(lu.n)), dim3(256), 0, s, t_gate, lu.n, lu.rowptr,
                       lu.col, lu.diag, lu.val, c, yin, yout);
  else
    hipLaunchKernelGGL(k_jacobi_sweep<1>, dim3(rows_grid(lu.n)), dim3(256), 0, s, t_gate, lu.n, lu.rowptr,
                       lu.col, lu.diag, lu.val, c, yin, yout);
}

void launch_add(int n, const double* d, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_add, dim3(cdiv(n, 256)), dim3(256), 0, s, t_gate, n, d, x);
}

void launch_scale_div(int n, const double* x, const double* scal, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_div, dim3(cdiv(n, 256)), dim3(256), 0, s, n, x, scal, y);
}

void launch_givens(int j, int m, const double* h, const double* h2, const double* ww, double* H,
                   double* cs, double* sn, double* g, double* y, double* hn_out, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, s, j, m, h, h2, ww, H, cs, sn, g, y, hn_out);
}

void launch_arnoldi_start(int n, int m, const double* r, const double* rr, double* v0, double* g,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi_start, dim3(cdiv(std::max(n, m + 1), 256)), dim3(256), 0, s, n, m,
                     r, rr, v0, g);
}


void launch_grad_sddmm(int n, int nrhs, const int* arow_ptr, const int* acol, const double* lam,
                       const double* x, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_sddmm, dim3(rows_grid(n)), dim3(256), 0, s, n, nrhs, arow_ptr, acol,
                     lam, x, grad);
}

void launch_copy(int n, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3(cdiv(n, 256)), dim3(256), 0, s, t_gate, n, x, y);
}

}  // namespace kktlu
