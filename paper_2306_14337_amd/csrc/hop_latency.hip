// Hop latency of the device-coherent publication that the dependency-driven
// refactorization and triangular solves rely on: one workgroup stores a
// value with a device-scope store, a second polls it with device-scope loads
// and answers the same way, for many rounds.  One hop (store, then the
// poll that sees it) is half a round trip.  Run for two workgroups on the
// same XCD and for two on different XCDs; the XCD of each workgroup is read
// from the hardware register, not assumed.  Prints one JSON line.
//
// Depth bound of a dependency-driven launch = (dependency levels on its
// critical chain) x (one hop), the latency floor of publishing a finished row
// to the rows that wait for it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int SPIN_LIMIT = 1 << 22;

__device__ __forceinline__ int ld_dev(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int xcc_id() {
  int v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & 0xf;
}

// Workgroups 0 and `partner` play; the others return.  Workgroup 0 writes odd
// values and waits for even ones, the partner the reverse.  Every wait is
// bounded: on the limit both sides stop and *fail is raised.
__global__ void k_pingpong(int* flag, int partner, int rounds, long long* ticks, int* xcc,
                           int* fail) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0 || (b != 0 && b != partner)) return;
  xcc[b == 0 ? 0 : 1] = xcc_id();
  const bool lead = b == 0;
  long long t0 = wall_clock64();
  for (int r = 0; r < rounds; r++) {
    const int want = lead ? 2 * r : 2 * r + 1;
    int spins = 0;
    while (ld_dev(flag) != want) {
      if ((++spins & 1023) == 0 && (spins > SPIN_LIMIT || ld_dev(fail))) {
        st_dev(fail, 1);
        return;
      }
    }
    st_dev(flag, want + 1);
  }
  if (lead) ticks[0] = wall_clock64() - t0;
}

int run(int partner, int rounds, double* rt_ns, int* xa, int* xb) {
  int *flag = nullptr, *xcc = nullptr, *fail = nullptr;
  long long* ticks = nullptr;
  if (hipMalloc(&flag, 256) != hipSuccess || hipMalloc(&xcc, 256) != hipSuccess ||
      hipMalloc(&fail, 256) != hipSuccess || hipMalloc(&ticks, 256) != hipSuccess)
    return 1;
  if (hipMemset(flag, 0, 256) != hipSuccess || hipMemset(fail, 0, 256) != hipSuccess ||
      hipMemset(xcc, 0xff, 256) != hipSuccess)
    return 1;
  hipLaunchKernelGGL(k_pingpong, dim3(partner + 1), dim3(64), 0, 0, flag, partner, rounds, ticks,
                     xcc, fail);
  if (hipDeviceSynchronize() != hipSuccess) return 2;
  int hfail = 0, hx[2] = {-1, -1};
  long long ht = 0;
  int dev = 0, khz = 0;
  if (hipMemcpy(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hx, xcc, sizeof hx, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&ht, ticks, sizeof ht, hipMemcpyDeviceToHost) != hipSuccess ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
    return 2;
  (void)hipFree(flag);
  (void)hipFree(xcc);
  (void)hipFree(fail);
  (void)hipFree(ticks);
  if (hfail || khz <= 0) return 3;
  *rt_ns = (double)ht / rounds / (khz * 1e3) * 1e9;
  *xa = hx[0];
  *xb = hx[1];
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  const int rounds = argc > 1 ? std::atoi(argv[1]) : 20000;
  // partners: the workgroup with the same index mod 8 (same XCD when
  // workgroups go round-robin over eight XCDs) and the next one
  int best_same = -1, best_cross = -1;
  double same = 0.0, cross = 0.0;
  int xs[2] = {-1, -1}, xc[2] = {-1, -1};
  for (int partner : {8, 16, 1, 2}) {
    double rt = 0.0;
    int a = -1, b = -1;
    const int rc = run(partner, rounds, &rt, &a, &b);
    if (rc != 0) {
      std::printf("{\"error\": \"ping-pong with workgroup %d failed (%d)\"}\n", partner, rc);
      return 1;
    }
    if (a == b && best_same < 0) {
      best_same = partner;
      same = rt;
      xs[0] = a;
      xs[1] = b;
    } else if (a != b && best_cross < 0) {
      best_cross = partner;
      cross = rt;
      xc[0] = a;
      xc[1] = b;
    }
  }
  std::printf(
      "{\"rounds\": %d, \"same_xcd\": {\"round_trip_ns\": %.1f, \"hop_ns\": %.1f, \"xcc\": [%d, %d]}, "
      "\"cross_xcd\": {\"round_trip_ns\": %.1f, \"hop_ns\": %.1f, \"xcc\": [%d, %d]}}\n",
      rounds, same, same / 2, xs[0], xs[1], cross, cross / 2, xc[0], xc[1]);
  return (best_same < 0 || best_cross < 0) ? 1 : 0;
}
