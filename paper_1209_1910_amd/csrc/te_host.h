// Host-side declarations shared by the C-ABI entry points (te_api.hip) and the
// serving engine (te_server.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <mutex>
#include <vector>

#include "../../include/tridiag_eigvecs.h"
#include "te_internal.h"

namespace te {

// Records a HIP failure for te_last_hip_error() and returns TE_ERR_HIP.
int hip_fail(hipError_t e);

struct Resolved {
  int iters;
  uint64_t seed;
  double rtol;
  int coop_wgs;
  uint64_t ws_budget;
  int orth;       // TE_ORTH_CWY or TE_ORTH_MGS
};
Resolved resolve(const te_opts *o);

struct DeviceLimits {
  int device = -1;
  int coop = 0;   // co-resident chain workgroups (cooperative kernel)
  int small = 0;  // resident workgroups of the small-chain kernel
  int mgs = 0;    // resident workgroups of the MGS chain kernel
};
DeviceLimits limits();

// One problem: device inputs d, e; device outputs W (m) and Z (ldz x m).
struct ProblemDesc {
  const double *d, *e;
  int n, il, iu;
  double *W, *Z;
  int ldz;
  int *info = nullptr;   // device, 1 + m ints; null: the workspace's own
};

// The whole method for a set of problems on `stream` (synchronizes it before
// returning).  ws may be null (workspace from hipMallocAsync on the stream).
int solve_problems(const std::vector<ProblemDesc> &pd, const double *W_given, const Resolved &opt,
                   void *ws, size_t ws_bytes, int *info, hipStream_t stream);

// Workspace bytes solve_problems needs for problems [b0, b1) (upper bound).
size_t problems_bytes(const std::vector<ProblemDesc> &pd, size_t b0, size_t b1,
                      const DeviceLimits &lim);

// Default device budget: half the free device memory, at most 64 GiB.
uint64_t default_budget();

// Per-device admission gate for kernels of this library.
//
// The cooperative chain kernel needs all of its workgroups resident at once;
// every other kernel of the library runs to completion without waiting on
// another workgroup.  A cooperative kernel launched while other work still
// holds compute units would have its first workgroups spin until the rest
// find room, and two cooperative kernels launched together could each hold
// part of the device for good.  So, per device:
//   - a caller holds the gate SHARED while any of its other kernels may be in
//     flight (from before the first launch to after the stream sync);
//   - a cooperative launch holds `coop` from launch to completion (one such
//     kernel in flight at a time) and the gate EXCLUSIVE from before the
//     launch until every one of its workgroups has reported that it started;
//     waiting writers keep new readers out.
// After that point other streams may launch again; their kernels use the
// compute units the cooperative grid leaves free.
struct DeviceGate {
  std::mutex mu;
  std::condition_variable cv;
  int readers = 0;
  int writers_waiting = 0;
  bool writer = false;
  std::mutex coop;
  int *started_host = nullptr;  // host-coherent residency slots (never freed)
  int *started_dev = nullptr;   // the same memory as seen by kernels
  int started_cap = 0;

  void lock_shared();
  void unlock_shared();
  void lock_exclusive();
  void unlock_exclusive();
};
DeviceGate &device_gate(int device);

// RAII shared hold on the current device's gate.
class SharedHold {
 public:
  SharedHold();
  ~SharedHold() { release(); }
  void acquire();
  void release();
  SharedHold(const SharedHold &) = delete;
  SharedHold &operator=(const SharedHold &) = delete;

 private:
  DeviceGate *g_ = nullptr;
  bool held_ = false;
};

}  // namespace te
