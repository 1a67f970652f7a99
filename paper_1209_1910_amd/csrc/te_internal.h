// Internal declarations shared by the kernels (te_kernels.hip) and the host
// orchestration (te_api.hip) of the tridiagonal eigenvector library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tridiag_eigvecs.h"

namespace te {

constexpr int kWave = 64;            // CDNA wavefront width

// Per-problem scalars from the setup pass.
struct Params {
  double norm1;   // ||T||_1
  double tol;     // cluster gap threshold, rtol * ||T||_1
  double pivmin;  // Sturm-count pivot floor
  double pivthr;  // LU pivot floor, eps * ||T||_1
  double gl, gu;  // widened bisection bracket
  double tnorm;   // max(|gl|, |gu|) of the unwidened Gershgorin interval
  double rtol;    // cluster gap as a multiple of ||T||_1 (input)
};

// One problem as seen by the kernels.  All arrays are device memory.
// Per-eigenvalue arrays of n entries (LU factors of T - W[j] I and the
// iterate) are stored interleaved: entry (row i, eigenvalue j) at i * m + j,
// so that one lane per eigenvalue reads and writes coalesced.
struct Prob {
  const double *d;      // n
  const double *e;      // n - 1
  double *e2;           // n - 1: e_i^2
  Params *prm;          // 1
  double *W;            // m eigenvalues (ascending)
  double *Z;            // eigenvectors, column-major, ld ldz
  double *V;            // n * m iterate storage, interleaved
  double *Ll;           // n * m multipliers l
  double *Lu1i;         // n * m 1 / u1
  double *Lu2;          // n * m u2 / u1
  double *Lu3;          // n * m u3 / u1
  unsigned char *Lsw;   // n * m row-swap flags
  double *nrm;          // m: 2-norm of each final iterate of the parallel solve
  int *pos;             // m: position of eigenvalue j in its cluster
  int *cl_start;        // m: cluster starts (first *ncl valid)
  int *cl_size;         // m
  int *ncl;             // 1
  double *Lrec;         // n * m * 4: member-major LU records {l, 1/u1, u2/u1, u3/u1},
                        //   eigenvalue j row i at (j * n + i) * 4 (later cluster members)
  unsigned char *Lswb;  // n * m: member-major swap flags, j * n + i
  double *Y;            // ldy * m: compact-WY Y column-major; cluster column l at
                        //   (start + l) * ldy
  double *Yr;           // n * ldm: the same Y row-major; cluster row i at i * ldm + start
  double *T;            // ldm * m: compact-WY T column-major (diagonal blocks)
  double *Tr;           // m * ldm: the same T row-major
  int ldy;              // n rounded up to even (16-byte aligned columns)
  int ldm;              // m rounded up to even
  int *info;            // 1 + m (may be null)
  int n, m, ldz;
  int kbase;            // global 1-based index of W[0] (start-vector key)
};

// A cluster chain work item: cluster [start, start + size) of problem prob.
struct ChainItem {
  int prob;
  int start;
  int size;
  int pad;
};

// Cooperative-kernel group: WGs [wg0, wg0 + nwg) run items [it0, it0 + nit).
struct Group {
  int wg0, nwg;
  int it0, nit;
};

// Chain scratch: one slot of `stride` doubles per small-kernel workgroup or
// per cooperative group.
struct ChainScratch {
  double *base;
  size_t stride;
};

size_t chain_scratch_doubles(int nmax, int mmax, int nwg_in_group);
// Group barrier state, unsigned words per group: a two-level barrier (top
// counter, kBarSubs sub-counters and release flags, each in its own 128-byte
// line) for the whole group at 0, the sweep's progress word at kBarProg, and
// the same barrier for ranks 1..size-1 at kBarSubRegion.
constexpr int kBarLine = 32, kBarSubs = 16;
constexpr int kBarTop = 0, kBarSubCnt = kBarLine, kBarSubFlag = kBarLine * (1 + kBarSubs);
constexpr int kBarRegion = kBarLine * (1 + 2 * kBarSubs);
constexpr int kBarProg = kBarRegion, kBarSubRegion = kBarRegion + kBarLine;
constexpr size_t kBarWords = 2 * kBarRegion + kBarLine;

// Launch helpers (te_kernels.hip).  Multi-problem kernels map a flat lane
// index t to (problem b, index j) through loff (nprob + 1 prefix offsets).
hipError_t launch_setup(const Prob *probs, int nprob, hipStream_t s);
hipError_t launch_bisect(const Prob *probs, int nprob, const int64_t *loff, int64_t nlanes,
                         hipStream_t s);
hipError_t launch_copy_w(const Prob *probs, int nprob, const int64_t *loff, int64_t nlanes,
                         const double *Wsrc, hipStream_t s);
hipError_t launch_cluster(const Prob *probs, int nprob, hipStream_t s);
hipError_t launch_invit(const Prob *probs, int nprob, const int64_t *loff, int64_t nlanes,
                        int iters, uint64_t seed, hipStream_t s);
hipError_t launch_transpose(const Prob *probs, int nprob, int nmax, int mmax, hipStream_t s);
hipError_t launch_chain_small(const Prob *probs, const ChainItem *items, int nitems,
                              int *counter, int *abort_flag, ChainScratch scr, int nwg,
                              int iters, hipStream_t s);
// started: null, or one host-coherent int per workgroup that the workgroup
// sets to 1 when it begins (the host waits on it for residency).
hipError_t launch_chain_coop(const Prob *probs, const ChainItem *items, const Group *groups,
                             const int *wg_group, unsigned *bars, int *abort_flag, int *started,
                             ChainScratch scr, int nwg, int iters, hipStream_t s);
// Graph-capturable variant: the item count is read from nitems_dev (device)
// when it is not null; nitems_cap bounds it otherwise.  nt: threads per
// workgroup, 256 or 512 (identical results).
hipError_t launch_chain_small_dev(const Prob *probs, const ChainItem *items, int nitems_cap,
                                  const int *nitems_dev, int *counter, int *abort_flag,
                                  ChainScratch scr, int nwg, int nt, int iters, hipStream_t s);
// Device-side chain plan of nprob problems whose cluster tables are on the
// device: items (capacity: the problems' sum of m / 2) ordered by decreasing
// cost, their count in *nitems.  bins: 2 * kPlanBins ints of scratch.
constexpr int kPlanBins = 64;
hipError_t launch_plan(const Prob *probs, int nprob, int *bins, ChainItem *items, int *nitems,
                       hipStream_t s);
// MGS chains (Alg. 1), one kMgsThreads-thread workgroup per cluster; item
// count as for launch_chain_small_dev.  Problems of order n <= TE_MGS_MAX_N.
constexpr int kMgsThreads = 512;
hipError_t launch_chain_mgs(const Prob *probs, const ChainItem *items, int nitems_cap,
                            const int *nitems_dev, int *counter, int *abort_flag,
                            ChainScratch scr, int nwg, int iters, hipStream_t s);
int mgs_max_wgs(int device);
hipError_t launch_finalize(const Prob *probs, int nprob, const int64_t *loff, int64_t nlanes,
                           hipStream_t s);
hipError_t launch_fill_i32(int *p, size_t n, int v, hipStream_t s);
// Splitting into unreduced blocks.
hipError_t launch_split_flags(const double *d, const double *e, int n, unsigned char *flag,
                              hipStream_t s);
struct SplitCol {
  const double *src;   // the block's vector (nb entries)
  const double *w;     // its eigenvalue
  const int *st;       // its status word
  int s, nb;           // block rows [s, s + nb)
  int p;               // output column
  int pad;
};
// Bidiagonal singular vectors through the Golub-Kahan tridiagonal.
hipError_t launch_gk_build(const double *a, const double *b, int n, double *dg, double *eg,
                           hipStream_t s);
hipError_t launch_gk_split(const double *Zg, int n, int m, double *U, size_t ldu, double *V,
                           size_t ldv, hipStream_t s);
hipError_t launch_split_scatter(const SplitCol *cols, int m, int n, double *W, double *Z,
                                size_t ldz, int *info, hipStream_t s);
int coop_max_wgs(int device);
int small_max_wgs(int device, int nt = 0);
int device_cus(int device);

}  // namespace te
