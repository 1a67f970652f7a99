// HIP kernels (gfx950, FP64) for inverse iteration with compact-WY
// re-orthogonalization (Ishigami, Kimura, Nakamura, arXiv:1209.1910).
//
// Built with -ffp-contract=off: every multiply and add below is rounded on its
// own unless written as fma(), so the Sturm counts, the bisection midpoints
// and the LU factors follow the same IEEE operation sequence as a plain C
// implementation of the same formulas.  Dot products use explicit fma().
#include <hip/hip_runtime.h>
#include <hip/hip_cooperative_groups.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>

#include "te_internal.h"

namespace te {

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

// Pointers read from problem descriptors in memory are generic to the
// compiler, which then emits flat memory instructions; those also count
// against the LDS wait counter, so every LDS wait would drain them too.  All
// of the library's buffers are global memory: say so once, where a pointer
// enters a hot loop, and the global address space propagates to every use.
template <class T>
__device__ __forceinline__ T *as_global(T *p) {
  return (T *)(__attribute__((address_space(1))) T *)p;
}
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
using lptr = __attribute__((address_space(3))) T *;

// Store of data that other workgroups read after a group barrier: a relaxed
// device-scope atomic store, which writes through to the device coherence
// point instead of leaving a dirty line in this XCD's L2.  Measured: with
// plain stores, a barrier whose single thread-0 release follows the other
// waves' stores let those stores be missed now and then when two groups
// shared the device (results then differed in the last bits), and a release
// in every wave instead cost 40 % of the chain's time.
template <class T>
__device__ __forceinline__ void st_dev(T *p, T v) {
  __hip_atomic_store((gptr<T>)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v) {
  // Fixed butterfly: every lane ends with the same, deterministic sum.
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
  return v;
}

__device__ __forceinline__ int find_prob(const int64_t *loff, int nprob, int64_t t) {
  int lo = 0, hi = nprob;  // loff[lo] <= t < loff[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (loff[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Sturm count: number of eigenvalues of T below sigma (negative pivots of the
// LDL^T factorization of T - sigma I; pivots with |q| <= pivmin become -pivmin).
// Reads d and e2 at uniform addresses across the wave.
__device__ int sturm_count(int n, const double *__restrict__ d, const double *__restrict__ e2,
                           double pivmin, double sigma) {
  double q = d[0] - sigma;
  if (fabs(q) <= pivmin) q = -pivmin;
  int cnt = q < 0.0 ? 1 : 0;
  for (int i = 1; i < n; i++) {
    double t1 = d[i] - sigma;
    double t2 = e2[i - 1] / q;
    q = t1 - t2;
    if (fabs(q) <= pivmin) q = -pivmin;
    cnt += q < 0.0 ? 1 : 0;
  }
  return cnt;
}

// Entry i of the start vector of global eigenvalue index k: the
// (((k << 32) | i) + 1)-th output of the SplitMix64 stream seeded with `seed`
// (Steele, Lea, Flood 2014), mapped to [-1, 1).
__device__ __forceinline__ double start_entry(uint64_t seed, uint64_t k, uint32_t i) {
  uint64_t key = (k << 32) | (uint64_t)i;
  uint64_t z = seed + (key + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  double u = (double)(z >> 11) * 0x1.0p-53;
  return 2.0 * u - 1.0;
}

// The growth stop rule (the kernels' iteration argument is negative): a solve
// (T - lambda I) x = v with ||v||_2 = 1 has converged when
// ||x||_2 >= 1 / (n eps ||T||_1) (1/||x||_2 is the residual of x/||x||_2), with
// ||x||_2^2 summed from the last row up; the first converged solve is followed
// by kStopExtra more iterations, kStopMaxIts at most.
constexpr int kStopExtra = 2, kStopMaxIts = 5;
__device__ __forceinline__ bool growth_converged(double nrm, int n, double norm1) {
  return nrm * (((double)n * DBL_EPSILON) * norm1) >= 1.0;
}

// ---------------------------------------------------------------------------
// a1: norm, tolerance, pivot floors and bisection bracket (one WG / problem)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_setup(const Prob *__restrict__ probs) {
  const Prob P = probs[blockIdx.x];
  const int n = P.n, tid = threadIdx.x;
  __shared__ double s_red[4][4];
  __shared__ double s_lohi[2];
  __shared__ int s_cnt[2];
  __shared__ int s_done;
  double rmax = -INFINITY, lmin = INFINITY, hmax = -INFINITY, e2max = 0.0;
  for (int i = tid; i < n; i += 256) {
    double r = fabs(P.d[i]);
    double s = 0.0;
    if (i > 0) { r = r + fabs(P.e[i - 1]); s = s + fabs(P.e[i - 1]); }
    if (i < n - 1) {
      r = r + fabs(P.e[i]);
      s = s + fabs(P.e[i]);
      double q = P.e[i] * P.e[i];
      P.e2[i] = q;
      e2max = fmax(e2max, q);
    }
    rmax = fmax(rmax, r);
    lmin = fmin(lmin, P.d[i] - s);
    hmax = fmax(hmax, P.d[i] + s);
  }
  rmax = wave_max(rmax); lmin = wave_min(lmin); hmax = wave_max(hmax); e2max = wave_max(e2max);
  const int w = tid / kWave, lane = tid % kWave;
  if (lane == 0) { s_red[0][w] = rmax; s_red[1][w] = lmin; s_red[2][w] = hmax; s_red[3][w] = e2max; }
  __syncthreads();
  const double norm1 = fmax(fmax(s_red[0][0], s_red[0][1]), fmax(s_red[0][2], s_red[0][3]));
  const double gl = fmin(fmin(s_red[1][0], s_red[1][1]), fmin(s_red[1][2], s_red[1][3]));
  const double gu = fmax(fmax(s_red[2][0], s_red[2][1]), fmax(s_red[2][2], s_red[2][3]));
  const double me2 = fmax(fmax(s_red[3][0], s_red[3][1]), fmax(s_red[3][2], s_red[3][3]));
  const double pivmin = DBL_MIN * (me2 > 1.0 ? me2 : 1.0);
  const double tnorm = fabs(gl) > fabs(gu) ? fabs(gl) : fabs(gu);
  __syncthreads();  // e2 visible to every wave
  // Widen until count(lo) == 0 and count(hi) == n (the two counts run on two waves).
  double wd = (2.0 * DBL_EPSILON * tnorm) * (double)n + 2.0 * pivmin;
  if (tid == 0) s_done = 0;
  for (int t = 0; t < 64; t++) {
    const double lo = gl - wd, hi = gu + wd;
    if (tid == 0) s_cnt[0] = sturm_count(n, P.d, P.e2, pivmin, lo);
    if (tid == kWave) s_cnt[1] = sturm_count(n, P.d, P.e2, pivmin, hi);
    __syncthreads();
    if (tid == 0) {
      s_lohi[0] = lo; s_lohi[1] = hi;
      s_done = (s_cnt[0] == 0 && s_cnt[1] == n) ? 1 : 0;
    }
    __syncthreads();
    if (s_done) break;
    wd = 2.0 * wd;
    __syncthreads();
  }
  if (tid == 0) {
    Params *p = P.prm;
    const double rtol = p->rtol;
    p->norm1 = norm1;
    p->tol = rtol * norm1;
    p->pivmin = pivmin;
    p->pivthr = DBL_EPSILON * norm1;
    p->gl = s_lohi[0];
    p->gu = s_lohi[1];
    p->tnorm = tnorm;
  }
}

hipError_t launch_setup(const Prob *probs, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_setup, dim3(nprob), dim3(256), 0, s, probs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a2: Sturm-count bisection, one lane per requested eigenvalue
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_bisect(const Prob *__restrict__ probs, int nprob,
                                                const int64_t *__restrict__ loff, int64_t nlanes) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlanes) return;
  const int b = find_prob(loff, nprob, t);
  const Prob &P = probs[b];
  const int j = (int)(t - loff[b]);
  const Params prm = *P.prm;
  const int k = P.kbase + j;
  const double atol = 2.0 * DBL_EPSILON * prm.tnorm;
  double lo = prm.gl, hi = prm.gu;
  for (int it = 0; it < 128 && (hi - lo) > atol; it++) {
    const double mid = lo + 0.5 * (hi - lo);
    if (sturm_count(P.n, P.d, P.e2, prm.pivmin, mid) >= k) hi = mid;
    else lo = mid;
  }
  P.W[j] = lo + 0.5 * (hi - lo);
}

hipError_t launch_bisect(const Prob *probs, int nprob, const int64_t *loff, int64_t nlanes,
                         hipStream_t s) {
  if (nlanes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bisect, dim3((unsigned)((nlanes + 255) / 256)), dim3(256), 0, s, probs,
                     nprob, loff, nlanes);
  return hipGetLastError();
}

__global__ void k_copy_w(const Prob *__restrict__ probs, int nprob, const int64_t *__restrict__ loff,
                         int64_t nlanes, const double *__restrict__ src) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlanes) return;
  const int b = find_prob(loff, nprob, t);
  probs[b].W[t - loff[b]] = src[t];
}

hipError_t launch_copy_w(const Prob *probs, int nprob, const int64_t *loff, int64_t nlanes,
                         const double *Wsrc, hipStream_t s) {
  if (nlanes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_w, dim3((unsigned)((nlanes + 255) / 256)), dim3(256), 0, s, probs,
                     nprob, loff, nlanes, Wsrc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a3: clusters by gap threshold (chain rule), one WG per problem
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_cluster(const Prob *__restrict__ probs) {
  const Prob P = probs[blockIdx.x];
  const int m = P.m, tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
  const double tol = P.prm->tol;
  __shared__ int s_wcnt[4];
  __shared__ int s_base;
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int base = 0; base < m; base += 256) {
    const int j = base + tid;
    const int flag = (j < m) && (j == 0 || (P.W[j] - P.W[j - 1]) > tol);
    const unsigned long long bal = __ballot(flag);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) s_wcnt[w] = __popcll(bal);
    __syncthreads();
    int off = s_base;
    for (int q = 0; q < w; q++) off += s_wcnt[q];
    if (flag) P.cl_start[off + before] = j;
    __syncthreads();
    if (tid == 0) s_base += s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
    __syncthreads();
  }
  const int ncl = s_base;
  if (tid == 0) *P.ncl = ncl;
  for (int c = tid; c < ncl; c += 256)
    P.cl_size[c] = (c + 1 < ncl ? P.cl_start[c + 1] : m) - P.cl_start[c];
  for (int j = tid; j < m; j += 256) {
    int lo = 0, hi = ncl;  // cl_start[lo] <= j < cl_start[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (P.cl_start[mid] <= j) lo = mid; else hi = mid;
    }
    P.pos[j] = j - P.cl_start[lo];
  }
}

hipError_t launch_cluster(const Prob *probs, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(k_cluster, dim3(nprob), dim3(256), 0, s, probs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Device-side chain plan (no host round trip, so the whole path can be
// captured in a graph): every cluster of two or more members becomes a chain
// item; items are ordered by decreasing cost size^2 n, in power-of-two cost
// bins (bin 0 holds the most expensive), so that a persistent chain kernel
// taking items from a counter starts the long chains first.  The order inside
// a bin depends on atomic timing; every chain computes the same bits wherever
// and whenever it runs.  bins: kPlanBins counts, then kPlanBins cursors.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int plan_bin(int size, int n) {
  const double cost = (double)size * (double)size * (double)n;
  const int e = ilogb(cost);  // >= 2 for size >= 2
  return e >= kPlanBins - 1 ? 0 : kPlanBins - 1 - e;
}

__global__ void __launch_bounds__(256) k_plan_count(const Prob *__restrict__ probs, int *bins) {
  const Prob &P = probs[blockIdx.x];
  __shared__ int h[kPlanBins];
  for (int i = threadIdx.x; i < kPlanBins; i += 256) h[i] = 0;
  __syncthreads();
  const int ncl = *P.ncl;
  for (int c = threadIdx.x; c < ncl; c += 256) {
    const int sz = P.cl_size[c];
    if (sz >= 2) atomicAdd(&h[plan_bin(sz, P.n)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kPlanBins; i += 256)
    if (h[i]) atomicAdd(&bins[i], h[i]);
}

__global__ void k_plan_scan(int *bins, int *nitems) {
  if (threadIdx.x != 0) return;
  int acc = 0;
  for (int i = 0; i < kPlanBins; i++) {
    const int c = bins[i];
    bins[kPlanBins + i] = acc;
    acc += c;
  }
  *nitems = acc;
}

__global__ void __launch_bounds__(256) k_plan_scatter(const Prob *__restrict__ probs, int *bins,
                                                      ChainItem *__restrict__ items) {
  const Prob &P = probs[blockIdx.x];
  const int ncl = *P.ncl;
  for (int c = threadIdx.x; c < ncl; c += 256) {
    const int sz = P.cl_size[c];
    if (sz < 2) continue;
    const int at = atomicAdd(&bins[kPlanBins + plan_bin(sz, P.n)], 1);
    items[at] = ChainItem{(int)blockIdx.x, P.cl_start[c], sz, 0};
  }
}

hipError_t launch_plan(const Prob *probs, int nprob, int *bins, ChainItem *items, int *nitems,
                       hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  hipError_t e = launch_fill_i32(bins, 2 * kPlanBins, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_plan_count, dim3(nprob), dim3(256), 0, s, probs, bins);
  hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(64), 0, s, bins, nitems);
  hipLaunchKernelGGL(k_plan_scatter, dim3(nprob), dim3(256), 0, s, probs, bins, items);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a4-a6: start vectors, partial-pivoting LU of T - lambda_j I and the solves
// of Eq. (1); one lane per eigenvalue, interleaved storage.
//
// Elimination step i keeps the active row (alpha at column i, beta at i+1).
// Row i+1 of T - sigma I is (e_i, d_{i+1} - sigma, e_{i+1}).  Without a swap
// the pivot row is the active row: U row i = (alpha, beta, 0), l = e_i/alpha.
// With a swap (|e_i| > |alpha|) the pivot row is row i+1: U row i =
// (e_i, d_{i+1} - sigma, e_{i+1}), l = alpha/e_i.  Pivots below pivthr in
// magnitude become +-pivthr.  Stored per row: l, 1/u1, u2/u1, u3/u1, swap.
//
// The iterate lives in V (interleaved).  The forward sweep writes
// y'_i = y_i / u1_i in place (slot i is overwritten only after it was read as
// b_i); the back sweep x_i = y'_i - (u2/u1)_i x_{i+1} - (u3/u1)_i x_{i+2}
// overwrites it again.  Singletons and first cluster members run all `iters`
// iterations; later members run the first (chain-independent) one only.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_invit(const Prob *__restrict__ probs, int nprob,
                                               const int64_t *__restrict__ loff, int64_t nlanes,
                                               int iters, uint64_t seed) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlanes) return;
  const int b = find_prob(loff, nprob, t);
  const Prob &P = probs[b];
  const int j = (int)(t - loff[b]);
  const int n = P.n;
  const size_t m = (size_t)P.m;
  const double *__restrict__ d = P.d;
  const double *__restrict__ e = P.e;
  double *__restrict__ V = P.V + j;
  double *__restrict__ Ll = P.Ll + j;
  double *__restrict__ U1 = P.Lu1i + j;
  double *__restrict__ U2 = P.Lu2 + j;
  double *__restrict__ U3 = P.Lu3 + j;
  unsigned char *__restrict__ SW = P.Lsw + j;
  const double sigma = P.W[j];
  const double pivthr = P.prm->pivthr;
  const bool stop = iters < 0, own = P.pos[j] == 0;   // own: all iterations here
  int K = own ? (stop ? kStopMaxIts : iters) : 1;
  bool conv = false;
  const uint64_t kglob = (uint64_t)(P.kbase + j);

  bool replaced = false;   // a pivot of the LU fell below pivthr
  double ss = 0.0;
  for (int i = 0; i < n; i++) {
    const double v = start_entry(seed, kglob, (uint32_t)i);
    V[(size_t)i * m] = v;
    ss = fma(v, v, ss);
  }
  for (int k = 1; k <= K; k++) {
    const double rn = 1.0 / sqrt(ss);
    double cur = V[0] * rn;
    if (k == 1) {
      double alpha = d[0] - sigma;
      double beta = n > 1 ? e[0] : 0.0;
      for (int i = 0; i < n - 1; i++) {
        const double bi = e[i];
        const double a1 = d[i + 1] - sigma;
        const double b1 = (i + 1 < n - 1) ? e[i + 1] : 0.0;
        const double bn = V[(size_t)(i + 1) * m] * rn;
        double piv, u2, u3, l, y;
        unsigned char sw;
        if (fabs(alpha) >= fabs(bi)) {
          piv = alpha;
          if (fabs(piv) < pivthr) { piv = piv < 0.0 ? -pivthr : pivthr; replaced = true; }
          u2 = beta; u3 = 0.0; sw = 0;
          l = bi / piv;
          alpha = a1 - l * beta;
          beta = b1;
          y = cur;
          cur = bn - l * cur;
        } else {
          piv = bi;
          if (fabs(piv) < pivthr) { piv = piv < 0.0 ? -pivthr : pivthr; replaced = true; }
          u2 = a1; u3 = b1; sw = 1;
          l = alpha / piv;
          alpha = beta - l * a1;
          beta = -(l * b1);
          y = bn;
          cur = cur - l * bn;
        }
        const double inv = 1.0 / piv;
        const size_t o = (size_t)i * m;
        Ll[o] = l; U1[o] = inv; U2[o] = u2 * inv; U3[o] = u3 * inv; SW[o] = sw;
        V[o] = y * inv;
      }
      double piv = alpha;
      if (fabs(piv) < pivthr) { piv = piv < 0.0 ? -pivthr : pivthr; replaced = true; }
      const double inv = 1.0 / piv;
      const size_t o = (size_t)(n - 1) * m;
      Ll[o] = 0.0; U1[o] = inv; U2[o] = 0.0; U3[o] = 0.0; SW[o] = 0;
      V[o] = cur * inv;
    } else {
      for (int i = 0; i < n - 1; i++) {
        const size_t o = (size_t)i * m;
        const double bn = V[o + m] * rn;
        const double l = Ll[o];
        double y;
        if (SW[o]) { y = bn; cur = cur - l * bn; }
        else { y = cur; cur = bn - l * cur; }
        V[o] = y * U1[o];
      }
      const size_t o = (size_t)(n - 1) * m;
      V[o] = cur * U1[o];
    }
    // back substitution
    ss = 0.0;
    double x1 = 0.0, x2 = 0.0;
    for (int i = n - 1; i >= 0; i--) {
      const size_t o = (size_t)i * m;
      const double x = fma(-U2[o], x1, fma(-U3[o], x2, V[o]));
      V[o] = x;
      ss = fma(x, x, ss);
      x2 = x1;
      x1 = x;
    }
    if (stop && own && !conv && growth_converged(sqrt(ss), n, P.prm->norm1)) {
      conv = true;
      K = min(K, k + kStopExtra);
    }
  }
  P.nrm[j] = sqrt(ss);
  if (P.info)
    P.info[1 + j] = (replaced ? TE_INFO_PIVOT : 0) | (stop && own && !conv ? TE_INFO_NOCONV : 0);
}

hipError_t launch_invit(const Prob *probs, int nprob, const int64_t *loff, int64_t nlanes,
                        int iters, uint64_t seed, hipStream_t s) {
  if (nlanes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_invit, dim3((unsigned)((nlanes + 255) / 256)), dim3(256), 0, s, probs,
                     nprob, loff, nlanes, iters, seed);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// V (interleaved) -> Z (column-major), and the LU factors of every later
// cluster member (interleaved) -> one contiguous record per row and member
// ({l, 1/u1, u2/u1, u3/u1} and the swap flag), the layout the sequential
// chain solves stream.  Singletons and first cluster members are normalized
// here (the first member's unit vector seeds Y_1, T_1); later members keep
// the raw first-iteration solve, the input of their first compact-WY step.
// 32 x 32 tiles through LDS.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_transpose(const Prob *__restrict__ probs) {
  const Prob &P = probs[blockIdx.z];
  const int n = P.n, m = P.m;
  const int j0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
  if (j0 >= m || i0 >= n) return;
  __shared__ double tv[32][33], tl[32][33], t1[32][33], t2[32][33], t3[32][33];
  __shared__ unsigned char tsw[32][33];
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    if (i < n && j < m) {
      const size_t o = (size_t)i * m + j;
      tv[r][tx] = P.V[o];
      tl[r][tx] = P.Ll[o];
      t1[r][tx] = P.Lu1i[o];
      t2[r][tx] = P.Lu2[o];
      t3[r][tx] = P.Lu3[o];
      tsw[r][tx] = P.Lsw[o];
    }
  }
  __syncthreads();
  for (int cc = ty; cc < 32; cc += 8) {
    const int j = j0 + cc, i = i0 + tx;
    if (i < n && j < m) {
      const int pj = P.pos[j];
      const double sc = pj == 0 ? 1.0 / P.nrm[j] : 1.0;
      P.Z[(size_t)j * P.ldz + i] = tv[tx][cc] * sc;
      if (pj > 0) {
        double4 rec;
        rec.x = tl[tx][cc];
        rec.y = t1[tx][cc];
        rec.z = t2[tx][cc];
        rec.w = t3[tx][cc];
        reinterpret_cast<double4 *>(P.Lrec)[(size_t)j * n + i] = rec;
        P.Lswb[(size_t)j * n + i] = tsw[tx][cc];
      }
    }
  }
}

hipError_t launch_transpose(const Prob *probs, int nprob, int nmax, int mmax, hipStream_t s) {
  if (nprob <= 0 || nmax <= 0 || mmax <= 0) return hipSuccess;
  dim3 grid((mmax + 31) / 32, (nmax + 31) / 32, nprob);
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, probs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a7: the compact-WY chain of one cluster (Alg. 4 with section 3.3.2).
//
// A group of G workgroups (G = 1 for the small kernel) runs the members
// c = 1..M-1 of the cluster in order; member c runs `iters` steps, each a
// compact-WY orthogonalization of its current iterate v followed, except
// after the last step, by the solve of Eq. (1).  Y (n x M; column l holds
// y_l, zero above row l and never read there) and T (M x M upper triangular)
// are kept in HBM twice, column-major and row-major, so that every pass below
// is a set of contiguous dot products, one wavefront per dot product:
//
//  P1  x   = Y_c^T v                (L^T v_chk + Yhat^T v_hat; columns of Y)
//  P2  x'  = T_c^T x                (columns of T)
//  P3  u   = v_hat - Yhat_c x'      (rows c..n-1 of Y) and ||u||^2
//  P4  c_j = -sgn(u_c)||u||, t_j = 1/(c_j^2 - u_c c_j), y_hat = u with
//      u_c - c_j at row c; s = Yhat_c^T y_hat (columns of Y); column c of Y
//  P5  t_hat = -t_j T_c s and x'' = T_{c+1} r, r = row c of Y_{c+1}
//      (rows of T, both vectors in one pass); column c of T
//  P6  q = Y_{c+1} x'' - e_c        (rows of Y)
//  P7  v = (T - lambda I)^{-1} q/||q||  (rank-0 workgroup)
//
// The product in P5 uses T_{c+1}; the transposed factor printed for this
// step in section 3.3.2 does not give orthonormal columns.
// ---------------------------------------------------------------------------

struct Ctx {
  int rank, size;      // workgroup rank in the group, group size (WGs)
  unsigned *cnt;       // group arrival counter (unused when size == 1)
  unsigned *flag;      // group release flag: last completed generation
  unsigned gen;        // generation of the next barrier
  unsigned sgen;       // generation of the next barrier among ranks 1..size-1
  int *abort_flag;
  int gw, nw;          // wave index in the group, waves in the group
  int wave, lane;
};

constexpr unsigned long long kSpinLimit = 1ull << 24;  // only a broken run waits that long
// s_waitcnt immediate (gfx9 encoding): vmcnt = 0, expcnt = 7, lgkmcnt = 15.
constexpr int kWaitVmcnt0 = (0x7 << 4) | (0xF << 8);

// Device-scope acquire by one thread on behalf of its workgroup: the cache
// invalidation it issues must have completed before the workgroup barrier
// lets the other waves load, or their loads can still hit stale L2 lines.
__device__ __forceinline__ void wg_acquire() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
}

// Group barrier: arrive on the counter; the last arrival publishes the
// generation on the flag; the others poll the flag.  Returns false (in every
// thread of the WG) when the run was aborted; a wait that exceeds the spin
// limit sets the abort flag, so every workgroup of every group unwinds.
template <int NT>
__device__ bool grp_sync(Ctx &c) {
  // Arrival.  Everything other workgroups read after a group barrier is
  // written with write-through (device-scope) stores, and the back sweep
  // releases its own stores when it publishes progress; so arriving only
  // needs every wave's stores to have completed (s_waitcnt vmcnt 0, the
  // other counters at their maximum), and the counter and flag updates can
  // be relaxed: no L2 writeback per barrier.
  //
  // Two levels: the ranks k, k + s, k + 2 s, ... (s = min(size, kBarSubs))
  // arrive on sub-counter k; the last of them arrives on the top counter,
  // and the last arrival there sets every sub-group's release flag.  Each
  // counter and flag has its own cache line: about size / s workgroups update
  // a sub-counter and poll a flag, s update the top counter.  (One counter and
  // one flag for all 256 workgroups cost 40 us per compact-WY step more.)
  if (c.size > 1) __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  __syncthreads();
  if (c.size == 1) return true;
  __shared__ int s_ok;
  c.gen++;
  if (threadIdx.x == 0) {
    int ok = 1;
    const int ns = c.size < kBarSubs ? c.size : kBarSubs;
    const int k = c.rank % ns;
    const unsigned members = (unsigned)((c.size - k + ns - 1) / ns);
    unsigned *sub = c.cnt + kBarSubCnt + kBarLine * k;
    unsigned *flag = c.cnt + kBarSubFlag + kBarLine * k;
    const unsigned old = __hip_atomic_fetch_add(sub, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1u == c.gen * members) {
      const unsigned top =
          __hip_atomic_fetch_add(c.cnt + kBarTop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (top + 1u == c.gen * (unsigned)ns)
        for (int j = 0; j < ns; j++)
          __hip_atomic_store(c.cnt + kBarSubFlag + kBarLine * j, c.gen, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned long long spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < c.gen) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255ull) == 0) {
        if (__hip_atomic_load(c.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
        if (spins > kSpinLimit) {
          __hip_atomic_store(c.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    wg_acquire();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Scratch layout of one chain slot.  Vectors paired in dot products with
// rows of Y or T (x, x', s, r, x'') start at the parity of the cluster start,
// so both operands of every dot product have the same 16-byte alignment.
struct Scr {
  double *v, *q, *u, *P, *Q;       // n each (even offsets)
  double *x, *xp, *s, *r, *xpp;    // mmax + 2 each (offset by the start parity)
  double *carry;                   // n / 64 + 8: carries into the scan chunks
  double *csum;                    // 2 (n / 64) + 16: chunk summaries (A, B)
  // next member's first-iteration products (lookahead)
  double *vla, *upre;              // n each (even offsets)
  double *xla, *xpla;              // mmax + 2 each (offset by the start parity)
  double *xseg;                    // n / 1024 + 2: segment partials of one column dot
  double *misc;                    // 2: ||x||^2 of the last chain solve
  double *tr;                      // mmax + 2: T_c r of a member's first step (parity offset)
};

__host__ __device__ inline size_t even_up(size_t x) { return (x + 1) & ~(size_t)1; }

__host__ __device__ inline size_t scr_doubles(int nmax, int mmax) {
  return even_up(7 * even_up((size_t)nmax) + 8 * even_up((size_t)mmax + 2) +
                 even_up((size_t)nmax / 64 + 8) + even_up(2 * ((size_t)nmax / 64) + 16) +
                 even_up((size_t)nmax / 1024 + 2) + 64);
}

size_t chain_scratch_doubles(int nmax, int mmax, int nwg_in_group) {
  (void)nwg_in_group;
  return scr_doubles(nmax, mmax);
}

__device__ inline Scr make_scr(double *base, int nmax, int mmax, int parity) {
  Scr S;
  double *p = base;
  const size_t nn = even_up((size_t)nmax), mm = even_up((size_t)mmax + 2);
  S.v = p; p += nn;
  S.q = p; p += nn;
  S.u = p; p += nn;
  S.P = p; p += nn;
  S.Q = p; p += nn;
  S.x = p + parity; p += mm;
  S.xp = p + parity; p += mm;
  S.s = p + parity; p += mm;
  S.r = p + parity; p += mm;
  S.xpp = p + parity; p += mm;
  S.carry = p; p += even_up((size_t)nmax / 64 + 8);
  S.csum = p; p += even_up(2 * ((size_t)nmax / 64) + 16);
  S.vla = p; p += nn;
  S.upre = p; p += nn;
  S.xla = p + parity; p += mm;
  S.xpla = p + parity; p += mm;
  S.xseg = p; p += even_up((size_t)nmax / 1024 + 2);
  S.tr = p + parity; p += mm;
  S.misc = p;   // inside the 64 doubles of slack scr_doubles adds
  return S;
}

// Native two-double vector and global-memory pointer types for the dot
// products: loads through address-space-1 pointers compile to global (not
// flat) instructions, so the compiler can wait on them one group at a time.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) d2v *gd2p;
typedef const __attribute__((address_space(1))) double *gdp;

// Dot product of a[lo..hi) and b[lo..hi) by one wave: 16-byte loads, fixed
// combination order; every lane gets the sum.  a + lo and b + lo must have
// the same alignment modulo 16 bytes.
__device__ __forceinline__ double wave_dot(const double *a_, const double *b_, int lo, int hi,
                                           int lane) {
  const gdp a = (gdp)a_, b = (gdp)b_;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (lo < hi && (reinterpret_cast<uintptr_t>(a_ + lo) & 15)) {
    if (lane == 0) a0 = a[lo] * b[lo];
    lo++;
  }
  const int np = (hi - lo) >> 1;
  const gd2p A2 = (gd2p)(a + lo);
  const gd2p B2 = (gd2p)(b + lo);
  int p = lane;
  for (; p + 3 * kWave < np; p += 4 * kWave) {
    const d2v x0 = A2[p], x1 = A2[p + kWave], x2 = A2[p + 2 * kWave], x3 = A2[p + 3 * kWave];
    const d2v y0 = B2[p], y1 = B2[p + kWave], y2 = B2[p + 2 * kWave], y3 = B2[p + 3 * kWave];
    a0 = fma(x0.x, y0.x, a0); a0 = fma(x0.y, y0.y, a0);
    a1 = fma(x1.x, y1.x, a1); a1 = fma(x1.y, y1.y, a1);
    a2 = fma(x2.x, y2.x, a2); a2 = fma(x2.y, y2.y, a2);
    a3 = fma(x3.x, y3.x, a3); a3 = fma(x3.y, y3.y, a3);
  }
  for (; p < np; p += kWave) {
    const d2v x0 = A2[p], y0 = B2[p];
    a0 = fma(x0.x, y0.x, a0); a0 = fma(x0.y, y0.y, a0);
  }
  if (((hi - lo) & 1) && lane == 0) a1 = fma(a[hi - 1], b[hi - 1], a1);
  return wave_sum((a0 + a1) + (a2 + a3));
}

// R dot products a_r . b over [lo, hi) with a_r = a + r * stride (every a_r
// with the 16-byte alignment of a), each with exactly wave_dot's arithmetic,
// so each result has wave_dot's bits.  Only r < nr (wave-uniform) are read.
// Several dot products in flight per wave hide the load and reduction latency
// that one at a time exposes.
template <int R>
__device__ __forceinline__ void wave_dot_multi(const double *a_, size_t stride, int nr,
                                               const double *b_, int lo, int hi, int lane,
                                               double (&out)[R]) {
  const gdp a = (gdp)a_, b = (gdp)b_;
  double a0[R], a1[R], a2[R], a3[R];
#pragma unroll
  for (int r = 0; r < R; r++) a0[r] = a1[r] = a2[r] = a3[r] = 0.0;
  if (lo < hi && (reinterpret_cast<uintptr_t>(a_ + lo) & 15)) {
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < R; r++)
        if (r < nr) a0[r] = a[(size_t)r * stride + lo] * b[lo];
    }
    lo++;
  }
  const int np = (hi - lo) >> 1;
  const gd2p B2 = (gd2p)(b + lo);
  int p = lane;
  for (; p + 3 * kWave < np; p += 4 * kWave) {
    const d2v y0 = B2[p], y1 = B2[p + kWave], y2 = B2[p + 2 * kWave], y3 = B2[p + 3 * kWave];
#pragma unroll
    for (int r = 0; r < R; r++) {
      if (r < nr) {
        const gd2p A2 = (gd2p)(a + (size_t)r * stride + lo);
        const d2v x0 = A2[p], x1 = A2[p + kWave], x2 = A2[p + 2 * kWave], x3 = A2[p + 3 * kWave];
        a0[r] = fma(x0.x, y0.x, a0[r]); a0[r] = fma(x0.y, y0.y, a0[r]);
        a1[r] = fma(x1.x, y1.x, a1[r]); a1[r] = fma(x1.y, y1.y, a1[r]);
        a2[r] = fma(x2.x, y2.x, a2[r]); a2[r] = fma(x2.y, y2.y, a2[r]);
        a3[r] = fma(x3.x, y3.x, a3[r]); a3[r] = fma(x3.y, y3.y, a3[r]);
      }
    }
  }
  for (; p < np; p += kWave) {
    const d2v y0 = B2[p];
#pragma unroll
    for (int r = 0; r < R; r++) {
      if (r < nr) {
        const d2v x0 = ((gd2p)(a + (size_t)r * stride + lo))[p];
        a0[r] = fma(x0.x, y0.x, a0[r]); a0[r] = fma(x0.y, y0.y, a0[r]);
      }
    }
  }
  if (((hi - lo) & 1) && lane == 0) {
#pragma unroll
    for (int r = 0; r < R; r++)
      if (r < nr) a1[r] = fma(a[(size_t)r * stride + hi - 1], b[hi - 1], a1[r]);
  }
#pragma unroll
  for (int r = 0; r < R; r++) out[r] = wave_sum((a0[r] + a1[r]) + (a2[r] + a3[r]));
}

// R dot products a_r[lo_r, hi_r) . b[lo_r, hi_r), each with exactly
// wave_dot(a_r, b, lo_r, hi_r)'s arithmetic (same bits), in one loop so that
// the loads and reductions of the R products overlap.  Only r < nr
// (wave-uniform) are read; the others return 0.
template <int R>
__device__ __forceinline__ void wave_dot_var(const double *const (&a_)[R], const double *b_,
                                             const int (&lo_)[R], const int (&hi_)[R], int nr,
                                             int lane, double (&out)[R]) {
  const gdp b = (gdp)b_;
  double a0[R], a1[R], a2[R], a3[R];
  int lo[R], np[R];
  bool mainp[R];
  int pmax = 0;
#pragma unroll
  for (int r = 0; r < R; r++) {
    a0[r] = a1[r] = a2[r] = a3[r] = 0.0;
    lo[r] = lo_[r];
    np[r] = 0;
    mainp[r] = true;
    if (r < nr) {
      const gdp a = (gdp)a_[r];
      if (lo[r] < hi_[r] && (reinterpret_cast<uintptr_t>(a_[r] + lo[r]) & 15)) {
        if (lane == 0) a0[r] = a[lo[r]] * b[lo[r]];
        lo[r]++;
      }
      np[r] = (hi_[r] - lo[r]) >> 1;
      pmax = np[r] > pmax ? np[r] : pmax;
    }
  }
  // wave_dot's two loops per product: while p + 3*64 < np, four pairs into
  // a0..a3; then, from the first p that fails, single pairs into a0
  for (int p = lane; p < pmax; p += 4 * kWave) {
#pragma unroll
    for (int r = 0; r < R; r++) {
      if (r >= nr) continue;
      const gd2p A2 = (gd2p)((gdp)a_[r] + lo[r]);
      const gd2p B2 = (gd2p)(b + lo[r]);
      if (mainp[r] && p + 3 * kWave < np[r]) {
        const d2v x0 = A2[p], x1 = A2[p + kWave], x2 = A2[p + 2 * kWave], x3 = A2[p + 3 * kWave];
        const d2v y0 = B2[p], y1 = B2[p + kWave], y2 = B2[p + 2 * kWave], y3 = B2[p + 3 * kWave];
        a0[r] = fma(x0.x, y0.x, a0[r]); a0[r] = fma(x0.y, y0.y, a0[r]);
        a1[r] = fma(x1.x, y1.x, a1[r]); a1[r] = fma(x1.y, y1.y, a1[r]);
        a2[r] = fma(x2.x, y2.x, a2[r]); a2[r] = fma(x2.y, y2.y, a2[r]);
        a3[r] = fma(x3.x, y3.x, a3[r]); a3[r] = fma(x3.y, y3.y, a3[r]);
      } else if (mainp[r]) {
        mainp[r] = false;
        for (int q = p; q < np[r]; q += kWave) {
          const d2v x0 = A2[q], y0 = B2[q];
          a0[r] = fma(x0.x, y0.x, a0[r]); a0[r] = fma(x0.y, y0.y, a0[r]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; r++) {
    if (r < nr && ((hi_[r] - lo[r]) & 1) && lane == 0) {
      const gdp a = (gdp)a_[r];
      a1[r] = fma(a[hi_[r] - 1], b[hi_[r] - 1], a1[r]);
    }
    out[r] = (r < nr) ? wave_sum((a0[r] + a1[r]) + (a2[r] + a3[r])) : 0.0;
  }
}

// (a.b, a.c) over [lo, hi) with exactly wave_dot's arithmetic for each of the
// two: one pass over a serves both products bit for bit.
__device__ __forceinline__ void wave_dot_pair(const double *a_, const double *b_,
                                              const double *c_, int lo, int hi, int lane,
                                              double &ob, double &oc) {
  const gdp a = (gdp)a_, b = (gdp)b_, c = (gdp)c_;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
  if (lo < hi && (reinterpret_cast<uintptr_t>(a_ + lo) & 15)) {
    if (lane == 0) { a0 = a[lo] * b[lo]; c0 = a[lo] * c[lo]; }
    lo++;
  }
  const int np = (hi - lo) >> 1;
  const gd2p A2 = (gd2p)(a + lo);
  const gd2p B2 = (gd2p)(b + lo);
  const gd2p C2 = (gd2p)(c + lo);
  int p = lane;
  for (; p + 3 * kWave < np; p += 4 * kWave) {
    const d2v x0 = A2[p], x1 = A2[p + kWave], x2 = A2[p + 2 * kWave], x3 = A2[p + 3 * kWave];
    const d2v y0 = B2[p], y1 = B2[p + kWave], y2 = B2[p + 2 * kWave], y3 = B2[p + 3 * kWave];
    const d2v z0 = C2[p], z1 = C2[p + kWave], z2 = C2[p + 2 * kWave], z3 = C2[p + 3 * kWave];
    a0 = fma(x0.x, y0.x, a0); a0 = fma(x0.y, y0.y, a0);
    a1 = fma(x1.x, y1.x, a1); a1 = fma(x1.y, y1.y, a1);
    a2 = fma(x2.x, y2.x, a2); a2 = fma(x2.y, y2.y, a2);
    a3 = fma(x3.x, y3.x, a3); a3 = fma(x3.y, y3.y, a3);
    c0 = fma(x0.x, z0.x, c0); c0 = fma(x0.y, z0.y, c0);
    c1 = fma(x1.x, z1.x, c1); c1 = fma(x1.y, z1.y, c1);
    c2 = fma(x2.x, z2.x, c2); c2 = fma(x2.y, z2.y, c2);
    c3 = fma(x3.x, z3.x, c3); c3 = fma(x3.y, z3.y, c3);
  }
  for (; p < np; p += kWave) {
    const d2v x0 = A2[p], y0 = B2[p], z0 = C2[p];
    a0 = fma(x0.x, y0.x, a0); a0 = fma(x0.y, y0.y, a0);
    c0 = fma(x0.x, z0.x, c0); c0 = fma(x0.y, z0.y, c0);
  }
  if (((hi - lo) & 1) && lane == 0) {
    a1 = fma(a[hi - 1], b[hi - 1], a1);
    c1 = fma(a[hi - 1], c[hi - 1], c1);
  }
  ob = wave_sum((a0 + a1) + (a2 + a3));
  oc = wave_sum((c0 + c1) + (c2 + c3));
}

// Two dot products sharing the matrix row a: (a.b, a.c) over [0, len); a, b
// and c must have the same alignment modulo 16 bytes.
__device__ __forceinline__ void wave_dot2(const double *a_, const double *b_, const double *c_,
                                          int len, int lane, double &ob, double &oc) {
  const gdp a = (gdp)a_, b = (gdp)b_, c = (gdp)c_;
  double b0 = 0.0, b1 = 0.0, c0 = 0.0, c1 = 0.0;
  int lo = 0;
  if (len > 0 && (reinterpret_cast<uintptr_t>(a_) & 15)) {
    if (lane == 0) { b0 = a[0] * b[0]; c0 = a[0] * c[0]; }
    lo = 1;
  }
  const int np = (len - lo) >> 1;
  const gd2p A2 = (gd2p)(a + lo);
  const gd2p B2 = (gd2p)(b + lo);
  const gd2p C2 = (gd2p)(c + lo);
  int p = lane;
  for (; p + kWave < np; p += 2 * kWave) {
    const d2v m0 = A2[p], m1 = A2[p + kWave];
    const d2v y0 = B2[p], y1 = B2[p + kWave];
    const d2v z0 = C2[p], z1 = C2[p + kWave];
    b0 = fma(m0.x, y0.x, b0); b0 = fma(m0.y, y0.y, b0);
    c0 = fma(m0.x, z0.x, c0); c0 = fma(m0.y, z0.y, c0);
    b1 = fma(m1.x, y1.x, b1); b1 = fma(m1.y, y1.y, b1);
    c1 = fma(m1.x, z1.x, c1); c1 = fma(m1.y, z1.y, c1);
  }
  for (; p < np; p += kWave) {
    const d2v m0 = A2[p], y0 = B2[p], z0 = C2[p];
    b0 = fma(m0.x, y0.x, b0); b0 = fma(m0.y, y0.y, b0);
    c0 = fma(m0.x, z0.x, c0); c0 = fma(m0.y, z0.y, c0);
  }
  if (((len - lo) & 1) && lane == 0) {
    b1 = fma(a[len - 1], b[len - 1], b1);
    c1 = fma(a[len - 1], c[len - 1], c1);
  }
  ob = wave_sum(b0 + b1);
  oc = wave_sum(c0 + c1);
}

// Folded assignment of `cnt` dot products whose lengths grow (or shrink)
// linearly with their index: indices p and cnt - 1 - p form pair p, pairs go
// round-robin to the waves, so every wave's total length is about the same.
// Task t of wave gw is pair gw + (t / 2) nw, its front index for even t and
// its back index for odd t.
__device__ __forceinline__ int fold_index(int gw, int nw, int t, int cnt) {
  const int p = gw + (t >> 1) * nw;
  return (t & 1) ? cnt - 1 - p : p;
}

__device__ __forceinline__ bool fold_valid(int gw, int nw, int t, int cnt) {
  const int p = gw + (t >> 1) * nw;
  if (2 * p >= cnt) return false;
  return (t & 1) ? (cnt - 1 - p > p) : true;
}

// Sum of squares of x[i0..n) for the whole group, in one fixed order that
// depends on neither the number of workgroups nor their size: after the group
// barrier (which also publishes x), each workgroup reads the whole range with
// 256 virtual lanes (lane v takes i0 + v, i0 + v + 256, ... into eight
// accumulators combined pairwise), reduces each 64-lane wave by the fixed
// butterfly and adds the four wave totals pairwise.  So a cluster's chain
// gives the same bits on one workgroup or many, alone or batched.
// Returns false on abort.
constexpr int kSumLanes = 256;

template <int NT>
__device__ bool grp_sumsq(Ctx &c, const double *x, int i0, int n, double &out) {
  static_assert(NT >= kSumLanes, "group sums need 256 threads");
  constexpr int kStep = 8 * kSumLanes;
  __shared__ double s_p[kSumLanes / kWave];
  const gptr<const double> xg = (gptr<const double>)x;
  if (!grp_sync<NT>(c)) return false;
  if (threadIdx.x < kSumLanes) {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = i0 + (int)threadIdx.x;
    for (; i + 7 * kSumLanes < n; i += kStep) {
      double t[8];
#pragma unroll
      for (int r = 0; r < 8; r++) t[r] = xg[i + r * kSumLanes];
#pragma unroll
      for (int r = 0; r < 8; r++) a[r] = fma(t[r], t[r], a[r]);
    }
#pragma unroll
    for (int r = 0; r < 7; r++) {
      const int ir = i + r * kSumLanes;
      if (ir < n) a[r] = fma(xg[ir], xg[ir], a[r]);
    }
    double p = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    p = wave_sum(p);
    if (c.lane == 0) s_p[c.wave] = p;
  }
  __syncthreads();
  out = (s_p[0] + s_p[1]) + (s_p[2] + s_p[3]);
  return true;
}

struct CView {
  int n, M;
  double *Y;            // column-major: cluster column l at Y + l * ldy
  double *Yr;           // row-major:    cluster row i at Yr + i * ldm
  double *T;            // column-major: T[p, l] at T[p + l * ldm]
  double *Tr;           // row-major:    T[p, l] at Tr[p * ldm + l]
  size_t ldy, ldm;
  double *Z;            // column-major, ldz
  size_t ldz;
  const double4 *Lrec;  // member c's LU rows at Lrec + c * n
  const unsigned char *Lswb;
};

// Back substitution x_i = y'_i - a_i x_{i+1} - b_i x_{i+2} (a = u2/u1,
// b = u3/u1 from the LU records, y' = y / u1 of the forward sweep, x into v).
// The recurrence is sequential and latency-bound, so it runs in lane 0 of one
// wave alone (no broadcasts, no gathers); everything else is taken off that
// lane.  The workgroup's other waves (producers) form the rows {a, b, y'} in
// 64-row blocks from the bottom up and stage them in an LDS ring of SLOTS
// blocks, many blocks ahead, so global-memory latency never reaches the sweep
// (consumer).  Lane 0 of the consumer keeps its LDS reads kSweepRing rows
// ahead in a register ring (across block boundaries) and stores each x
// through a per-block global base pointer.
constexpr int kSweepRing = 4;

// staged[s] = k + 1 once block k sits in slot s = k % SLOTS; freed = number
// of blocks the consumer no longer reads; abort set by a wait that timed out.
// Reset before every sweep (a workgroup barrier separates sweeps).
struct alignas(16) SRow {
  double a, b, y, pad;   // u2/u1, u3/u1, y'
};

template <int SLOTS>
struct SweepRing {
  SRow row[SLOTS][kWave];
  int staged[SLOTS];
  int freed;
  int abort;
};

typedef const __attribute__((address_space(3))) SRow *ldrp;
__device__ __forceinline__ SRow lds_row(ldrp p) {   // field by field: C++ copies are generic-only
  SRow r;
  r.a = p->a;
  r.b = p->b;
  r.y = p->y;
  r.pad = 0.0;
  return r;
}
constexpr unsigned kRingSpinLimit = 1u << 22;   // only a broken run waits that long

// Whole-wave wait until the LDS word w reaches target; later LDS reads of
// the wave see what the writer stored before it set w.  A wait past the spin
// limit marks the ring aborted (and the run, through abort_flag); a marked
// ring ends every other wait.
__device__ __forceinline__ bool ring_wait(lptr<int> w, int target, lptr<int> ring_abort,
                                          int *abort_flag) {
  unsigned spins = 0;
  while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
    if (__hip_atomic_load(ring_abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
      return false;
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kRingSpinLimit) {
      __hip_atomic_store(ring_abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (abort_flag)
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  return true;
}

// Sweep of one full block from LDS slot cur; the ring reads run on into the
// next block's slot nxt.  x into xb[0..63].
// With SS, ss accumulates x_i^2 from the bottom row up (fused multiply-adds).
template <bool SS>
__device__ __forceinline__ void sweep_block(ldrp cur, ldrp nxt, SRow (&ring)[kSweepRing],
                                            double &x1, double &x2, double &ss, gptr<double> xb) {
#pragma unroll
  for (int t = kWave - 1; t >= 0; t--) {
    const int slot = (kWave - 1 - t) % kSweepRing;
    const SRow c = ring[slot];
    ring[slot] = lds_row((t - kSweepRing >= 0) ? cur + (t - kSweepRing) : nxt + (t - kSweepRing + kWave));
    const double x = fma(-c.a, x1, fma(-c.b, x2, c.y));
    x2 = x1;
    x1 = x;
    xb[t] = x;
    if (SS) ss = fma(x, x, ss);
  }
}

// Rows of the solution become final from the bottom; when `prog` is non-null
// lane 0 publishes, each time a kSegRows-row segment (counted from row 0) is
// complete, the word (seq << 32) | (rows final), after a device-scope release
// of its stores, for consumers that overlap work with the sweep.
constexpr int kSegRows = 1024;

// Consumer: the back sweep.  Block k holds rows n - 64 (k + 1) + j, j = 0..63
// (rows below 0 are zero).  Returns false if a ring wait failed.
// ss_out: null, or where lane 0 stores ||x||_2^2 of the solution (summed
// from the last row up), written through for the other workgroups.
template <int SLOTS>
__device__ bool sweep_consume(SweepRing<SLOTS> &sr, double *v_, int n, int lane,
                              unsigned long long *prog, unsigned long long seq, int *abort_flag,
                              double *ss_out) {
  static_assert(kWave % kSweepRing == 0, "ring must tile a block");
  int pub_next = ((n - 1) / kSegRows) * kSegRows;   // start of the next segment to publish
  auto publish = [&](int done_lo) {                  // rows >= done_lo are final
    if (!prog || done_lo > pub_next) return;
    if (lane == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(prog, (seq << 32) | (unsigned long long)(n - done_lo), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    pub_next = done_lo > 0 ? ((done_lo - 1) / kSegRows) * kSegRows : -1;
  };
  const gptr<double> v = (gptr<double>)v_;
  const lptr<int> ab = (lptr<int>)&sr.abort;
  const int nblk = (n + kWave - 1) / kWave;
  const int nfull = (n % kWave == 0) ? nblk : nblk - 1;
  if (!ring_wait((lptr<int>)&sr.staged[0], 1, ab, abort_flag)) return false;
  if (nblk > 1 && !ring_wait((lptr<int>)&sr.staged[1 % SLOTS], 2, ab, abort_flag)) return false;
  double x1 = 0.0, x2 = 0.0, ss = 0.0;
  SRow ring[kSweepRing];
#pragma unroll
  for (int d = 0; d < kSweepRing; d++) ring[d] = lds_row((ldrp)sr.row[0] + (kWave - 1 - d));
  int k = 0;
  for (; k < nfull; k++) {
    // the ring reads reach into block k + 1 (stale rows past the last block
    // are read and never used)
    if (k + 1 < nblk &&
        !ring_wait((lptr<int>)&sr.staged[(k + 1) % SLOTS], k + 2, ab, abort_flag))
      return false;
    if (lane == 0) {
      if (ss_out)
        sweep_block<true>((ldrp)sr.row[k % SLOTS], (ldrp)sr.row[(k + 1) % SLOTS], ring, x1, x2, ss,
                          v + (n - kWave * (k + 1)));
      else
        sweep_block<false>((ldrp)sr.row[k % SLOTS], (ldrp)sr.row[(k + 1) % SLOTS], ring, x1, x2,
                           ss, v + (n - kWave * (k + 1)));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    if (lane == 0) __hip_atomic_store((lptr<int>)&sr.freed, k + 1, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
    publish(n - kWave * (k + 1));
  }
  if (k < nblk) {  // the partial last block (rows 0 .. n mod 64 - 1), already waited for
    if (lane == 0) {
      const ldrp cur = (ldrp)sr.row[k % SLOTS];
      const int base = n - kWave * (k + 1);
      for (int t = kWave - 1; t >= 0 && base + t >= 0; t--) {
        const SRow c = lds_row(cur + t);
        const double x = fma(-c.a, x1, fma(-c.b, x2, c.y));
        x2 = x1;
        x1 = x;
        v[base + t] = x;
        ss = fma(x, x, ss);
      }
    }
    publish(0);
  }
  if (ss_out && lane == 0) st_dev(ss_out, ss);
  return true;
}

// Producer p of np (one wave each): stages blocks p, p + np, ...  The row of
// block k for lane j is i = n - 64 (k + 1) + j; its y'_i = y_i / u1_i comes
// from the chunk scans: the carry into row i's chunk advanced by the chunk's
// prefix map (or, where rows were swapped, the right-hand side itself).  The
// loads of the producer's next block are issued before it waits for a slot.
template <int SLOTS>
__device__ bool sweep_produce(SweepRing<SLOTS> &sr, int p, int np, const double4 *R_,
                              const double *q_, double rn, const double *P_, const double *Q_,
                              lptr<const double> carry_lds, const double *carry_glb,
                              const unsigned char *SW, int n, int lane, int *abort_flag) {
  const gptr<const double> rd = (gptr<const double>)(R_);   // record i at rd[4i .. 4i+3]
  const gptr<const double> q = (gptr<const double>)q_;
  const gptr<const double> P = (gptr<const double>)P_;
  const gptr<const double> Q = (gptr<const double>)Q_;
  const gptr<const double> cg = (gptr<const double>)carry_glb;
  const gptr<const unsigned char> sw = (gptr<const unsigned char>)SW;
  const lptr<int> ab = (lptr<int>)&sr.abort;
  const int nblk = (n + kWave - 1) / kWave;
  struct Raw {
    double u, a, b, p, qq, qn;
    int s;
  };
  auto row = [&](int k) { return (k < nblk) ? n - kWave * (k + 1) + lane : -1; };
  auto load = [&](int k) {
    Raw r;
    const int i = row(k);
    r.u = r.a = r.b = r.p = r.qq = r.qn = 0.0;
    r.s = 0;
    if (i >= 0) {
      const size_t o = 4 * (size_t)i;
      r.u = rd[o + 1];
      r.a = rd[o + 2];
      r.b = rd[o + 3];
      if (i % kWave != 0) { r.p = P[i - 1]; r.qq = Q[i - 1]; }
      if (i < n - 1) { r.qn = q[i + 1]; r.s = sw[i]; }
    }
    return r;
  };
  Raw nx = load(p);
  for (int k = p; k < nblk; k += np) {
    const Raw r = nx;
    nx = load(k + np);
    // slot k % SLOTS last held block k - SLOTS
    if (k >= SLOTS && !ring_wait((lptr<int>)&sr.freed, k - SLOTS + 1, ab, abort_flag))
      return false;
    const int i = row(k);
    SRow w = {0.0, 0.0, 0.0, 0.0};
    if (i >= 0) {
      const double ck = carry_lds ? carry_lds[i / kWave] : cg[i / kWave];
      double y = (i % kWave == 0) ? ck : fma(r.p, ck, r.qq);
      if (r.s) y = r.qn * rn;
      w = {r.a, r.b, y * r.u, 0.0};
    }
    __attribute__((address_space(3))) SRow *dst = (__attribute__((address_space(3))) SRow *)sr.row[k % SLOTS] + lane;
    dst->a = w.a;
    dst->b = w.b;
    dst->y = w.y;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    if (lane == 0)
      __hip_atomic_store((lptr<int>)&sr.staged[k % SLOTS], k + 1, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  return true;
}

// P1 arithmetic, x_l = Y[:, l] . v over rows l..n-1 (column l of Y is zero
// above row l), in kSegRows-row segments counted from row 0: each segment's
// dot by one wave, the segments added from the bottom up.  The plain pass and
// the pass overlapped with the back sweep produce the same bits.
__device__ __forceinline__ double seg_dot(const double *col, const double *v, int l, int n, int s,
                                          int lane) {
  const int lo = s * kSegRows > l ? s * kSegRows : l;
  const int hi = (s + 1) * kSegRows < n ? (s + 1) * kSegRows : n;
  return wave_dot(col, v, lo, hi, lane);
}

__device__ __forceinline__ double col_dot_segmented(const double *col, const double *v, int l,
                                                    int n, int lane) {
  const int top = (n - 1) / kSegRows;
  double acc = 0.0;
  for (int s = top; s >= l / kSegRows; s--) {
    const double d = seg_dot(col, v, l, n, s, lane);
    acc = (s == top) ? d : acc + d;
  }
  return acc;
}

// The next iteration's P1 (x = Y_c^T v) computed while rank 0 runs the back
// sweep: the workgroups of ranks 1..size-1 take the columns, follow the
// sweep's published progress segment by segment (thread 0 polls, then an
// acquire), and accumulate each column (owned by one wave) from the bottom
// segment up, the running sums of a wave's first kAcc columns in LDS (a
// global read-modify-write per column and segment would put a memory round
// trip on every step), writing x[l] once the column is complete.  With v2
// given, the same pass also accumulates x2_l = Y[:, l] . v2 (the lookahead's
// products), from the same loads.  Returns false on abort.
template <int NT>
__device__ bool p1_overlapped(Ctx &cx, const CView &cv, int c, const double *v, double *x,
                              const double *v2, double *x2, const unsigned long long *prog,
                              unsigned long long seq) {
  const int n = cv.n;
  const int top = (n - 1) / kSegRows;
  const int gw = (cx.rank - 1) * (NT / kWave) + cx.wave;
  const int nw = (cx.size - 1) * (NT / kWave);
  __shared__ int s_go;
  constexpr int kAcc = 64;   // partial sums kept in LDS per wave
  __shared__ double s_acc[NT / kWave][kAcc], s_acc2[NT / kWave][kAcc];
  for (int s = top; s >= 0; s--) {
    if (threadIdx.x == 0) {
      const unsigned long long target = (seq << 32) | (unsigned long long)(n - s * kSegRows);
      int ok = 1;
      unsigned long long spins = 0;
      while (__hip_atomic_load(prog, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        if ((++spins & 255ull) == 0) {
          if (__hip_atomic_load(cx.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = 0;
            break;
          }
          if (spins > kSpinLimit) {
            __hip_atomic_store(cx.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
        }
      }
      wg_acquire();
      s_go = ok;
    }
    __syncthreads();
    if (!s_go) return false;
    int j = 0;
    for (int l = gw; l < c; l += nw, j++) {
      if (s < l / kSegRows) continue;   // segment above row l
      const double *col = cv.Y + (size_t)l * cv.ldy;
      const bool last = (s == l / kSegRows);
      if (v2) {   // both products from one read of the column segment
        const int lo = s * kSegRows > l ? s * kSegRows : l;
        const int hi = (s + 1) * kSegRows < n ? (s + 1) * kSegRows : n;
        double d, d2;
        wave_dot_pair(col, v, v2, lo, hi, cx.lane, d, d2);
        if (cx.lane == 0) {
          if (j < kAcc) {
            const double a = (s == top) ? d : s_acc[cx.wave][j] + d;
            const double a2 = (s == top) ? d2 : s_acc2[cx.wave][j] + d2;
            s_acc[cx.wave][j] = a;
            s_acc2[cx.wave][j] = a2;
            if (last) { st_dev(&x[l], a); st_dev(&x2[l], a2); }
          } else {
            st_dev(&x[l], (s == top) ? d : x[l] + d);
            st_dev(&x2[l], (s == top) ? d2 : x2[l] + d2);
          }
        }
      } else {
        const double d = seg_dot(col, v, l, n, s, cx.lane);
        if (cx.lane == 0) {
          if (j < kAcc) {
            const double a = (s == top) ? d : s_acc[cx.wave][j] + d;
            s_acc[cx.wave][j] = a;
            if (last) st_dev(&x[l], a);
          } else {
            st_dev(&x[l], (s == top) ? d : x[l] + d);
          }
        }
      }
    }
  }
  return true;
}

// Lookahead for member c + 1, prepared while member c iterates.  Member
// c + 1's first compact-WY step needs, with v its raw first iterate (column
// c + 1 of Z):
//   x_l = Y[:, l] . v, x'_l = T[0..l, l] . x, u_i = v_i - Yhat[i, :] x'.
// Columns 0..c-1 of Y and T do not change while member c iterates, so
//   vla = v, xla_l = x_l and xpla_l = x'_l for l < c, and
//   upre_i = (vla_i - Yhat[i, 0..c-1) . xpla) - Y[i, c-1] xpla_{c-1}, rows i > c,
// are prepared in the same arithmetic the plain passes use (the term of
// column c follows once member c is final; a plain first step takes the last
// two columns apart for that reason): in the first back sweep the ranks
// 1..size-1 stage vla and xla rides along the overlapped P1's reads of Y;
// xpla rides along the P2 reads of T and upre along the P3 reads of Yhat of
// member c's last step.
// Barriers here are among the ranks taking part.  Return false on abort.
// Row passes (P3, P6) while the cluster has few columns (c <= kShortRows):
// a wave per row would leave most lanes idle on rows this short, so each
// thread takes whole rows instead, reading Y column-major (coalesced across
// the threads; row_dot_cm).  Every chain,
// whatever kernel or group runs it, takes this path for the same c, so the
// results still do not depend on where a chain runs.
constexpr int kShortRows = 256;
constexpr int kColsInFlight = 4;   // column dots per wave at a time while c <= kShortRows
constexpr int kColsVar = 2;        // the same for dots of different ranges (Y^T v, T^T x)

// sum_{l < len} Y[i + l ldy] x[l] for one row i of column-major Y, by one
// thread: eight interleaved partial sums (l mod 8) added pairwise, which keeps
// the rounding error growth near that of a tree sum.
__device__ __forceinline__ double row_dot_cm(const double *Y_, size_t ldy, int i,
                                             const double *x_, int len) {
  const gdp Y = (gdp)Y_, x = (gdp)x_;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int l = 0;
  for (; l + 8 <= len; l += 8) {
#pragma unroll
    for (int r = 0; r < 8; r++) a[r] = fma(Y[(size_t)(l + r) * ldy + i], x[l + r], a[r]);
  }
#pragma unroll
  for (int r = 0; r < 8; r++)
    if (l + r < len) a[r] = fma(Y[(size_t)(l + r) * ldy + i], x[l + r], a[r]);
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// row_dot_cm for two vectors at once, each with row_dot_cm's arithmetic.
__device__ __forceinline__ void row_dot_cm2(const double *Y_, size_t ldy, int i, const double *x_,
                                            const double *z_, int len, double &ox,
                                            double &oz) {
  const gdp Y = (gdp)Y_, x = (gdp)x_, z = (gdp)z_;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double b[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int l = 0;
  for (; l + 8 <= len; l += 8) {
#pragma unroll
    for (int r = 0; r < 8; r++) {
      const double y = Y[(size_t)(l + r) * ldy + i];
      a[r] = fma(y, x[l + r], a[r]);
      b[r] = fma(y, z[l + r], b[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < 8; r++) {
    if (l + r < len) {
      const double y = Y[(size_t)(l + r) * ldy + i];
      a[r] = fma(y, x[l + r], a[r]);
      b[r] = fma(y, z[l + r], b[r]);
    }
  }
  ox = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  oz = ((b[0] + b[1]) + (b[2] + b[3])) + ((b[4] + b[5]) + (b[6] + b[7]));
}

template <int NT>
__device__ Ctx la_sub(const Ctx &cx) {
  Ctx sub = cx;
  sub.rank = cx.rank - 1;
  sub.size = cx.size - 1;
  sub.cnt = cx.cnt + kBarSubRegion;
  sub.flag = nullptr;
  sub.gen = cx.sgen;
  sub.gw = sub.rank * (NT / kWave) + cx.wave;
  sub.nw = sub.size * (NT / kWave);
  return sub;
}

template <int NT>
__device__ bool la_stage(Ctx &cx, const CView &cv, int c, const Scr &S) {
  Ctx sub = la_sub<NT>(cx);
  const int gtid = sub.rank * NT + (int)threadIdx.x, gthreads = sub.size * NT;
  const double *zn = cv.Z + (size_t)(c + 1) * cv.ldz;
  for (int i = gtid; i < cv.n; i += gthreads) st_dev(&S.vla[i], zn[i]);
  const bool ok = grp_sync<NT>(sub);
  cx.sgen = sub.gen;
  return ok;
}

// Solve (T - lambda I) v = q/||q|| with the stored LU of member c.
// rn = 1/||q|| comes from the pass that produced q.
//  S1  the waves of the group scan 64-row chunks of the affine maps
//      cur_{i+1} = A_i cur_i + B_i of the forward sweep (|A_i| <= 1 under
//      partial pivoting, so the scan is as stable as the recurrence);
//  S2  wave 0 of rank 0 scans the chunk summaries for the carries into
//      each chunk (in LDS);
//  S3  the back sweep x_i = y'_i - (u2/u1)_i x_{i+1} - (u3/u1)_i x_{i+2}
//      runs sequentially in lane 0 of wave 0 of rank 0 (a blocked version
//      of it is not stable) while the other waves of rank 0 form
//      y'_i = y_i / u1_i and stage the rows ahead of it (sweep_consume,
//      sweep_produce).  Meanwhile the other ranks do overlapped work.
// Returns false on abort.
constexpr int kLdsCarries = 2048;

template <int NT>
__device__ bool grp_solve(Ctx &cx, const CView &cv, int c, const double *__restrict__ q,
                          double *__restrict__ v, const Scr &S, double rn, bool overlap_p1,
                          bool la, double *ss_out) {
  const int n = cv.n;
  const int tid = threadIdx.x, lane = cx.lane, wave = cx.wave;
  constexpr int NW = NT / kWave;
  const double4 *__restrict__ R = as_global(cv.Lrec + (size_t)c * n);
  const unsigned char *__restrict__ SW = as_global(cv.Lswb + (size_t)c * n);
  q = as_global(q);
  v = as_global(v);
  __shared__ double s_carry[kLdsCarries + 1];
  constexpr int kSlots = NT >= 512 ? 16 : 8;
  __shared__ SweepRing<kSlots> s_ring;

  // S1: chunk scans over the whole group (chunk summaries in S.csum)
  const int nmaps = n - 1;
  const int nch = (nmaps + kWave - 1) / kWave;
  const gptr<const double> rd = (gptr<const double>)R;
  const gptr<const unsigned char> sw = (gptr<const unsigned char>)SW;
  const gptr<const double> qg = (gptr<const double>)q;
  for (int k = cx.gw; k < nch; k += cx.nw) {
    const int i = k * kWave + lane;
    double A = 1.0, B = 0.0;
    if (i < nmaps) {
      const double bn = qg[i + 1] * rn;
      const double l = rd[4 * (size_t)i];
      if (sw[i]) { A = 1.0; B = -(l * bn); }
      else { A = -l; B = bn; }
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const double Ap = __shfl_up(A, off, kWave);
      const double Bp = __shfl_up(B, off, kWave);
      if (lane >= off) { B = fma(A, Bp, B); A = A * Ap; }
    }
    if (i < nmaps) { st_dev(&S.P[i], A); st_dev(&S.Q[i], B); }
    if (lane == kWave - 1) { st_dev(&S.csum[2 * k], A); st_dev(&S.csum[2 * k + 1], B); }
  }
  if (!grp_sync<NT>(cx)) return false;

  // carries into the chunks: in LDS when they fit, else in the scratch slot
  const bool lds_carry = nch <= kLdsCarries;
  lptr<double> carry_lds = lds_carry ? (lptr<double>)s_carry : nullptr;
  const gptr<double> carry_glb = (gptr<double>)S.carry;
  if (cx.rank == 0) {
    // S2: carries into each chunk (scan of the chunk summaries, 64 at a time)
    if (wave == 0) {
      double cur = q[0] * rn;
      for (int k0 = 0; k0 < nch; k0 += kWave) {
        const int k = k0 + lane;
        double A = 1.0, B = 0.0;
        if (k < nch) { A = S.csum[2 * k]; B = S.csum[2 * k + 1]; }
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
          const double Ap = __shfl_up(A, off, kWave);
          const double Bp = __shfl_up(B, off, kWave);
          if (lane >= off) { B = fma(A, Bp, B); A = A * Ap; }
        }
        const double Ae = __shfl_up(A, 1, kWave), Be = __shfl_up(B, 1, kWave);
        const double ck = lane == 0 ? cur : fma(Ae, cur, Be);
        if (k < nch) {
          if (lds_carry) carry_lds[k] = ck;
          else carry_glb[k] = ck;
        }
        const double Al = __shfl(A, kWave - 1, kWave), Bl = __shfl(B, kWave - 1, kWave);
        cur = fma(Al, cur, Bl);
      }
      if (lane == 0) {
        if (lds_carry) carry_lds[nch] = cur;
        else carry_glb[nch] = cur;
      }
    } else if (wave == 1) {   // reset the sweep ring (the last sweep ended at a barrier)
      if (lane < kSlots) s_ring.staged[lane] = 0;
      if (lane == 0) { s_ring.freed = 0; s_ring.abort = 0; }
    }
    __syncthreads();
  }

  // S3: back substitution, one lane of one wave; with overlap_p1 (groups of
  // two or more workgroups) the other ranks compute the next P1 meanwhile,
  // and with la the lookahead's first part for member c + 1 (stage vla, and
  // xla from the same reads of Y).
  unsigned long long *prog = reinterpret_cast<unsigned long long *>(cx.cnt + kBarProg);
  const unsigned long long seq = cx.gen;
  if (cx.rank == 0) {
    // wave 0 sweeps, the other waves stage its rows; a failed ring wait
    // marks the ring, and the workgroup leaves together
    if (wave == 0)
      sweep_consume<kSlots>(s_ring, v, n, lane, overlap_p1 ? prog : nullptr, seq, cx.abort_flag,
                            ss_out);
    else
      sweep_produce<kSlots>(s_ring, wave - 1, NW - 1, R, q, rn, S.P, S.Q, carry_lds, S.carry, SW,
                            n, lane, cx.abort_flag);
    __syncthreads();
    if (__hip_atomic_load((lptr<int>)&s_ring.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
      return false;
  } else if (overlap_p1) {
    if (la && !la_stage<NT>(cx, cv, c, S)) return false;
    if (!p1_overlapped<NT>(cx, cv, c, v, S.x, la ? S.vla : nullptr, la ? S.xla : nullptr,
                           prog, seq))
      return false;
  }
  return grp_sync<NT>(cx);
}


// Runs the chain of one cluster with the group described by ctx.  Returns
// false if the run was aborted.
template <int NT>
__device__ bool run_chain(Ctx &cx, const Prob &P, const ChainItem &it, const Scr &S, int iters) {
  CView cv;
  const size_t s0 = (size_t)it.start;
  cv.n = P.n; cv.M = it.size;
  cv.ldy = (size_t)P.ldy;
  cv.ldm = (size_t)P.ldm;
  cv.Y = as_global(P.Y + s0 * cv.ldy);
  cv.Yr = as_global(P.Yr + s0);
  cv.T = as_global(P.T + s0 + s0 * cv.ldm);
  cv.Tr = as_global(P.Tr + s0 + s0 * cv.ldm);
  cv.Z = as_global(P.Z + s0 * P.ldz);
  cv.ldz = (size_t)P.ldz;
  cv.Lrec = as_global(reinterpret_cast<const double4 *>(P.Lrec) + s0 * P.n);
  cv.Lswb = as_global(P.Lswb + s0 * P.n);
  const int n = cv.n;
  const size_t ldy = cv.ldy, ldm = cv.ldm;
  const int tid = threadIdx.x, lane = cx.lane;
  const int gtid = cx.rank * NT + tid, gthreads = cx.size * NT;

  // Y_1, T_1 from the first member's unit vector z (Alg. 4, first step of the
  // second member): c_1 = -sgn(z_0)||z||, y_1 = z - c_1 e_0, t_1 = 1/(c_1^2 - z_0 c_1).
  // The raw first iterate of member 1 is staged into the aligned scratch v.
  {
    const double *z = cv.Z;
    const double *z1 = cv.Z + cv.ldz;
    for (int i = gtid; i < n; i += gthreads) st_dev(&S.v[i], z1[i]);
    double nz2;
    if (!grp_sumsq<NT>(cx, z, 0, n, nz2)) return false;
    const double z0 = z[0];
    const double g = -(z0 >= 0.0 ? 1.0 : -1.0) * sqrt(nz2);
    for (int i = gtid; i < n; i += gthreads) {
      const double y = (i == 0) ? z0 - g : z[i];
      st_dev(&cv.Y[i], y);
      st_dev(&cv.Yr[(size_t)i * ldm], y);
    }
    if (gtid == 0) {
      const double t = (g == 0.0) ? 0.0 : 1.0 / (g * g - z0 * g);
      st_dev(&cv.T[0], t);
      st_dev(&cv.Tr[0], t);
    }
    if (!grp_sync<NT>(cx)) return false;
  }

  const double *vin = S.v;
  const bool overlap_p1 = cx.size > 1;
  const bool stop = iters < 0;   // the growth rule: at least 1 + kStopExtra iterations
  // member c + 1's first step prepared during member c (needs a back sweep of
  // member c to overlap with, hence two or more iterations, and a group to
  // share it with)
  const bool use_la = overlap_p1 && (stop || iters >= 2);
  bool x_ready = false;   // P1 already done beside the last back sweep
  bool la_ready = false;  // this member's first step prepared by the lookahead
  __shared__ double s_xpc;
  for (int c = 1; c < cv.M; c++) {
    const bool la_next = use_la && c + 1 < cv.M;
    const double *yprev = cv.Y + (size_t)(c - 1) * ldy;   // column c - 1 of Y
    int kend = iters;   // the last iteration of this member
    bool conv = false;
    if (stop) {         // the first solve ran with the parallel solves
      conv = growth_converged(P.nrm[it.start + c], n, P.prm->norm1);
      kend = conv ? 1 + kStopExtra : kStopMaxIts;
    }
    for (int k = 1; k <= kend; k++) {
      if (k == 1 && la_ready) {
        // P1-P3 from the lookahead: x_{c-1} arrived with member c - 1's last
        // step; x'_{c-1} = T[0..c-1, c-1] . x is formed by every workgroup
        // (same bits everywhere); then u = upre - y_{c-1} x'_{c-1}.
        if (cx.wave == 0) {
          const double xpc = wave_dot(cv.T + (size_t)(c - 1) * ldm, S.xla, 0, c, lane);
          if (lane == 0) s_xpc = xpc;
        }
        __syncthreads();
        const double xpc = s_xpc;
        for (int i = c + gtid; i < n; i += gthreads) st_dev(&S.u[i], S.upre[i] - yprev[i] * xpc);
      } else {
        // P1: x = Y_c^T v
        if (!x_ready) {
          if (c <= kShortRows) {   // few columns: kColsVar per wave (same bits)
            const int top = (n - 1) / kSegRows;
            for (int l0 = cx.gw; l0 < c; l0 += kColsVar * cx.nw) {
              const int nr = min(kColsVar, (c - 1 - l0) / cx.nw + 1);
              const double *col[kColsVar];
              int lo[kColsVar], hi[kColsVar];
              double acc[kColsVar], d[kColsVar];
#pragma unroll
              for (int r = 0; r < kColsVar; r++) {
                col[r] = cv.Y + (size_t)(l0 + r * cx.nw) * ldy;
                acc[r] = 0.0;
              }
              // col_dot_segmented's order: segments from the top, added bottom-up
              for (int sg = top; sg >= 0; sg--) {
                int ns = 0;   // columns reaching segment sg (a prefix: l grows with r)
#pragma unroll
                for (int r = 0; r < kColsVar; r++) {
                  const int l = l0 + r * cx.nw;
                  if (r < nr && sg >= l / kSegRows) ns = r + 1;
                  lo[r] = sg * kSegRows > l ? sg * kSegRows : l;
                  hi[r] = (sg + 1) * kSegRows < n ? (sg + 1) * kSegRows : n;
                }
                if (ns == 0) break;
                wave_dot_var<kColsVar>(col, vin, lo, hi, ns, lane, d);
#pragma unroll
                for (int r = 0; r < kColsVar; r++)
                  if (r < ns) acc[r] = (sg == top) ? d[r] : acc[r] + d[r];
              }
              if (lane == 0) {
#pragma unroll
                for (int r = 0; r < kColsVar; r++)
                  if (r < nr) st_dev(&S.x[l0 + r * cx.nw], acc[r]);
              }
            }
          } else {
            for (int l = cx.gw; l < c; l += cx.nw) {
              const double acc = col_dot_segmented(cv.Y + (size_t)l * ldy, vin, l, n, lane);
              if (lane == 0) st_dev(&S.x[l], acc);
            }
          }
          if (!grp_sync<NT>(cx)) return false;
        }
        // P2: x' = T_c^T x (column l has l + 1 entries: folded assignment),
        // kColsVar columns per wave at a time while c is small (same bits).
        // In the last step of a member with a lookahead the same reads of T
        // also give xpla = T_c^T xla for member c + 1 (wave_dot's bits).
        const bool share2 = (k == kend) && la_next;
        if (c <= kShortRows) {
          for (int t0 = 0; fold_valid(cx.gw, cx.nw, t0, c); t0 += kColsVar) {
            const double *col[kColsVar];
            int lo[kColsVar], hi[kColsVar], ls[kColsVar];
            double d[kColsVar];
            int nr = 0;
#pragma unroll
            for (int r = 0; r < kColsVar; r++) {
              const bool ok = fold_valid(cx.gw, cx.nw, t0 + r, c);
              ls[r] = ok ? fold_index(cx.gw, cx.nw, t0 + r, c) : 0;
              if (ok && nr == r) nr = r + 1;
              col[r] = cv.T + (size_t)ls[r] * ldm;
              lo[r] = 0;
              hi[r] = ls[r] + 1;
            }
            wave_dot_var<kColsVar>(col, S.x, lo, hi, nr, lane, d);
            if (lane == 0) {
#pragma unroll
              for (int r = 0; r < kColsVar; r++)
                if (r < nr) st_dev(&S.xp[ls[r]], d[r]);
            }
          }
        } else {
          for (int t = 0; fold_valid(cx.gw, cx.nw, t, c); t++) {
            const int l = fold_index(cx.gw, cx.nw, t, c);
            if (share2) {
              double acc, acc2;
              wave_dot_pair(cv.T + (size_t)l * ldm, S.x, S.xla, 0, l + 1, lane, acc, acc2);
              if (lane == 0) { st_dev(&S.xp[l], acc); st_dev(&S.xpla[l], acc2); }
            } else {
              const double acc = wave_dot(cv.T + (size_t)l * ldm, S.x, 0, l + 1, lane);
              if (lane == 0) st_dev(&S.xp[l], acc);
            }
          }
        }
        if (share2 && c <= kShortRows) {
          for (int t = 0; fold_valid(cx.gw, cx.nw, t, c); t++) {
            const int l = fold_index(cx.gw, cx.nw, t, c);
            const double acc2 = wave_dot(cv.T + (size_t)l * ldm, S.xla, 0, l + 1, lane);
            if (lane == 0) st_dev(&S.xpla[l], acc2);
          }
        }
        if (!grp_sync<NT>(cx)) return false;
        // P3: u = v_hat - Yhat_c x' over rows c..n-1, the last column's term
        // taken apart: u_i = (v_i - Yhat[i, 0..c-1) . x') - y_{c-1,i} x'_{c-1};
        // a member's first step takes the last two columns apart (the
        // lookahead's arithmetic).  In the last step of a member with a
        // lookahead, the same reads of Yhat also give upre for member c + 1
        // (rows c + 1..n-1, with member c + 1's choice of row path).
        const double xpc = S.xp[c - 1];
        const bool first = (k == 1 && c >= 2);
        const int nd = first ? c - 2 : c - 1;
        const double *ypp = cv.Y + (size_t)(first ? c - 2 : 0) * ldy;   // column c - 2
        const double xppc = first ? S.xp[c - 2] : 0.0;
        const bool share = (k == kend) && la_next && !first;
        const bool short_u = c <= kShortRows, short_la = c + 1 <= kShortRows;
        const double xplc = share ? S.xpla[c - 1] : 0.0;
        auto u_of = [&](int i, double acc) {
          const double w = vin[i] - acc;
          return first ? (w - ypp[i] * xppc) - yprev[i] * xpc : w - yprev[i] * xpc;
        };
        if (short_u) {   // short rows: one thread per row over column-major Y
          for (int i = c + gtid; i < n; i += gthreads) {
            if (share && short_la) {
              double acc, acc2;
              row_dot_cm2(cv.Y, ldy, i, S.xp, S.xpla, nd, acc, acc2);
              st_dev(&S.u[i], u_of(i, acc));
              if (i > c) st_dev(&S.upre[i], (S.vla[i] - acc2) - yprev[i] * xplc);
            } else {
              st_dev(&S.u[i], u_of(i, row_dot_cm(cv.Y, ldy, i, S.xp, nd)));
            }
          }
        } else {
          for (int i = c + cx.gw; i < n; i += cx.nw) {
            if (share) {
              double acc, acc2;
              wave_dot_pair(cv.Yr + (size_t)i * ldm, S.xp, S.xpla, 0, nd, lane, acc, acc2);
              if (lane == 0) {
                st_dev(&S.u[i], u_of(i, acc));
                if (i > c) st_dev(&S.upre[i], (S.vla[i] - acc2) - yprev[i] * xplc);
              }
            } else {
              const double acc = wave_dot(cv.Yr + (size_t)i * ldm, S.xp, 0, nd, lane);
              if (lane == 0) st_dev(&S.u[i], u_of(i, acc));
            }
          }
        }
        if (share && short_u && !short_la) {   // c = kShortRows: upre by member c + 1's path
          for (int i = c + 1 + cx.gw; i < n; i += cx.nw) {
            const double acc2 = wave_dot(cv.Yr + (size_t)i * ldm, S.xpla, 0, nd, lane);
            if (lane == 0) st_dev(&S.upre[i], (S.vla[i] - acc2) - yprev[i] * xplc);
          }
        }
      }
      x_ready = false;
      double beta2;
      if (!grp_sumsq<NT>(cx, S.u, c, n, beta2)) return false;
      // P4: Householder vector and s = Yhat_c^T y_hat
      const double alpha = S.u[c];
      const double beta = sqrt(beta2);
      const double gam = -(alpha >= 0.0 ? 1.0 : -1.0) * beta;
      const double tj = (gam == 0.0) ? 0.0 : 1.0 / (gam * gam - alpha * gam);
      const double yc = alpha - gam;
      if (gam == 0.0 && gtid == 0 && P.info)   // reflector breakdown: H = I
        P.info[1 + it.start + c] |= TE_INFO_BREAKDOWN;
      if (c <= kShortRows) {   // few columns: kColsInFlight per wave (wave_dot's bits)
        for (int l0 = cx.gw; l0 < c; l0 += kColsInFlight * cx.nw) {
          const int nr = min(kColsInFlight, (c - 1 - l0) / cx.nw + 1);
          double acc[kColsInFlight];
          wave_dot_multi<kColsInFlight>(cv.Y + (size_t)l0 * ldy, (size_t)cx.nw * ldy, nr, S.u,
                                        c + 1, n, lane, acc);
          if (lane == 0) {
#pragma unroll
            for (int r = 0; r < kColsInFlight; r++) {
              if (r < nr) {
                const int l = l0 + r * cx.nw;
                const double rl = cv.Y[(size_t)l * ldy + c];
                st_dev(&S.s[l], fma(rl, yc, acc[r]));
                st_dev(&S.r[l], rl);
              }
            }
          }
        }
      } else {
        for (int l = cx.gw; l < c; l += cx.nw) {
          const double *col = cv.Y + (size_t)l * ldy;
          const double rl = col[c];   // loaded ahead of the dot's reduction
          const double acc = wave_dot(col, S.u, c + 1, n, lane);
          if (lane == 0) {
            st_dev(&S.s[l], fma(rl, yc, acc));
            st_dev(&S.r[l], rl);
          }
        }
      }
      {
        double *ycol = cv.Y + (size_t)c * ldy;
        for (int i = c + gtid; i < n; i += gthreads) {
          const double y = (i == c) ? yc : S.u[i];
          st_dev(&ycol[i], y);
          st_dev(&cv.Yr[(size_t)i * ldm + c], y);
        }
        if (gtid == 0) {
          st_dev(&cv.T[(size_t)c + (size_t)c * ldm], tj);
          st_dev(&cv.Tr[(size_t)c * ldm + c], tj);
        }
      }
      if (!grp_sync<NT>(cx)) return false;
      const bool last = (k == kend);
      // P5: t_hat = -t_j T_c s (column c of T) and x'' = T_{c+1} r
      // (row p has c - p entries: folded assignment).  Lookahead: the
      // segment dots of x_c = Y[:, c] . vla for member c + 1, one wave each
      // from the last wave down.
      if (last && la_next) {
        const int top = (n - 1) / kSegRows, s0 = c / kSegRows;
        for (int sg = top - (cx.nw - 1 - cx.gw); sg >= s0; sg -= cx.nw) {
          const double d = seg_dot(cv.Y + (size_t)c * ldy, S.vla, c, n, sg, lane);
          if (lane == 0) st_dev(&S.xseg[sg], d);
        }
      }
      if (c <= kShortRows) {   // short rows of T: one thread per row p
        const gdp Tc = (gdp)cv.T, sv = (gdp)S.s, rv = (gdp)S.r;
        for (int p = gtid; p < c; p += gthreads) {
          // l = c-1 down to p (the same l across the threads: coalesced), in
          // eight interleaved partial sums added pairwise
          double bs[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
          double br[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
          const int len = c - p;
          int k = 0;
          for (; k + 8 <= len; k += 8) {
#pragma unroll
            for (int r = 0; r < 8; r++) {
              const int l = c - 1 - (k + r);
              const double t = Tc[(size_t)p + (size_t)l * ldm];
              bs[r] = fma(t, sv[l], bs[r]);
              br[r] = fma(t, rv[l], br[r]);
            }
          }
#pragma unroll
          for (int r = 0; r < 8; r++) {
            if (k + r < len) {
              const int l = c - 1 - (k + r);
              const double t = Tc[(size_t)p + (size_t)l * ldm];
              bs[r] = fma(t, sv[l], bs[r]);
              br[r] = fma(t, rv[l], br[r]);
            }
          }
          const double ts = ((bs[0] + bs[1]) + (bs[2] + bs[3])) + ((bs[4] + bs[5]) + (bs[6] + bs[7]));
          const double tr = ((br[0] + br[1]) + (br[2] + br[3])) + ((br[4] + br[5]) + (br[6] + br[7]));
          const double th = -tj * ts;
          st_dev(&cv.T[(size_t)p + (size_t)c * ldm], th);
          st_dev(&cv.Tr[(size_t)p * ldm + c], th);
          st_dev(&S.xpp[p], fma(th, yc, tr));
        }
      } else {
        // r (row c of Y_c) and T_c stay the same through a member's steps,
        // so T_c r is formed in its first step and reused after; later steps
        // read T against s alone.
        for (int t = 0; fold_valid(cx.gw, cx.nw, t, c); t++) {
          const int p = fold_index(cx.gw, cx.nw, t, c);
          double ts, tr;
          if (k == 1) {
            wave_dot2(cv.Tr + (size_t)p * ldm + p, S.s + p, S.r + p, c - p, lane, ts, tr);
            if (lane == 0) st_dev(&S.tr[p], tr);
          } else {
            tr = S.tr[p];
            ts = wave_dot(cv.Tr + (size_t)p * ldm, S.s, p, c, lane);
          }
          if (lane == 0) {
            const double th = -tj * ts;
            st_dev(&cv.T[(size_t)p + (size_t)c * ldm], th);
            st_dev(&cv.Tr[(size_t)p * ldm + c], th);
            st_dev(&S.xpp[p], fma(th, yc, tr));
          }
        }
      }
      if (gtid == 0) st_dev(&S.xpp[c], tj * yc);
      if (!grp_sync<NT>(cx)) return false;
      // P6: q = Y_{c+1} x'' - e_c; after the last step, also stage the next
      // member's raw first iterate into the aligned scratch v.  Rows below c
      // are shorter (min(i, c) + 1 entries): folded assignment.  Lookahead:
      // the last wave adds the segment dots of x_c bottom-up (the order of
      // col_dot_segmented).
      if (last && la_next && cx.gw == cx.nw - 1 && lane == 0) {
        const int top = (n - 1) / kSegRows, s0 = c / kSegRows;
        double acc = S.xseg[top];
        for (int sg = top - 1; sg >= s0; sg--) acc = acc + S.xseg[sg];
        st_dev(&S.xla[c], acc);
      }
      double *qout = last ? (cv.Z + (size_t)c * cv.ldz) : S.q;
      if (c <= kShortRows) {   // short rows: one thread per row over column-major Y
        for (int i = gtid; i < n; i += gthreads) {
          const double acc = row_dot_cm(cv.Y, ldy, i, S.xpp, (i < c ? i : c) + 1);
          st_dev(&qout[i], (i == c) ? acc - 1.0 : acc);
        }
      } else {
        for (int t = 0; fold_valid(cx.gw, cx.nw, t, n); t++) {
          const int i = fold_index(cx.gw, cx.nw, t, n);
          const int l1 = (i < c ? i : c) + 1;
          const double acc = wave_dot(cv.Yr + (size_t)i * ldm, S.xpp, 0, l1, lane);
          if (lane == 0) st_dev(&qout[i], (i == c) ? acc - 1.0 : acc);
        }
      }
      if (last) {
        if (c + 1 < cv.M) {
          const double *zn = cv.Z + (size_t)(c + 1) * cv.ldz;
          for (int i = gtid; i < n; i += gthreads) st_dev(&S.v[i], zn[i]);
        }
        if (!grp_sync<NT>(cx)) return false;
      } else {
        // P7: next iterate v = (T - lambda I)^{-1} q / ||q||
        double qn2;
        if (!grp_sumsq<NT>(cx, S.q, 0, n, qn2)) return false;
        // the lookahead's first part rides along the first sweep
        const bool la = la_next && k == 1;
        const bool test = stop && !conv;
        if (!grp_solve<NT>(cx, cv, c, S.q, S.v, S, 1.0 / sqrt(qn2), overlap_p1, la,
                           test ? S.misc : nullptr))
          return false;
        x_ready = overlap_p1;
        if (test) {   // solve k + 1; its norm was written through before the barrier
          const double nx =
              sqrt(__hip_atomic_load(S.misc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (growth_converged(nx, n, P.prm->norm1)) {
            conv = true;
            kend = min(kend, k + 1 + kStopExtra);
          }
        }
      }
    }
    if (stop && !conv && gtid == 0 && P.info) P.info[1 + it.start + c] |= TE_INFO_NOCONV;
    la_ready = la_next;
  }
  return true;
}

constexpr int kSmallThreads = 256;
constexpr int kCoopThreads = 512;

// Small clusters: one workgroup of NT threads per cluster, items taken from a
// work counter.  The item count is nitems, or *nitems_dev when that is not
// null (a plan written on the device by k_plan_scatter).  Every chain sum has
// one order for any NT (see grp_sumsq), so the variants give identical bits.
template <int NT>
__global__ void __launch_bounds__(NT) k_chain_small(const Prob *__restrict__ probs,
                                                    const ChainItem *__restrict__ items,
                                                    int nitems, const int *nitems_dev,
                                                    int *counter, int *abort_flag,
                                                    ChainScratch scr, int iters) {
  __shared__ int s_item;
  Ctx cx;
  cx.rank = 0; cx.size = 1; cx.cnt = nullptr; cx.flag = nullptr; cx.gen = 0; cx.sgen = 0;
  cx.abort_flag = abort_flag;
  cx.wave = threadIdx.x / kWave; cx.lane = threadIdx.x % kWave;
  cx.gw = cx.wave; cx.nw = NT / kWave;
  if (nitems_dev) nitems = *nitems_dev;
  double *base = as_global(scr.base + (size_t)blockIdx.x * scr.stride);
  for (;;) {
    // after a failed run (abort flag set) no further items are taken
    if (threadIdx.x == 0)
      s_item = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   ? nitems
                   : atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_item;
    __syncthreads();
    if (idx >= nitems) break;
    const ChainItem it = items[idx];
    const Prob &P = probs[it.prob];
    const Scr S = make_scr(base, P.n, P.m, it.start & 1);
    run_chain<NT>(cx, P, it, S, iters);
  }
}

static const void *small_kernel(int nt) {
  switch (nt) {
    case 512: return (const void *)k_chain_small<512>;
    default: return (const void *)k_chain_small<kSmallThreads>;
  }
}

// ---------------------------------------------------------------------------
// The paper's baseline re-orthogonalization, modified Gram-Schmidt (Alg. 1,
// the DSTEIN scheme): after every solve of member c of a cluster,
// v <- v - <v, z_r> z_r for r = 0 .. c-1 in order, against the earlier
// members' final unit vectors.  Each projection needs the result of the one
// before it, so a member's step is c dependent dot products: one workgroup
// runs a chain, with v in registers (entry i in thread i mod NT, slot i / NT)
// and the next column's loads issued ahead of the reduction that closes the
// current projection.  The solves are those of the compact-WY chain
// (grp_solve).  Every reduction has one fixed order (wave butterflies, then
// the wave totals in wave order), so results do not depend on timing.
// ---------------------------------------------------------------------------
constexpr int kMgsSlots = 16;   // n <= kMgsThreads * kMgsSlots (TE_MGS_MAX_N)
static_assert(kMgsThreads * kMgsSlots == TE_MGS_MAX_N, "MGS size limit");

template <int NT, int K>
__device__ bool run_chain_mgs(Ctx &cx, const Prob &P, const ChainItem &it, const Scr &S,
                              int iters) {
  constexpr int NW = NT / kWave;
  CView cv;
  const size_t s0 = (size_t)it.start;
  cv.n = P.n; cv.M = it.size;
  cv.Y = nullptr; cv.Yr = nullptr; cv.T = nullptr; cv.Tr = nullptr;
  cv.ldy = 0; cv.ldm = 0;
  cv.Z = as_global(P.Z + s0 * P.ldz);
  cv.ldz = (size_t)P.ldz;
  cv.Lrec = as_global(reinterpret_cast<const double4 *>(P.Lrec) + s0 * P.n);
  cv.Lswb = as_global(P.Lswb + s0 * P.n);
  const int n = cv.n, tid = threadIdx.x;
  __shared__ double s_red[2][NW];
  int buf = 0;
  // Workgroup sum in a fixed order; the two buffers alternate, so one
  // barrier per sum suffices (a buffer is rewritten two sums later, after
  // every thread has passed the barrier of the sum in between).
  auto wg_sum = [&](double p) {
    p = wave_sum(p);
    if (cx.lane == 0) s_red[buf][cx.wave] = p;
    __syncthreads();
    double a = s_red[buf][0];
#pragma unroll
    for (int w = 1; w < NW; w++) a += s_red[buf][w];
    buf ^= 1;
    return a;
  };
  double v[K];
  for (int c = 1; c < cv.M; c++) {
    // the raw first solve of member c (written by the parallel solves)
    const gptr<double> zc = (gptr<double>)(cv.Z + (size_t)c * cv.ldz);
#pragma unroll
    for (int t = 0; t < K; t++) {
      const int i = tid + t * NT;
      v[t] = i < n ? zc[i] : 0.0;
    }
    int kend = iters;   // the last iteration of this member
    bool conv = false;
    if (iters < 0) {    // the growth rule; the first solve ran with the parallel solves
      conv = growth_converged(P.nrm[it.start + c], n, P.prm->norm1);
      kend = conv ? 1 + kStopExtra : kStopMaxIts;
    }
    for (int k = 1; k <= kend; k++) {
      if (k > 1) {   // normalize and solve Eq. (1)
        double p = 0.0;
#pragma unroll
        for (int t = 0; t < K; t++) {
          const int i = tid + t * NT;
          if (i < n) st_dev(&S.q[i], v[t]);
          p = fma(v[t], v[t], p);
        }
        const double ss = wg_sum(p);   // its barrier also orders the stores of q
        const bool test = iters < 0 && !conv;
        if (!grp_solve<NT>(cx, cv, c, S.q, S.v, S, 1.0 / sqrt(ss), false, 0,
                           test ? S.misc : nullptr))
          return false;
        if (test) {   // solve k
          const double nx =
              sqrt(__hip_atomic_load(S.misc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
          if (growth_converged(nx, n, P.prm->norm1)) {
            conv = true;
            kend = min(kend, k + kStopExtra);
          }
        }
        const gptr<const double> vg = (gptr<const double>)S.v;
#pragma unroll
        for (int t = 0; t < K; t++) {
          const int i = tid + t * NT;
          v[t] = i < n ? vg[i] : 0.0;
        }
      }
      // v <- v - <v, z_r> z_r, r = 0 .. c-1 (za: z_r, zb: z_{r+1} in flight)
      double za[K], zb[K];
      double p = 0.0;
      {
        const gptr<const double> z0 = (gptr<const double>)cv.Z;
#pragma unroll
        for (int t = 0; t < K; t++) {
          const int i = tid + t * NT;
          za[t] = i < n ? z0[i] : 0.0;
          p = fma(v[t], za[t], p);
        }
      }
      for (int r = 0; r < c; r++) {
        const bool more = r + 1 < c;
        if (more) {
          const gptr<const double> zn = (gptr<const double>)(cv.Z + (size_t)(r + 1) * cv.ldz);
#pragma unroll
          for (int t = 0; t < K; t++) {
            const int i = tid + t * NT;
            zb[t] = i < n ? zn[i] : 0.0;
          }
        }
        const double sr = wg_sum(p);
        p = 0.0;
        if (more) {
#pragma unroll
          for (int t = 0; t < K; t++) {
            v[t] = fma(-sr, za[t], v[t]);
            p = fma(v[t], zb[t], p);
            za[t] = zb[t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < K; t++) v[t] = fma(-sr, za[t], v[t]);
        }
      }
    }
    if (iters < 0 && !conv && tid == 0 && P.info) P.info[1 + it.start + c] |= TE_INFO_NOCONV;
    // z_c = v / ||v||, the unit vector later members project against
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < K; t++) p = fma(v[t], v[t], p);
    const double nv = sqrt(wg_sum(p));
#pragma unroll
    for (int t = 0; t < K; t++) {
      const int i = tid + t * NT;
      if (i < n) st_dev(cv.Z + (size_t)c * cv.ldz + i, v[t] / nv);
    }
    __syncthreads();
  }
  return true;
}

// MGS chains: one workgroup per cluster, items taken from a work counter
// (item count nitems, or *nitems_dev when that is not null).
__global__ void __launch_bounds__(kMgsThreads) k_chain_mgs(const Prob *__restrict__ probs,
                                                           const ChainItem *__restrict__ items,
                                                           int nitems, const int *nitems_dev,
                                                           int *counter, int *abort_flag,
                                                           ChainScratch scr, int iters) {
  __shared__ int s_item;
  Ctx cx;
  cx.rank = 0; cx.size = 1; cx.cnt = nullptr; cx.flag = nullptr; cx.gen = 0; cx.sgen = 0;
  cx.abort_flag = abort_flag;
  cx.wave = threadIdx.x / kWave; cx.lane = threadIdx.x % kWave;
  cx.gw = cx.wave; cx.nw = kMgsThreads / kWave;
  if (nitems_dev) nitems = *nitems_dev;
  double *base = as_global(scr.base + (size_t)blockIdx.x * scr.stride);
  for (;;) {
    if (threadIdx.x == 0)
      s_item = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   ? nitems
                   : atomicAdd(counter, 1);
    __syncthreads();
    const int idx = s_item;
    __syncthreads();
    if (idx >= nitems) break;
    const ChainItem it = items[idx];
    const Prob &P = probs[it.prob];
    const Scr S = make_scr(base, P.n, P.m, it.start & 1);
    run_chain_mgs<kMgsThreads, kMgsSlots>(cx, P, it, S, iters);
  }
}

hipError_t launch_chain_mgs(const Prob *probs, const ChainItem *items, int nitems_cap,
                            const int *nitems_dev, int *counter, int *abort_flag,
                            ChainScratch scr, int nwg, int iters, hipStream_t s) {
  if (nwg <= 0 || (!nitems_dev && nitems_cap <= 0)) return hipSuccess;
  hipLaunchKernelGGL(k_chain_mgs, dim3(nwg), dim3(kMgsThreads), 0, s, probs, items, nitems_cap,
                     nitems_dev, counter, abort_flag, scr, iters);
  return hipGetLastError();
}

int mgs_max_wgs(int device) {
  int ncu = 0, per = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_chain_mgs, kMgsThreads,
                                                   0) != hipSuccess)
    return 0;
  return ncu * per;
}

hipError_t launch_chain_small(const Prob *probs, const ChainItem *items, int nitems, int *counter,
                              int *abort_flag, ChainScratch scr, int nwg, int iters,
                              hipStream_t s) {
  if (nitems <= 0 || nwg <= 0) return hipSuccess;
  return launch_chain_small_dev(probs, items, nitems, nullptr, counter, abort_flag, scr, nwg,
                                kSmallThreads, iters, s);
}

hipError_t launch_chain_small_dev(const Prob *probs, const ChainItem *items, int nitems_cap,
                                  const int *nitems_dev, int *counter, int *abort_flag,
                                  ChainScratch scr, int nwg, int nt, int iters, hipStream_t s) {
  if (nwg <= 0) return hipSuccess;
  if (nt != kSmallThreads && nt != 512) return hipErrorInvalidValue;
  switch (nt) {
    case 512:
      hipLaunchKernelGGL(k_chain_small<512>, dim3(nwg), dim3(512), 0, s, probs, items, nitems_cap,
                         nitems_dev, counter, abort_flag, scr, iters);
      break;
    default:
      hipLaunchKernelGGL(k_chain_small<kSmallThreads>, dim3(nwg), dim3(kSmallThreads), 0, s,
                         probs, items, nitems_cap, nitems_dev, counter, abort_flag, scr, iters);
  }
  return hipGetLastError();
}

// Large clusters: cooperative launch; workgroup w belongs to group
// wg_group[w] and runs that group's items in order with group barriers.
// bars holds kBarWords words per group: the group's two-level barrier (word
// 0), the back-sweep progress word (kBarProg) and the barrier of ranks
// 1..size-1 that the lookahead uses (kBarSubRegion).
__global__ void __launch_bounds__(kCoopThreads) k_chain_coop(const Prob *__restrict__ probs,
                                                             const ChainItem *__restrict__ items,
                                                             const Group *__restrict__ groups,
                                                             const int *__restrict__ wg_group,
                                                             unsigned *bars, int *abort_flag,
                                                             int *started, ChainScratch scr,
                                                             int iters) {
  // Residency report to the host (host-coherent memory; may be null).
  if (started && threadIdx.x == 0)
    __hip_atomic_store(started + blockIdx.x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  const int g = wg_group[blockIdx.x];
  if (g < 0) return;
  const Group G = groups[g];
  Ctx cx;
  cx.rank = (int)blockIdx.x - G.wg0;
  cx.size = G.nwg;
  cx.cnt = bars + (size_t)g * kBarWords;
  cx.flag = nullptr;
  cx.gen = 0;
  cx.sgen = 0;
  cx.abort_flag = abort_flag;
  cx.wave = threadIdx.x / kWave;
  cx.lane = threadIdx.x % kWave;
  cx.gw = cx.rank * (kCoopThreads / kWave) + cx.wave;
  cx.nw = cx.size * (kCoopThreads / kWave);
  double *base = as_global(scr.base + (size_t)g * scr.stride);
  for (int q = 0; q < G.nit; q++) {
    const ChainItem it = items[G.it0 + q];
    const Prob &P = probs[it.prob];
    const Scr S = make_scr(base, P.n, P.m, it.start & 1);
    if (!run_chain<kCoopThreads>(cx, P, it, S, iters)) return;
    if (!grp_sync<kCoopThreads>(cx)) return;   // scratch reuse across items
  }
}

// The chain kernel relies on all of its workgroups being resident at once
// (one per CU, within the occupancy limit checked by coop_max_wgs); the
// cooperative launch guarantees that.  TE_COOP_LAUNCH=0 in the environment
// dispatches the same grid with a regular launch instead, for profilers that
// cannot handle cooperative dispatches; a workgroup that were not resident
// would time out in its first barrier and abort the run with TE_ERR_KERNEL.
static bool coop_launch_enabled() {
  static const bool on = [] {
    const char *v = getenv("TE_COOP_LAUNCH");
    return !(v && v[0] == '0' && v[1] == '\0');
  }();
  return on;
}

hipError_t launch_chain_coop(const Prob *probs, const ChainItem *items, const Group *groups,
                             const int *wg_group, unsigned *bars, int *abort_flag, int *started,
                             ChainScratch scr, int nwg, int iters, hipStream_t s) {
  if (nwg <= 0) return hipSuccess;
  if (!coop_launch_enabled()) {
    hipLaunchKernelGGL(k_chain_coop, dim3(nwg), dim3(kCoopThreads), 0, s, probs, items, groups,
                       wg_group, bars, abort_flag, started, scr, iters);
    return hipGetLastError();
  }
  void *args[] = {(void *)&probs,     (void *)&items,   (void *)&groups,
                  (void *)&wg_group,  (void *)&bars,    (void *)&abort_flag,
                  (void *)&started,   (void *)&scr,     (void *)&iters};
  return hipLaunchCooperativeKernel((const void *)k_chain_coop, dim3(nwg), dim3(kCoopThreads),
                                    args, 0, s);
}

// One cooperative workgroup (8 waves, up to 256 VGPRs each) per compute unit
// keeps the group barriers cheap (their cost grows with the number of
// arriving workgroups) while 8 waves per CU with 8 KB of loads in flight
// each still saturate HBM on the streaming passes.
int coop_max_wgs(int device) {
  int ncu = 0, per = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_chain_coop,
                                                   kCoopThreads, 0) != hipSuccess)
    return 0;
  return per >= 1 ? ncu : 0;
}

int small_max_wgs(int device, int nt) {
  int ncu = 0, per = 0;
  if (nt <= 0) nt = kSmallThreads;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, small_kernel(nt), nt, 0) != hipSuccess)
    return 0;
  return ncu * per;
}

int device_cus(int device) {
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  return ncu;
}

// ---------------------------------------------------------------------------
// a8: normalize each column, largest-magnitude entry positive (lowest index on
// ties); add the non-finite bit to the vector's status word (the pivot bit
// came from k_invit, the breakdown bit from the chain) and count the vectors
// with any bit set.  One wave per column.
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_finalize(const Prob *__restrict__ probs, int nprob,
                                                  const int64_t *__restrict__ loff, int64_t nlanes) {
  const int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x % kWave;
  if (wv >= nlanes) return;
  const int b = find_prob(loff, nprob, wv);
  const Prob &P = probs[b];
  const int j = (int)(wv - loff[b]);
  double *z = P.Z + (size_t)j * P.ldz;
  const int n = P.n;
  double ss = 0.0, best = -1.0;
  int bi = 0x7fffffff;
  for (int i = lane; i < n; i += kWave) {
    const double v = z[i];
    ss = fma(v, v, ss);
    const double a = fabs(v);
    if (a > best) { best = a; bi = i; }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(best, off, kWave);
    const int oi = __shfl_xor(bi, off, kWave);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  ss = wave_sum(ss);
  const bool finite = isfinite(ss) && ss > 0.0;
  const double sgn = (bi < n && z[bi] < 0.0) ? -1.0 : 1.0;
  const double sc = finite ? sgn / sqrt(ss) : 1.0;
  for (int i = lane; i < n; i += kWave) z[i] = z[i] * sc;
  if (P.info && lane == 0) {
    const int st = P.info[1 + j] | (finite ? 0 : TE_INFO_NONFINITE);
    P.info[1 + j] = st;
    if (st) atomicAdd(P.info, 1);
  }
}

hipError_t launch_finalize(const Prob *probs, int nprob, const int64_t *loff, int64_t nlanes,
                           hipStream_t s) {
  if (nlanes <= 0) return hipSuccess;
  const int64_t threads = nlanes * kWave;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, probs,
                     nprob, loff, nlanes);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Splitting into unreduced blocks: flag[i] = 1 when e_i is negligible,
// e_i^2 <= eps^2 |d_i d_{i+1}| + DBL_MIN (each operation rounded on its own).
// ---------------------------------------------------------------------------

__global__ void k_split_flags(const double *__restrict__ d, const double *__restrict__ e, int n,
                              unsigned char *__restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const double lim = (DBL_EPSILON * DBL_EPSILON) * fabs(d[i] * d[i + 1]) + DBL_MIN;
  flag[i] = (e[i] * e[i] <= lim) ? 1 : 0;
}

hipError_t launch_split_flags(const double *d, const double *e, int n, unsigned char *flag,
                              hipStream_t s) {
  if (n < 2) return hipSuccess;
  hipLaunchKernelGGL(k_split_flags, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s, d, e,
                     n, flag);
  return hipGetLastError();
}

// Block results -> the caller's columns: column p of Z (leading dimension
// ldz, n rows) is zero outside rows [s, s + nb) and holds the block's vector
// (src, nb entries) inside; W[p] and the status word follow.  One 256-thread
// workgroup per column.
__global__ void __launch_bounds__(256) k_split_scatter(const SplitCol *__restrict__ cols, int n,
                                                       double *__restrict__ W,
                                                       double *__restrict__ Z, size_t ldz,
                                                       int *__restrict__ info) {
  const SplitCol c = cols[blockIdx.x];
  double *z = Z + (size_t)c.p * ldz;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    z[i] = (i >= c.s && i < c.s + c.nb) ? c.src[i - c.s] : 0.0;
  if (threadIdx.x == 0) {
    W[c.p] = *c.w;
    if (info) {
      const int st = *c.st;
      info[1 + c.p] = st;
      if (st) atomicAdd(info, 1);
    }
  }
}

hipError_t launch_split_scatter(const SplitCol *cols, int m, int n, double *W, double *Z,
                                size_t ldz, int *info, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_scatter, dim3((unsigned)m), dim3(256), 0, s, cols, n, W, Z, ldz,
                     info);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Singular vectors of an upper bidiagonal B (diagonal a, superdiagonal b)
// through its Golub-Kahan tridiagonal of order 2n: zero diagonal, off-diagonal
// (a_0, b_0, a_1, ..., b_{n-2}, a_{n-1}).  An eigenvector (x_0, y_0, x_1, ...)
// of +sigma gives the right (x) and left (y) singular vectors.
// ---------------------------------------------------------------------------

__global__ void k_gk_build(const double *__restrict__ a, const double *__restrict__ b, int n,
                           double *__restrict__ dg, double *__restrict__ eg) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * n) return;
  dg[t] = 0.0;
  if (t < 2 * n - 1) eg[t] = (t & 1) ? b[t >> 1] : a[t >> 1];
}

hipError_t launch_gk_build(const double *a, const double *b, int n, double *dg, double *eg,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_gk_build, dim3((unsigned)((2 * n + 255) / 256)), dim3(256), 0, s, a, b, n,
                     dg, eg);
  return hipGetLastError();
}

// Column j of Zg (2n entries): V column = even entries, U column = odd
// entries, each scaled to unit 2-norm.  One 256-thread workgroup per column;
// the sums of squares in a fixed order (per-thread strided partial sums, then
// the workgroup tree), so the result does not depend on timing.
__global__ void __launch_bounds__(256) k_gk_split(const double *__restrict__ Zg, int n,
                                                  double *__restrict__ U, size_t ldu,
                                                  double *__restrict__ V, size_t ldv) {
  __shared__ double sx[256], sy[256];
  const double *z = Zg + (size_t)blockIdx.x * (size_t)(2 * n);
  double px = 0.0, py = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    const double x = z[2 * k], y = z[2 * k + 1];
    px = fma(x, x, px);
    py = fma(y, y, py);
  }
  sx[threadIdx.x] = px;
  sy[threadIdx.x] = py;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sx[threadIdx.x] = sx[threadIdx.x] + sx[threadIdx.x + w];
      sy[threadIdx.x] = sy[threadIdx.x] + sy[threadIdx.x + w];
    }
    __syncthreads();
  }
  const double rx = 1.0 / sqrt(sx[0]), ry = 1.0 / sqrt(sy[0]);
  double *u = U + (size_t)blockIdx.x * ldu;
  double *v = V + (size_t)blockIdx.x * ldv;
  for (int k = threadIdx.x; k < n; k += 256) {
    v[k] = z[2 * k] * rx;
    u[k] = z[2 * k + 1] * ry;
  }
}

hipError_t launch_gk_split(const double *Zg, int n, int m, double *U, size_t ldu, double *V,
                           size_t ldv, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gk_split, dim3((unsigned)m), dim3(256), 0, s, Zg, n, U, ldu, V, ldv);
  return hipGetLastError();
}

__global__ void k_fill_i32(int *p, size_t n, int v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int *p, size_t n, int v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace te
