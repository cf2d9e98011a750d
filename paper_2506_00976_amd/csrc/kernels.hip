// HIP kernels for gfx950 (CDNA4): fine-grid stages of the quantization bounds.
//
// Every kernel works on a table of jobs (DevJob), so one launch serves one
// pair or a batch of pairs of uneven sizes.  Work items are mapped to jobs by
// a prefix table (find_job); the c-transform is a persistent launch over a
// planner-built item table (one item per work-group, the rest through a
// counter).  Reductions are deterministic:
// per-work-group partials in a fixed tree order, combined by a finalize
// kernel in a fixed order - repeated runs are bitwise identical.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>

#include "qbw_internal.h"

namespace qbw {

#define HIP_TRY(x)                                                        \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      set_error("%s failed: %s", #x, hipGetErrorString(e_));              \
      return QBW_E_HIP;                                                   \
    }                                                                     \
  } while (0)

__device__ __forceinline__ int find_job(const int* __restrict__ off, int njobs, int item) {
  // a batch of equal jobs: the quotient by the first job's count, checked
  // against its two prefix entries (two dependent loads, not log2 njobs);
  // otherwise the last job whose prefix entry is at most the item
  const int per = off[1] - off[0];
  if (per > 0) {
    const int g = min(item / per, njobs - 1);
    if (off[g] <= item && item < off[g + 1]) return g;
  }
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int NT>
__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Coordinates of a flat pixel index (C order).
__device__ __forceinline__ void pix_coords(int i, int N, int d, int& x0, int& x1, int& x2) {
  if (d == 2) { x0 = 0; x1 = i / N; x2 = i - x1 * N; }
  else { x0 = i / (N * N); int r = i - x0 * N * N; x1 = r / N; x2 = r - x1 * N; }
}

// Flat index of member m (0 <= m < k^d) of coarse block K.
__device__ __forceinline__ int block_member(int K, int m, int N, int n, int k, int d) {
  if (d == 2) {
    int b0 = K / n, b1 = K - b0 * n;
    int u0 = m / k, u1 = m - u0 * k;
    return (b0 * k + u0) * N + b1 * k + u1;
  }
  int b0 = K / (n * n), r = K - b0 * n * n, b1 = r / n, b2 = r - b1 * n;
  int u0 = m / (k * k), s = m - u0 * k * k, u1 = s / k, u2 = s - u1 * k;
  return ((b0 * k + u0) * N + b1 * k + u1) * N + b2 * k + u2;
}

// Ground cost in float64 between two pixels: |x - y|^p (exact integer for p = 2).
__device__ __forceinline__ double cost64(int i, int j, int N, int d, int p) {
  int a0, a1, a2, b0, b1, b2;
  pix_coords(i, N, d, a0, a1, a2);
  pix_coords(j, N, d, b0, b1, b2);
  int e0 = a0 - b0, e1 = a1 - b1, e2 = a2 - b2;
  double d2 = (double)(e0 * e0 + e1 * e1 + e2 * e2);
  return p == 2 ? d2 : sqrt(d2);
}

// Correctly rounded float32 square root for exact nonnegative integers below
// 2^24 (no denormals): hardware estimate, then the two neighbouring floats
// are tested with exact fused residuals.
__device__ __forceinline__ float sqrt_rn_int(float x) {
  float s = __builtin_amdgcn_sqrtf(x);
  float sd = __int_as_float(__float_as_int(s) - 1);
  float su = __int_as_float(__float_as_int(s) + 1);
  float rd = __builtin_fmaf(-sd, s, x);
  float ru = __builtin_fmaf(-su, s, x);
  s = (rd <= 0.0f) ? sd : s;
  s = (ru > 0.0f) ? su : s;
  return s;
}

// t[n] = sqrt_rn_int(n) for n < count (integers below 2^24 are exact floats).
__global__ __launch_bounds__(256) void k_sqrt_table(float* __restrict__ t, int count) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) t[i] = sqrt_rn_int((float)i);
}

// ------------------------------------------------------------------ pooling

// Blocks are reduced by groups of g lanes, g the smallest power of two
// >= min(k^d, 64): a wave takes 64 / g blocks (small blocks share a wave, a
// large block spreads over all 64 lanes).  Group sums use a butterfly over the
// group's lanes, in a fixed order.
__device__ __forceinline__ double group_sum(double v, int g) {
  for (int o = g >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}


// ------------------------------------------------------------------ upscaling

// Per axis: x = centre(K0) + w * k, clamped to the hull of the block centres.
__device__ __forceinline__ void axis_weight(int x, int k, int n, int& K0, int& K1, double& w) {
  const int t = 2 * x - (k - 1);
  const int den = 2 * k;
  if (t <= 0 || n == 1) { K0 = 0; K1 = 0; w = 0.0; return; }
  const int q = t / den;
  if (q >= n - 1) { K0 = n - 1; K1 = n - 1; w = 0.0; return; }
  K0 = q;
  K1 = q + 1;
  // a power-of-two denominator divides exactly as a product with its reciprocal
  const double r = (double)(t - den * q);
  w = (den & (den - 1)) == 0 ? r * (1.0 / (double)den) : r / (double)den;
}

__device__ __forceinline__ double lerp_nc(double a, double b, double w) {
#pragma clang fp contract(off)
  return a + w * (b - a);
}

// Catmull-Rom cubic convolution along one axis at fine coordinate x: the four
// tap indices (clamped to the coarse grid) and weights.  The pixel's coarse
// position t = (2x - (k-1)) / (2k) is clamped to [0, n-1]; i = floor(t),
// s = t - i = r / (2k) from the integer remainder r.  Every float64 operation
// is rounded on its own, in the order written.
__device__ __forceinline__ void axis_cubic(int x, int k, int n, int (&K)[4], double (&w)[4]) {
#pragma clang fp contract(off)
  const int t = 2 * x - (k - 1);
  const int den = 2 * k;
  int i, r;
  if (t <= 0) { i = 0; r = 0; }
  else {
    i = t / den;
    r = t - den * i;
    if (i >= n - 1) { i = n - 1; r = 0; }
  }
  for (int o = 0; o < 4; ++o) K[o] = min(max(i + o - 1, 0), n - 1);
  const double s = (den & (den - 1)) == 0 ? (double)r * (1.0 / (double)den) : (double)r / (double)den;
  const double s2 = s * s;
  const double s3 = s2 * s;
  w[0] = 0.5 * ((2.0 * s2 - s3) - s);
  w[1] = 0.5 * ((3.0 * s3 - 5.0 * s2) + 2.0);
  w[2] = 0.5 * ((4.0 * s2 - 3.0 * s3) + s);
  w[3] = 0.5 * (s3 - s2);
}

__device__ __forceinline__ double cubic_sum(const double (&w)[4], double v0, double v1, double v2, double v3) {
#pragma clang fp contract(off)
  return ((w[0] * v0 + w[1] * v1) + w[2] * v2) + w[3] * v3;
}

// f^ at pixel (x0, x1, x2) (2D: x1 row, x2 column) from the job's coarse
// potential, by its interpolation rule.
__device__ __forceinline__ float upscale_value(const DevJob& J, int x0, int x1, int x2) {
  const double* __restrict__ F = J.ftil;
  const int n = J.n;
  double val;
  if (J.interp == 1) {
    // nearest centre = the centre of the pixel's own block
    const int b1 = x1 / J.k, b2 = x2 / J.k;
    val = J.d == 2 ? F[b1 * n + b2] : F[((x0 / J.k) * n + b1) * n + b2];
  } else if (J.interp == 2) {
    int B[4], C[4];
    double wb[4], wc[4];
    axis_cubic(x1, J.k, n, B, wb);
    axis_cubic(x2, J.k, n, C, wc);
    if (J.d == 2) {
      double r[4];
      for (int u = 0; u < 4; ++u) {
        const double* row = F + B[u] * n;
        r[u] = cubic_sum(wc, row[C[0]], row[C[1]], row[C[2]], row[C[3]]);
      }
      val = cubic_sum(wb, r[0], r[1], r[2], r[3]);
    } else {
      int A[4];
      double wa[4];
      axis_cubic(x0, J.k, n, A, wa);
      double sa[4];
      for (int t = 0; t < 4; ++t) {
        double r[4];
        for (int u = 0; u < 4; ++u) {
          const double* row = F + (A[t] * n + B[u]) * n;
          r[u] = cubic_sum(wc, row[C[0]], row[C[1]], row[C[2]], row[C[3]]);
        }
        sa[t] = cubic_sum(wb, r[0], r[1], r[2], r[3]);
      }
      val = cubic_sum(wa, sa[0], sa[1], sa[2], sa[3]);
    }
  } else if (J.d == 2) {
    int A0, A1, B0, B1;
    double wa, wb;
    axis_weight(x1, J.k, n, A0, A1, wa);
    axis_weight(x2, J.k, n, B0, B1, wb);
    const double r0 = lerp_nc(F[A0 * n + B0], F[A0 * n + B1], wb);
    const double r1 = lerp_nc(F[A1 * n + B0], F[A1 * n + B1], wb);
    val = lerp_nc(r0, r1, wa);
  } else {
    int A0, A1, B0, B1, C0, C1;
    double wa, wb, wc;
    axis_weight(x0, J.k, n, A0, A1, wa);
    axis_weight(x1, J.k, n, B0, B1, wb);
    axis_weight(x2, J.k, n, C0, C1, wc);
    auto at = [&](int a, int b, int c) { return F[(a * n + b) * n + c]; };
    const double s00 = lerp_nc(at(A0, B0, C0), at(A0, B0, C1), wc);
    const double s01 = lerp_nc(at(A0, B1, C0), at(A0, B1, C1), wc);
    const double s10 = lerp_nc(at(A1, B0, C0), at(A1, B0, C1), wc);
    const double s11 = lerp_nc(at(A1, B1, C0), at(A1, B1, C1), wc);
    const double t0 = lerp_nc(s00, s01, wb);
    const double t1 = lerp_nc(s10, s11, wb);
    val = lerp_nc(t0, t1, wa);
  }
  return (float)val;
}

// f^ over chunks of pixels.  skip_small: only jobs with k > 64 (the pooling
// launch upscales the others along with its block strips).
__global__ __launch_bounds__(256) void k_upscale(const DevJob* __restrict__ jobs, int njobs,
                                                 const int* __restrict__ off, int total, int skip_small) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (skip_small && J.k <= 64) continue;
    const int base = (it - off[jb]) * kChunk;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int i = base + q;
      if (i >= J.P) break;
      int x0, x1, x2;
      pix_coords(i, J.N, J.d, x0, x1, x2);
      J.fhat[i] = upscale_value(J, x0, x1, x2);
    }
  }
}

// ------------------------------------------------------------------ c-transform
//
// psi_j = min_i RN32(c_ij - phi_i) over all sources i.
//
// Mapping: one wave per work item = (job, target tile, source split).  Lane
// l owns R consecutive targets of one grid row (the last axis): columns
// v0 .. v0+R-1 of row r.  Sources are swept row by row; within a source row
// every lane needs, at source column t, the costs c(A, t - v0 - q) for
// q = 0..R-1, where A is the squared distance over the other axes.  Moving
// from t to t+1 shifts that window by one: R-1 values are reused and only
// c(A, t + 1 - v0) is new (an exact integer update for p = 2, plus one
// correctly rounded square root for p = 1).  With the window held in R
// registers whose roles rotate through a fully unrolled block of R steps,
// each (source, target) pair costs one subtraction plus half of a v_min3:
// the block runs over pairs of sources, and for every target the two
// candidates and the running minimum meet in one v_min3 (so only two
// candidates are live at a time and R = 32 fits in 128 VGPRs).
// The source potential is wave-uniform and comes through scalar loads.
// Source potentials are read through the constant address space: the data
// is not written during the launch and every lane reads the same address, so
// the loads become scalar (s_load) and the values feed the VALU as SGPRs.
// The next block's potentials are requested before the current block's
// arithmetic, so the scalar-load latency hides behind it.
typedef const __attribute__((address_space(4))) float* const_fptr;

template <int R, int PP>
__device__ __forceinline__ void ct_tile(const float* __restrict__ src, float* __restrict__ out,
                                        int N, int d, int P, int tile, int r0, int r1) {
  const int lane = threadIdx.x & 63;
  const int j0 = tile * 64 * R + lane * R;
  const bool valid = j0 < P;
  const int jj = valid ? j0 : 0;
  const int trow = jj / N;
  const int v0 = jj - trow * N;
  int ta, tb;
  if (d == 2) { ta = 0; tb = trow; } else { ta = trow / N; tb = trow - ta * N; }
  float mn[R];
#pragma unroll
  for (int q = 0; q < R; ++q) mn[q] = INFINITY;
  const float sq0 = (float)(v0 * v0);
  const float inc0 = (float)(2 * v0 + 1);
  const_fptr cbase = (const_fptr)src;
  const size_t end = (size_t)r1 * N;
  float nxt[R];
  if (r0 < r1) {
#pragma unroll
    for (int m = 0; m < R; ++m) nxt[m] = cbase[(size_t)r0 * N + m];
  }

  for (int sr = r0; sr < r1; ++sr) {
    int sa, sb;
    if (d == 2) { sa = 0; sb = sr; } else { sa = sr / N; sb = sr - sa * N; }
    const int da = sa - ta, db = sb - tb;
    const float A = (float)(da * da + db * db);
    // W[q] = A + (v0 + q)^2 by exact increments 2 (v0 + q) - 1.  The chain
    // starts from a copy the compiler cannot see through, so it is rebuilt
    // per source row instead of R row-invariant squares being kept live (and
    // spilled) across the whole sweep.
    float inc = inc0;
    __asm__ volatile("" : "+v"(inc));
    float W[R];
    float nk = A + sq0;
    const float n0_row = nk;
    W[0] = (PP == 2) ? nk : sqrt_rn_int(nk);
#pragma unroll
    for (int q = 1; q < R; ++q) {
      nk = nk + inc;
      inc = inc + 2.0f;
      W[q] = (PP == 2) ? nk : sqrt_rn_int(nk);
    }
    float n0 = n0_row;
    float D = (float)(1 - 2 * v0);
    for (int b = 0; b < N; b += R) {
      float cur[R];
#pragma unroll
      for (int m = 0; m < R; ++m) cur[m] = nxt[m];
      // prefetch the next block of source potentials (the next row's first
      // block at the end of a row; the current block again after the last)
      {
        const size_t cb = (size_t)sr * N + b;
        const size_t nb = cb + R;
        const_fptr np = cbase + (nb < end ? nb : cb);
#pragma unroll
        for (int m = 0; m < R; ++m) nxt[m] = np[m];
      }
      // keep the prefetch ahead of the block's arithmetic
      __builtin_amdgcn_sched_barrier(0);
      if (R == 1) {
        float p0 = cur[0];
        __asm__("" : "+v"(p0));
        mn[0] = fminf(mn[0], W[0] - p0);
        if (PP == 2) { W[0] = W[0] + D; } else { n0 = n0 + D; W[0] = sqrt_rn_int(n0); }
        D += 2.0f;
      } else {
#pragma unroll
        for (int m = 0; m < R; m += 2) {
          // two sources per step pair; each is moved to a VGPR once (on
          // gfx950 a VALU op with an SGPR operand issues at about half rate)
          float p0 = cur[m], p1 = cur[m + 1];
          __asm__("" : "+v"(p0));
          __asm__("" : "+v"(p1));
          // Target q = R-1 first: it is the last reader of the two window
          // slots this pair of steps replaces, so their new values can take
          // the same registers (no register rotation at the loop back-edge).
          {
            const float t0 = W[(R - 1 - m + R) % R] - p0;
            const float t1 = W[(R - 2 - m + 2 * R) % R] - p1;
            mn[R - 1] = fminf(mn[R - 1], fminf(t0, t1));
            __asm__("" : "+v"(mn[R - 1]));
          }
          // slot (R-1-m) % R takes the cost of the source after m; target 0
          // reads it for source m+1
          if (PP == 2) {
            W[(R - 1 - m + R) % R] = W[(R - m) % R] + D;
          } else {
            n0 = n0 + D;
            W[(R - 1 - m + R) % R] = sqrt_rn_int(n0);
          }
#pragma unroll
          for (int q = 0; q < R - 1; ++q) {
            const float t0 = W[(q - m + R) % R] - p0;
            const float t1 = W[(q - m - 1 + 2 * R) % R] - p1;
            mn[q] = fminf(mn[q], fminf(t0, t1));
            // keep the running minimum a chain of v_min3 (no re-association)
            __asm__("" : "+v"(mn[q]));
          }
          if (PP == 2) {
            W[(R - 2 - m + 2 * R) % R] = W[(R - 1 - m + R) % R] + (D + 2.0f);
          } else {
            n0 = n0 + (D + 2.0f);
            W[(R - 2 - m + 2 * R) % R] = sqrt_rn_int(n0);
          }
          D += 4.0f;
        }
      }
    }
  }
  if (valid) {
    if constexpr (R % 4 == 0) {
      // 16-byte stores: j0 and the split's row start are multiples of 4 floats
      float4* o4 = reinterpret_cast<float4*>(out + j0);
#pragma unroll
      for (int q = 0; q < R; q += 4) o4[q / 4] = make_float4(mn[q], mn[q + 1], mn[q + 2], mn[q + 3]);
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) out[j0 + q] = mn[q];
    }
  }
}

// p = 1 with a table instead of a square root per step.  For a source row
// and a target row the costs are RN32(sqrt(A + a^2)), a = |source column -
// target column| in [0, N], A the squared distance over the other axes.  At
// every source row the wave writes, for each of its target rows, that row of
// N values to LDS (R correctly rounded square roots per lane, the same
// sqrt_rn_int as the direct path), and the sweep then reads each new window
// value from LDS.  Within a block of R sources the column offset b + m + 1 - v0
// keeps one sign per lane (blocks and v0 are multiples of R), so its table
// position moves by one slot per step (+1 on the increasing side's last step
// where it crosses a multiple of 32): one address multiply-add per step.  Row
// entries are stored at a + (a >> 5), rows S = (N + N/32) | 1 apart, so lanes
// whose offsets differ by 32 (or whose rows differ) hit different banks.
// Applies when the wave's targets cover whole rows (64R a multiple of N, or
// N a multiple of 64R) and N <= 2048; the table holds at most 2176 floats.
constexpr int kCtTab = 2176 + 64;
__device__ __forceinline__ bool ct_p1_table_ok(int N, int R) {
  return R >= 4 && N <= 2048 && (((64 * R) % N) == 0 || (N % (64 * R)) == 0);
}

// One table for every tile variant (separate per-variant arrays made the
// compiler give up the four-waves-per-SIMD register budget).
__shared__ float ct_tab[kCtTab];

template <int R>
__device__ __forceinline__ void ct_tile_p1(const float* __restrict__ src, float* __restrict__ out,
                                           const float* __restrict__ sq, int N, int d, int P, int tile,
                                           int r0, int r1) {
  float* tab = ct_tab;
  const int lane = threadIdx.x & 63;
  const int j0 = tile * 64 * R + lane * R;
  const bool valid = j0 < P;
  const int wj0 = tile * 64 * R;
  const int wrow0 = wj0 / N;                       // first target row of the wave
  const int rpw = 64 * R >= N ? 64 * R / N : 1;    // target rows per wave
  const int S = (N + (N >> 5)) | 1;                // table row stride
  const int jj = valid ? j0 : wj0;
  const int trow = jj / N;
  const int v0 = jj - trow * N;
  const int lr = min(max(trow - wrow0, 0), rpw - 1);
  // the table row this lane fills and its target row's coordinates
  const int er = lane % rpw, G = 64 / rpw, cnt = N / G;
  // rows past the grid's end (a last wave covering fewer rows) are filled
  // from the last row: only lanes without targets read them, and every
  // squared distance stays within (d - 1)(N - 1)^2
  const int erow = min(wrow0 + er, P / N - 1);
  int eta, etb;
  if (d == 2) { eta = 0; etb = erow; } else { eta = erow / N; etb = erow - eta * N; }
  float mn[R];
#pragma unroll
  for (int q = 0; q < R; ++q) mn[q] = INFINITY;
  const_fptr cbase = (const_fptr)src;
  const size_t end = (size_t)r1 * N;
  float nxt[R];
  if (r0 < r1) {
#pragma unroll
    for (int m = 0; m < R; ++m) nxt[m] = cbase[(size_t)r0 * N + m];
  }
  const int rowbase = lr * S;
  for (int sr = r0; sr < r1; ++sr) {
    int sa, sb;
    if (d == 2) { sa = 0; sb = sr; } else { sa = sr / N; sb = sr - sa * N; }
    {
      const int da = sa - eta, db = sb - etb;
      const int A = da * da + db * db;
      __syncthreads();   // the previous row's reads are done
      if (sq) {
        // the same values from the context's square-root table (small grids,
        // where the fill is a large share of a row's work)
#pragma unroll 8
        for (int q = 0; q < cnt; ++q) {
          const int a = lane / rpw + G * q;
          tab[er * S + a + (a >> 5)] = sq[A + a * a];
        }
      } else {
        for (int q = 0; q < cnt; ++q) {
          const int a = lane / rpw + G * q;
          tab[er * S + a + (a >> 5)] = sqrt_rn_int((float)(A + a * a));
        }
      }
      __syncthreads();
    }
    // window at source column 0: W[q] = cost(0, v0 + q), one aligned group of R
    float W[R];
    {
      const float* wp = tab + rowbase + v0 + (v0 >> 5);
#pragma unroll
      for (int q = 0; q < R; ++q) W[q] = wp[q];
    }
    for (int b = 0; b < N; b += R) {
      float cur[R];
#pragma unroll
      for (int m = 0; m < R; ++m) cur[m] = nxt[m];
      {
        const size_t cb = (size_t)sr * N + b;
        const size_t nb = cb + R;
        const_fptr np = cbase + (nb < end ? nb : cb);
#pragma unroll
        for (int m = 0; m < R; ++m) nxt[m] = np[m];
      }
      __builtin_amdgcn_sched_barrier(0);
      // table positions of the new values (source b + m + 1, target v0)
      const int s = b >= v0 ? 1 : -1;
      const int a0 = s * (b + 1 - v0);                       // |offset| at m = 0
      const int lo = s > 0 ? b - v0 : v0 - b - R;            // the block's aligned group
      int pa = rowbase + a0 + (lo >> 5);   // position of the next new value
      const int jmp = (s > 0 && ((b - v0 + R) & 31) == 0) ? 1 : 0;
#pragma unroll
      for (int m = 0; m < R; m += 2) {
        // one running position, stepped as the values are consumed (not R
        // precomputed addresses held across the block)
        const float nv0 = tab[pa];
        pa += s;
        const float nv1 = tab[pa + (m + 1 == R - 1 ? jmp : 0)];
        pa += s;
        __asm__ volatile("" : "+v"(pa));
        float p0 = cur[m], p1 = cur[m + 1];
        __asm__("" : "+v"(p0));
        __asm__("" : "+v"(p1));
        {
          const float t0 = W[(R - 1 - m + R) % R] - p0;
          const float t1 = W[(R - 2 - m + 2 * R) % R] - p1;
          mn[R - 1] = fminf(mn[R - 1], fminf(t0, t1));
          __asm__("" : "+v"(mn[R - 1]));
        }
        W[(R - 1 - m + R) % R] = nv0;
#pragma unroll
        for (int q = 0; q < R - 1; ++q) {
          const float t0 = W[(q - m + R) % R] - p0;
          const float t1 = W[(q - m - 1 + 2 * R) % R] - p1;
          mn[q] = fminf(mn[q], fminf(t0, t1));
          __asm__("" : "+v"(mn[q]));
        }
        W[(R - 2 - m + 2 * R) % R] = nv1;
      }
    }
  }
  if (valid) {
    float4* o4 = reinterpret_cast<float4*>(out + j0);
#pragma unroll
    for (int q = 0; q < R; q += 4) o4[q / 4] = make_float4(mn[q], mn[q + 1], mn[q + 2], mn[q + 3]);
  }
}

// Persistent c-transform.  The planner lays the items out so that position
// b < G (the grid) is work-group b's item for the first round, positions
// b = q (mod 8) holding XCD q's share: the dispatcher deals work-groups to the
// XCDs in turn, so each XCD's source potentials stay in its own L2.  No atomics
// are needed for that round, which matters: the counter is shared by all
// XCDs, so every read-modify-write on it goes to the memory side and thousands
// of them at a launch's start and end serialize.  Only when there are more
// items than work-groups does a wave take further items (largest first) from
// the tail through the counter; every wave exits once the tail is empty.
__device__ __forceinline__ void ct_item(const DevJob* __restrict__ jobs, const CtItem& w, int phase) {
  const DevJob& J = jobs[w.job];
  const float* src = phase == 0 ? J.fhat : J.g;
  float* out = J.part + (size_t)w.split * J.P;
  const int r0 = (int)(((long long)w.split * J.rows) / J.S);
  const int r1 = (int)(((long long)(w.split + 1) * J.rows) / J.S);
  if (J.p == 1 && J.R >= 4 && ct_p1_table_ok(J.N, J.R)) {
    switch (J.R) {
      case 32: ct_tile_p1<32>(src, out, J.sqrt_tab, J.N, J.d, J.P, w.tile, r0, r1); return;
      case 16: ct_tile_p1<16>(src, out, J.sqrt_tab, J.N, J.d, J.P, w.tile, r0, r1); return;
      case 8: ct_tile_p1<8>(src, out, J.sqrt_tab, J.N, J.d, J.P, w.tile, r0, r1); return;
      default: ct_tile_p1<4>(src, out, J.sqrt_tab, J.N, J.d, J.P, w.tile, r0, r1); return;
    }
  }
  const int key = J.R * 4 + J.p;
  switch (key) {
    case 32 * 4 + 2: ct_tile<32, 2>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 32 * 4 + 1: ct_tile<32, 1>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 16 * 4 + 2: ct_tile<16, 2>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 16 * 4 + 1: ct_tile<16, 1>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 8 * 4 + 2: ct_tile<8, 2>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 8 * 4 + 1: ct_tile<8, 1>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 4 * 4 + 2: ct_tile<4, 2>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 4 * 4 + 1: ct_tile<4, 1>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 2 * 4 + 2: ct_tile<2, 2>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 2 * 4 + 1: ct_tile<2, 1>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    case 1 * 4 + 2: ct_tile<1, 2>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
    default: ct_tile<1, 1>(src, out, J.N, J.d, J.P, w.tile, r0, r1); break;
  }
}

// Four waves per SIMD: the R = 32 tile holds 32 running minima, a 32-entry
// cost window and the step pair's temporaries in at most 128 VGPRs.
__attribute__((amdgpu_waves_per_eu(4)))
__global__ __launch_bounds__(64) void k_ctransform(const DevJob* __restrict__ jobs,
                                                   const CtItem* __restrict__ items, int n_items,
                                                   int* __restrict__ counter, int phase) {
  const int G = gridDim.x;
  if ((int)blockIdx.x < n_items) ct_item(jobs, items[blockIdx.x], phase);
  if (n_items <= G) return;
  for (;;) {
    int it = 0;
    if (threadIdx.x == 0) it = G + atomicAdd(counter, 1);
    it = __shfl(it, 0);
    it = __builtin_amdgcn_readfirstlane(it);
    if (it >= n_items) break;
    ct_item(jobs, items[it], phase);
  }
}

__global__ void k_reset_counter(int* counter, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counter[i] = 0;
}

// Minimum over source splits; the winning split is the lowest one attaining it.
// One thread per target: blockIdx.y picks the quarter of the 1024-target chunk,
// and four splits are read per step to keep several loads in flight.
__global__ __launch_bounds__(256) void k_merge(const DevJob* __restrict__ jobs, int njobs,
                                               const int* __restrict__ off, int total, int phase) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (J.sep || J.xs) continue;
    const int j = (it - off[jb]) * kChunk + blockIdx.y * 256 + threadIdx.x;
    if (j >= J.P) continue;
    float* dst = phase == 0 ? J.g : J.f;
    const float* pp = J.part + j;
    const size_t P = (size_t)J.P;
    float best = INFINITY;
    int win = 0;
    int s = 0;
    for (; s + 4 <= J.S; s += 4) {
      const float v0 = pp[(size_t)s * P], v1 = pp[(size_t)(s + 1) * P];
      const float v2 = pp[(size_t)(s + 2) * P], v3 = pp[(size_t)(s + 3) * P];
      if (v0 < best) { best = v0; win = s; }
      if (v1 < best) { best = v1; win = s + 1; }
      if (v2 < best) { best = v2; win = s + 2; }
      if (v3 < best) { best = v3; win = s + 3; }
    }
    for (; s < J.S; ++s) {
      const float v = pp[(size_t)s * P];
      if (v < best) { best = v; win = s; }
    }
    dst[j] = best;
    J.win[j] = win;
  }
}

// Lowest source index attaining the minimum: rescan the winning split only.
__global__ __launch_bounds__(256) void k_argmin(const DevJob* __restrict__ jobs, int njobs,
                                                const int* __restrict__ off, int total, int phase) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (J.sep || J.xs) continue;
    const int base = (it - off[jb]) * kChunk;
    const float* src = phase == 0 ? J.fhat : J.g;
    const float* dst = phase == 0 ? J.g : J.f;
    int* arg = phase == 0 ? J.arg_g : J.arg_f;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int j = base + q;
      if (j >= J.P) break;
      const int s = J.win[j];
      const int r0 = (int)(((long long)s * J.rows) / J.S);
      const int r1 = (int)(((long long)(s + 1) * J.rows) / J.S);
      int y0, y1, y2;
      pix_coords(j, J.N, J.d, y0, y1, y2);
      const float target = dst[j];
      int found = -1;
      for (int i = r0 * J.N; i < r1 * J.N && found < 0; ++i) {
        int x0, x1, x2;
        pix_coords(i, J.N, J.d, x0, x1, x2);
        const int e0 = x0 - y0, e1 = x1 - y1, e2 = x2 - y2;
        const float c2 = (float)(e0 * e0 + e1 * e1 + e2 * e2);
        const float c = J.p == 2 ? c2 : sqrt_rn_int(c2);
        if (c - src[i] == target) found = i;
      }
      arg[j] = found;
    }
  }
}

// ------------------------------------------------------------------ exact separable c-transform (p = 2)
//
// The all-pairs reading is psi(y) = min_x RN32(c(x, y) - phi(x)) with c an
// exact integer, and the arg-min is the lowest x attaining psi.  Rounding is
// monotone, so psi(y) = RN32(V(y)) with V(y) = min_x (c(x, y) - phi(x)) taken
// exactly, and for p = 2 that exact minimum separates over the axes:
//   V(y) = min_{x_0} ((x_0 - y_0)^2 + min_{x_1} ((x_1 - y_1)^2 + ...
//          min_{x_{d-1}} ((x_{d-1} - y_{d-1})^2 - phi(x)))).
// Stage k (k = 0 .. d-1) takes axis a = d-1-k from source to target
// coordinates along every line of the other axes, in float64: per target it
// keeps the smallest candidate value (lowest source coordinate on equal
// values), that candidate's flat source index over the axes done so far, and
// the smallest value over all other sources (the runner-up), which is the
// smaller of the other candidates' values and the winner's own runner-up.
// Every float64 operation rounds, so a value is known to within
// delta(w) = d 2^-51 (|w| + 2 d (N-1)^2 + 1).  The last stage certifies each
// target: psi = RN32(w1) holds if w1 - delta and w1 + delta round to the same
// float32, and the arg-min holds if the runner-up minus its delta rounds
// above psi (no other source can round to psi).  Targets that fail either
// test (near ties, exact ties, non-finite potentials) are queued and
// evaluated by brute force exactly as the all-pairs kernel does.
constexpr int kXsOff = 2904;   // squares table: xs_sq[i] = (i - kXsOff)^2, 0 <= i <= 2 kXsOff (any valid N)
constexpr int kXsWinCap = 72;  // argmin windows staged in LDS up to this many sources (64 lines each)

__global__ __launch_bounds__(256) void k_xs_squares(double* __restrict__ t) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i <= 2 * kXsOff; i += gridDim.x * 256) {
    const double v = (double)(i - kXsOff);
    t[i] = v * v;
  }
}

typedef const __attribute__((address_space(4))) double* const_dptr;
typedef const __attribute__((address_space(1))) double* gdptr;

// min of two doubles with quiet NaN operands ignored (IEEE mode), as one
// v_min_f64: the asm keeps the compiler from re-canonicalising the
// loop-carried minima (a max of each with itself) at every unrolled block.
__device__ __forceinline__ double vmin_f64(double a, double b) {
  double r;
  __asm__("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Value-only stage candidates for one block of T sources r0 .. r0+T-1 and the
// lane's T targets t0 .. t0+T-1: h + (r - t0 - t)^2.  The squares of the T
// offsets a - t a source meets (a = r - t0) sit in a window of T registers;
// from one source to the next the window moves by one offset, so each step
// writes one new square, (a)^2 = (a-1)^2 + (2a-1), exact in float64, into the
// slot the last step's target T-1 no longer needs, and the slots' roles
// rotate through the unrolled block (target t at step j reads slot
// (t - j) mod T).  Every candidate is then one all-VGPR add and one min.
// On entry W[1] holds (r0 - t0 - 1)^2 and W[q] = (r0 - t0 - q)^2 for q >= 1;
// inc = 2 (r0 - t0) - 1.  H(j) gives the line's value at source r0 + j.
template <int T, typename H>
__device__ __forceinline__ void xs_window_block(double (&m1)[T], double (&W)[T], double& inc, H&& hval) {
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const int s = (T - j) % T, sp = (T - j + 1) % T;
    W[s] = W[sp] + inc;
    inc += 2.0;
    const double h = hval(j);
#pragma unroll
    for (int t = 0; t < T; ++t) m1[t] = vmin_f64(m1[t], h + W[(t - j + T) % T]);
    // one step at a time: without this the scheduler pulls later steps'
    // work (and so the waits for their sources' loads) up into this one
    __builtin_amdgcn_sched_barrier(0);
  }
}

// The same block when the lane's targets are the wave's (t0 wave-uniform):
// the squares (a0 + q)^2, a0 = r0 - t0, |q| < T, are the same in every lane,
// so they are read once per block from the table into scalar registers and
// each candidate is one add with a scalar operand and one min, with no
// per-lane window.  sqa points at the table entry of a0.
template <int T, int PARTS, typename H>
__device__ __forceinline__ void xs_sq_block(double (&m1)[T], const_dptr sqa, H&& hval) {
  // in PARTS runs of T / PARTS steps, each with the T + T / PARTS - 1 squares
  // it uses, so that fewer scalar registers hold squares at a time
  constexpr int TP = T / PARTS, NS = T + TP - 1;
#pragma unroll
  for (int hf = 0; hf < PARTS; ++hf) {
    double sq[NS];   // offsets hf TP - (T - 1) ... hf TP + TP - 1
#pragma unroll
    for (int q = 0; q < NS; ++q) sq[q] = sqa[hf * TP + q - (T - 1)];
#pragma unroll
    for (int jj = 0; jj < TP; ++jj) {
      const int j = hf * TP + jj;
      const double h = hval(j);
#pragma unroll
      for (int t = 0; t < T; ++t) m1[t] = vmin_f64(m1[t], h + sq[jj - t + T - 1]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// One item of stage k: 64 lines x T targets along the axis.  `tile` is the
// work-group's LDS staging area of the first stage (64 x 17 floats).  ARG:
// the job wants arg-mins, so the index and the runner-up are tracked; without
// them a candidate is one add and one min, and only the value is certified.
template <bool FIRST, int kXsT, bool ARG>
__device__ __forceinline__ void xs_item(const DevJob& J, int jb, int local, int phase, int k,
                                        const double* __restrict__ sqt, int2* __restrict__ list,
                                        int* __restrict__ count, float* tile, int wv, int SW,
                                        double* red) {
  const int lane = threadIdx.x & 63;
  {
    const int N = J.N, P = J.P;
    const int lines = P / N;
    const int nchunk = (lines + 63) >> 6;
    // Lanes are (line, target group) pairs.  Later stages: 64 consecutive
    // lines of one target group per wave (their loads are coalesced along
    // the last axis, and the wave's targets, so the squares its candidates
    // add, are the same in every lane).  First stage without arg-mins: the
    // lanes run along the rows, G groups per row, so the lanes of a row read
    // the same source values (a few distinct addresses per load, no
    // staging); with arg-mins it keeps the line-per-lane layout and its LDS
    // tiles.  Either way a launch has nchunk x G items of 64 lanes.
    constexpr bool ROWLANES = FIRST && !ARG;
    const int G = (N + kXsT - 1) / kXsT;
    int e, t0;
    if constexpr (ROWLANES) {
      const int gi = local * 64 + lane;
      e = gi / G;
      t0 = (gi - e * G) * kXsT;
    } else {
      const int group = local / nchunk, chunk = local - group * nchunk;
      t0 = group * kXsT;
      e = chunk * 64 + lane;
    }
    int st = 1;
    for (int q = 0; q < k; ++q) st *= N;   // stride of axis d-1-k
    const bool valid = e < lines;
    const int ee = valid ? e : 0;
    const int outer = ee / st, inner = ee - outer * st;
    const int base = outer * N * st + inner;
    const float* src = phase == 0 ? J.fhat : J.g;
    const double* v1in = J.xs_v + (size_t)((k + 1) & 1) * 2 * P;   // stage k reads buffer (k+1)&1
    const double* v2in = v1in + P;
    const int* ixin = J.xs_i + (size_t)((k + 1) & 1) * P;
    double m1[kXsT], m2[kXsT];
    int ix[kXsT];
#pragma unroll
    for (int t = 0; t < kXsT; ++t) { m1[t] = INFINITY; m2[t] = INFINITY; ix[t] = -1; }
    const_dptr sq = (const_dptr)sqt;
    // one source step: candidates h + (r - t0 - t)^2 for the lane's targets,
    // the costs the same for every lane (one run of scalar loads)
    auto step = [&](double h, int r) {
      const_dptr sr = sq + (r - t0 + kXsOff - (kXsT - 1));
#pragma unroll
      for (int t = 0; t < kXsT; ++t) {
        const double w = h + sr[kXsT - 1 - t];
        if (ARG) {
          m2[t] = fmin(m2[t], fmax(m1[t], w));
          ix[t] = w < m1[t] ? r : ix[t];
          m1[t] = fmin(m1[t], w);
        } else {
          // each candidate's add next to its min, so that the scheduler does
          // not hold all T candidates in registers at once
          m1[t] = vmin_f64(m1[t], w);
        }
      }
    };
    // The SW waves of the work-group split the sources: wave wv takes
    // [rlo, rhi), a multiple of 16 long (the first stage's tile width, so
    // also of kXsT), and the minima meet in LDS at the end.  Arg-mins keep
    // one wave per item (SW = 1).
    const int chunkS = ((N + 16 * SW - 1) / (16 * SW)) * 16;
    const int rlo = min(N, wv * chunkS), rhi = min(N, rlo + chunkS);
    // value-only: squares from a rotating register window (all-VGPR adds)
    // over whole blocks of kXsT sources; the last (rhi - rlo) mod kXsT
    // sources take them from the table
    double W[kXsT];
    double inc = 2.0 * (double)(rlo - t0) - 1.0;
    if constexpr (!ARG) {
#pragma unroll
      for (int q = 1; q < kXsT; ++q) W[q] = (double)(rlo - t0 - q) * (double)(rlo - t0 - q);
      W[0] = 0.0;
    }
    const int NB = ARG ? rlo : rhi - (rhi - rlo) % kXsT;   // sources in whole window blocks end here
    if constexpr (ROWLANES) {
      // the lane's row, loaded one source at a time four steps ahead (all
      // lanes of a row load the same address), converted to -phi in float64
      typedef const __attribute__((address_space(1))) float* gfptr;
      const gfptr rp = (gfptr)(src + (size_t)ee * N);
      if constexpr (kXsT >= 8) {
        float hb[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) hb[u] = rlo + u < NB ? rp[rlo + u] : 0.0f;
        for (int r0 = rlo; r0 < NB; r0 += kXsT) {
          xs_window_block<kXsT>(m1, W, inc, [&](int j) {
            hb[(j + 4) & 7] = rp[min(r0 + j + 4, NB - 1)];
            return -(double)hb[j & 7];
          });
        }
      } else {
        for (int r0 = rlo; r0 < NB; r0 += kXsT) {
          float hc[kXsT];
#pragma unroll
          for (int u = 0; u < kXsT; ++u) hc[u] = rp[r0 + u];
          xs_window_block<kXsT>(m1, W, inc, [&](int j) { return -(double)hc[j]; });
        }
      }
      // the remaining sources: per-lane targets, so the squares are formed
      // here (exact small integers) rather than read as wave-uniform values
      for (int r = NB; r < rhi; ++r) {
        const double h = -(double)rp[r];
#pragma unroll
        for (int t = 0; t < kXsT; ++t) {
          const double dd = (double)(r - t0 - t);
          m1[t] = vmin_f64(m1[t], h + dd * dd);
        }
      }
    } else if (FIRST) {
      // the lines are rows (stride 1): tiles of 64 rows x 16 columns are read
      // coalesced (the next tile while the current one is in use) into LDS,
      // then each lane walks its own row there (stride 17 words, no bank
      // conflicts), instead of 64 rows' cache lines per load
      constexpr int TC = 16;
      const int row0 = e - lane;   // the chunk's first line
      const int sub = lane / TC, cl = lane % TC;   // 4 rows of 16 columns per load
      float nx[64 / 4];
      // a wave-uniform base per group of four rows plus the lane's 32-bit
      // offset inside the group: the loads take the scalar-base form and no
      // per-row 64-bit addresses stay live across the tiles
      const unsigned loff = (unsigned)(sub * N + cl);
      auto fetch = [&](int rb) {
#pragma unroll
        for (int i = 0; i < 64 / 4; ++i) {
          const int row = row0 + 4 * i + sub, col = rb + cl;
          const float* ub = src + ((size_t)(row0 + 4 * i) * N + rb);
          nx[i] = (row < lines && col < N) ? ub[loff] : 0.0f;
        }
      };
      // each wave has its own tile: ordering its LDS writes and reads needs
      // only a wave-level barrier
      auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      };
      if (rlo < rhi) fetch(rlo);
      for (int rb = rlo; rb < rhi; rb += TC) {
        const int nc = min(TC, rhi - rb);
        wave_sync();
#pragma unroll
        for (int i = 0; i < 64 / 4; ++i) tile[(4 * i + sub) * (TC + 1) + cl] = nx[i];
        wave_sync();
        if (rb + TC < rhi) fetch(rb + TC);
        // unrolled so that the loop-carried minima are re-canonicalised (a
        // max with itself, for min/max in IEEE mode) once per four steps
#pragma unroll 4
        for (int j = 0; j < nc; ++j) step(-(double)tile[lane * (TC + 1) + j], rb + j);
      }
    } else if constexpr (!ARG) {
      // whole window blocks; each source is loaded four steps before its use
      // into a ring of eight (a block of 8 or 16 sources starts at a multiple
      // of 8, so the ring slots are fixed), or for 2 and 4 targets per lane a
      // block's sources while the previous block is in use
      if constexpr (kXsT >= 8) {
        // buffer loads: the lane's byte offset in a vector register, the
        // source's (r st 8 bytes) in a scalar one, so a load takes no vector
        // address arithmetic.  The resource spans this stage's two input
        // halves (v1in, v2in: 2P doubles); the loads four steps ahead of the
        // last whole block stay inside it and go unused.
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(v1in), 0, 16 * P, 0x00020000);
        const int lob = base * 8;   // the lane's byte offset
        const int st8 = st * 8;
        // the next load's source offset, advanced by one source per load; the
        // empty asm keeps it one running scalar (rather than sixteen
        // precomputed per-step offsets that would not fit the scalar
        // registers)
        int soff = rlo * st8;
        auto next = [&]() {
          const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, lob, soff, 0);
          soff += st8;
          __asm__ volatile("" : "+s"(soff));
          double x;
          __builtin_memcpy(&x, &w, 8);
          return x;
        };
        double hb[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) hb[u] = next();
        for (int r0 = rlo; r0 < NB; r0 += kXsT) {
          xs_sq_block<kXsT, 4>(m1, sq + (r0 - t0 + kXsOff), [&](int j) {
            hb[(j + 4) & 7] = next();   // source r0 + j + 4
            return hb[j & 7];
          });
        }
      } else {
        double hc[kXsT], hn[kXsT];
        if (NB > rlo) {
#pragma unroll
          for (int u = 0; u < kXsT; ++u) hn[u] = v1in[base + (rlo + u) * st];
        }
        for (int r0 = rlo; r0 < NB; r0 += kXsT) {
#pragma unroll
          for (int u = 0; u < kXsT; ++u) hc[u] = hn[u];
          if (r0 + kXsT < NB) {
#pragma unroll
            for (int u = 0; u < kXsT; ++u) hn[u] = v1in[base + (r0 + kXsT + u) * st];
          }
          xs_window_block<kXsT>(m1, W, inc, [&](int j) { return hc[j]; });
        }
      }
      for (int r = NB; r < rhi; ++r) step(v1in[base + r * st], r);
    } else {
      // four sources per round, the next four loaded while these are used
      const int N4 = N & ~3;
      double hn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) hn[u] = u < N4 ? v1in[base + u * st] : 0.0;
      for (int r = 0; r < N4; r += 4) {
        double hc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) hc[u] = hn[u];
        if (r + 4 < N4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) hn[u] = v1in[base + (r + 4 + u) * st];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) step(hc[u], r + u);
      }
      for (int r = N4; r < N; ++r) step(v1in[base + r * st], r);
    }
    if constexpr (!ARG) {
      // the waves' minima meet in wave 0 as a tree: the upper half of the
      // waves hands its minima to the lower half, which halves again (the
      // barrier before each round's writes also keeps them behind the reads
      // of the round before, and of the previous item's last round), so the
      // LDS holds SW / 2 waves' minima at most and more work-groups fit a CU
      for (int half = SW >> 1; half > 0; half >>= 1) {
        __syncthreads();
        if (wv >= half && wv < 2 * half) {
#pragma unroll
          for (int t = 0; t < kXsT; ++t) red[((wv - half) * kXsT + t) * 64 + lane] = m1[t];
        }
        __syncthreads();
        if (wv < half) {
#pragma unroll
          for (int t = 0; t < kXsT; ++t) m1[t] = vmin_f64(m1[t], red[(wv * kXsT + t) * 64 + lane]);
        }
      }
      if (wv > 0) return;
    }
    if (!valid) return;
    const bool last = k == J.d - 1;
    float* dst = phase == 0 ? J.g : J.f;
    int* arg = phase == 0 ? J.arg_g : J.arg_f;
    double* v1out = J.xs_v + (size_t)(k & 1) * 2 * P;
    double* v2out = v1out + P;
    int* ixout = J.xs_i + (size_t)(k & 1) * P;
    const double dk = (double)J.d * 4.440892098500626e-16;    // d 2^-51
    const double c0 = 2.0 * J.d * (double)(N - 1) * (N - 1) + 1.0;
#pragma unroll
    for (int t = 0; t < kXsT; ++t) {
      const int tt = t0 + t;
      if (tt >= N) break;
      const int o = base + tt * st;
      if (!ARG) {
        if (!last) {
          v1out[o] = m1[t];
          continue;
        }
        const double w1 = m1[t];
        const double del1 = dk * (fabs(w1) + c0);
        const float lo = (float)(w1 - del1), hi = (float)(w1 + del1);
        if (lo == hi) {   // false for NaN and infinite values
          dst[o] = lo;
        } else {
          const int slot = atomicAdd(count, 1);
          list[slot] = make_int2(jb, o);
        }
        continue;
      }
      const int rs = ix[t];
      double s1 = INFINITY;
      int idx = -1;
      if (rs >= 0) {
        const double c = (double)(rs - tt) * (double)(rs - tt);
        s1 = FIRST ? INFINITY : c + v2in[base + rs * st];
        idx = rs * st + (FIRST ? 0 : ixin[base + rs * st]);
      }
      const double w2 = fmin(m2[t], s1);
      if (!last) {
        v1out[o] = m1[t];
        v2out[o] = w2;
        ixout[o] = idx;
        continue;
      }
      const double w1 = m1[t];
      const double del1 = dk * (fabs(w1) + c0);
      const float lo = (float)(w1 - del1), hi = (float)(w1 + del1);
      bool ok = lo == hi && idx >= 0;   // false for NaN and infinite values
      if (ok && arg && w2 != INFINITY) {
        const double del2 = dk * (fabs(w2) + c0);
        ok = (float)(w2 - del2) > lo;
      }
      if (ok) {
        dst[o] = lo;
        if (arg) arg[o] = idx;
      } else {
        const int slot = atomicAdd(count, 1);
        list[slot] = make_int2(jb, o);
      }
    }
  }
}

// Two-dimensional jobs without arg-mins, 8 or 16 targets per lane: axis 0
// first, then axis 1.  Both stages give a wave 64 consecutive lines (the
// columns x_1 in the first, the target rows y_0 in the second) whose sources
// lie N apart, so every load is coalesced across the lanes and the wave's
// targets, hence the squares its candidates add, are common to its lanes
// (scalar registers, as in the later stages above).  The first stage writes
// its minima line by line, [x_1][y_0], the layout the second reads along its
// lanes.  Each candidate still takes one float64 rounding per axis, of the
// same magnitudes, so the error bound and the certification are those of the
// other order, and so are the certified values.
template <bool FIRST, int kXsT>
__device__ __forceinline__ void xs_item_xt(const DevJob& J, int jb, int local, int phase,
                                           const double* __restrict__ sqt, int2* __restrict__ list,
                                           int* __restrict__ count, int wv, int SW, double* red) {
  const int lane = threadIdx.x & 63;
  const int N = J.N, P = J.P;
  const int nchunk = (N + 63) >> 6;
  const int group = local / nchunk, chunk = local - group * nchunk;
  const int t0 = group * kXsT;
  const int e = chunk * 64 + lane;   // the lane's line
  const bool valid = e < N;
  const int ee = valid ? e : 0;
  double m1[kXsT];
#pragma unroll
  for (int t = 0; t < kXsT; ++t) m1[t] = INFINITY;
  const_dptr sq = (const_dptr)sqt;
  const int chunkS = ((N + 16 * SW - 1) / (16 * SW)) * 16;
  const int rlo = min(N, wv * chunkS), rhi = min(N, rlo + chunkS);
  const int NB = rhi - (rhi - rlo) % kXsT;   // sources in whole blocks end here
  // source r of line e at r N + e: the first stage reads the potential
  // (float32, negated), the second the first stage's minima (buffer 0);
  // buffer loads with the lane's byte offset in a vector register and the
  // source's in a scalar one, clamped to the last source (the loads four
  // steps ahead of the last block go unused)
  constexpr int EB = FIRST ? 4 : 8;
  const void* base = FIRST ? (const void*)(phase == 0 ? J.fhat : J.g) : (const void*)J.xs_v;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, EB * P, 0x00020000);
  const int lob = ee * EB;
  const int st8 = N * EB, last_off = (N - 1) * st8;
  int soff = rlo * st8;
  // a ring of eight raw loads (float32 or float64 bits), each converted only
  // when its step uses it
  typedef typename std::conditional<FIRST, float, double>::type HT;
  auto next = [&]() {
    HT x;
    if constexpr (FIRST) {
      x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lob, soff, 0));
    } else {
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, lob, soff, 0);
      __builtin_memcpy(&x, &w, 8);
    }
    soff = min(soff + st8, last_off);
    __asm__ volatile("" : "+s"(soff));
    return x;
  };
  HT hb[8];
#pragma unroll
  for (int u = 0; u < 4; ++u) hb[u] = next();
  for (int r0 = rlo; r0 < NB; r0 += kXsT) {
    xs_sq_block<kXsT, 4>(m1, sq + (r0 - t0 + kXsOff), [&](int j) {
      hb[(j + 4) & 7] = next();   // source r0 + j + 4
      return FIRST ? -(double)hb[j & 7] : (double)hb[j & 7];
    });
  }
  // the last (rhi - rlo) mod kXsT sources: squares from the table per step
  for (int r = NB; r < rhi; ++r) {
    const double h = FIRST ? -(double)(phase == 0 ? J.fhat : J.g)[(size_t)r * N + ee]
                           : J.xs_v[(size_t)r * N + ee];
    const_dptr sr = sq + (r - t0 + kXsOff - (kXsT - 1));
#pragma unroll
    for (int t = 0; t < kXsT; ++t) m1[t] = vmin_f64(m1[t], h + sr[kXsT - 1 - t]);
  }
  // the waves' minima meet in wave 0 (as in xs_item)
  for (int half = SW >> 1; half > 0; half >>= 1) {
    __syncthreads();
    if (wv >= half && wv < 2 * half) {
#pragma unroll
      for (int t = 0; t < kXsT; ++t) red[((wv - half) * kXsT + t) * 64 + lane] = m1[t];
    }
    __syncthreads();
    if (wv < half) {
#pragma unroll
      for (int t = 0; t < kXsT; ++t) m1[t] = vmin_f64(m1[t], red[(wv * kXsT + t) * 64 + lane]);
    }
  }
  if (wv > 0 || !valid) return;
  if constexpr (FIRST) {
#pragma unroll
    for (int t = 0; t < kXsT; ++t)
      if (t0 + t < N) J.xs_v[(size_t)e * N + t0 + t] = m1[t];
  } else {
    float* dst = phase == 0 ? J.g : J.f;
    const double dk = 2.0 * 4.440892098500626e-16;    // d 2^-51, d = 2
    const double c0 = 4.0 * (double)(N - 1) * (N - 1) + 1.0;
#pragma unroll
    for (int t = 0; t < kXsT; ++t) {
      if (t0 + t >= N) break;
      const int o = e * N + t0 + t;   // target (y_0 = e, y_1 = t0 + t)
      const double w1 = m1[t];
      const double del1 = dk * (fabs(w1) + c0);
      const float lo = (float)(w1 - del1), hi = (float)(w1 + del1);
      if (lo == hi) {   // false for NaN and infinite values
        dst[o] = lo;
      } else {
        const int slot = atomicAdd(count, 1);
        list[slot] = make_int2(jb, o);
      }
    }
  }
}

// The window minima of a wave's TPW targets: the first stage stores them, the
// second certifies them (as in xs_item_xt).
template <bool FIRST, int TPW>
__device__ __forceinline__ void xs_win_store(const DevJob& J, int jb, int phase, int2* __restrict__ list,
                                             int* __restrict__ count, int e, bool valid, int tw0,
                                             const double (&m)[TPW]) {
  const int N = J.N;
  if (!valid) return;
  if constexpr (FIRST) {
#pragma unroll
    for (int j = 0; j < TPW; ++j)
      if (tw0 + j < N) J.xs_v[(size_t)e * N + tw0 + j] = m[j];
  } else {
    float* dst = phase == 0 ? J.g : J.f;
    const double dk = 2.0 * 4.440892098500626e-16;    // d 2^-51, d = 2
    const double c0 = 4.0 * (double)(N - 1) * (N - 1) + 1.0;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      if (tw0 + j >= N) break;
      const int o = e * N + tw0 + j;   // target (y_0 = e, y_1 = tw0 + j)
      const double w1 = m[j];
      const double del1 = dk * (fabs(w1) + c0);
      const float lo = (float)(w1 - del1), hi = (float)(w1 + del1);
      if (lo == hi) {   // false for NaN and infinite values
        dst[o] = lo;
      } else {
        const int slot = atomicAdd(count, 1);
        list[slot] = make_int2(jb, o);
      }
    }
  }
}

// The same stage by windows (the default for these jobs).  Along one axis the
// candidate matrix a[r] + (r - t)^2 is Monge, so the first exact minimiser of
// a target never lies left of the first one of a smaller target, nor the last
// one right of the last one of a larger target.  Rounding is monotone: every
// exact minimiser of t attains the rounded minimum of t, and the rounded
// minimum is the rounding of the exact one.  Hence, for the targets t0 <= t <=
// t1 of an item, the sources from the first one attaining the rounded minimum
// of t0 to the last one attaining that of t1 hold a minimiser of each t, and
// the minimum over that window equals the minimum over all sources, bit for
// bit (no source whose value is NaN ever bounds a window; a line without a
// finite candidate keeps +inf).  Phase 1: the item's waves split the sources
// and scan the two boundary targets, keeping each one's rounded minimum and
// the start of the first, or the end of the last, block of eight sources
// attaining it (bounds on the first and last sources attaining it); the
// waves' partials meet through LDS.
// Phase 2: each wave scans the window (the union over its 64 lines, so that
// loads stay coalesced and the squares wave-uniform) for T / SW of the
// item's targets, and certifies and stores them as above; a window of up to
// kXsWinCap sources is first staged in LDS by the work-group, so that its
// waves read it from the L2 once between them.
template <bool FIRST, int TPW>
__device__ __forceinline__ void xs_win_scan(const DevJob& J, int jb, int phase, const_dptr sq,
                                            int2* __restrict__ list, int* __restrict__ count, int e,
                                            bool valid, int tw0, int wlo, int whi,
                                            __amdgpu_buffer_rsrc_t rs, int lob, int st8) {
  double m[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) m[j] = INFINITY;
  typedef typename std::conditional<FIRST, float, double>::type HT;
  auto load = [&](int off) {   // the source at byte offset off (a scalar)
    HT x;
    if constexpr (FIRST) {
      x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lob, off, 0));
    } else {
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, lob, off, 0);
      __builtin_memcpy(&x, &w, 8);
    }
    return x;
  };
  if (wlo <= whi) {
    // blocks of sixteen through a ring of loads eight ahead; in the last
    // block the sources past the window load the window's last source and
    // count as +inf
    const int whi8 = whi * st8;
    int soff = wlo * st8;
    auto next = [&]() {
      const HT x = load(soff);
      soff = min(soff + st8, whi8);
      __asm__ volatile("" : "+s"(soff));
      return x;
    };
    HT hb[16];
#pragma unroll
    for (int u = 0; u < 8; ++u) hb[u] = next();
    auto block = [&](int r0, auto partial) {   // sixteen sources
#pragma unroll
      for (int bk = 0; bk < 2; ++bk) {
        // sb[j + TPW - 1 - t] = (r0 + 8 bk + j - tw0 - t)^2
        const_dptr sb = sq + (r0 + 8 * bk - tw0 + kXsOff - (TPW - 1));
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          hb[(8 * bk + j + 8) & 15] = next();   // source r0 + 8 bk + j + 8
          double h = FIRST ? -(double)hb[8 * bk + j] : (double)hb[8 * bk + j];
          if constexpr (decltype(partial)::value) h = r0 + 8 * bk + j <= whi ? h : INFINITY;
#pragma unroll
          for (int t = 0; t < TPW; ++t) m[t] = vmin_f64(m[t], h + sb[j + TPW - 1 - t]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    int r0 = wlo;
    for (; r0 + 15 <= whi; r0 += 16) block(r0, std::false_type());
    if (r0 <= whi) block(r0, std::true_type());
  }
  xs_win_store<FIRST, TPW>(J, jb, phase, list, count, e, valid, tw0, m);
}

// Phase 2 from a window staged in LDS by the work-group, wb[(r - wlo) 64 +
// lane] the source r of the lane's line, in blocks of eight (the last one
// masked past the window).
template <bool FIRST, int TPW>
__device__ __forceinline__ void xs_win_scan_lds(const DevJob& J, int jb, int phase, const_dptr sq,
                                                int2* __restrict__ list, int* __restrict__ count, int e,
                                                bool valid, int tw0, int wlo, int whi,
                                                const typename std::conditional<FIRST, float, double>::type* wb) {
  const int lane = threadIdx.x & 63;
  double m[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) m[j] = INFINITY;
  const int last = whi - wlo;
  auto block = [&](int r0, auto partial) {
    // sb[j + TPW - 1 - t] = (r0 + j - tw0 - t)^2
    const_dptr sb = sq + (r0 - tw0 + kXsOff - (TPW - 1));
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int sidx = decltype(partial)::value ? min(r0 + j - wlo, last) : r0 + j - wlo;
      double h = FIRST ? -(double)wb[sidx * 64 + lane] : (double)wb[sidx * 64 + lane];
      if constexpr (decltype(partial)::value) h = r0 + j <= whi ? h : INFINITY;
#pragma unroll
      for (int t = 0; t < TPW; ++t) m[t] = vmin_f64(m[t], h + sb[j + TPW - 1 - t]);
    }
  };
  int r0 = wlo;
  for (; r0 + 7 <= whi; r0 += 8) block(r0, std::false_type());
  if (r0 <= whi) block(r0, std::true_type());
  xs_win_store<FIRST, TPW>(J, jb, phase, list, count, e, valid, tw0, m);
}

template <bool FIRST, int kXsT>
__device__ __forceinline__ void xs_item_win(const DevJob& J, int jb, int local, int phase,
                                            const double* __restrict__ sqt, int2* __restrict__ list,
                                            int* __restrict__ count, int wv, int SW, double* red) {
  const int lane = threadIdx.x & 63;
  const int N = J.N, P = J.P;
  const int ngroup = (N + kXsT - 1) / kXsT;
  const int chunk = local / ngroup, group = local - chunk * ngroup;   // chunk-major
  const int t0 = group * kXsT;
  const int tb1 = min(t0 + kXsT - 1, N - 1);   // the item's last target
  const int e = chunk * 64 + lane;
  const bool valid = e < N;
  const int ee = valid ? e : 0;
  const_dptr sq = (const_dptr)sqt;
  const int chunkS = ((N + 16 * SW - 1) / (16 * SW)) * 16;
  const int rlo = min(N, wv * chunkS), rhi = min(N, rlo + chunkS);
  const int NB = rhi - (rhi - rlo) % 16;   // sources in whole pairs of blocks of 8 end here
  // phase 1: rounded minima of t0 and tb1 over this wave's sources, with the
  // start of the first block of eight attaining the one and the end of the
  // last block attaining the other
  double b0 = INFINITY, b1 = INFINITY;
  int lo = 0x7fffffff, hi = -1;
  constexpr int EB = FIRST ? 4 : 8;
  const void* base = FIRST ? (const void*)(phase == 0 ? J.fhat : J.g) : (const void*)J.xs_v;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, EB * P, 0x00020000);
  const int lob = ee * EB;
  const int st8 = N * EB, last_off = (N - 1) * st8;
  int soff = rlo * st8;
  typedef typename std::conditional<FIRST, float, double>::type HT;
  auto next = [&]() {
    HT x;
    if constexpr (FIRST) {
      x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lob, soff, 0));
    } else {
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, lob, soff, 0);
      __builtin_memcpy(&x, &w, 8);
    }
    soff = min(soff + st8, last_off);
    __asm__ volatile("" : "+s"(soff));
    return x;
  };
  auto load_src = [&](int r) {   // source r of the lane's line (r a scalar)
    HT x;
    if constexpr (FIRST) {
      x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, lob, r * st8, 0));
    } else {
      const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, lob, r * st8, 0);
      __builtin_memcpy(&x, &w, 8);
    }
    return x;
  };
  // a block's minima update the running ones: lo is the first block start
  // and hi the last block end at which they are attained (bounds on the
  // first and last sources attaining them, at most seven sources wider)
  auto take = [&](double m0, double m1, int first, int last) {
    lo = m0 < b0 ? first : lo;
    hi = m1 <= b1 ? last : hi;
    b0 = vmin_f64(b0, m0);
    b1 = vmin_f64(b1, m1);
  };
  // a ring of sixteen loads, eight ahead: a step does a few instructions
  // per load, so the loads in flight, not the arithmetic, hide the latency
  HT hb[16];
#pragma unroll
  for (int u = 0; u < 8; ++u) hb[u] = next();
  for (int r0 = rlo; r0 < NB; r0 += 16) {
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) {
      const int rb = r0 + 8 * bk;
      const_dptr q0 = sq + (rb - t0 + kXsOff), q1 = sq + (rb - tb1 + kXsOff);
      double m0 = INFINITY, m1 = INFINITY;
      // in two halves, each with its own eight squares in scalar registers
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        double s0[4], s1[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) { s0[j] = q0[4 * hf + j]; s1[j] = q1[4 * hf + j]; }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int j = 8 * bk + 4 * hf + jj;
          hb[(j + 8) & 15] = next();   // source r0 + j + 8
          const double h = FIRST ? -(double)hb[j] : (double)hb[j];
          m0 = vmin_f64(m0, h + s0[jj]);
          m1 = vmin_f64(m1, h + s1[jj]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      take(m0, m1, rb, rb + 7);
    }
  }
  for (int r = NB; r < rhi; ++r) {
    const double h = FIRST ? -(double)(phase == 0 ? J.fhat : J.g)[(size_t)r * N + ee]
                           : J.xs_v[(size_t)r * N + ee];
    take(h + sq[r - t0 + kXsOff], h + sq[r - tb1 + kXsOff], r, r);
  }
  // the waves' partials, combined in wave order by every wave
  double* rb = red;                                        // SW x 64 x (b0, b1)
  int* ri = reinterpret_cast<int*>(red + 2 * 64 * SW);     // SW x 64 x (lo, hi)
  rb[(wv * 64 + lane) * 2] = b0;
  rb[(wv * 64 + lane) * 2 + 1] = b1;
  ri[(wv * 64 + lane) * 2] = lo;
  ri[(wv * 64 + lane) * 2 + 1] = hi;
  __syncthreads();
  b0 = INFINITY; b1 = INFINITY; lo = 0x7fffffff; hi = -1;
  for (int w = 0; w < SW; ++w) {
    const double c0 = rb[(w * 64 + lane) * 2], c1 = rb[(w * 64 + lane) * 2 + 1];
    const int l0 = ri[(w * 64 + lane) * 2], h1 = ri[(w * 64 + lane) * 2 + 1];
    lo = c0 < b0 ? l0 : (c0 == b0 ? min(lo, l0) : lo);
    hi = c1 < b1 ? h1 : (c1 == b1 ? max(hi, h1) : hi);
    b0 = vmin_f64(b0, c0);
    b1 = vmin_f64(b1, c1);
  }
  // the window over the wave's lines
  if (!valid) { lo = 0x7fffffff; hi = -1; }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  const int wlo = __builtin_amdgcn_readfirstlane(max(lo, 0));
  const int whi = __builtin_amdgcn_readfirstlane(min(hi, N - 1));
  // phase 2: this wave's targets
  const int tpw = kXsT / SW;
  const int tw0 = t0 + wv * tpw;
  const int nw = whi - wlo + 1;   // the same in every wave of the work-group
  if (nw > 0 && nw <= kXsWinCap) {
    // the window staged once in LDS (over the partials, once every wave has
    // read them), each wave loading every SW-th source of it
    HT* wb = reinterpret_cast<HT*>(red);
    __syncthreads();
    for (int sidx = wv; sidx < nw; sidx += SW) wb[sidx * 64 + lane] = load_src(wlo + sidx);
    __syncthreads();
    if (tw0 >= N) return;
    if (tpw == 2) {
      xs_win_scan_lds<FIRST, 2>(J, jb, phase, sq, list, count, e, valid, tw0, wlo, whi, wb);
    } else {
      for (int c = 0; c < tpw; c += 4)
        xs_win_scan_lds<FIRST, 4>(J, jb, phase, sq, list, count, e, valid, tw0 + c, wlo, whi, wb);
    }
    return;
  }
  if (tw0 >= N) return;
  // (four targets per pass at most, which keeps one pass within the
  // stage's registers; more passes re-read the window from the caches)
  if (tpw == 2) {
    xs_win_scan<FIRST, 2>(J, jb, phase, sq, list, count, e, valid, tw0, wlo, whi, rs, lob, st8);
  } else {
    for (int c = 0; c < tpw; c += 4)
      xs_win_scan<FIRST, 4>(J, jb, phase, sq, list, count, e, valid, tw0 + c, wlo, whi, rs, lob, st8);
  }
}

// One instance per (stage kind, targets per lane T, arg-mins): each has its
// own register budget.  T (16, 8, 4 or 2) is the plan's: fewer for small
// plans, so that a launch still has enough waves (16 only without arg-mins,
// where a target holds one running minimum).  A work-group of SW = blockDim / 64
// waves takes one item, its waves splitting the sources.
template <bool FIRST, int T, bool ARG, int XT>
__attribute__((amdgpu_waves_per_eu((ARG || (FIRST && XT == 0)) ? 4 : 8)))
__global__ __launch_bounds__(XT == 2 ? 512 : 256) void k_xs_stage(const DevJob* __restrict__ jobs, int njobs,
                                                  const int* __restrict__ off, int total, int phase, int k,
                                                  const double* __restrict__ sqt, int2* __restrict__ list,
                                                  int* __restrict__ count) {
  // dynamic LDS, sized by the launcher (xs_lds_bytes): the first stage's
  // per-wave tiles (64 x 17 floats, with arg-mins only), then SW / 2 x 64 x T
  // doubles for the waves' minima on their way to wave 0 (argmin windows:
  // SW x 64 x (two minima, two source bounds) for the waves' partials, then
  // the window's sources, up to kXsWinCap x 64)
  extern __shared__ double xs_lds[];
  const int SW = blockDim.x >> 6;
  // the wave index, known wave-uniform: source ranges and load addresses
  // derived from it stay in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float* tiles = reinterpret_cast<float*>(xs_lds);
  double* red = xs_lds + (FIRST && ARG ? (SW * 64 * 17 + 1) / 2 : 0);
  if constexpr (XT > 0) {
    // one item per work-group (the launcher's grid is the item count): with
    // the source loop not nested in an item loop, the wait before each block
    // is for the load four sources back, not for every load in flight.  XT 2:
    // argmin windows (xs_item_win), XT 1: every source (xs_item_xt), each in
    // its own instance with its own registers
    int it = blockIdx.x;
    if (it >= total) return;
    // argmin windows: work-groups go to the eight XCDs in turn, so XCD x
    // takes the x-th eighth of the items, whole line chunks (chunk-major
    // items), each chunk's sources read into one L2
    if (XT == 2 && (total & 7) == 0) it = (it & 7) * (total >> 3) + (it >> 3);
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (!J.xs || k >= J.d || J.xs_xt != XT) return;
    if constexpr (XT == 2)
      xs_item_win<FIRST, T>(J, jb, it - off[jb], phase, sqt, list, count, wv, SW, red);
    else
      xs_item_xt<FIRST, T>(J, jb, it - off[jb], phase, sqt, list, count, wv, SW, red);
  } else {
    for (int it = blockIdx.x; it < total; it += gridDim.x) {
      const int jb = find_job(off, njobs, it);
      const DevJob& J = jobs[jb];
      if (!J.xs || k >= J.d || J.xs_xt) continue;
      xs_item<FIRST, T, ARG>(J, jb, it - off[jb], phase, k, sqt, list, count, tiles + wv * 64 * 17, wv, SW, red);
    }
  }
}

// LDS bytes of one k_xs_stage work-group (matches the kernel's carving).
static size_t xs_lds_bytes(bool first, int T, bool arg, int waves, bool xt, bool first_src32) {
  const size_t tiles = first && arg ? 8 * (size_t)((waves * 64 * 17 + 1) / 2) : 0;
  // the waves' minima on their way to wave 0, or the windows' partials and
  // then the staged window (float32 sources in the first stage, else float64)
  const size_t red = xt ? std::max<size_t>((size_t)waves * 64 * (16 + 8), (size_t)kXsWinCap * 64 * (first_src32 ? 4 : 8))
                        : arg ? 0 : 8 * (size_t)(waves / 2) * 64 * T;
  return std::max<size_t>(8, tiles + red);
}

// The queued targets, one wave each, with the all-pairs arithmetic:
// RN32((float)c - phi), smallest value over non-NaN candidates (+inf if there
// is none), lowest source index attaining it (-1 if none).  Only sources
// whose value can round to that minimum matter, and the stage buffers bound
// them from below: a row (2D: one value of the first coordinate; 3D: one
// (x_0, x_1)) holds no candidate below its stage minimum plus the cost of the
// remaining axes, less the error bound.  The float64 best w1 gives
// psi <= hi = RN32(w1 + delta), so every source that can round to psi lies
// below T = hi + 2^-22 |hi| (beyond the upper end of hi's rounding interval);
// rows whose bound exceeds T are skipped, the others scanned in index order.
// NaN or infinite bounds never skip anything.
__device__ __forceinline__ void xs_take(float v, int i, float& best, int& bi) {
  if (v < best || (v == best && bi == 0x7fffffff)) { best = v; bi = i; }
}

__global__ __launch_bounds__(64) void k_xs_fallback(const DevJob* __restrict__ jobs, const int2* __restrict__ list,
                                                    const int* __restrict__ count, int phase) {
  const int n = *count;
  const int lane = threadIdx.x;
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int2 ent = list[q];
    const DevJob& J = jobs[ent.x];
    const int y = ent.y, N = J.N, P = J.P, d = J.d;
    const float* src = phase == 0 ? J.fhat : J.g;
    int y0, y1, y2;
    pix_coords(y, N, d, y0, y1, y2);
    const double* b0 = J.xs_v;           // stage 0: min over x_{d-1} per (x_0.., y_{d-1})
    const double* b1 = J.xs_v + 2 * P;   // stage 1 (3D): min over (x_1, x_2) per (x_0, y_1, y_2)
    const double dk = (double)d * 4.440892098500626e-16;
    const double c0 = 2.0 * d * (double)(N - 1) * (N - 1) + 1.0;
    // outer index o: 2D the row x_1 (coordinate y1 of the target), or the
    // column x_2 for jobs whose first stage ran along axis 0 (its buffer
    // [x_2][y_1]); 3D the plane x_0
    const bool xt = d == 2 && J.xs_xt;
    const int oy = d == 2 ? (xt ? y2 : y1) : y0;
    auto outer_bound = [&](int o) -> double {
      const double c = (double)(o - oy) * (double)(o - oy);
      return d == 2 ? b0[(size_t)o * N + (xt ? y1 : y2)] + c : b1[(size_t)o * N * N + (size_t)y1 * N + y2] + c;
    };
    // the lane's outer bounds (o = lane + 64 i), kept for the scan below
    // when N <= 256
    double obv[4];
    double w1 = INFINITY;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = lane + 64 * i;
      obv[i] = o < N ? outer_bound(o) : INFINITY;
      w1 = fmin(w1, obv[i]);
    }
    for (int o = lane + 256; o < N; o += 64) w1 = fmin(w1, outer_bound(o));
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) w1 = fmin(w1, __shfl_xor(w1, s, 64));
    const float hi = (float)(w1 + dk * (fabs(w1) + c0));
    const double T = (double)hi + 2.384185791015625e-07 * fabs((double)hi);   // + 2^-22 |hi|
    auto skip = [&](double bnd) { return bnd - dk * (fabs(bnd) + c0) > T; };
    float best = INFINITY;
    int bi = 0x7fffffff;
    auto scan_row = [&](int rowbase, int cost_rest, int ya) {
      // sources rowbase + x, x = 0 .. N-1 along the last axis (four loads in
      // flight per lane)
#pragma unroll 4
      for (int x = lane; x < N; x += 64) {
        const int e = x - ya;
        xs_take((float)(cost_rest + e * e) - src[rowbase + x], rowbase + x, best, bi);
      }
    };
    for (int oc = 0; oc < N; oc += 64) {
      const int o = oc + lane;
      const int ci = oc >> 6;
      const double bo = ci == 0 ? obv[0] : ci == 1 ? obv[1] : ci == 2 ? obv[2] : ci == 3 ? obv[3] : 0.0;
      unsigned long long m = __ballot(o < N && !skip(ci < 4 ? bo : outer_bound(o)));
      if (xt) {
        // value only: the selected columns four at a time, the sources (r, ob)
        // of each, r = 0 .. N-1, loaded 256 rows at a time before any is used
        while (m) {
          int cols[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            cols[c] = m ? oc + __ffsll((long long)m) - 1 : -1;
            m &= m - 1;
          }
          for (int r0 = 0; r0 < N; r0 += 256) {
            float v[4][4];
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const int r = r0 + lane + 64 * k;
                v[c][k] = (cols[c] >= 0 && r < N) ? src[r * N + cols[c]] : 0.0f;
              }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              if (cols[c] < 0) continue;
              const int co = (cols[c] - oy) * (cols[c] - oy);
#pragma unroll
              for (int k = 0; k < 4; ++k) {
                const int r = r0 + lane + 64 * k;
                if (r < N) {
                  const int e = r - y1;
                  xs_take((float)(co + e * e) - v[c][k], r * N + cols[c], best, bi);
                }
              }
            }
          }
        }
        continue;
      }
      while (m) {
        const int ob = oc + __ffsll((long long)m) - 1;
        m &= m - 1;
        const int co = (ob - oy) * (ob - oy);
        if (d == 2) {
          scan_row(ob * N, co, y2);
        } else {
          // rows (ob, x_1) of the plane, bounded by stage 0
          for (int rc = 0; rc < N; rc += 64) {
            const int r1 = rc + lane;
            bool ok = false;
            if (r1 < N) {
              const double bnd = b0[(size_t)ob * N * N + (size_t)r1 * N + y2] +
                                 (double)(co + (r1 - y1) * (r1 - y1));
              ok = !skip(bnd);
            }
            unsigned long long mr = __ballot(ok);
            while (mr) {
              const int rb = rc + __ffsll((long long)mr) - 1;
              mr &= mr - 1;
              scan_row(ob * N * N + rb * N, co + (rb - y1) * (rb - y1), y2);
            }
          }
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob < best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) {
      (phase == 0 ? J.g : J.f)[y] = best;
      int* arg = phase == 0 ? J.arg_g : J.arg_f;
      if (arg) arg[y] = bi == 0x7fffffff ? -1 : bi;
    }
  }
}

// ------------------------------------------------------------------ separable c-transform (p = 2)
//
// |x - y|^2 is a sum over axes, so the c-transform is d nested 1-D transforms.
// Pass k (0-based) runs along axis a = d-1-k; a line is one index tuple of the
// other axes and its element e sits at base + e * N^k.  Pass 0 subtracts the
// potential, later passes add the previous pass's result:
//   dst[v] = min_t RN32((t - v)^2 -/+ src[t]),  arg = lowest t attaining it.
// One wave per (job, line, chunk of 64 targets); the cost is updated exactly
// (c += D, D += 2) and the source values are wave-uniform scalar loads.
__global__ __launch_bounds__(64) void k_ct1d(const DevJob* __restrict__ jobs, int njobs,
                                             const int* __restrict__ off, int total, int phase,
                                             int pass) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (!J.sep || J.sep_R != 0 || pass >= J.d) continue;
    const int N = J.N, P = J.P;
    const int chunks = (N + 63) / 64;
    const int local = it - off[jb];
    const int line = local / chunks, ch = local - line * chunks;
    int stride = 1;
    for (int q = 0; q < pass; ++q) stride *= N;
    const int hi = line / stride, lo = line - hi * stride;
    const int base = hi * stride * N + lo;
    const float* src = pass == 0 ? (phase == 0 ? J.fhat : J.g) : J.sep_tmp + (size_t)((pass - 1) & 1) * P;
    float* dst = pass == J.d - 1 ? (phase == 0 ? J.g : J.f) : J.sep_tmp + (size_t)(pass & 1) * P;
    int* arg = J.sep_arg ? J.sep_arg + (size_t)pass * P : nullptr;
    const_fptr s = (const_fptr)(src + base);
    const int v = ch * 64 + (int)(threadIdx.x & 63);
    float c = (float)(v * v);
    float D = (float)(1 - 2 * v);
    float best = INFINITY;
    int barg = 0;
    if (pass == 0) {
      for (int t = 0; t < N; ++t) {
        const float val = c - s[(size_t)t * stride];
        if (val < best) { best = val; barg = t; }
        c += D;
        D += 2.0f;
      }
    } else {
      for (int t = 0; t < N; ++t) {
        const float val = c + s[(size_t)t * stride];
        if (val < best) { best = val; barg = t; }
        c += D;
        D += 2.0f;
      }
    }
    if (v < N) {
      dst[base + (size_t)v * stride] = best;
      if (arg) arg[base + (size_t)v * stride] = barg;
    }
  }
}

// The same pass without arg-mins, for power-of-two N in [32, 1024]: one wave
// per (job, line).  Lane l takes R consecutive targets v = (l mod TL) R + r
// (TL = N / R target lanes) and the sources of group l / TL, one of
// G = 64 / TL equal slices; the groups' minima are combined by lane exchange
// at the end.  Sources go in blocks of R: for a block starting at t0 the
// costs (v - t)^2 = (D + r - q)^2, D = (l mod TL) R - t0, take only 2R - 1
// values, exact float32 squares of small integers, so a pair costs one
// subtraction (addition in later passes; fused with the exact square) and
// half a v_min3, and the candidate is rounded exactly as in k_ct1d.  The
// line's sources are staged in LDS.
template <int R>
__global__ __launch_bounds__(64) void k_ct1d_fast(const DevJob* __restrict__ jobs, int njobs,
                                                  const int* __restrict__ off, int total, int phase, int pass) {
  __shared__ float line_v[1024];   // the line's signed source values
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (!J.sep || J.sep_R != R || pass >= J.d) continue;
    const int N = J.N, P = J.P;
    const int line = it - off[jb];
    int stride = 1;
    for (int q = 0; q < pass; ++q) stride *= N;
    const int hi = line / stride, lo = line - hi * stride;
    const size_t base = (size_t)hi * stride * N + lo;
    const float* src = pass == 0 ? (phase == 0 ? J.fhat : J.g) : J.sep_tmp + (size_t)((pass - 1) & 1) * P;
    float* dst = pass == J.d - 1 ? (phase == 0 ? J.g : J.f) : J.sep_tmp + (size_t)(pass & 1) * P;
    const int TL = N / R;            // target lanes per line (<= 64)
    const int SG = N * TL / 64;      // sources per group (a multiple of R)
    const int lane = threadIdx.x & 63;
    const int tl = lane & (TL - 1), grp = lane / TL;
    const float sgn = pass == 0 ? -1.0f : 1.0f;
    __syncthreads();
    for (int t = lane; t < N; t += 64) line_v[t] = sgn * src[base + (size_t)t * stride];
    __syncthreads();
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = INFINITY;
    const int t_begin = grp * SG, t_end = t_begin + SG;
    for (int t0 = t_begin; t0 < t_end; t0 += R) {
      float sv[R];
#pragma unroll
      for (int q = 0; q < R; ++q) sv[q] = line_v[t0 + q];
      // W[k] = (D + k - (R - 1))^2, k = r - q + R - 1
      const float b0 = (float)(tl * R - t0 - (R - 1));
      float W[2 * R - 1];
#pragma unroll
      for (int k = 0; k < 2 * R - 1; ++k) {
        const float e = b0 + (float)k;
        W[k] = e * e;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int q = 0; q < R; q += 2) {
          const float c0 = W[r - q + R - 1] + sv[q];
          const float c1 = W[r - q - 1 + R - 1] + sv[q + 1];
          acc[r] = __builtin_fminf(acc[r], __builtin_fminf(c0, c1));
          __asm__("" : "+v"(acc[r]));   // keep the running minimum a chain of v_min3
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      for (int o = TL; o < 64; o <<= 1) acc[r] = __builtin_fminf(acc[r], __shfl_xor(acc[r], o, 64));
    if (grp == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) dst[base + (size_t)(tl * R + r) * stride] = acc[r];
    }
  }
}

// Compose the passes' arg-mins into the source index (last pass fixes axis 0).
__global__ __launch_bounds__(256) void k_sep_argmin(const DevJob* __restrict__ jobs, int njobs,
                                                    const int* __restrict__ off, int total, int phase) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (!J.sep || !J.sep_arg) continue;
    int* out = phase == 0 ? J.arg_g : J.arg_f;
    if (!out) continue;
    const int base = (it - off[jb]) * kChunk;
    const int N = J.N, P = J.P;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int j = base + q;
      if (j >= P) break;
      int x[3];
      pix_coords(j, N, J.d, x[0], x[1], x[2]);   // 2D: x[1], x[2] hold the coordinates
      const int a0 = J.d == 2 ? 1 : 0;           // first used slot
      for (int pass = J.d - 1; pass >= 0; --pass) {
        const int slot = a0 + (J.d - 1 - pass);   // axis d-1-pass
        const int cur = J.d == 2 ? x[1] * N + x[2] : (x[0] * N + x[1]) * N + x[2];
        x[slot] = J.sep_arg[(size_t)pass * P + cur];
      }
      out[j] = J.d == 2 ? x[1] * N + x[2] : (x[0] * N + x[1]) * N + x[2];
    }
  }
}

// ------------------------------------------------------------------ IPF (Algorithm 4)
//
// With the uniform kernel, pi^ b is constant on every block:
//   (pi^ b)_i = k^(-2d) sum_L pi~_KL B_L,  B_L = sum_{j in Y_L} b_j,
// so the fitting runs on coarse vectors.  With a = mu / u (u = pi^ b) and
// b = nu / v (v = pi^T a) the block sums are A_K = mu~_K / u_K and
// B_L = nu~_L / v_L; b = 1 at the start gives B^0 = k^d.  Every iterate u^t,
// v^t is kept for the backward pass.  One work-group per job.
// The coarse coupling and per-block vectors a coarse kernel reads, in LDS
// when they fit the launch's dynamic allocation (lds_bytes), else in global
// memory; the arithmetic and its order are the same either way.
struct CoarseView {
  const int *csr, *csc, *cidx, *erow, *ecol;
  const double* ev;
  double* vec;   // nvec x Q doubles of scratch vectors (LDS), or null
  bool in_lds;
};

__device__ CoarseView coarse_view(const DevJob& J, double* lds, size_t lds_bytes, int nvec) {
  CoarseView c;
  const int Q = J.Q, nnz = J.nnz;
  c.in_lds = lds_bytes > 0 && coarse_lds_need(Q, nnz, nvec) <= lds_bytes;
  if (!c.in_lds) {
    c.csr = J.csr_ptr; c.csc = J.csc_ptr; c.cidx = J.csc_idx; c.erow = J.e_row; c.ecol = J.e_col;
    c.ev = J.e_val; c.vec = nullptr;
    return c;
  }
  double* ev = lds + (size_t)nvec * Q;
  int* ip = reinterpret_cast<int*>(ev + nnz);
  int* csr = ip;
  int* csc = csr + Q + 1;
  int* cidx = csc + Q + 1;
  int* erow = cidx + nnz;
  int* ecol = erow + nnz;
  for (int i = threadIdx.x; i < nnz; i += blockDim.x) {
    ev[i] = J.e_val[i];
    cidx[i] = J.csc_idx[i];
    erow[i] = J.e_row[i];
    ecol[i] = J.e_col[i];
  }
  for (int i = threadIdx.x; i <= Q; i += blockDim.x) {
    csr[i] = J.csr_ptr[i];
    csc[i] = J.csc_ptr[i];
  }
  c.csr = csr; c.csc = csc; c.cidx = cidx; c.erow = erow; c.ecol = ecol; c.ev = ev;
  c.vec = lds;
  __syncthreads();
  return c;
}

__device__ void coarse_reverse(const DevJob& J, const CoarseView& C, double* sc);
__device__ void coarse_plancost2(const DevJob& J, const CoarseView& C, int T);

// Iterative proportional fitting on coarse vectors (uniform kernel): with
// b-block sums B (B^0 = k^d), u^t = cc pi~ B^{t-1}, A^t = mu~ / u^t,
// v^t = cc pi~^T A^t, B^t = nu~ / v^t (0/0 := 0); the residual after
// iteration t is ||mu^ - mu||_1 (from u^{t+1} / u^t per block) plus the mass
// of unmatched target blocks.  One work-group per job; u^t and v^t are
// written out for the backward pass and the fine sweeps.  For p = 2 jobs the
// same work-group then forms the plan-cost entries (flags bit 0) and runs the
// reverse pass of the backward (bit 1, which needs bit 0), on the coupling it
// already holds: the whole coarse part of a step in one launch.
__global__ __launch_bounds__(1024) void k_ipf(const DevJob* __restrict__ jobs, int njobs, size_t lds_bytes,
                                              int flags, double* __restrict__ scratch_all, int stride) {
  extern __shared__ double lds[];
  __shared__ double sh[1024];
  const DevJob& J = jobs[blockIdx.x];
  const int Q = J.Q;
  const double kd = J.d == 2 ? (double)J.k * J.k : (double)J.k * J.k * J.k;
  const double cc = 1.0 / (kd * kd);
  double* U = J.ipf_u;  // row t holds u^t, t = 1 .. T+1
  double* V = J.ipf_v;  // row t holds v^t
  const CoarseView C = coarse_view(J, lds, lds_bytes, 6);
  // scratch vectors: LDS, or the job's global scratch and checkpoint rows
  double* Bprev = C.in_lds ? C.vec : J.gbar_nu;            // B^{t-1}
  double* Acur = C.in_lds ? C.vec + Q : J.gbar_mu;         // A^t
  double* ucur = C.in_lds ? C.vec + 2 * Q : nullptr;       // u^t (else row t of U)
  double* vcur = C.in_lds ? C.vec + 3 * Q : nullptr;       // v^t (else row t of V)
  double* muL = C.in_lds ? C.vec + 4 * Q : nullptr;
  double* nuL = C.in_lds ? C.vec + 5 * Q : nullptr;
  const double* mu_t = C.in_lds ? muL : J.mu_t;
  const double* nu_t = C.in_lds ? nuL : J.nu_t;
  for (int L = threadIdx.x; L < Q; L += 1024) {
    Bprev[L] = kd;
    if (C.in_lds) { muL[L] = J.mu_t[L]; nuL[L] = J.nu_t[L]; }
  }
  __syncthreads();
  // u^1
  {
    double* u = C.in_lds ? ucur : U + (size_t)1 * Q;
    for (int K = threadIdx.x; K < Q; K += 1024) {
      double s = 0.0;
      for (int e = C.csr[K]; e < C.csr[K + 1]; ++e) s += C.ev[e] * Bprev[C.ecol[e]];
      u[K] = cc * s;
      if (C.in_lds) U[(size_t)1 * Q + K] = u[K];
    }
  }
  __syncthreads();
  int T = 0;
  double resid = INFINITY;
  for (int t = 1; t <= J.max_iter; ++t) {
    const double* u = C.in_lds ? ucur : U + (size_t)t * Q;
    double* v = C.in_lds ? vcur : V + (size_t)t * Q;
    for (int K = threadIdx.x; K < Q; K += 1024) Acur[K] = u[K] > 0.0 ? mu_t[K] / u[K] : 0.0;
    __syncthreads();
    for (int L = threadIdx.x; L < Q; L += 1024) {
      double s = 0.0;
      for (int q = C.csc[L]; q < C.csc[L + 1]; ++q) {
        const int e = C.cidx[q];
        s += C.ev[e] * Acur[C.erow[e]];
      }
      v[L] = cc * s;
      if (C.in_lds) V[(size_t)t * Q + L] = v[L];
      Bprev[L] = v[L] > 0.0 ? nu_t[L] / v[L] : 0.0;
    }
    __syncthreads();
    // u^{t+1} (also the next iteration's u^t) and the residual of iteration t
    double part = 0.0;
    for (int K = threadIdx.x; K < Q; K += 1024) {
      double s = 0.0;
      for (int e = C.csr[K]; e < C.csr[K + 1]; ++e) s += C.ev[e] * Bprev[C.ecol[e]];
      const double un = cc * s;
      U[(size_t)(t + 1) * Q + K] = un;
      // ||mu^ - mu||_1 on block K: mu^_i = mu_i u^{t+1}_K / u^t_K
      const double m = mu_t[K];
      const double uk = u[K];
      if (uk > 0.0) part += m * fabs(un / uk - 1.0);
      else part += m;
      if (C.in_lds) Acur[K] = un;   // staged; copied into ucur below (Acur is free here)
    }
    for (int L = threadIdx.x; L < Q; L += 1024) {
      // nu^_j = b_j (pi^T a)_j = nu_j exactly when v^t_L > 0
      if (!(v[L] > 0.0)) part += nu_t[L];
    }
    resid = block_sum<1024>(part, sh);   // its barriers also order the writes above
    T = t;
    if (resid < J.xi) break;
    if (C.in_lds) {
      for (int K = threadIdx.x; K < Q; K += 1024) ucur[K] = Acur[K];
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    J.result[RS_IPF_ITERS] = (double)T;
    J.result[RS_IPF_RESID] = resid;
    J.result[RS_WARN] = (resid < J.xi) ? 0.0 : (double)QBW_WARN_IPF_NOT_CONVERGED;
  }
  if (J.p != 2 || !(flags & 1)) return;
  __syncthreads();   // the iterates and the results above, for the whole work-group
  coarse_plancost2(J, C, T);
  if (!(flags & 2)) return;
  __syncthreads();
  coarse_reverse(J, C, C.in_lds ? C.vec : scratch_all + (size_t)blockIdx.x * 4 * stride);
}

// Fine scalings of the last iterate: a_s = mu / u^T, b_s = nu / v^T (0/0 := 0).
__global__ __launch_bounds__(256) void k_scalings(const DevJob* __restrict__ jobs, int njobs,
                                                  const int* __restrict__ off, int total) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    const int T = (int)J.result[RS_IPF_ITERS];
    const double* u = J.ipf_u + (size_t)T * J.Q;
    const double* v = J.ipf_v + (size_t)T * J.Q;
    const int base = (it - off[jb]) * kChunk;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int i = base + q;
      if (i >= J.P) break;
      int x0, x1, x2;
      pix_coords(i, J.N, J.d, x0, x1, x2);
      const int n = J.n, k = J.k;
      const int K = J.d == 2 ? (x1 / k) * n + x2 / k : ((x0 / k) * n + x1 / k) * n + x2 / k;
      J.a_s[i] = u[K] > 0.0 ? J.mu[i] / u[K] : 0.0;
      J.b_s[i] = v[K] > 0.0 ? J.nu[i] / v[K] : 0.0;
    }
  }
}

// The forward pass's pixel sweep after IPF (one read of f, g, f^, mu, nu for
// three jobs): per chunk the lower-bound sums <f, mu>, <g, nu> and the maxima
// |f^|, |g|, |f| of the feasibility shift; the fine scalings of k_scalings
// (written out for p = 1 jobs, whose plan cost and gradient sum pixel pairs;
// p = 2 jobs take block moments instead); the weighted-TV
// partials of k_tv_partial, with the same arithmetic as those two kernels.
// Every partial goes to its chunk's slot; k_finalize adds them in order.
// NS sums and NM maxima of per-thread values over a 256-thread work-group, in
// a fixed order: a butterfly within each wave, then the four waves' results
// added in wave order.  Two barriers for all of them.  Results in every thread.
template <int NS, int NM>
__device__ __forceinline__ void block_reduce_many(double (&s)[NS], double (&m)[NM], double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int i = 0; i < NS; ++i) s[i] += __shfl_xor(s[i], o, 64);
#pragma unroll
    for (int i = 0; i < NM; ++i) m[i] = fmax(m[i], __shfl_xor(m[i], o, 64));
  }
  constexpr int W = NS + NM;
  const int w = threadIdx.x >> 6;
  __syncthreads();   // earlier readers of sh are done
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NS; ++i) sh[w * W + i] = s[i];
#pragma unroll
    for (int i = 0; i < NM; ++i) sh[w * W + NS + i] = m[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NS; ++i) s[i] = ((sh[i] + sh[W + i]) + sh[2 * W + i]) + sh[3 * W + i];
#pragma unroll
  for (int i = 0; i < NM; ++i)
    m[i] = fmax(fmax(sh[NS + i], sh[W + NS + i]), fmax(sh[2 * W + NS + i], sh[3 * W + NS + i]));
}

// clear[0 .. nclear): counters of the step's c-transforms, done with here,
// zeroed for the next step.
__global__ __launch_bounds__(256) void k_fwd_pixels(const DevJob* __restrict__ jobs, int njobs,
                                                    const int* __restrict__ off, int total,
                                                    int* __restrict__ clear, int nclear) {
  __shared__ double sh[256];
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < nclear; i += 256) clear[i] = 0;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    const int T = (int)J.result[RS_IPF_ITERS];
    const double* u = J.ipf_u + (size_t)T * J.Q;
    const double* un = J.ipf_u + (size_t)(T + 1) * J.Q;
    const double* v = J.ipf_v + (size_t)T * J.Q;
    const int c = it - off[jb];
    const int base = c * kChunk;
    const double hN = 0.5 * (J.N - 1);
    const int n = J.n, k = J.k;
    double sf = 0.0, sg = 0.0, mh = 0.0, mg = 0.0, mf = 0.0;
    double tm = 0.0, tn = 0.0, wm = 0.0, wn = 0.0;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int i = base + q;
      if (i >= J.P) break;
      const double mu = J.mu[i], nu = J.nu[i];
      // lower bound
      const double f = J.f[i], g = J.g[i];
      sf += f * mu;
      sg += g * nu;
      mh = fmax(mh, fabs((double)J.fhat[i]));
      mg = fmax(mg, fabs(g));
      mf = fmax(mf, fabs(f));
      // scalings
      int x0, x1, x2;
      pix_coords(i, J.N, J.d, x0, x1, x2);
      const int K = J.d == 2 ? (x1 / k) * n + x2 / k : ((x0 / k) * n + x1 / k) * n + x2 / k;
      const double as = u[K] > 0.0 ? mu / u[K] : 0.0;
      const double bs = v[K] > 0.0 ? nu / v[K] : 0.0;
      if (J.p == 1) {   // the p = 1 plan cost and gradient read them; p = 2 uses block moments
        J.a_s[i] = as;
        J.b_s[i] = bs;
      }
      // weighted TV
      const double d0 = J.d == 2 ? 0.0 : x0 - hN, d1 = x1 - hN, d2 = x2 - hN;
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double w = J.p == 2 ? r2 : sqrt(r2);
      const double muh = as * un[K];
      const double nuh = bs * v[K];
      tm += w * fabs(muh - mu);
      tn += w * fabs(nu - nuh);
      wm += w * mu;
      wn += w * nu;
    }
    double sv[6] = {sf, sg, tm, tn, wm, wn};
    double mv[3] = {mh, mg, mf};
    block_reduce_many<6, 3>(sv, mv, sh);
    if (threadIdx.x == 0) {
      double* r = J.red_lb + (size_t)c * kRedSlotsLB;
      r[0] = sv[0]; r[1] = sv[1]; r[2] = mv[0]; r[3] = mv[1]; r[4] = mv[2];
      double* t = J.red_tv + (size_t)c * kRedSlotsTV;
      t[0] = sv[2]; t[1] = sv[3]; t[2] = sv[4]; t[3] = sv[5];
    }
  }
}

// Weighted TV sums: w_i = |x_i - x-bar|^p; mu^_i = a_s_i u^{T+1}_K, nu^_j = b_s_j v^T_L.
__global__ __launch_bounds__(256) void k_tv_partial(const DevJob* __restrict__ jobs, int njobs,
                                                    const int* __restrict__ off, int total) {
  __shared__ double sh[256];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    const int T = (int)J.result[RS_IPF_ITERS];
    const double* un = J.ipf_u + (size_t)(T + 1) * J.Q;
    const double* v = J.ipf_v + (size_t)T * J.Q;
    const int c = it - off[jb];
    const int base = c * kChunk;
    const double h = 0.5 * (J.N - 1);
    double tm = 0.0, tn = 0.0, wm = 0.0, wn = 0.0;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int i = base + q;
      if (i >= J.P) break;
      int x0, x1, x2;
      pix_coords(i, J.N, J.d, x0, x1, x2);
      const double d0 = J.d == 2 ? 0.0 : x0 - h, d1 = x1 - h, d2 = x2 - h;
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double w = J.p == 2 ? r2 : sqrt(r2);
      const int n = J.n, k = J.k;
      const int K = J.d == 2 ? (x1 / k) * n + x2 / k : ((x0 / k) * n + x1 / k) * n + x2 / k;
      const double muh = J.a_s[i] * un[K];
      const double nuh = J.b_s[i] * v[K];
      tm += w * fabs(muh - J.mu[i]);
      tn += w * fabs(J.nu[i] - nuh);
      wm += w * J.mu[i];
      wn += w * J.nu[i];
    }
    tm = block_sum<256>(tm, sh);
    tn = block_sum<256>(tn, sh);
    wm = block_sum<256>(wm, sh);
    wn = block_sum<256>(wn, sh);
    if (threadIdx.x == 0) {
      double* r = J.red_tv + (size_t)c * kRedSlotsTV;
      r[0] = tm; r[1] = tn; r[2] = wm; r[3] = wn;
    }
  }
}

// ------------------------------------------------------------------ plan cost
//
// S_e = sum over X_K x Y_L of a_s_i b_s_j c_ij for every support entry (K, L).
//
// p = 2: with block centres c_K, offsets delta_i = x_i - c_K, eps_j = y_j - c_L
// and D = c_K - c_L, |x - y|^2 = |D + delta - eps|^2, so
//   S_e = A0 B0 |D|^2 + 2 D.(A1 B0 - A0 B1) + A2 B0 + A0 B2 - 2 A1.B1
// with the block moments (A0, A1, A2) of a_s and (B0, B1, B2) of b_s: one
// thread per entry.  p = 1: brute force, one work-group per entry, target
// block staged in LDS (value and integer coordinates).
__device__ __forceinline__ double moment_pair_sq(const double* __restrict__ A, const double* __restrict__ B,
                                                 double D0, double D1, double D2) {
  const double dd = D0 * D0 + D1 * D1 + D2 * D2;
  return A[0] * B[0] * dd
       + 2.0 * (D0 * (A[1] * B[0] - A[0] * B[1]) + D1 * (A[2] * B[0] - A[0] * B[2]) + D2 * (A[3] * B[0] - A[0] * B[3]))
       + A[4] * B[0] + A[0] * B[4]
       - 2.0 * (A[1] * B[1] + A[2] * B[2] + A[3] * B[3]);
}

__device__ __forceinline__ void block_delta(int K, int L, const DevJob& J, double& D0, double& D1, double& D2) {
  int k0, k1, k2, l0, l1, l2;
  pix_coords(K, J.n, J.d, k0, k1, k2);
  pix_coords(L, J.n, J.d, l0, l1, l2);
  D0 = (double)J.k * (k0 - l0);
  D1 = (double)J.k * (k1 - l1);
  D2 = (double)J.k * (k2 - l2);
}

__global__ __launch_bounds__(256) void k_plancost2(const DevJob* __restrict__ jobs, int njobs,
                                                   const int* __restrict__ off, int total) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    const int e = (it - off[jb]) * 256 + threadIdx.x;
    if (J.p != 2 || e >= J.nnz) continue;
    const int K = J.e_row[e], L = J.e_col[e];
    double D0, D1, D2;
    block_delta(K, L, J, D0, D1, D2);
    const double* A = J.mom_as + 5 * (size_t)K;
    const double* Bm = J.mom_bs + 5 * (size_t)L;
    J.red_pc[e] = moment_pair_sq(A, Bm, D0, D1, D2);
    // A0 B0 (|D| + 2 rho)^2 bounds the absolute values of the moment form's
    // terms (rho the largest offset of a pixel from its block centre): the
    // scale of this entry's rounding error, summed by k_finalize
    const double dn = sqrt(D0 * D0 + D1 * D1 + D2 * D2) + sqrt((double)J.d) * (double)(J.k - 1);
    J.red_pm[e] = (A[0] * Bm[0]) * (dn * dn);
  }
}

// The same entries from the pooled moments of mu and nu (k_moments) and the
// last iterates: on block K the scaling a_s = mu / u^T_K has one divisor, so
// its block moments are those of mu divided by u^T_K (and those of b_s are
// nu's divided by v^T_L); 0 where the divisor is 0, as a_s and b_s are.  The
// work-group of the coarse fitting, one thread per entry.
__device__ void coarse_plancost2(const DevJob& J, const CoarseView& C, int T) {
  const double* uT = J.ipf_u + (size_t)T * J.Q;
  const double* vT = J.ipf_v + (size_t)T * J.Q;
  const double rho2 = sqrt((double)J.d) * (double)(J.k - 1);
  for (int e = threadIdx.x; e < J.nnz; e += blockDim.x) {
    const int K = C.erow[e], L = C.ecol[e];
    double D0, D1, D2;
    block_delta(K, L, J, D0, D1, D2);
    const double uk = uT[K], vl = vT[L];
    const double* Mm = J.mom_mu + 5 * (size_t)K;
    const double* Mn = J.mom_nu + 5 * (size_t)L;
    double A[5], Bm[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      A[q] = uk > 0.0 ? Mm[q] / uk : 0.0;
      Bm[q] = vl > 0.0 ? Mn[q] / vl : 0.0;
    }
    J.red_pc[e] = moment_pair_sq(A, Bm, D0, D1, D2);
    const double dn = sqrt(D0 * D0 + D1 * D1 + D2 * D2) + rho2;
    J.red_pm[e] = (A[0] * Bm[0]) * (dn * dn);
  }
}

// sqrt(n) for an integer 0 <= n < 2^24 in float64 to a relative error below
// 2^-42: the float32 reciprocal square root r (within a few units of 2^-24)
// refined by one Newton step on y = n r, y + (r/2)(n - y^2), whose error is
// 1.5 times the square of r's.  Used for the p = 1 plan cost and gradient
// sums; the emitted upper bound's outward allowance covers it.
__device__ __forceinline__ double sqrt_int_f64(int n) {
  const double r = (double)__builtin_amdgcn_rsqf((float)n);
  const double dn = (double)n;
  const double y = dn * r;
  const double z = fma(0.5 * r, fma(-y, y, dn), y);
  return n > 0 ? z : 0.0;
}

// sum_r w[r] |x - y_r| over an LDS tile (p = 1 cost of the exact integer
// squared distance), in four interleaved partial sums so that the additions
// do not form one long dependency chain.
__device__ __forceinline__ double dist_dot(int x0, int x1, int x2, const double* w, const int (*c)[3], int tn) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int r = 0;
  auto term = [&](int q) {
    const int e0 = x0 - c[q][0], e1 = x1 - c[q][1], e2 = x2 - c[q][2];
    return w[q] * sqrt_int_f64(e0 * e0 + e1 * e1 + e2 * e2);
  };
  for (; r + 4 <= tn; r += 4) {
    s0 += term(r);
    s1 += term(r + 1);
    s2 += term(r + 2);
    s3 += term(r + 3);
  }
  for (; r < tn; ++r) s0 += term(r);
  return (s0 + s1) + (s2 + s3);
}

// p = 1 plan cost: item = (support entry e = (K, L), 64 of K's pixels); the
// work-group's partial sum of a_s_i b_s_j |x_i - y_j| goes to part1, and
// k_pc1_sum adds an entry's partials in order into red_pc[e] = S_e.
__global__ __launch_bounds__(64) void k_plancost(const DevJob* __restrict__ jobs, int njobs,
                                                 const int* __restrict__ off, int total) {
  __shared__ double sh[64];
  __shared__ double sb[1024];
  __shared__ int sc[1024][3];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (J.p == 2 || J.p1_nt) continue;   // table-path jobs: k_pc1_tab
    const int m = J.d == 2 ? J.k * J.k : J.k * J.k * J.k;
    if (m <= 32) {
      // small blocks: the wave takes 64 / g entries (g = reduce_group(m) lanes
      // each), lane a of a group holds source a and stages target a of its entry
      const int gsz = reduce_group(m), sub = threadIdx.x / gsz, a = threadIdx.x - sub * gsz;
      const int e = (it - off[jb]) * (64 / gsz) + sub;
      const bool act = e < J.nnz && a < m;
      int x0 = 0, x1 = 0, x2 = 0;
      double wa = 0.0;
      __syncthreads();
      if (act) {
        const int i = block_member(J.e_row[e], a, J.N, J.n, J.k, J.d);
        const int j = block_member(J.e_col[e], a, J.N, J.n, J.k, J.d);
        pix_coords(i, J.N, J.d, x0, x1, x2);
        wa = J.a_s[i];
        sb[threadIdx.x] = J.b_s[j];
        pix_coords(j, J.N, J.d, sc[threadIdx.x][0], sc[threadIdx.x][1], sc[threadIdx.x][2]);
      }
      __syncthreads();
      double v = act ? wa * dist_dot(x0, x1, x2, sb + sub * gsz, sc + sub * gsz, m) : 0.0;
      v = group_sum(v, gsz);
      if (a == 0 && e < J.nnz) J.part1[e] = v;   // one partial per entry
      continue;
    }
    const int pcc = (m + 63) / 64;
    const int li = it - off[jb];
    const int e = li / pcc, c = li - e * pcc;
    const int K = J.e_row[e], L = J.e_col[e];
    const int a = c * 64 + threadIdx.x;
    int x0 = 0, x1 = 0, x2 = 0;
    double wa = 0.0;
    if (a < m) {
      const int i = block_member(K, a, J.N, J.n, J.k, J.d);
      pix_coords(i, J.N, J.d, x0, x1, x2);
      wa = J.a_s[i];
    }
    double acc = 0.0;
    for (int t0 = 0; t0 < m; t0 += 1024) {
      const int tn = min(1024, m - t0);
      __syncthreads();
      for (int q = threadIdx.x; q < tn; q += 64) {
        const int j = block_member(L, t0 + q, J.N, J.n, J.k, J.d);
        sb[q] = J.b_s[j];
        pix_coords(j, J.N, J.d, sc[q][0], sc[q][1], sc[q][2]);
      }
      __syncthreads();
      if (a < m) acc += wa * dist_dot(x0, x1, x2, sb, sc, tn);
    }
    acc = block_sum<64>(acc, sh);
    if (threadIdx.x == 0) J.part1[(size_t)e * pcc + c] = acc;
  }
}

// Distance-table kernels (p = 1, blocks of m = k^d pixels with m > 32): for a
// block pair (B, O) the distance between offset u of B and offset v of O is
// |k (B - O) + u - v|, and u - v takes only (2k-1)^d values.  Each item builds
// that table in LDS (float64 square roots of exact integers), stages the
// other block's weights, and sums weight x table entry over the other block's
// pixels: the index of u - v is I(u) - I(v) + C with I linear in the offset.
__device__ __forceinline__ int p1_lin(int a, int k, int d, int w) {
  if (d == 2) { const int u1 = a / k; return u1 * w + (a - u1 * k); }
  const int u0 = a / (k * k), r = a - u0 * k * k, u1 = r / k;
  return (u0 * w + u1) * w + (r - u1 * k);
}

template <int NT>
__device__ __forceinline__ void p1_build_table(double* tab, const DevJob& J, int B, int O) {
  const int k = J.k, w = 2 * k - 1;
  int b0, b1, b2, o0, o1, o2;
  pix_coords(B, J.n, J.d, b0, b1, b2);
  pix_coords(O, J.n, J.d, o0, o1, o2);
  const int D0 = k * (b0 - o0) - (k - 1), D1 = k * (b1 - o1) - (k - 1), D2 = k * (b2 - o2) - (k - 1);
  const int size = J.d == 2 ? w * w : w * w * w;
  for (int q = threadIdx.x; q < size; q += NT) {
    int e0 = 0, r = q;
    if (J.d == 3) { e0 = q / (w * w); r = q - e0 * w * w; }
    const int e1 = r / w, e2 = r - e1 * w;
    const long long x0 = J.d == 3 ? D0 + e0 : 0, x1 = D1 + e1, x2 = D2 + e2;
    const long long r2 = x0 * x0 + x1 * x1 + x2 * x2;
    // the refined float32 root (relative error below 2^-42, inside the upper
    // bound's allowance) where the squared distance fits its range
    tab[q] = r2 < (1ll << 24) ? sqrt_int_f64((int)r2) : sqrt((double)r2);
  }
}

// sum over the other block's pixels v of wv[v] tab[I(u) - I(v) + C], v in C order
__device__ __forceinline__ double p1_table_dot(const double* tab, const double* wv, int Iu, int k, int d, int w) {
  const int C = (k - 1) * (d == 2 ? w + 1 : w * w + w + 1);
  double s0 = 0.0, s1 = 0.0;
  int t = 0;
  const int n0 = d == 2 ? 1 : k;
  for (int v0 = 0; v0 < n0; ++v0) {
    for (int v1 = 0; v1 < k; ++v1) {
      const double* trow = tab + (Iu + C - (v0 * w + v1) * w);
      int v2 = 0;
      for (; v2 + 2 <= k; v2 += 2, t += 2) {
        s0 += wv[t] * trow[-v2];
        s1 += wv[t + 1] * trow[-v2 - 1];
      }
      for (; v2 < k; ++v2, ++t) s0 += wv[t] * trow[-v2];
    }
  }
  return s0 + s1;
}

// The same sum with k and d known at compile time: fully unrolled, every LDS
// read at an immediate offset from one base, four partial sums.
template <int KT, int DT>
__device__ __forceinline__ double p1_table_dot_fixed(const double* tab, const double* wv, int Iu) {
  constexpr int w = 2 * KT - 1;
  constexpr int C = (KT - 1) * (DT == 2 ? w + 1 : w * w + w + 1);
  const double* base = tab + (Iu + C);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int v0 = 0; v0 < (DT == 2 ? 1 : KT); ++v0)
#pragma unroll
    for (int v1 = 0; v1 < KT; ++v1)
#pragma unroll
      for (int v2 = 0; v2 < KT; ++v2) {
        const int t = (v0 * KT + v1) * KT + v2;
        acc[t & 3] += wv[t] * base[-((v0 * w + v1) * w + v2)];
      }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

__device__ __forceinline__ double p1_dot_any(const double* tab, const double* wv, int Iu, int k, int d, int w) {
  if (d == 3 && k == 8) return p1_table_dot_fixed<8, 3>(tab, wv, Iu);
  if (d == 3 && k == 4) return p1_table_dot_fixed<4, 3>(tab, wv, Iu);
  if (d == 2 && k == 8) return p1_table_dot_fixed<8, 2>(tab, wv, Iu);
  if (d == 2 && k == 16) return p1_table_dot_fixed<16, 2>(tab, wv, Iu);
  return p1_table_dot(tab, wv, Iu, k, d, w);
}

// p = 1 plan cost, table path: item = (support entry e = (K, L), NT pixels of
// K); the work-group's partial sum goes to part1 slot e * ceil(m/64) +
// (NT/64) c, the other slots of its range get 0, and k_pc1_sum adds an
// entry's slots in order.
// LDS per table kernel: NT = 64 serves blocks of at most 64 pixels (2D k <= 8,
// 3D k <= 4: tables of at most 15^2 and 7^3 entries), NT = 256 the rest.
template <int NT> struct P1Lds {
  static constexpr int tab = NT == 64 ? 512 : 4096;
  static constexpr int blk = NT == 64 ? 64 : 1024;
};

template <int NT>
__global__ __launch_bounds__(NT) void k_pc1_tab(const DevJob* __restrict__ jobs, int njobs,
                                                const int* __restrict__ off, int total) {
  __shared__ double tab[P1Lds<NT>::tab];
  __shared__ double sb[P1Lds<NT>::blk];
  __shared__ double sh[NT];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (J.p == 2 || J.p1_nt != NT) continue;
    const int k = J.k, w = 2 * k - 1;
    const int m = J.d == 2 ? k * k : k * k * k;
    const int nch = (m + NT - 1) / NT, pcc = (m + 63) / 64;
    const int li = it - off[jb];
    const int e = li / nch, c = li - e * nch;
    const int K = J.e_row[e], L = J.e_col[e];
    __syncthreads();
    p1_build_table<NT>(tab, J, K, L);
    for (int t = threadIdx.x; t < m; t += NT) sb[t] = J.b_s[block_member(L, t, J.N, J.n, J.k, J.d)];
    __syncthreads();
    const int a = c * NT + threadIdx.x;
    double v = 0.0;
    if (a < m) v = J.a_s[block_member(K, a, J.N, J.n, J.k, J.d)] * p1_dot_any(tab, sb, p1_lin(a, k, J.d, w), k, J.d, w);
    v = block_sum<NT>(v, sh);
    const int s0 = c * (NT / 64);
    if ((int)threadIdx.x < NT / 64 && s0 + (int)threadIdx.x < pcc)
      J.part1[(size_t)e * pcc + s0 + threadIdx.x] = threadIdx.x == 0 ? v : 0.0;
  }
}

// p = 1 upper-bound gradient, table path: item = (support entry e, NT pixels
// of the entry's block on this side); part1 layout as in k_ub_grad.
template <int NT>
__global__ __launch_bounds__(NT) void k_ubg_tab(const DevJob* __restrict__ jobs, int njobs,
                                                const int* __restrict__ off, int total, int side) {
  __shared__ double tab[P1Lds<NT>::tab];
  __shared__ double sb[P1Lds<NT>::blk];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    double* grad = side == 0 ? J.grad_a : J.grad_b;
    if (!grad || J.p == 2 || J.p1_nt != NT) continue;
    const int k = J.k, w = 2 * k - 1;
    const int m = J.d == 2 ? k * k : k * k * k;
    const int nch = (m + NT - 1) / NT, per = (m + 63) / 64;
    const int li = it - off[jb];
    const int e = li / nch, c = li - e * nch;
    const int B = side == 0 ? J.e_row[e] : J.e_col[e];
    const int O = side == 0 ? J.e_col[e] : J.e_row[e];
    const double* other = side == 0 ? J.nu : J.mu;
    __syncthreads();
    p1_build_table<NT>(tab, J, B, O);
    for (int t = threadIdx.x; t < m; t += NT) sb[t] = other[block_member(O, t, J.N, J.n, J.k, J.d)];
    __syncthreads();
    const int a = c * NT + threadIdx.x;
    if (a < m) J.part1[(size_t)e * per * 64 + a] = J.coef[e] * p1_dot_any(tab, sb, p1_lin(a, k, J.d, w), k, J.d, w);
  }
}

// S_e of every p = 1 entry: its partials added in order (one work-group per job).
__global__ __launch_bounds__(256) void k_pc1_sum(const DevJob* __restrict__ jobs) {
  const DevJob& J = jobs[blockIdx.x];
  if (J.p == 2) return;
  const int m = J.d == 2 ? J.k * J.k : J.k * J.k * J.k;
  const int pcc = (m + 63) / 64;
  for (int e = threadIdx.x; e < J.nnz; e += 256) {
    double s = 0.0;
    for (int c = 0; c < pcc; ++c) s += J.part1[(size_t)e * pcc + c];
    J.red_pc[e] = s;
  }
}

// ------------------------------------------------------------------ finalize

// Additions on the longest path of a pooled block sum in k_moments (the
// accumulators start at zero, so the first term adds exactly): k <= 64, a
// thread's share of a column (ceil(rows / RG) terms), the RG row groups, the
// block's k columns; k > 64, every g-th pixel in a lane, then the butterfly.
__device__ __forceinline__ int pool_depth(const DevJob& J) {
  const int k = J.k;
  if (k <= 64) {
    const int W = (256 / k) * k, Wc = min(W, J.N), RG = 256 / Wc;
    const int nrows = J.d == 2 ? k : k * k;
    return (nrows + RG - 1) / RG - 1 + (RG - 1) + (k - 1);
  }
  const int m = J.d == 2 ? k * k : k * k * k;
  const int g = reduce_group(m);
  int lg = 0;
  while ((1 << lg) < g) ++lg;
  return (m + g - 1) / g - 1 + lg;
}

// gamma(n) = n u / (1 - n u), u = 2^-53: a float64 evaluation n roundings deep
// (a sum of nonnegative terms along any tree of that height, a chain of
// products and quotients) is within a relative gamma(n) of its exact value.
__device__ __forceinline__ double gam(double n) {
  const double t = n * 1.1102230246251565e-16;
  return t / (1.0 - t);
}

// Outward allowances of the emitted upper bound.  The lemma on the triangle
// inequality upper bound holds for the coupling the kernels formed, diag(a_s)
// pi^ diag(b_s) with the float64 scalings as computed, so the emitted value must
// dominate that coupling's exact plan cost and the exact weighted TV of its
// exact marginals; it also dominates the exact-arithmetic value of Algorithm 4
// on the same inputs and any float64 evaluation of it whose sums stay within
// about one rounding of exact (such an evaluation's fitted marginals carry at
// most 14 T u of relative error after T iterations).  With r, c the longest
// row and column of the coarse coupling and s_p the depth of the pooled block
// sums, each fitting step of the coarse iteration (row sum, pooled-mass
// quotient, column sum, pooled-mass quotient) adds at most
//   D = gamma(r+1) + gamma(c+1) + 2 gamma(s_p) + 4u
// of relative error to the iterates against exact arithmetic, starting from
// gamma(r+1) + u, so the fitted mu^ = a_s (pi^ b_s) is within
//   e_G = 2 (gamma(r+1) + u) + (2T - 1) D + 2u
// of the exact iterate's, and within gamma(r+1) + gamma(s_p) + 4u <= e_G of the
// exact marginal of the formed coupling; nu^ is within
//   e_nu = gamma(c+1) + gamma(s_p) + 4u
// of nu on both counts (the column update fits nu exactly in exact
// arithmetic).  A weighted TV sum T computed over pixels n_s additions deep
// then satisfies T_exact <= Z + e (W + Z) / (1 - e_G), with Z = T (1 +
// gamma(n_s + 3)), W = <w, mu> (1 + gamma(n_s + 2)) and e = e_G + 14 T u (resp.
// e_nu).  The plan cost: p = 2 sums block moments, each entry within
// (2 gamma(s_m + 4) + gamma(16)) M_e of exact, M_e = A0 B0 (|D_KL| + 2 rho)^2
// bounding the absolute values of its terms (rho the largest offset of a pixel
// from its block centre) and s_m = max(k^d, s_p): a moment of the scalings is
// a pooled moment of the measure (at most s_p + 2 roundings deep, the offset
// products included) divided by u^T_K (one more), against the sum of the
// scalings as rounded (one more), or the same moments summed from the scalings
// themselves; p = 1 sums nonnegative terms (gamma(k^2d + nnz + 8) plus 2^-41
// for the refined square roots).  Both are then widened by the scalings'
// e_G + 14 T u.
// One job's bounds by a 256-thread work-group (sh: 256 doubles of LDS).
__device__ void finalize_job(const DevJob& J, double* sh) {
  double* res = J.result;
  // the pixel chunks' partials of the lower bound (sums and maxima) and of
  // the TV terms, one loop so that both rows' loads are in flight together
  double sf = 0, sg = 0, mh = 0, mg = 0, mf = 0;
  double tm = 0, tn = 0, wm = 0, wn = 0;
  for (int c = threadIdx.x; c < J.chunks; c += 256) {
    const double* r = J.red_lb + (size_t)c * kRedSlotsLB;
    const double* t = J.red_tv + (size_t)c * kRedSlotsTV;
    sf += r[0]; sg += r[1];
    mh = fmax(mh, r[2]); mg = fmax(mg, r[3]); mf = fmax(mf, r[4]);
    tm += t[0]; tn += t[1]; wm += t[2]; wn += t[3];
  }
  // upper bound
  const int kdi = J.d == 2 ? J.k * J.k : J.k * J.k * J.k;
  const double kd = (double)kdi;
  const double cc = 1.0 / (kd * kd);
  double pc = 0, mm = 0;
  // eight of a thread's entries at a time, all their loads issued before the
  // first is used (the sums keep their order: entry e, e + 256, ...)
  {
    const int nnz = J.nnz;
    const double* ev = J.e_val;
    const double* rp = J.red_pc;
    const double* rm = J.p == 2 ? J.red_pm : J.red_pc;
    for (int e0 = threadIdx.x; e0 < nnz; e0 += 256 * 8) {
      double a[8], b[8], c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = min(e0 + 256 * u, nnz - 1);
        a[u] = ev[e];
        b[u] = rp[e];
        c[u] = rm[e];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (e0 + 256 * u < nnz) {
          const double ce = cc * a[u];
          pc += ce * b[u];
          if (J.p == 2) mm += ce * c[u];
        }
      }
    }
  }
  const double rmax = (double)J.row_max, cmax = (double)J.col_max;
  // all sums and maxima in one work-group reduction
  {
    double sv[8] = {sf, sg, pc, tm, tn, wm, wn, mm};
    double mv[3] = {mh, mg, mf};
    block_reduce_many<8, 3>(sv, mv, sh);
    sf = sv[0]; sg = sv[1]; pc = sv[2]; tm = sv[3]; tn = sv[4]; wm = sv[5]; wn = sv[6]; mm = sv[7];
    mh = mv[0]; mg = mv[1]; mf = mv[2];
  }
  if (threadIdx.x != 0) return;
  // float32 feasibility shift (first order in u = 2^-24; see the oracle's derivation)
  const double u = 5.9604644775390625e-08;
  const double up = J.p == 1 ? u : 0.0;
  const double F = mh * (1.0 + 2.0 * u);
  double e_g, e_f;
  if (J.sep) {
    // separable evaluation: one rounding per axis of partial values <= |g| + d (N-1)^2
    const double Cm = (double)J.d * (J.N - 1) * (J.N - 1);
    e_g = u * (F + J.d * mg + (J.d - 1) * Cm);
    e_f = u * (J.d * mf + (J.d - 1) * Cm) + e_g;
  } else {
    e_g = (u + up) * (mg + F);
    e_f = u * mf + up * (mf + mg) + e_g;
  }
  const double shift = (e_f + e_g) * (1.0 + 0.0009765625) + 2.220446049250313e-16 * J.P * (mf + mg);
  const double S32 = sf + sg;
  const double Se = S32 - shift;
  unsigned warn = (unsigned)res[RS_WARN];
  double lower = 0.0;
  if (Se > 0.0) lower = J.p == 2 ? sqrt(Se) : Se;
  else warn |= QBW_WARN_LB_CLIPPED;
  // upper bound with the outward allowances derived above
  const double u53 = 1.1102230246251565e-16;
  const double T = fmax(1.0, res[RS_IPF_ITERS]);
  const double s_pool = (double)pool_depth(J);
  const double n_s = 4 + 6 + 3 + (J.chunks + 255) / 256 + 9;   // pixel sums: thread, wave, work-group, chunks
  const double n_e = (J.nnz + 255) / 256 + 9;                   // entry sums
  const double a1 = gam(rmax + 1) + u53;
  const double Dg = gam(rmax + 1) + gam(cmax + 1) + 2.0 * gam(s_pool) + 4.0 * u53;
  const double eG = 2.0 * a1 + (2.0 * T - 1.0) * Dg + 2.0 * u53;
  const double eO = 14.0 * T * u53;
  const double emu = (eG + eO) * (1.0 + 0x1p-40);
  const double enu = (gam(cmax + 1) + gam(s_pool) + 4.0 * u53) * (1.0 + 0x1p-40);
  const double Zm = tm * (1.0 + gam(n_s + 3)), Zn = tn * (1.0 + gam(n_s + 3));
  const double Wm = wm * (1.0 + gam(n_s + 2)), Wn = wn * (1.0 + gam(n_s + 2));
  const double Tm = (Zm + emu * (Wm + Zm) / (1.0 - eG)) * (1.0 + 8.0 * u53);
  const double Tn = (Zn + enu * (Wn + Zn) / (1.0 - enu)) * (1.0 + 8.0 * u53);
  double Pv;
  if (J.p == 2)
    Pv = pc + (2.0 * gam(fmax(kd, s_pool) + 4) + gam(16) + 2.0 * gam(n_e + 4)) * mm * (1.0 + gam(n_e + 10));
  else
    Pv = pc * (1.0 + gam(kd * kd + J.nnz + 8) + 0x1p-41);
  const double pe = Pv * (1.0 + eG + eO + 6.0 * u53) * (1.0 + 4.0 * u53);
  const double c1 = J.p == 2 ? 1.4142135623730951 : 1.0;   // RN(sqrt 2) > sqrt 2
  auto root = [&](double x) { return J.p == 2 ? sqrt(x) : x; };
  const double tvm = c1 * root(Tm) * (1.0 + 2.0 * u53);
  const double tvn = c1 * root(Tn) * (1.0 + 2.0 * u53);
  const double upper = (root(pe) * (1.0 + u53) + tvm + tvn) * (1.0 + 2.0 * u53);
  res[RS_LOWER] = lower;
  res[RS_UPPER] = upper;
  res[RS_LOWER_S] = Se;
  res[RS_SHIFT] = shift;
  res[RS_UPPER_COST] = pe;
  res[RS_TV_MU] = tvm;
  res[RS_TV_NU] = tvn;
  res[RS_COARSE_OBJ] = J.coarse_obj;
  res[RS_WARN] = (double)warn;
  res[RS_S32] = S32;
  res[RS_PCOST_RAW] = pc;
  res[RS_MAX_FHAT] = mh;
  res[RS_MAX_G] = mg;
  res[RS_MAX_F] = mf;
  res[RS_TVSUM_MU] = tm;
  res[RS_TVSUM_NU] = tn;
  res[RS_MW_MU] = wm;
  res[RS_MW_NU] = wn;
  res[RS_TV_RAW_MU] = c1 * root(tm);
  res[RS_TV_RAW_NU] = c1 * root(tn);
}

// The bounds of every job, one work-group per job.
__global__ __launch_bounds__(256) void k_finalize(const DevJob* __restrict__ jobs, int njobs) {
  __shared__ double sh[256];
  finalize_job(jobs[blockIdx.x], sh);
}

// ------------------------------------------------------------------ C-bar (Section 3.2)
//
// p = 2: with block centres c_K and offsets delta = x - c_K the block-pair sum
// of |x - y|^2 mu(x) nu(y) expands into pooled moments (mass, first moment,
// second moment); p = 1: brute force over the k^(2d) pixel pairs.
__global__ __launch_bounds__(256) void k_cbar(const DevJob* __restrict__ jobs, int njobs,
                                              const int* __restrict__ off, int total,
                                              double* const* __restrict__ outs) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    const long long pr = (long long)(it - off[jb]) * 256 + threadIdx.x;
    const int Q = J.Q;
    if (pr >= (long long)Q * Q) continue;
    const int K = (int)(pr / Q), L = (int)(pr - (long long)K * Q);
    double D0, D1, D2;
    block_delta(K, L, J, D0, D1, D2);
    const double dc2 = D0 * D0 + D1 * D1 + D2 * D2;
    const double mK = J.mu_t[K], nL = J.nu_t[L];
    double val;
    if (J.p == 2) {
      if (mK > 0.0 && nL > 0.0) {
        val = moment_pair_sq(J.mom_mu + 5 * (size_t)K, J.mom_nu + 5 * (size_t)L, D0, D1, D2) / (mK * nL);
      } else {
        val = dc2;
      }
    } else {
      if (mK > 0.0 && nL > 0.0) {
        const int m = J.d == 2 ? J.k * J.k : J.k * J.k * J.k;
        double s = 0.0;
        for (int a = 0; a < m; ++a) {
          const int i = block_member(K, a, J.N, J.n, J.k, J.d);
          const double x = J.mu[i];
          if (x == 0.0) continue;
          double r = 0.0;
          for (int b = 0; b < m; ++b) {
            const int j = block_member(L, b, J.N, J.n, J.k, J.d);
            r += J.nu[j] * cost64(i, j, J.N, J.d, 1);
          }
          s += x * r;
        }
        val = s / (mK * nL);
      } else {
        val = sqrt(dc2);
      }
    }
    outs[jb][(size_t)K * Q + L] = val;
  }
}

// Block moments about the block centre (5 slots): which = 0 -> (mu, nu) into
// (mom_mu, mom_nu); which = 1 -> (a_s, b_s) into (mom_as, mom_bs); which = 2
// -> as 0, and also the pooled masses (SumPool: the block sums, slot 0) into
// (mu_t, nu_t) and the input checks (negative entry, NaN) into the job's flags;
// which = 3 -> as 2, and for k <= 64 also f^ on the strip's pixels (the
// upscaled coarse potential, which depends on neither measure).
//
// k <= 64: one work-group per strip of blocks along the last axis (the k or
// k^2 pixel rows of one block row), both fields.  The strip goes in chunks of
// W = k floor(256 / k) columns (whole blocks); a chunk's Wc columns each get
// 256 / Wc threads that split the strip's rows, every thread sums its share
// of a column (coalesced row reads), and each block's k columns and their
// row shares are then added in a fixed order from LDS.  k > 64: one lane group per
// (side, block), g lanes summing every g-th pixel, then a butterfly (block
// rows are then long enough to coalesce).  pool_depth gives the additions a
// block sum takes.
__global__ __launch_bounds__(256) void k_moments(const DevJob* __restrict__ jobs, int njobs,
                                                 const int* __restrict__ off, int total, int which) {
  __shared__ double cs[10][256];   // five column sums per side
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (J.k <= 64) {
      const int k = J.k, N = J.N, n = J.n;
      const int strip = it - off[jb];
      const int b0 = J.d == 2 ? 0 : strip / n, b1 = J.d == 2 ? strip : strip - (strip / n) * n;
      const int W = (256 / k) * k;            // columns per chunk (whole blocks)
      const int Wc = min(W, N);               // columns present in a chunk
      const int RG = 256 / Wc;                // row groups: threads t, t + Wc, ... share a column
      const int col = (int)threadIdx.x % Wc, rg = (int)threadIdx.x / Wc;
      const int nrows = J.d == 2 ? k : k * k;
      const double h = 0.5 * (k - 1);
      // both fields in one sweep (each with its own sums, in the same order
      // as a sweep of its own)
      const double* ma = which != 1 ? J.mu : J.a_s;
      const double* mb = which != 1 ? J.nu : J.b_s;
      double* moa = which != 1 ? J.mom_mu : J.mom_as;
      double* mob = which != 1 ? J.mom_nu : J.mom_bs;
      for (int c0 = 0; c0 < N; c0 += W) {
        const int x2 = c0 + col;
        double sa0 = 0.0, sa1 = 0.0, sa2 = 0.0, sa4 = 0.0;
        double sb0 = 0.0, sb1 = 0.0, sb2 = 0.0, sb4 = 0.0;
        int bad = 0;
        if (rg < RG && x2 < N) {
#pragma unroll 4
          for (int r = rg; r < nrows; r += RG) {
            const int u0 = J.d == 2 ? 0 : r / k, u1 = J.d == 2 ? r : r - (r / k) * k;
            const size_t row = J.d == 2 ? (size_t)(b1 * k + u1)
                                        : ((size_t)(b0 * k + u0) * N + (size_t)(b1 * k + u1));
            const double wa = ma[row * N + x2], wb = mb[row * N + x2];
            bad |= (wa < 0.0 ? 1 : 0) | (wa != wa ? 2 : 0) | (wb < 0.0 ? 1 : 0) | (wb != wb ? 2 : 0);
            const double d0 = J.d == 2 ? 0.0 : u0 - h, d1 = u1 - h;
            sa0 += wa;
            sa1 += wa * d0;
            sa2 += wa * d1;
            sa4 += wa * (d0 * d0 + d1 * d1);
            sb0 += wb;
            sb1 += wb * d0;
            sb2 += wb * d1;
            sb4 += wb * (d0 * d0 + d1 * d1);
          }
        }
        if (bad && which >= 2) atomicOr(J.flags, bad);
        const double d2 = (double)(x2 % k) - h;
        __syncthreads();
        cs[0][threadIdx.x] = sa0;
        cs[1][threadIdx.x] = sa1;
        cs[2][threadIdx.x] = sa2;
        cs[3][threadIdx.x] = sa0 * d2;
        cs[4][threadIdx.x] = sa4 + sa0 * (d2 * d2);
        cs[5][threadIdx.x] = sb0;
        cs[6][threadIdx.x] = sb1;
        cs[7][threadIdx.x] = sb2;
        cs[8][threadIdx.x] = sb0 * d2;
        cs[9][threadIdx.x] = sb4 + sb0 * (d2 * d2);
        __syncthreads();
        // column totals over the row groups (in place, in group order) ...
        if (RG > 1 && (int)threadIdx.x < Wc) {
#pragma unroll
          for (int q = 0; q < 10; ++q) {
            double v = cs[q][threadIdx.x];
            for (int g = 1; g < RG; ++g) v += cs[q][g * Wc + threadIdx.x];
            cs[q][threadIdx.x] = v;
          }
        }
        __syncthreads();
        // ... then each (side, block, moment) adds its k columns in order
        const int nb = min(W, N - c0) / k;   // whole blocks in this chunk
        for (int id = threadIdx.x; id < 10 * nb; id += 256) {
          const int side = id >= 5 * nb ? 1 : 0;
          const int rest = id - side * 5 * nb;
          const int bq = rest / 5, q = rest - bq * 5;
          const int K2 = c0 / k + bq;
          const int K = J.d == 2 ? b1 * n + K2 : (b0 * n + b1) * n + K2;
          double v = 0.0;
          for (int c = 0; c < k; ++c) v += cs[side * 5 + q][bq * k + c];
          (side ? mob : moa)[5 * (size_t)K + q] = v;
          if (q == 0 && which >= 2) (side ? J.nu_t : J.mu_t)[K] = v;
        }
      }
      if (which == 3) {
        // f^ of the strip's pixels, each by the thread that read them above
        for (int c0 = 0; c0 < N; c0 += W) {
          const int x2 = c0 + col;
          if (rg >= RG || x2 >= N) continue;
          if (J.interp == 0 && J.d == 2) {
            // bilinear: a 2D strip's rows lie between the coarse rows b1 - 1
            // and b1 + 1, so the three interpolations along x_2 are formed
            // once (the same operations as upscale_value's), then each
            // pixel's along x_1
            const double* __restrict__ F = J.ftil;
            int B0, B1;
            double wb;
            axis_weight(x2, k, n, B0, B1, wb);
            const int a0 = max(b1 - 1, 0);
            double rr[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              const int a = min(a0 + q, n - 1);
              rr[q] = lerp_nc(F[a * n + B0], F[a * n + B1], wb);
            }
            for (int r = rg; r < nrows; r += RG) {
              const int X1 = b1 * k + r;
              int A0, A1;
              double wa;
              axis_weight(X1, k, n, A0, A1, wa);
              const double v0 = A0 - a0 == 0 ? rr[0] : rr[1];
              const double v1 = A1 - a0 == 1 ? rr[1] : (A1 - a0 == 2 ? rr[2] : rr[0]);
              J.fhat[(size_t)X1 * N + x2] = (float)lerp_nc(v0, v1, wa);
            }
            continue;
          }
          for (int r = rg; r < nrows; r += RG) {
            const int u0 = J.d == 2 ? 0 : r / k, u1 = J.d == 2 ? r : r - (r / k) * k;
            const int X0 = J.d == 2 ? 0 : b0 * k + u0, X1 = b1 * k + u1;
            const size_t row = J.d == 2 ? (size_t)X1 : ((size_t)X0 * N + (size_t)X1);
            J.fhat[row * N + x2] = upscale_value(J, X0, X1, x2);
          }
        }
      }
      continue;
    }
    // k > 64: (side, block) pairs reduced by lane groups as in k_pool
    const int mm = J.d == 2 ? J.k * J.k : J.k * J.k * J.k;
    const int g = reduce_group(mm);
    const int idx = ((it - off[jb]) * 4 + wv) * (64 / g) + lane / g;
    const int sub = lane & (g - 1);
    const bool ok = idx < 2 * J.Q;
    const int side = ok ? idx / J.Q : 0, K = ok ? idx - side * J.Q : 0;
    const double* m = which != 1 ? (side == 0 ? J.mu : J.nu) : (side == 0 ? J.a_s : J.b_s);
    const double h = 0.5 * (J.k - 1);
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    int bad = 0;
    if (ok) {
      for (int a = sub; a < mm; a += g) {
        const int i = block_member(K, a, J.N, J.n, J.k, J.d);
        int u0, u1, u2;
        pix_coords(a, J.k, J.d, u0, u1, u2);
        const double d0 = J.d == 2 ? 0.0 : u0 - h, d1 = u1 - h, d2 = u2 - h;
        const double w = m[i];
        bad |= (w < 0.0 ? 1 : 0) | (w != w ? 2 : 0);
        s0 += w;
        s1 += w * d0; s2 += w * d1; s3 += w * d2;
        s4 += w * (d0 * d0 + d1 * d1 + d2 * d2);
      }
    }
    s0 = group_sum(s0, g); s1 = group_sum(s1, g); s2 = group_sum(s2, g);
    s3 = group_sum(s3, g); s4 = group_sum(s4, g);
    if (bad && which >= 2) atomicOr(J.flags, bad);
    if (ok && sub == 0) {
      double* o = (which != 1 ? (side == 0 ? J.mom_mu : J.mom_nu) : (side == 0 ? J.mom_as : J.mom_bs)) + 5 * (size_t)K;
      o[0] = s0; o[1] = s1; o[2] = s2; o[3] = s3; o[4] = s4;
      if (which >= 2) (side == 0 ? J.mu_t : J.nu_t)[K] = s0;
    }
  }
}

// ------------------------------------------------------------------ backward

__global__ __launch_bounds__(256) void k_lb_grad(const DevJob* __restrict__ jobs, int njobs,
                                                 const int* __restrict__ off, int total,
                                                 const double* __restrict__ dl) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (!J.grad_a || !J.grad_b || J.p == 2) continue;   // p = 2: k_grad2
    const double Se = J.result[RS_LOWER_S];
    const double s = Se > 0.0 ? (J.p == 2 ? 0.5 / sqrt(Se) : 1.0) * dl[jb] : 0.0;
    const int base = (it - off[jb]) * kChunk;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int i = base + q;
      if (i >= J.P) break;
      J.grad_a[i] += s * (double)J.f[i];
      J.grad_b[i] += s * (double)J.g[i];
    }
  }
}

// Reverse mode through the coarse IPF recurrence (one work-group per job).
// Produces d P / d mu~ (gbar_mu), d P / d nu~ (gbar_nu) and, per support
// entry, coef_e = k^(-2d) pi~_e / (u^T_K v^T_L), the weight of
// S_e = sum mu_i nu_j c_ij in P.
// Quadratic coefficients of the direct upper-bound gradient term for p = 2
// at block K: both sides' h(x) = A |z|^2 + B.z + C, z = x - centre of K, from
// the other side's block moments and the entries' coefficients.
__device__ void grad2_quad_block(const DevJob& J, const CoarseView& C, int K) {
  const int n = J.n;
  int k0, k1, k2;
  pix_coords(K, n, J.d, k0, k1, k2);
  for (int side = 0; side < 2; ++side) {
    const double* omom = side == 0 ? J.mom_nu : J.mom_mu;
    const int e0 = side == 0 ? C.csr[K] : C.csc[K];
    const int e1 = side == 0 ? C.csr[K + 1] : C.csc[K + 1];
    double A = 0.0, B0 = 0.0, B1 = 0.0, B2 = 0.0, Cc = 0.0;
    for (int q = e0; q < e1; ++q) {
      const int e = side == 0 ? q : C.cidx[q];
      const int O = side == 0 ? C.ecol[e] : C.erow[e];
      int o0, o1, o2;
      pix_coords(O, n, J.d, o0, o1, o2);
      const double D0 = J.d == 2 ? 0.0 : (double)(J.k * (k0 - o0));
      const double D1 = (double)(J.k * (k1 - o1)), D2 = (double)(J.k * (k2 - o2));
      const double* W = omom + 5 * (size_t)O;
      const double cf = J.coef[e];
      A += cf * W[0];
      B0 += cf * (2.0 * W[0] * D0 - 2.0 * W[1]);
      B1 += cf * (2.0 * W[0] * D1 - 2.0 * W[2]);
      B2 += cf * (2.0 * W[0] * D2 - 2.0 * W[3]);
      Cc += cf * (W[0] * (D0 * D0 + D1 * D1 + D2 * D2) - 2.0 * (D0 * W[1] + D1 * W[2] + D2 * W[3]) + W[4]);
    }
    double* o = J.gquad + (size_t)10 * K + 5 * side;
    o[0] = A; o[1] = B0; o[2] = B1; o[3] = B2; o[4] = Cc;
  }
}

// The reverse pass of one job, by its work-group: the four adjoint vectors
// live in sc (LDS or the job's global scratch).
__device__ void coarse_reverse(const DevJob& J, const CoarseView& C, double* sc) {
  const int Q = J.Q;
  const int T = (int)J.result[RS_IPF_ITERS];
  const double kd = J.d == 2 ? (double)J.k * J.k : (double)J.k * J.k * J.k;
  const double cc = 1.0 / (kd * kd);
  double* ub = sc;          // adjoint of u^t
  double* vb = sc + Q;      // adjoint of v^t
  double* Ab = sc + 2 * Q;  // adjoint of A^t
  double* Bb = sc + 3 * Q;  // adjoint of B^{t-1}
  const double* uT = J.ipf_u + (size_t)T * Q;
  const double* vT = J.ipf_v + (size_t)T * Q;
  for (int e = threadIdx.x; e < J.nnz; e += blockDim.x) {
    const int K = C.erow[e], L = C.ecol[e];
    J.coef[e] = (uT[K] > 0.0 && vT[L] > 0.0) ? cc * C.ev[e] / (uT[K] * vT[L]) : 0.0;
  }
  for (int K = threadIdx.x; K < Q; K += blockDim.x) { J.gbar_mu[K] = 0.0; J.gbar_nu[K] = 0.0; }
  __syncthreads();
  // p = 2: the direct term's per-block quadratic (needs the coefficients above)
  if (J.p == 2)
    for (int K = threadIdx.x; K < Q; K += blockDim.x) grad2_quad_block(J, C, K);
  // direct terms: P = sum_e cc val_e red_pc[e], red_pc = S_e / (u_K v_L)
  for (int K = threadIdx.x; K < Q; K += blockDim.x) {
    double s = 0.0;
    for (int e = C.csr[K]; e < C.csr[K + 1]; ++e) s += cc * C.ev[e] * J.red_pc[e];
    ub[K] = uT[K] > 0.0 ? -s / uT[K] : 0.0;
  }
  for (int L = threadIdx.x; L < Q; L += blockDim.x) {
    double s = 0.0;
    for (int q = C.csc[L]; q < C.csc[L + 1]; ++q) {
      const int e = C.cidx[q];
      s += cc * C.ev[e] * J.red_pc[e];
    }
    vb[L] = vT[L] > 0.0 ? -s / vT[L] : 0.0;
  }
  __syncthreads();
  for (int t = T; t >= 1; --t) {
    const double* u = J.ipf_u + (size_t)t * Q;
    // v^t = cc pi^T A^t  ->  Ab
    for (int K = threadIdx.x; K < Q; K += blockDim.x) {
      double s = 0.0;
      for (int e = C.csr[K]; e < C.csr[K + 1]; ++e) s += C.ev[e] * vb[C.ecol[e]];
      Ab[K] = cc * s;
    }
    __syncthreads();
    // A^t = mu~ / u^t
    for (int K = threadIdx.x; K < Q; K += blockDim.x) {
      if (u[K] > 0.0) {
        J.gbar_mu[K] += Ab[K] / u[K];
        ub[K] += -Ab[K] * J.mu_t[K] / (u[K] * u[K]);
      }
    }
    __syncthreads();
    if (t == 1) break;
    const double* vp = J.ipf_v + (size_t)(t - 1) * Q;
    // u^t = cc pi B^{t-1}  ->  Bb
    for (int L = threadIdx.x; L < Q; L += blockDim.x) {
      double s = 0.0;
      for (int q = C.csc[L]; q < C.csc[L + 1]; ++q) {
        const int e = C.cidx[q];
        s += C.ev[e] * ub[C.erow[e]];
      }
      Bb[L] = cc * s;
    }
    __syncthreads();
    // B^{t-1} = nu~ / v^{t-1}
    for (int L = threadIdx.x; L < Q; L += blockDim.x) {
      if (vp[L] > 0.0) {
        J.gbar_nu[L] += Bb[L] / vp[L];
        vb[L] = -Bb[L] * J.nu_t[L] / (vp[L] * vp[L]);
      } else {
        vb[L] = 0.0;
      }
    }
    for (int K = threadIdx.x; K < Q; K += blockDim.x) ub[K] = 0.0;
    __syncthreads();
  }
}

// The reverse pass as a launch of its own (one work-group per job), for jobs
// whose forward did not run it: with skip_p2, p = 2 jobs are left alone (their
// forward coarse kernel ran it).
__global__ __launch_bounds__(1024) void k_ub_coarse_bwd(const DevJob* __restrict__ jobs, int njobs,
                                                        double* __restrict__ scratch_all,
                                                        int stride, size_t lds_bytes, int skip_p2) {
  extern __shared__ double lds[];
  const DevJob& J = jobs[blockIdx.x];
  if (skip_p2 && J.p == 2) return;
  const CoarseView C = coarse_view(J, lds, lds_bytes, 4);
  coarse_reverse(J, C, C.in_lds ? C.vec : scratch_all + (size_t)blockIdx.x * 4 * stride);  // stride >= every job's Q
}

// d upper / d mu (side 0) or d nu (side 1).  For a member x of block B the
// direct term is
//   h(x) = sum over entries e of B's row (column) of coef_e sum_{y in O_e} w(y) c(x, y)
// with w = nu (side 0) or mu (side 1) and O_e the other block of the entry.
// k_ub_grad (p = 1) sums it y by y through LDS tiles, one 64-thread
// work-group per (support entry, 64 pixels of the block), each entry's share
// kept apart; k_ub_grad_sum adds a pixel's shares in a fixed order.
// For p = 2 the direct upper-bound term of a pixel x in block K is a quadratic
// in z = x - c_K (c_K the block centre).  With D_e = c_K - c_L for the other
// block L of a support entry e and the moments W0 = sum w_y, W1 = sum w_y
// (y - c_L), W2 = sum w_y |y - c_L|^2 of w (nu for side 0, mu for side 1)
// over L:
//   sum_y w_y |x - y|^2 = W0 |z + D_e|^2 - 2 (z + D_e).W1 + W2,
// so h(x) = sum_e coef_e (...) = A |z|^2 + B.z + C with
//   A = sum coef_e W0,  B = sum coef_e (2 W0 D_e - 2 W1),
//   C = sum coef_e (W0 |D_e|^2 - 2 D_e.W1 + W2).
// One thread per coarse block and side writes (A, B0, B1, B2, C).

// Gradients of dl * lower + du * upper for p = 2 jobs, one thread per pixel
// (coalesced): the lower-bound term s_L f_i (resp. s_L g_j), then the
// upper-bound term s_U (h(x_i) + gbar_K) from the block's quadratic.
__global__ __launch_bounds__(256) void k_grad2(const DevJob* __restrict__ jobs, int njobs,
                                               const int* __restrict__ off, int total,
                                               const double* __restrict__ dl, const double* __restrict__ du) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    if (J.p != 2) continue;
    const bool lb = J.grad_a && J.grad_b;
    const double Se = J.result[RS_LOWER_S];
    const double sL = Se > 0.0 ? 0.5 / sqrt(Se) * dl[jb] : 0.0;
    const double Pc = J.result[RS_PCOST_RAW];
    const double sU = Pc > 0.0 ? 0.5 / sqrt(Pc) * du[jb] : 0.0;
    const int base = (it - off[jb]) * kChunk;
    const int n = J.n, k = J.k;
    const double hk = 0.5 * (k - 1);
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int i = base + q;
      if (i >= J.P) break;
      int x0, x1, x2;
      pix_coords(i, J.N, J.d, x0, x1, x2);
      const int b0 = x0 / k, b1 = x1 / k, b2 = x2 / k;
      const int K = J.d == 2 ? b1 * n + b2 : (b0 * n + b1) * n + b2;
      const double z0 = J.d == 2 ? 0.0 : x0 - (k * b0 + hk);
      const double z1 = x1 - (k * b1 + hk), z2 = x2 - (k * b2 + hk);
      const double zz = z0 * z0 + z1 * z1 + z2 * z2;
      for (int side = 0; side < 2; ++side) {
        double* grad = side == 0 ? J.grad_a : J.grad_b;
        if (!grad) continue;
        const double* c = J.gquad + (size_t)10 * K + 5 * side;
        const double h = c[0] * zz + (c[1] * z0 + c[2] * z1 + c[3] * z2) + c[4];
        double g = grad[i];
        if (lb) g += sL * (double)(side == 0 ? J.f[i] : J.g[i]);
        g += sU * (h + (side == 0 ? J.gbar_mu[K] : J.gbar_nu[K]));
        grad[i] = g;
      }
    }
  }
}

__global__ __launch_bounds__(64) void k_ub_grad(const DevJob* __restrict__ jobs, int njobs,
                                                const int* __restrict__ off, int total,
                                                const double* __restrict__ du, int side) {
  __shared__ double sw[512];
  __shared__ int sc[512][3];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    double* grad = side == 0 ? J.grad_a : J.grad_b;
    if (!grad || J.p == 2 || J.p1_nt) continue;   // p = 2 jobs: k_grad2; table-path jobs: k_ubg_tab
    const int m = J.d == 2 ? J.k * J.k : J.k * J.k * J.k;
    const double* other = side == 0 ? J.nu : J.mu;
    if (m <= 32) {
      // small blocks: 64 / g entries per wave, as in k_plancost
      const int gsz = reduce_group(m), sub = threadIdx.x / gsz, a = threadIdx.x - sub * gsz;
      const int e = (it - off[jb]) * (64 / gsz) + sub;
      const bool act = e < J.nnz && a < m;
      int x0 = 0, x1 = 0, x2 = 0;
      __syncthreads();
      if (act) {
        const int B = side == 0 ? J.e_row[e] : J.e_col[e];
        const int O = side == 0 ? J.e_col[e] : J.e_row[e];
        pix_coords(block_member(B, a, J.N, J.n, J.k, J.d), J.N, J.d, x0, x1, x2);
        const int j = block_member(O, a, J.N, J.n, J.k, J.d);
        sw[threadIdx.x] = other[j];
        pix_coords(j, J.N, J.d, sc[threadIdx.x][0], sc[threadIdx.x][1], sc[threadIdx.x][2]);
      }
      __syncthreads();
      if (act) J.part1[(size_t)e * 64 + a] = J.coef[e] * dist_dot(x0, x1, x2, sw + sub * gsz, sc + sub * gsz, m);
      continue;
    }
    // item = (support entry e, 64 pixels of its block on this side)
    const int per = (m + 63) / 64;
    const int li = it - off[jb];
    const int e = li / per, c = li - e * per;
    const int B = side == 0 ? J.e_row[e] : J.e_col[e];
    const int O = side == 0 ? J.e_col[e] : J.e_row[e];
    const int a = c * 64 + threadIdx.x;
    int x0 = 0, x1 = 0, x2 = 0;
    if (a < m) pix_coords(block_member(B, a, J.N, J.n, J.k, J.d), J.N, J.d, x0, x1, x2);
    double acc = 0.0;
    for (int t0 = 0; t0 < m; t0 += 512) {
      const int tn = min(512, m - t0);
      __syncthreads();
      for (int r = threadIdx.x; r < tn; r += 64) {
        const int j = block_member(O, t0 + r, J.N, J.n, J.k, J.d);
        sw[r] = other[j];
        pix_coords(j, J.N, J.d, sc[r][0], sc[r][1], sc[r][2]);
      }
      __syncthreads();
      if (a < m) acc += dist_dot(x0, x1, x2, sw, sc, tn);
    }
    J.part1[((size_t)e * per + c) * 64 + threadIdx.x] = J.coef[e] * acc;
  }
}

// p = 1: h(x) = sum over the entries of x's block row (side 0) or column
// (side 1), in the order of the coupling's lists, of the partials above; then
// grad += du (h + gbar).  One thread per pixel.
__global__ __launch_bounds__(256) void k_ub_grad_sum(const DevJob* __restrict__ jobs, int njobs,
                                                     const int* __restrict__ off, int total,
                                                     const double* __restrict__ du, int side) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    double* grad = side == 0 ? J.grad_a : J.grad_b;
    if (!grad || J.p == 2) continue;
    const double s = J.result[RS_PCOST_RAW] > 0.0 ? du[jb] : 0.0;   // d P / d P for p = 1
    const int m = J.d == 2 ? J.k * J.k : J.k * J.k * J.k;
    const int per = (m + 63) / 64;
    const int k = J.k, n = J.n;
    const int base = (it - off[jb]) * kChunk;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int i = base + q;
      if (i >= J.P) break;
      int x0, x1, x2;
      pix_coords(i, J.N, J.d, x0, x1, x2);
      const int B = J.d == 2 ? (x1 / k) * n + x2 / k : ((x0 / k) * n + x1 / k) * n + x2 / k;
      const int a = J.d == 2 ? (x1 % k) * k + x2 % k : ((x0 % k) * k + x1 % k) * k + x2 % k;
      const int e0 = side == 0 ? J.csr_ptr[B] : J.csc_ptr[B];
      const int e1 = side == 0 ? J.csr_ptr[B + 1] : J.csc_ptr[B + 1];
      double h = 0.0;
      for (int qq = e0; qq < e1; ++qq) {
        const int e = side == 0 ? qq : J.csc_idx[qq];
        h += J.part1[(size_t)e * per * 64 + a];
      }
      grad[i] += s * (h + (side == 0 ? J.gbar_mu[B] : J.gbar_nu[B]));
    }
  }
}

// d lower / d fhat through the arg-mins: sum_i mu_i [argmin_g(argmin_f(i)) = r] - sum_j nu_j [argmin_g(j) = r].
__global__ __launch_bounds__(256) void k_fhat_grad(const DevJob* __restrict__ jobs, int njobs,
                                                   const int* __restrict__ off, int total,
                                                   const double* __restrict__ dl,
                                                   double* const* __restrict__ outs) {
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int jb = find_job(off, njobs, it);
    const DevJob& J = jobs[jb];
    double* out = outs[jb];
    if (!out || !J.arg_g || !J.arg_f) continue;
    const double Se = J.result[RS_LOWER_S];
    const double s = Se > 0.0 ? (J.p == 2 ? 0.5 / sqrt(Se) : 1.0) * dl[jb] : 0.0;
    const int base = (it - off[jb]) * kChunk;
    for (int q = threadIdx.x; q < kChunk; q += 256) {
      const int i = base + q;
      if (i >= J.P) break;
      const int jf = J.arg_f[i];
      const int r1 = (jf >= 0 && jf < J.P) ? J.arg_g[jf] : -1;
      const int r2 = J.arg_g[i];
      if (r1 >= 0 && r1 < J.P) atomicAdd(out + r1, s * J.mu[i]);
      if (r2 >= 0 && r2 < J.P) atomicAdd(out + r2, -s * J.nu[i]);
    }
  }
}

// For caller-supplied scalings (a_s, b_s): block sums A_K = sum a_s, B_L = sum b_s,
// then (pi^ b_s) on block K = k^(-2d) sum_L pi~_KL B_L and (pi^T a_s) on block
// L = k^(-2d) sum_K pi~_KL A_K, stored where k_tv_partial reads u^{T+1}, v^T
// (with T = 1).  One work-group per job.
__global__ __launch_bounds__(1024) void k_tv_prep(const DevJob* __restrict__ jobs, int njobs) {
  const DevJob& J = jobs[blockIdx.x];
  const int Q = J.Q;
  const int m = J.d == 2 ? J.k * J.k : J.k * J.k * J.k;
  const double kd = (double)m;
  const double cc = 1.0 / (kd * kd);
  double* A = J.gbar_mu;
  double* B = J.gbar_nu;
  for (int K = threadIdx.x; K < Q; K += 1024) {
    double sa = 0.0, sb = 0.0;
    for (int t = 0; t < m; ++t) {
      const int i = block_member(K, t, J.N, J.n, J.k, J.d);
      sa += J.a_s[i];
      sb += J.b_s[i];
    }
    A[K] = sa;
    B[K] = sb;
  }
  __syncthreads();
  for (int K = threadIdx.x; K < Q; K += 1024) {
    double s = 0.0;
    for (int e = J.csr_ptr[K]; e < J.csr_ptr[K + 1]; ++e) s += J.e_val[e] * B[J.e_col[e]];
    J.ipf_u[2 * (size_t)Q + K] = cc * s;
  }
  for (int L = threadIdx.x; L < Q; L += 1024) {
    double s = 0.0;
    for (int q = J.csc_ptr[L]; q < J.csc_ptr[L + 1]; ++q) {
      const int e = J.csc_idx[q];
      s += J.e_val[e] * A[J.e_row[e]];
    }
    J.ipf_v[(size_t)Q + L] = cc * s;
  }
  if (threadIdx.x == 0) J.result[RS_IPF_ITERS] = 1.0;
}

// ------------------------------------------------------------------ upper bound with any upscaling kernel
//
// Section 3.4 upscales the coarse coupling by a Kronecker product with a
// normalised nonnegative kernel tensor on [k]^(2d); Algorithm 4 takes the
// uniform one.  For a general kernel, pi^ restricted to X_K x Y_L is
// pi~_KL times the m x m kernel matrix (m = k^d, rows and columns indexed by
// the in-block offsets in C order), so
//   (pi^ x)_i   = sum_{L: (K,L) in supp} pi~_KL sum_t Kst[s(i), t] x_(L,t),
//   (pi^T y)_j  = sum_{K: (K,L) in supp} pi~_KL sum_s Kst[s, t(j)] y_(K,s),
// and the fitting runs on fine vectors.  Both sums are linear in x (y), so a
// pass first adds the other side's blocks, weighted by pi~, into one m-vector
// z in LDS and then takes a single product with the kernel matrix:
//   (pi^ x)_(K,s) = sum_t Kst[s, t] z_t,  z_t = sum_{L: (K,L) in supp} pi~_KL x_(L,t).
// One work-group handles nt offsets of one block (grid Q x cpb) and reads the
// kernel matrix coalesced (Kts for rows, Kst for columns).  Every pass returns
// at once after the fitting has stopped.
//
// Iteration t (t = 1 .. T) of Algorithm 4 is k_kub_col(t) then k_kub_row(t):
//   col(t): v = pi^T a^t, b^t = nu / v, nu^ = b^t v        (0/0 := 0)
//   row(t): u = pi^ b^t,  mu^ = a^t u, a^(t+1) = mu / u
// with a^1 = mu / (pi^ 1) from row(0); k_kub_check(t) then adds the L1
// residual partials in a fixed order and stops the fitting once it is below
// xi (or at max_iter).  a^t alternates
// between a0 (t even) and a1 (t odd), so a^T survives the row pass that
// follows it.

// z_q = sum over block blk's coupling entries e (stored order) of
// pi~_e x_(B_e, q) into xs[0, m), B_e the other side's block (x null: all
// ones).  ROWS walks the CSR list of a source block, else the CSC list of a
// target block.  Ends with a barrier.
template <bool ROWS>
__device__ __forceinline__ void kub_stage(const KubJob& J, int blk, const double* __restrict__ x, double* xs) {
  const int m = J.m;
  const int r0 = ROWS ? J.csr_ptr[blk] : J.csc_ptr[blk];
  const int r1 = ROWS ? J.csr_ptr[blk + 1] : J.csc_ptr[blk + 1];
  for (int q = threadIdx.x; q < m; q += 256) {
    double z = 0.0;
    for (int r = r0; r < r1; ++r) {
      const int e = ROWS ? r : J.csc_idx[r];
      const int B = ROWS ? J.e_col[e] : J.e_row[e];
      z += J.e_val[e] * (x ? x[block_member(B, q, J.N, J.n, J.k, J.d)] : 1.0);
    }
    xs[q] = z;
  }
  __syncthreads();
}

// Thread share g (of S) of sum_q Kmat[q m + o] xs[q], in four independent
// partial sums so that several loads of the kernel matrix are in flight.
template <int S>
__device__ __forceinline__ double kub_dot(const double* __restrict__ Km, const double* xs, int m, int o, int g) {
  const int per = (m + S - 1) / S;
  const int q0 = min(m, g * per), q1 = min(m, q0 + per);
  double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
  int q = q0;
#pragma unroll 2
  for (; q + 4 <= q1; q += 4) {
    r0 += Km[(size_t)q * m + o] * xs[q];
    r1 += Km[(size_t)(q + 1) * m + o] * xs[q + 1];
    r2 += Km[(size_t)(q + 2) * m + o] * xs[q + 2];
    r3 += Km[(size_t)(q + 3) * m + o] * xs[q + 3];
  }
  for (; q < q1; ++q) r0 += Km[(size_t)q * m + o] * xs[q];
  return (r0 + r1) + (r2 + r3);
}

// Adds the S shares of each offset (threads o, o + OFF, ...) in order; the
// result is valid in the first OFF threads.  Called by every thread.
template <int S, int OFF>
__device__ __forceinline__ double kub_combine(double v, double* sh) {
  if (S == 1) return v;
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  double r = v;
  if ((int)threadIdx.x < OFF) {
    r = sh[threadIdx.x];
    for (int g = 1; g < S; ++g) r += sh[g * OFF + threadIdx.x];
  }
  __syncthreads();
  return r;
}

// The passes run 256 threads per work-group over OFF offsets of one block:
// OFF = 64 (k^d <= 64) splits each offset's sum over four waves, OFF = 256
// gives every thread its own offset.
template <int OFF>
__global__ __launch_bounds__(256) void k_kub_row(KubJob J, int t) {
  constexpr int S = 256 / OFF;
  if (J.state[0]) return;
  extern __shared__ double xs[];  // z over the target blocks
  __shared__ double sh[256];
  const int K = blockIdx.x, c = blockIdx.y, m = J.m;
  const int g = threadIdx.x / OFF;
  const int s = c * OFF + (threadIdx.x - g * OFF);
  kub_stage<true>(J, K, t == 0 ? nullptr : J.b, xs);
  double acc = s < m ? kub_dot<S>(J.Kts, xs, m, s, g) : 0.0;
  acc = kub_combine<S, OFF>(acc, sh);
  double part = 0.0;
  if (g == 0 && s < m) {
    const int i = block_member(K, s, J.N, J.n, J.k, J.d);
    const double mu = J.mu[i];
    if (J.hist_u) J.hist_u[(size_t)(t + 1) * J.P + i] = acc;
    if (t >= 1) {
      const double muh = ((t & 1) ? J.a1 : J.a0)[i] * acc;
      J.muh[i] = muh;
      part = fabs(muh - mu);
    }
    (((t + 1) & 1) ? J.a1 : J.a0)[i] = acc > 0.0 ? mu / acc : 0.0;
  }
  if (t >= 1) {
    part = block_sum<256>(part, sh);
    if (threadIdx.x == 0) J.part_mu[(size_t)K * J.cpb + c] = part;
  }
}

template <int OFF>
__global__ __launch_bounds__(256) void k_kub_col(KubJob J, int t) {
  constexpr int S = 256 / OFF;
  if (J.state[0]) return;
  extern __shared__ double xs[];  // z over the source blocks
  __shared__ double sh[256];
  const int L = blockIdx.x, c = blockIdx.y, m = J.m;
  const int g = threadIdx.x / OFF;
  const int o = c * OFF + (threadIdx.x - g * OFF);
  kub_stage<false>(J, L, (t & 1) ? J.a1 : J.a0, xs);
  double acc = o < m ? kub_dot<S>(J.Kst, xs, m, o, g) : 0.0;
  acc = kub_combine<S, OFF>(acc, sh);
  double part = 0.0;
  if (g == 0 && o < m) {
    const int j = block_member(L, o, J.N, J.n, J.k, J.d);
    const double nu = J.nu[j];
    if (J.hist_v) J.hist_v[(size_t)t * J.P + j] = acc;
    const double b = acc > 0.0 ? nu / acc : 0.0;
    const double nuh = b * acc;
    J.b[j] = b;
    J.nuh[j] = nuh;
    part = fabs(nu - nuh);
  }
  part = block_sum<256>(part, sh);
  if (threadIdx.x == 0) J.part_nu[(size_t)L * J.cpb + c] = part;
}

// Stop test of iteration t after col(t) and row(t): the L1 residual partials
// of both passes added in a fixed order, then the stop flag.
__global__ __launch_bounds__(256) void k_kub_check(KubJob J, int t) {
  if (J.state[0]) return;
  __shared__ double sh[256];
  const int n = J.Q * J.cpb;
  double sm = 0.0, sn = 0.0;
  for (int q = threadIdx.x; q < n; q += 256) {
    sm += J.part_mu[q];
    sn += J.part_nu[q];
  }
  double sv[2] = {sm, sn}, mv[1] = {0.0};
  block_reduce_many<2, 1>(sv, mv, sh);
  if (threadIdx.x == 0) {
    const double err = sv[0] + sv[1];
    J.result[RS_IPF_RESID] = err;
    J.result[RS_IPF_ITERS] = (double)t;
    const bool conv = err < J.xi;
    if (conv || t >= J.max_iter) {
      J.result[RS_WARN] = conv ? 0.0 : (double)QBW_WARN_IPF_NOT_CONVERGED;
      J.state[0] = 1;
    }
  }
}

// Plan cost: per (coupling entry e = (K, L), nt source offsets) the sum over
// the offsets s and all target offsets t of a_(K,s) Kst[s,t] b_(L,t) c_st,
// target block staged in LDS by tiles of 1024 (values and coordinates);
// k_kub_finalize multiplies by pi~_e and adds everything in a fixed order.
template <int NT>
__global__ __launch_bounds__(NT) void k_kub_plancost(KubJob J) {
  __shared__ double sh[NT];
  __shared__ double sb[1024];
  __shared__ int sc[1024][3];
  const int e = blockIdx.x, c = blockIdx.y, m = J.m;
  const int T = (int)J.result[RS_IPF_ITERS];
  const double* a = (T & 1) ? J.a1 : J.a0;
  const int K = J.e_row[e], L = J.e_col[e];
  const int s = c * NT + threadIdx.x;
  int x0 = 0, x1 = 0, x2 = 0;
  double wa = 0.0;
  if (s < m) {
    const int i = block_member(K, s, J.N, J.n, J.k, J.d);
    pix_coords(i, J.N, J.d, x0, x1, x2);
    wa = a[i];
  }
  double acc = 0.0;
  for (int t0 = 0; t0 < m; t0 += 1024) {
    const int tn = min(1024, m - t0);
    __syncthreads();
    for (int q = threadIdx.x; q < tn; q += NT) {
      const int j = block_member(L, t0 + q, J.N, J.n, J.k, J.d);
      sb[q] = J.b[j];
      pix_coords(j, J.N, J.d, sc[q][0], sc[q][1], sc[q][2]);
    }
    __syncthreads();
    if (s < m) {
      for (int q = 0; q < tn; ++q) {
        const int e0 = x0 - sc[q][0], e1 = x1 - sc[q][1], e2 = x2 - sc[q][2];
        const double d2 = (double)(e0 * e0 + e1 * e1 + e2 * e2);
        const double cst = J.p == 2 ? d2 : sqrt(d2);
        acc += J.Kts[(size_t)(t0 + q) * m + s] * sb[q] * cst;
      }
    }
  }
  acc = block_sum<NT>(wa * acc, sh);
  if (threadIdx.x == 0) J.pc_part[(size_t)e * J.cpb + c] = acc;
}

// Weighted-TV partials per chunk of kChunk pixels: w_i = |x_i - x-bar|^p.
__global__ __launch_bounds__(256) void k_kub_tv(KubJob J) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  const double h = 0.5 * (J.N - 1);
  double tm = 0.0, tn = 0.0, wm = 0.0, wn = 0.0;
  for (int q = threadIdx.x; q < kChunk; q += 256) {
    const int i = c * kChunk + q;
    if (i >= J.P) break;
    int x0, x1, x2;
    pix_coords(i, J.N, J.d, x0, x1, x2);
    const double d0 = J.d == 2 ? 0.0 : x0 - h, d1 = x1 - h, d2 = x2 - h;
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const double w = J.p == 2 ? r2 : sqrt(r2);
    const double mu = J.mu[i], nu = J.nu[i];
    tm += w * fabs(J.muh[i] - mu);
    tn += w * fabs(nu - J.nuh[i]);
    wm += w * mu;
    wn += w * nu;
  }
  double sv[4] = {tm, tn, wm, wn}, mv[1] = {0.0};
  block_reduce_many<4, 1>(sv, mv, sh);
  if (threadIdx.x == 0) {
    double* r = J.red_tv + (size_t)c * kRedSlotsTV;
    r[0] = sv[0]; r[1] = sv[1]; r[2] = sv[2]; r[3] = sv[3];
  }
}

// The bound with outward allowances derived as for the uniform kernel (see
// k_finalize), for fitting on fine vectors: a row pass forms, per pixel, the
// pi~-weighted sum of r entries' blocks (gamma(r+1)) and its product with a
// kernel row of m nonnegative weights (gamma(m+2)); a column pass likewise with
// c entries.  Each iteration then adds D = gamma(r+1) + gamma(c+1) +
// 2 gamma(m+2) + 2u to the iterates' relative error against exact arithmetic,
// from gamma(r+1) + gamma(m+2) at the first row pass, so the fitted
// mu^ is within e_G = 2 (gamma(r+1) + gamma(m+2)) + (2T - 1) D + 2u and nu^ within
// e_nu = gamma(c+1) + gamma(m+2) + 4u.  The plan cost sums nonnegative terms
// m + cpb + ceil(nnz/256) + 24 additions deep (plus 2^-41 for p = 1's roots),
// widened by the scalings' e_G + 14 T u.
__global__ __launch_bounds__(256) void k_kub_finalize(KubJob J) {
  __shared__ double sh[256];
  double pc = 0.0;
  for (int e = threadIdx.x; e < J.nnz; e += 256) {
    double s = 0.0;
    for (int c = 0; c < J.cpb; ++c) s += J.pc_part[(size_t)e * J.cpb + c];
    pc += J.e_val[e] * s;
  }
  double rmax = 0, cmax = 0;
  if (J.nnz > 0)
    for (int K = threadIdx.x; K < J.Q; K += 256) {
      rmax = fmax(rmax, (double)(J.csr_ptr[K + 1] - J.csr_ptr[K]));
      cmax = fmax(cmax, (double)(J.csc_ptr[K + 1] - J.csc_ptr[K]));
    }
  double tm = 0.0, tn = 0.0, wm = 0.0, wn = 0.0;
  for (int c = threadIdx.x; c < J.chunks; c += 256) {
    const double* r = J.red_tv + (size_t)c * kRedSlotsTV;
    tm += r[0]; tn += r[1]; wm += r[2]; wn += r[3];
  }
  {
    double sv[5] = {pc, tm, tn, wm, wn}, mv[2] = {rmax, cmax};
    block_reduce_many<5, 2>(sv, mv, sh);
    pc = sv[0]; tm = sv[1]; tn = sv[2]; wm = sv[3]; wn = sv[4];
    rmax = mv[0]; cmax = mv[1];
  }
  if (threadIdx.x != 0) return;
  double* res = J.result;
  const double u53 = 1.1102230246251565e-16;
  const double T = fmax(1.0, res[RS_IPF_ITERS]);
  const double m = (double)J.m;
  const double n_s = 4 + 9 + (J.chunks + 255) / 256 + 9;
  const double a1 = gam(rmax + 1) + gam(m + 2);
  const double Dg = gam(rmax + 1) + gam(cmax + 1) + 2.0 * gam(m + 2) + 2.0 * u53;
  const double eG = 2.0 * a1 + (2.0 * T - 1.0) * Dg + 2.0 * u53;
  const double eO = 14.0 * T * u53;
  const double emu = (eG + eO) * (1.0 + 0x1p-40);
  const double enu = (gam(cmax + 1) + gam(m + 2) + 4.0 * u53) * (1.0 + 0x1p-40);
  const double Zm = tm * (1.0 + gam(n_s + 3)), Zn = tn * (1.0 + gam(n_s + 3));
  const double Wm = wm * (1.0 + gam(n_s + 2)), Wn = wn * (1.0 + gam(n_s + 2));
  const double Tm = (Zm + emu * (Wm + Zm) / (1.0 - eG)) * (1.0 + 8.0 * u53);
  const double Tn = (Zn + enu * (Wn + Zn) / (1.0 - enu)) * (1.0 + 8.0 * u53);
  const double Pv = pc * (1.0 + gam(m + J.cpb + (J.nnz + 255) / 256 + 24) + (J.p == 1 ? 0x1p-41 : 0.0));
  const double pe = Pv * (1.0 + eG + eO + 6.0 * u53) * (1.0 + 4.0 * u53);
  const double c1 = J.p == 2 ? 1.4142135623730951 : 1.0;
  auto root = [&](double x) { return J.p == 2 ? sqrt(x) : x; };
  const double tvm = c1 * root(Tm) * (1.0 + 2.0 * u53);
  const double tvn = c1 * root(Tn) * (1.0 + 2.0 * u53);
  res[RS_UPPER] = (root(pe) * (1.0 + u53) + tvm + tvn) * (1.0 + 2.0 * u53);
  res[RS_UPPER_COST] = pe;
  res[RS_TV_MU] = tvm;
  res[RS_TV_NU] = tvn;
  res[RS_COARSE_OBJ] = J.coarse_obj;
  res[RS_PCOST_RAW] = pc;
  res[RS_TVSUM_MU] = tm;
  res[RS_TVSUM_NU] = tn;
  res[RS_MW_MU] = wm;
  res[RS_MW_NU] = wn;
  res[RS_TV_RAW_MU] = c1 * root(tm);
  res[RS_TV_RAW_NU] = c1 * root(tn);
}

// Gradient of the plan cost P = sum a^T_i pi^_ij b^T_j c_ij through the T
// fitting iterations (coarse coupling, kernel and T frozen), from the
// checkpointed u^t, v^t.  With a^t = mu / u^t, b^t = nu / v^t (0 where the
// denominator is 0), reverse mode gives, for t = T .. 1,
//   b-bar = (t = T ? d P / d b^T : pi^T u-bar^(t+1)),
//   d mu_nu += b-bar / v^t,   v-bar = -b-bar nu / (v^t)^2,
//   a-bar = (t = T ? d P / d a^T : 0) + pi^ v-bar,
//   d mu += a-bar / u^t,      u-bar = -a-bar mu / (u^t)^2,
// with d P / d a^T = (pi^ o C) b^T and d P / d b^T = (pi^ o C)^T a^T.  The
// column half of step t is fused into the pass that produces b-bar.

// Cost-weighted passes for d P / d a^T (rows) and d P / d b^T (columns, with
// step T's column half).  Other-side block staged in LDS by tiles of 1024.
template <int NT, bool COLS>
__global__ __launch_bounds__(NT) void k_kub_pgrad(KubJob J, int T) {
  __shared__ double sb[1024];
  __shared__ int sc[1024][3];
  const int B = blockIdx.x, c = blockIdx.y, m = J.m;
  const int o = c * NT + threadIdx.x;
  const double* aT = (T & 1) ? J.a1 : J.a0;
  int x0 = 0, x1 = 0, x2 = 0, i = 0;
  if (o < m) {
    i = block_member(B, o, J.N, J.n, J.k, J.d);
    pix_coords(i, J.N, J.d, x0, x1, x2);
  }
  double acc = 0.0;
  const int q0 = COLS ? J.csc_ptr[B] : J.csr_ptr[B];
  const int q1 = COLS ? J.csc_ptr[B + 1] : J.csr_ptr[B + 1];
  for (int q = q0; q < q1; ++q) {
    const int e = COLS ? J.csc_idx[q] : q;
    const int O = COLS ? J.e_row[e] : J.e_col[e];   // the other side's block
    const double* w = COLS ? aT : J.b;
    double r = 0.0;
    for (int t0 = 0; t0 < m; t0 += 1024) {
      const int tn = min(1024, m - t0);
      __syncthreads();
      for (int z = threadIdx.x; z < tn; z += NT) {
        const int j = block_member(O, t0 + z, J.N, J.n, J.k, J.d);
        sb[z] = w[j];
        pix_coords(j, J.N, J.d, sc[z][0], sc[z][1], sc[z][2]);
      }
      __syncthreads();
      if (o < m) {
        for (int z = 0; z < tn; ++z) {
          const int e0 = x0 - sc[z][0], e1 = x1 - sc[z][1], e2 = x2 - sc[z][2];
          const double d2 = (double)(e0 * e0 + e1 * e1 + e2 * e2);
          const double cst = J.p == 2 ? d2 : sqrt(d2);
          // rows: Kst[o, t0+z] = Kts[(t0+z) m + o]; columns: Kst[t0+z, o]
          const double kw = COLS ? J.Kst[(size_t)(t0 + z) * m + o] : J.Kts[(size_t)(t0 + z) * m + o];
          r += kw * sb[z] * cst;
        }
      }
    }
    acc += J.e_val[e] * r;
  }
  if (o >= m) return;
  if (!COLS) {
    J.g_abar[i] = acc;
  } else {
    const double v = J.hist_v[(size_t)T * J.P + i];
    J.g_nu[i] = v > 0.0 ? acc / v : 0.0;
    J.g_vbar[i] = v > 0.0 ? -acc * J.nu[i] / (v * v) : 0.0;
  }
}

// Row half of reverse step t: a-bar = (t = T ? g_abar : 0) + pi^ v-bar.
template <int OFF>
__global__ __launch_bounds__(256) void k_kub_rev_row(KubJob J, int t, int T) {
  constexpr int S = 256 / OFF;
  extern __shared__ double xs[];
  __shared__ double sh[256];
  const int K = blockIdx.x, c = blockIdx.y, m = J.m;
  const int g = threadIdx.x / OFF;
  const int s = c * OFF + (threadIdx.x - g * OFF);
  kub_stage<true>(J, K, J.g_vbar, xs);
  double acc = s < m ? kub_dot<S>(J.Kts, xs, m, s, g) : 0.0;
  acc = kub_combine<S, OFF>(acc, sh);
  if (g != 0 || s >= m) return;
  const int i = block_member(K, s, J.N, J.n, J.k, J.d);
  const double abar = (t == T ? J.g_abar[i] : 0.0) + acc;
  const double u = J.hist_u[(size_t)t * J.P + i];
  const double gm = u > 0.0 ? abar / u : 0.0;
  J.g_mu[i] = (t == T ? 0.0 : J.g_mu[i]) + gm;
  J.g_ubar[i] = u > 0.0 ? -abar * J.mu[i] / (u * u) : 0.0;
}

// b-bar = pi^T u-bar^(t+1), then the column half of step t (t < T).
template <int OFF>
__global__ __launch_bounds__(256) void k_kub_rev_col(KubJob J, int t) {
  constexpr int S = 256 / OFF;
  extern __shared__ double xs[];
  __shared__ double sh[256];
  const int L = blockIdx.x, c = blockIdx.y, m = J.m;
  const int g = threadIdx.x / OFF;
  const int o = c * OFF + (threadIdx.x - g * OFF);
  kub_stage<false>(J, L, J.g_ubar, xs);
  double acc = o < m ? kub_dot<S>(J.Kst, xs, m, o, g) : 0.0;
  acc = kub_combine<S, OFF>(acc, sh);
  if (g != 0 || o >= m) return;
  const int j = block_member(L, o, J.N, J.n, J.k, J.d);
  const double v = J.hist_v[(size_t)t * J.P + j];
  J.g_nu[j] += v > 0.0 ? acc / v : 0.0;
  J.g_vbar[j] = v > 0.0 ? -acc * J.nu[j] / (v * v) : 0.0;
}

// grad += dupper d(P^(1/p)) / d(mu, nu), P^(1/p)' = P^(1/p - 1) / p (0 at P = 0).
__global__ __launch_bounds__(256) void k_kub_grad_out(KubJob J, double dupper, double* __restrict__ ga,
                                                      double* __restrict__ gb) {
  const double pc = J.result[RS_PCOST_RAW];
  const double sc = pc > 0.0 ? dupper * (J.p == 2 ? 0.5 / sqrt(pc) : 1.0) : 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < J.P; i += gridDim.x * 256) {
    if (ga) ga[i] += sc * J.g_mu[i];
    if (gb) gb[i] += sc * J.g_nu[i];
  }
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int total, int cap = 65535) { return total < 1 ? 1 : (total < cap ? total : cap); }

int launch_upscale(const DevJob* jobs, int njobs, const int* off, int total, int skip_small, void* stream) {
  hipLaunchKernelGGL(k_upscale, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total,
                     skip_small);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int ctransform_waves_per_cu() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_ctransform, 64, 0) != hipSuccess) return 0;
  return blocks;   // one wave per work-group
}
int launch_reset_counter(int* counter, int n, void* stream) {
  hipLaunchKernelGGL(k_reset_counter, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, counter, n);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_ctransform(const DevJob* jobs, const CtItem* items, int n_items, int* counter, int phase, int grid,
                      void* stream) {
  hipLaunchKernelGGL(k_ctransform, dim3(grid), dim3(64), 0, (hipStream_t)stream, jobs, items, n_items, counter,
                     phase);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_sqrt_table(float* t, int n, void* stream) {
  hipLaunchKernelGGL(k_sqrt_table, dim3(grid_for((n + 255) / 256, 1024)), dim3(256), 0, (hipStream_t)stream, t, n);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_merge(const DevJob* jobs, int njobs, const int* off, int total, int phase, void* stream) {
  hipLaunchKernelGGL(k_merge, dim3(grid_for(total), kChunk / 256), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off,
                     total, phase);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_argmin(const DevJob* jobs, int njobs, const int* off, int total, int phase, void* stream) {
  hipLaunchKernelGGL(k_argmin, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total, phase);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_ipf(const DevJob* jobs, int njobs, size_t lds_bytes, int flags, double* scratch, int stride,
               void* stream) {
  hipLaunchKernelGGL(k_ipf, dim3(njobs), dim3(1024), lds_bytes, (hipStream_t)stream, jobs, njobs, lds_bytes, flags,
                     scratch, stride);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_scalings(const DevJob* jobs, int njobs, const int* off, int total, void* stream) {
  hipLaunchKernelGGL(k_scalings, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_tv_partial(const DevJob* jobs, int njobs, const int* off, int total, void* stream) {
  hipLaunchKernelGGL(k_tv_partial, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_plancost(const DevJob* jobs, int njobs, const P1Items& it, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (it.total[0])
    hipLaunchKernelGGL(k_plancost, dim3(grid_for(it.total[0])), dim3(64), 0, st, jobs, njobs, it.off[0], it.total[0]);
  if (it.total[1])
    hipLaunchKernelGGL(k_pc1_tab<64>, dim3(grid_for(it.total[1])), dim3(64), 0, st, jobs, njobs, it.off[1], it.total[1]);
  if (it.total[2])
    hipLaunchKernelGGL(k_pc1_tab<256>, dim3(grid_for(it.total[2])), dim3(256), 0, st, jobs, njobs, it.off[2],
                       it.total[2]);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_plancost2(const DevJob* jobs, int njobs, const int* off, int total, void* stream) {
  hipLaunchKernelGGL(k_plancost2, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_finalize(const DevJob* jobs, int njobs, void* stream) {
  hipLaunchKernelGGL(k_finalize, dim3(njobs), dim3(256), 0, (hipStream_t)stream, jobs, njobs);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_pool(const DevJob* jobs, int njobs, const int* off_mom, int total_mom, int upscale, void* stream) {
  return launch_moments(jobs, njobs, off_mom, total_mom, upscale ? 3 : 2, stream);
}
int launch_moments(const DevJob* jobs, int njobs, const int* off, int total, int which, void* stream) {
  hipLaunchKernelGGL(k_moments, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total, which);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_cbar2(const DevJob* jobs, int njobs, const int* off, int total, double* const* outs,
                 void* stream) {
  hipLaunchKernelGGL(k_cbar, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total, outs);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_lb_grad(const DevJob* jobs, int njobs, const int* off, int total, const double* dl, void* stream) {
  hipLaunchKernelGGL(k_lb_grad, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total, dl);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_ub_coarse_bwd2(const DevJob* jobs, int njobs, double* scratch, int stride, size_t lds_bytes,
                          int skip_p2, void* stream) {
  hipLaunchKernelGGL(k_ub_coarse_bwd, dim3(njobs), dim3(1024), lds_bytes, (hipStream_t)stream, jobs, njobs, scratch,
                     stride, lds_bytes, skip_p2);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_ub_grad(const DevJob* jobs, int njobs, const P1Items& it, const double* du, int side, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (it.total[0])
    hipLaunchKernelGGL(k_ub_grad, dim3(grid_for(it.total[0])), dim3(64), 0, st, jobs, njobs, it.off[0], it.total[0],
                       du, side);
  if (it.total[1])
    hipLaunchKernelGGL(k_ubg_tab<64>, dim3(grid_for(it.total[1])), dim3(64), 0, st, jobs, njobs, it.off[1],
                       it.total[1], side);
  if (it.total[2])
    hipLaunchKernelGGL(k_ubg_tab<256>, dim3(grid_for(it.total[2])), dim3(256), 0, st, jobs, njobs, it.off[2],
                       it.total[2], side);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_fwd_pixels(const DevJob* jobs, int njobs, const int* off, int total, int* clear, int nclear,
                      void* stream) {
  hipLaunchKernelGGL(k_fwd_pixels, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total,
                     clear, nclear);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_pc1_sum(const DevJob* jobs, int njobs, void* stream) {
  hipLaunchKernelGGL(k_pc1_sum, dim3(njobs), dim3(256), 0, (hipStream_t)stream, jobs);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_ub_grad_sum(const DevJob* jobs, int njobs, const int* off, int total, const double* du, int side,
                       void* stream) {
  hipLaunchKernelGGL(k_ub_grad_sum, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off,
                     total, du, side);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_grad2(const DevJob* jobs, int njobs, const int* off, int total, const double* dl, const double* du,
                 void* stream) {
  hipLaunchKernelGGL(k_grad2, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total, dl, du);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_tv_prep(const DevJob* jobs, int njobs, void* stream) {
  hipLaunchKernelGGL(k_tv_prep, dim3(njobs), dim3(1024), 0, (hipStream_t)stream, jobs, njobs);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_ct1d(const DevJob* jobs, int njobs, const int* off, int total, int phase, int pass,
                void* stream) {
  hipLaunchKernelGGL(k_ct1d, dim3(grid_for(total)), dim3(64), 0, (hipStream_t)stream, jobs, njobs, off, total, phase, pass);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_ct1d_fast(const DevJob* jobs, int njobs, const int* off, int total, int phase, int pass, int R,
                     void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (R == 16) hipLaunchKernelGGL(k_ct1d_fast<16>, dim3(grid_for(total)), dim3(64), 0, st, jobs, njobs, off, total, phase, pass);
  else if (R == 8) hipLaunchKernelGGL(k_ct1d_fast<8>, dim3(grid_for(total)), dim3(64), 0, st, jobs, njobs, off, total, phase, pass);
  else hipLaunchKernelGGL(k_ct1d_fast<4>, dim3(grid_for(total)), dim3(64), 0, st, jobs, njobs, off, total, phase, pass);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_xs_squares(double* t, void* stream) {
  hipLaunchKernelGGL(k_xs_squares, dim3((2 * kXsOff + 256) / 256), dim3(256), 0, (hipStream_t)stream, t);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
template <bool FIRST>
static void launch_xs_kind(int T, bool arg, int xt, int waves, const DevJob* jobs, int njobs, const int* off,
                           int total, int phase, int k, const double* sqt, int2* list, int* count, hipStream_t st) {
  const dim3 g(xt ? total : grid_for(total)), b(64 * waves);
  const size_t lds = xs_lds_bytes(FIRST && !xt, T, arg, waves, xt == 2, FIRST);
#define QBW_XS(TT, AA, XX) hipLaunchKernelGGL((k_xs_stage<FIRST, TT, AA, XX>), g, b, lds, st, jobs, njobs, off, total, \
                                              phase, k, sqt, list, count)
  if (xt == 2) {
    if (T == 32) QBW_XS(32, false, 2);
    else if (T == 16) QBW_XS(16, false, 2);
    else QBW_XS(8, false, 2);
  } else if (xt == 1) {
    if (T == 16) QBW_XS(16, false, 1);
    else QBW_XS(8, false, 1);
  } else if (arg) {
    if (T == 2) QBW_XS(2, true, 0);
    else if (T == 4) QBW_XS(4, true, 0);
    else QBW_XS(8, true, 0);
  } else {
    if (T == 2) QBW_XS(2, false, 0);
    else if (T == 4) QBW_XS(4, false, 0);
    else if (T == 16) QBW_XS(16, false, 0);
    else QBW_XS(8, false, 0);
  }
#undef QBW_XS
}

int launch_xs_stage(const DevJob* jobs, int njobs, const int* off, int total, int phase, int k, const double* sqt,
                    int* list, int* count, int T, int argmin, int waves, int xt, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  int2* l2 = reinterpret_cast<int2*>(list);
  if (argmin) waves = 1;
  if (xt < 0 || xt > 2 || (xt && (argmin || T < 8)) || (xt != 2 && T > 16) || waves > (xt == 2 ? 8 : 4))
    return QBW_E_INVAL;
  if (xt && total > (1 << 23)) {   // one work-group per item: the grid's threads must stay below 2^32
    set_error("launch_xs_stage: %d items exceed one work-group per item", total);
    return QBW_E_INVAL;
  }
  if (k == 0) launch_xs_kind<true>(T, argmin != 0, xt, waves, jobs, njobs, off, total, phase, 0, sqt, l2, count, st);
  else launch_xs_kind<false>(T, argmin != 0, xt, waves, jobs, njobs, off, total, phase, k, sqt, l2, count, st);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_xs_fallback(const DevJob* jobs, const int* list, const int* count, int phase, int grid, void* stream) {
  hipLaunchKernelGGL(k_xs_fallback, dim3(grid), dim3(64), 0, (hipStream_t)stream, jobs,
                     reinterpret_cast<const int2*>(list), count, phase);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_sep_argmin(const DevJob* jobs, int njobs, const int* off, int total, int phase, void* stream) {
  hipLaunchKernelGGL(k_sep_argmin, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total, phase);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_fhat_grad2(const DevJob* jobs, int njobs, const int* off, int total, const double* dl,
                      double* const* outs, void* stream) {
  hipLaunchKernelGGL(k_fhat_grad, dim3(grid_for(total)), dim3(256), 0, (hipStream_t)stream, jobs, njobs, off, total, dl, outs);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}

int launch_kub_row(const KubJob& J, int t, void* stream) {
  const size_t lds = sizeof(double) * (size_t)J.m;
  if (J.nt == 64)
    hipLaunchKernelGGL(k_kub_row<64>, dim3(J.Q, J.cpb), dim3(256), lds, (hipStream_t)stream, J, t);
  else
    hipLaunchKernelGGL(k_kub_row<256>, dim3(J.Q, J.cpb), dim3(256), lds, (hipStream_t)stream, J, t);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_kub_col(const KubJob& J, int t, void* stream) {
  const size_t lds = sizeof(double) * (size_t)J.m;
  if (J.nt == 64)
    hipLaunchKernelGGL(k_kub_col<64>, dim3(J.Q, J.cpb), dim3(256), lds, (hipStream_t)stream, J, t);
  else
    hipLaunchKernelGGL(k_kub_col<256>, dim3(J.Q, J.cpb), dim3(256), lds, (hipStream_t)stream, J, t);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_kub_check(const KubJob& J, int t, void* stream) {
  hipLaunchKernelGGL(k_kub_check, dim3(1), dim3(256), 0, (hipStream_t)stream, J, t);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_kub_plancost(const KubJob& J, void* stream) {
  if (J.nt == 64)
    hipLaunchKernelGGL(k_kub_plancost<64>, dim3(J.nnz, J.cpb), dim3(64), 0, (hipStream_t)stream, J);
  else
    hipLaunchKernelGGL(k_kub_plancost<256>, dim3(J.nnz, J.cpb), dim3(256), 0, (hipStream_t)stream, J);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_kub_tv(const KubJob& J, void* stream) {
  hipLaunchKernelGGL(k_kub_tv, dim3(J.chunks), dim3(256), 0, (hipStream_t)stream, J);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}
int launch_kub_finalize(const KubJob& J, void* stream) {
  hipLaunchKernelGGL(k_kub_finalize, dim3(1), dim3(256), 0, (hipStream_t)stream, J);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}

int launch_kub_backward(const KubJob& J, int T, double dupper, double* grad_a, double* grad_b, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const size_t lds = sizeof(double) * (size_t)J.m;
  const dim3 g(J.Q, J.cpb);
  if (J.nt == 64) {
    hipLaunchKernelGGL((k_kub_pgrad<64, false>), g, dim3(64), 0, st, J, T);
    hipLaunchKernelGGL((k_kub_pgrad<64, true>), g, dim3(64), 0, st, J, T);
    for (int t = T; t >= 1; --t) {
      hipLaunchKernelGGL(k_kub_rev_row<64>, g, dim3(256), lds, st, J, t, T);
      if (t > 1) hipLaunchKernelGGL(k_kub_rev_col<64>, g, dim3(256), lds, st, J, t - 1);
    }
  } else {
    hipLaunchKernelGGL((k_kub_pgrad<256, false>), g, dim3(256), 0, st, J, T);
    hipLaunchKernelGGL((k_kub_pgrad<256, true>), g, dim3(256), 0, st, J, T);
    for (int t = T; t >= 1; --t) {
      hipLaunchKernelGGL(k_kub_rev_row<256>, g, dim3(256), lds, st, J, t, T);
      if (t > 1) hipLaunchKernelGGL(k_kub_rev_col<256>, g, dim3(256), lds, st, J, t - 1);
    }
  }
  HIP_TRY(hipGetLastError());
  const int blocks = std::min((J.P + 255) / 256, 4096);
  hipLaunchKernelGGL(k_kub_grad_out, dim3(blocks), dim3(256), 0, st, J, dupper, grad_a, grad_b);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}

// ------------------------------------------------------------------ static scratch
//
// Device memory of the allocation-free c-transform entry point: one array per
// GPU, which the GPU holds until the process ends.  On the host the name is
// only a stand-in for the symbol: its address on a device comes from
// hipGetSymbolAddress with that device current, taken once per device here
// and handed to the kernels as a plain pointer.
static __device__ __align__(256) char scratch[kScratchBytes];

// Set-up of the allocation-free c-transform: the job record (passed by value),
// its chunk prefix table, the work-item table and zeroed counters, written into
// the static scratch by one launch, so the call needs no host-to-device copy.
// Item b is tile b mod tiles of split b / tiles: with a multiple of eight
// tiles that is the planner's per-XCD layout for a single job.
__global__ __launch_bounds__(256) void k_noalloc_setup(DevJob D, DevJob* __restrict__ dj, int* __restrict__ off,
                                                       CtItem* __restrict__ items, int n_items, int tiles,
                                                       int* __restrict__ ints, int n_ints) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i == 0) {
    *dj = D;
    off[0] = 0;
    off[1] = D.chunks;
  }
  if (i < n_ints) ints[i] = 0;
  for (int b = i; b < n_items; b += gridDim.x * 256) items[b] = CtItem{0, b % tiles, b / tiles, 0};
}

int launch_noalloc_setup(const DevJob& D, DevJob* dj, int* off, CtItem* items, int n_items, int tiles, int* ints,
                         int n_ints, void* stream) {
  const int blocks = std::max(1, std::min((std::max(n_items, n_ints) + 255) / 256, 1024));
  hipLaunchKernelGGL(k_noalloc_setup, dim3(blocks), dim3(256), 0, (hipStream_t)stream, D, dj, off, items, n_items,
                     tiles, ints, n_ints);
  HIP_TRY(hipGetLastError());
  return QBW_OK;
}

int scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[kMaxScratchDevices] = {};
  if (device < 0 || device >= kMaxScratchDevices) {
    set_error("device %d beyond the %d devices the static scratch table covers", device, kMaxScratchDevices);
    return QBW_E_HIP;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
      return QBW_E_HIP;
    }
    addr[device] = p;
  }
  *out = addr[device];
  return QBW_OK;
}

}  // namespace qbw
