// Large-rank route of the PAM sweep (Algorithm 1) for jobs with an edge rank
// above the fused kernels' limit, up to 36 (the largest value of the rank
// grid of the multispectral experiments of Sec. 5).
//
// Column j of G_{k,i} solves eq. (updateG): the slice i_k = j of iFCTN(G)
// is A_j g with A_j(x, r) = G_{i,k}(r, x_i) prod_{a != k,i} W_{k,a}(j, x_a)
// D_{-k}(x), x the indices of the modes other than k and D_{-k} the product
// of the edge matrices W_ab with a, b != k.  So
//   A_j^T A_j = G_{i,k} diag(c_j) G_{i,k}^T with
//   c_j(y) = sum_{x: x_i = y} prod_{a != k,i} W_{k,a}(j, x_a)^2 D_{-k}(x)^2,
//   A_j^T X(j, .) = contraction of U_k(j, .) = sum_x X(j, x) D_{-k}(x)
//                   prod_{a != k} G_{a,k}(r_a, x_a) with g_{k,a}(., j), a != k,i,
// which the kernels below form as plain float64 dense steps: the mode
// products of U_k and H_j = c_j . (G_{i,k} (x) G_{i,k}) are tiled GEMMs with
// LDS staging; the Cholesky factorisation runs on one wave per column with
// the matrix in LDS.  Every sum runs in a fixed order (no atomics).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ifctn_internal.h"

namespace ifctn {
namespace {

__device__ __forceinline__ double w_at(const double* __restrict__ W, const LrEdge& e, int x, int y) {
  return W[e.off + (long long)x * e.s1 + (long long)y * e.s2];
}

// --------------------------------------------------------------------------
// Y = X o D_{-k}
// --------------------------------------------------------------------------
template <typename TX>
__global__ __launch_bounds__(NT) void k_lr_y(LrYArgs a) {
  if (a.stop && *a.stop) return;
  const long long L = (long long)blockIdx.x * NT + threadIdx.x;
  if (L >= a.nX) return;
  int idx[MAXN];
  long long t = L;
  for (int m = a.N - 1; m >= 0; --m) {
    idx[m] = (int)(t % a.dims[m]);
    t /= a.dims[m];
  }
  double v = (double)((const TX*)a.X)[L];
  for (int e = 0; e < a.ne; ++e) v *= a.W64[a.woff[e] + (long long)idx[a.ea[e]] * a.dims[a.eb[e]] + idx[a.eb[e]]];
  a.Y[L] = v;
}

// --------------------------------------------------------------------------
// out[a][n][b] = sum_x in[a][x][b] B(n, x): 64 rows (a, b) x 32 columns n per
// workgroup, x in chunks of 16 staged through LDS; each thread keeps 8
// accumulators (one row, 8 columns).
// --------------------------------------------------------------------------
constexpr int LG_TM = 64, LG_TN = 32, LG_TK = 16;

__global__ __launch_bounds__(NT) void k_lr_gemm(LrGemmArgs a) {
  if (a.stop && *a.stop) return;
  __shared__ double As[LG_TK][LG_TM];
  __shared__ double Bs[LG_TK][LG_TN];
  __shared__ int pr[LG_TN];
  const int tid = threadIdx.x;
  const long long M = a.A * a.Bn;
  const long long m0 = (long long)blockIdx.x * LG_TM;
  const int n0 = blockIdx.y * LG_TN;
  if (tid < LG_TN) {
    int n = n0 + tid, r = 0;
    if (a.pairR > 0 && n < a.Nn) {
      while (n >= a.pairR - r) {
        n -= a.pairR - r;
        ++r;
      }
      pr[tid] = r | ((r + n) << 8);
    } else {
      pr[tid] = 0;
    }
  }
  // the A elements this thread stages: with Bn > 1 one row (adjacent lanes,
  // adjacent b), four x; with Bn == 1 four rows, one x (adjacent lanes, adjacent x)
  const bool wide = a.Bn > 1;
  const int lr = wide ? (tid & 63) : (tid >> 4);
  const int lx = wide ? (tid >> 6) : (tid & 15);
  long long rbase[4];
  bool rok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long long m = m0 + (wide ? lr : lr + 16 * q);
    rok[q] = m < M;
    const long long mm = rok[q] ? m : 0;
    const long long aa = mm / a.Bn, b = mm - aa * a.Bn;
    rbase[q] = aa * a.I * a.Bn + b;
  }
  const int mm = tid & 63, ng = tid >> 6;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  __syncthreads();
  for (int x0 = 0; x0 < a.I; x0 += LG_TK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int xx = wide ? lx + 4 * q : lx;
      const int row = wide ? lr : lr + 16 * q;
      const int x = x0 + xx;
      const bool ok = wide ? (rok[0] && x < a.I) : (rok[q] && x < a.I);
      const long long base = wide ? rbase[0] : rbase[q];
      As[xx][row] = ok ? a.in[base + (long long)x * a.Bn] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = tid + q * NT;
      const int xx = e & 15, nn = e >> 4;
      const int n = n0 + nn, x = x0 + xx;
      double v = 0.0;
      if (n < a.Nn && x < a.I) {
        if (a.pairR > 0) {
          const int rp = pr[nn];
          v = a.Bm[(long long)(rp & 255) * a.ldb + x] * a.Bm[(long long)(rp >> 8) * a.ldb + x];
        } else {
          v = a.Bm[(long long)n * a.ldb + x];
        }
      }
      Bs[xx][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int xx = 0; xx < LG_TK; ++xx) {
      const double av = As[xx][mm];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += av * Bs[xx][ng * 8 + q];
    }
    __syncthreads();
  }
  const long long m = m0 + mm;
  if (m < M) {
    const long long aa = m / a.Bn, b = m - aa * a.Bn;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int n = n0 + ng * 8 + q;
      if (n < a.Nn) a.out[(aa * a.Nn + n) * a.Bn + b] = acc[q];
    }
  }
}

// --------------------------------------------------------------------------
// c(j, y): one work-item per (j, y), the other modes walked as a mixed-radix
// counter (last fastest)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_lr_c(LrCArgs a) {
  if (a.stop && *a.stop) return;
  const long long e = (long long)blockIdx.x * NT + threadIdx.x;
  if (e >= (long long)a.Ik * a.Ii) return;
  const int j = (int)(e / a.Ii), y = (int)(e - (long long)j * a.Ii);
  long long total = 1;
  for (int p = 0; p < a.nr; ++p) total *= a.rdim[p];
  int x[MAXN - 2] = {};
  double sum = 0.0;
  for (long long q = 0; q < total; ++q) {
    double v = 1.0;
#pragma unroll
    for (int p = 0; p < MAXN - 2; ++p) {
      if (p < a.nr) {
        const double f = w_at(a.W64, a.ek[p], j, x[p]) * w_at(a.W64, a.ei[p], y, x[p]);
        v *= f * f;
      }
    }
    for (int t = 0; t < a.npr; ++t) {
      const double f = w_at(a.W64, a.ep[t], x[a.pa[t]], x[a.pb[t]]);
      v *= f * f;
    }
    sum += v;
#pragma unroll
    for (int p = MAXN - 3; p >= 0; --p) {       // advance the counter
      if (p < a.nr) {
        if (++x[p] < a.rdim[p]) break;
        x[p] = 0;
      }
    }
  }
  a.c[e] = sum;
}

// --------------------------------------------------------------------------
// Solve of one column j (one wave): b_j, H_j + rho I in LDS, Cholesky
// H = L L^T (right-looking, one row per lane), L y = b, L^T g = y; then G_{k,i}
// column j, ||g - g_old||^2 and row j of W_{k,i} = G_{k,i}^T G_{i,k}.
// --------------------------------------------------------------------------
constexpr int LS_NT = 64;

template <typename TC>
__global__ __launch_bounds__(LS_NT) void k_lr_solve(LrSolveArgs a) {
  if (a.stop && *a.stop) return;
  __shared__ double Hs[LR_MAXR][LR_MAXR + 1];
  __shared__ double gl[MAXN][LR_MAXR];
  __shared__ double gold[LR_MAXR];
  __shared__ double vs[LR_MAXR];
  __shared__ double red[LS_NT];
  const int lane = threadIdx.x;
  const int j = blockIdx.x;
  const int R = a.R, Ik = a.Ik;
  for (int p = 0; p < a.nr; ++p)
    for (int r = lane; r < a.urank[p]; r += LS_NT) gl[p][r] = a.G[a.goff_o[p] + (long long)r * Ik + j];
  if (lane < R) gold[lane] = a.G[a.goff_ki + (long long)lane * Ik + j];
  // H_j + rho I from the packed pairs p(r, r') = r R - r (r - 1) / 2 + (r' - r)
  const int P = R * (R + 1) / 2;
  const double* Hj = a.H + (long long)j * P;
  for (int e = lane; e < R * R; e += LS_NT) {
    const int r = e / R, rr = e - r * R;
    const int lo = min(r, rr), hi = max(r, rr);
    Hs[r][rr] = Hj[lo * R - lo * (lo - 1) / 2 + (hi - lo)] + (r == rr ? a.rho : 0.0);
  }
  __syncthreads();
  // b_j(r) + rho g_old(r): lane r sums U_k(j, r, .) against the other g columns
  double v = 0.0;
  if (lane < R) {
    long long total = 1;
    for (int p = 0; p < a.nr; ++p) total *= a.urank[p];
    int x[MAXN - 2] = {};
    const double* Ur = a.U + (long long)j * a.ustr_j + (long long)lane * a.ustr_i;
    for (long long q = 0; q < total; ++q) {
      double w = 1.0;
      long long off = 0;
#pragma unroll
      for (int p = 0; p < MAXN - 2; ++p)
        if (p < a.nr) {
          w *= gl[p][x[p]];
          off += (long long)x[p] * a.ustr[p];
        }
      v += Ur[off] * w;
#pragma unroll
      for (int p = MAXN - 3; p >= 0; --p) {
        if (p < a.nr) {
          if (++x[p] < a.urank[p]) break;
          x[p] = 0;
        }
      }
    }
    v += a.rho * gold[lane];
  }
  // Cholesky: step c scales column c below the diagonal, then lane r > c
  // updates row r of the trailing matrix
  for (int c = 0; c < R; ++c) {
    const double d = sqrt(Hs[c][c]);
    const double lrc = lane > c && lane < R ? Hs[lane][c] / d : 0.0;
    __syncthreads();
    if (lane == c) Hs[c][c] = d;
    if (lane > c && lane < R) Hs[lane][c] = lrc;
    __syncthreads();
    if (lane > c && lane < R)
      for (int rr = c + 1; rr <= lane; ++rr) Hs[lane][rr] -= lrc * Hs[rr][c];
    __syncthreads();
  }
  // forward substitution, lane r holding entry r of the right-hand side
  for (int c = 0; c < R; ++c) {
    if (lane == c) vs[c] = v / Hs[c][c];
    __syncthreads();
    if (lane > c && lane < R) v -= Hs[lane][c] * vs[c];
  }
  __syncthreads();
  if (lane < R) v = vs[lane];
  // back substitution with L^T
  for (int c = R - 1; c >= 0; --c) {
    if (lane == c) vs[c] = v / Hs[c][c];
    __syncthreads();
    if (lane < c) v -= Hs[c][lane] * vs[c];
  }
  __syncthreads();
  double dg = 0.0;
  if (lane < R) {
    const double g = vs[lane];
    a.G[a.goff_ki + (long long)lane * Ik + j] = g;
    const double d = g - gold[lane];
    dg = d * d;
  }
  red[lane] = dg;
  __syncthreads();
  if (lane == 0) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += red[r];
    a.dgpart[j] = s;
  }
  // row j of W_{k,i}
  const double* Gik = a.G + a.goff_ik;
  for (int y = lane; y < a.Ii; y += LS_NT) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += vs[r] * Gik[(long long)r * a.Ii + y];
    const long long o = a.w.off + (long long)j * a.w.s1 + (long long)y * a.w.s2;
    a.W64[o] = s;
    ((TC*)a.Wc)[o] = (TC)s;
  }
}

// --------------------------------------------------------------------------
// X step (eq. (updateX)) with Xhat = prod over the edges of W_ab(i_a, i_b),
// grid-stride over a fixed grid; each workgroup writes its three partial sums
// --------------------------------------------------------------------------
template <typename TX>
__global__ __launch_bounds__(NT) void k_lr_x(LrXArgs a) {
  if (a.stop && *a.stop) return;
  __shared__ double red[NT / 64][3];
  TX* X = (TX*)a.X;
  double dx2 = 0.0, x2 = 0.0, f2 = 0.0;
  for (long long L = (long long)blockIdx.x * NT + threadIdx.x; L < a.nX; L += (long long)gridDim.x * NT) {
    int idx[MAXN];
    long long t = L;
    for (int m = a.N - 1; m >= 0; --m) {
      idx[m] = (int)(t % a.dims[m]);
      t /= a.dims[m];
    }
    double xh = 1.0;
    for (int e = 0; e < a.ne; ++e) xh *= a.W64[a.woff[e] + (long long)idx[a.ea[e]] * a.dims[a.eb[e]] + idx[a.eb[e]]];
    const TX x = X[L];
    const bool obs = (a.bits[L >> 5] >> (L & 31)) & 1u;
    const TX xn = obs ? x : (TX)((xh + a.rx * (double)x) * a.inv1);
    if (!obs) X[L] = xn;
    const double d = (double)xn - (double)x;
    dx2 += d * d;
    x2 += (double)x * (double)x;
    const double rr = (double)xn - xh;
    f2 += rr * rr;
  }
  for (int o = 32; o > 0; o >>= 1) {
    dx2 += __shfl_down(dx2, o, 64);
    x2 += __shfl_down(x2, o, 64);
    f2 += __shfl_down(f2, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w][0] = dx2;
    red[w][1] = x2;
    red[w][2] = f2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int q = 0; q < NT / 64; ++q) s += red[q][threadIdx.x];
    a.normpart[(long long)blockIdx.x * 3 + threadIdx.x] = s;
  }
}

unsigned cdivu(long long n, int d) { return (unsigned)((n + d - 1) / d); }

}  // namespace

hipError_t launch_lr_y(int dtype, const LrYArgs& a, hipStream_t s) {
  if (a.nX <= 0) return hipSuccess;
  if (dtype)
    hipLaunchKernelGGL(k_lr_y<double>, dim3(cdivu(a.nX, NT)), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL(k_lr_y<float>, dim3(cdivu(a.nX, NT)), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lr_gemm(const LrGemmArgs& a, hipStream_t s) {
  const long long M = a.A * a.Bn;
  if (M <= 0 || a.Nn <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lr_gemm, dim3(cdivu(M, LG_TM), cdivu(a.Nn, LG_TN)), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lr_c(const LrCArgs& a, hipStream_t s) {
  const long long n = (long long)a.Ik * a.Ii;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lr_c, dim3(cdivu(n, NT)), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lr_solve(const LrSolveArgs& a, hipStream_t s) {
  if (a.Ik <= 0) return hipSuccess;
  if (a.dtype)
    hipLaunchKernelGGL(k_lr_solve<double>, dim3((unsigned)a.Ik), dim3(LS_NT), 0, s, a);
  else
    hipLaunchKernelGGL(k_lr_solve<float>, dim3((unsigned)a.Ik), dim3(LS_NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lr_x(int dtype, const LrXArgs& a, int nblk, hipStream_t s) {
  if (dtype)
    hipLaunchKernelGGL(k_lr_x<double>, dim3((unsigned)nblk), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL(k_lr_x<float>, dim3((unsigned)nblk), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace ifctn
