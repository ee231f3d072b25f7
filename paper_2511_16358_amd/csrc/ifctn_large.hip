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

// An empty register pin: the value counts as used here, so the compiler
// cannot sink the load that produced it into a later conditional (which would
// make every load of a batch wait for the one before it).
__device__ __forceinline__ double pin(double v) {
  asm volatile("" : "+v"(v));
  return v;
}

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
  unsigned t = (unsigned)L;                  // nX < 2^31
  for (int m = a.N - 1; m >= 0; --m) {
    const unsigned d = (unsigned)a.dims[m], q = t / d;
    idx[m] = (int)(t - q * d);
    t = q;
  }
  double v = (double)((const TX*)a.X)[L];
  for (int e = 0; e < a.ne; ++e) v *= a.W64[a.woff[e] + (long long)idx[a.ea[e]] * a.dims[a.eb[e]] + idx[a.eb[e]]];
  a.Y[L] = v;
}

// --------------------------------------------------------------------------
// out[a][n][b] = sum_x in[a][x][b] B(n, x): 64 rows (a, b) x 32 columns n per
// workgroup, x in chunks of 64 staged through LDS (padded rows: no bank
// conflicts on either the stores or the reads).  Each thread stages 16 A and
// 8 B values per chunk, all loads of the next chunk in flight while the
// current one is multiplied; it keeps 8 accumulators (one row, 8 columns).
// --------------------------------------------------------------------------
constexpr int LG_TM = 64, LG_TN = 32, LG_TK = 64;
constexpr int LG_AV = LG_TM * LG_TK / NT, LG_BV = LG_TN * LG_TK / NT;   // 16 and 8 values per thread

// WIDE: Bn > 1 (rows (a, b) adjacent in b); PAIR: B(n, x) is a Gram pair.
// Every staging load is unconditional at a clamped index (out-of-range
// values are replaced by zero afterwards), so a thread's 24 loads are all in
// flight together.
template <bool WIDE, bool PAIR>
__global__ __launch_bounds__(NT) void k_lr_gemm(LrGemmArgs a) {
  if (a.stop && *a.stop) return;
  __shared__ double As[LG_TK][LG_TM + 1];
  __shared__ __align__(16) double Bs[LG_TK][LG_TN + 2];
  __shared__ int pr[LG_TN];
  const int tid = threadIdx.x;
  const long long M = a.A * a.Bn;
  const long long m0 = (long long)blockIdx.x * LG_TM;
  const int n0 = blockIdx.y * LG_TN;
  if (tid < LG_TN) {
    int n = min(n0 + tid, a.Nn - 1), r = 0;
    if (PAIR) {
      while (n >= a.pairR - r) {
        n -= a.pairR - r;
        ++r;
      }
      pr[tid] = r | ((r + n) << 8);
    } else {
      pr[tid] = n;
    }
  }
  __syncthreads();
  // A staging: WIDE -- one row per thread (adjacent lanes, adjacent b) and
  // x = (tid >> 6) + 4 q; otherwise x = tid & 63 (adjacent lanes, adjacent x)
  // and rows (tid >> 6) + 4 q
  long long wbase = 0;
  if (WIDE) {
    const long long mc = min(m0 + (tid & 63), M - 1);
    const long long aa = mc / a.Bn, b = mc - aa * a.Bn;
    wbase = aa * a.I * a.Bn + b;
  }
  const int bx = tid & 63, bn = tid >> 6;
  int brow0[LG_BV], brow1[LG_BV];
#pragma unroll
  for (int q = 0; q < LG_BV; ++q) {
    const int rp = pr[bn + 4 * q];
    brow0[q] = PAIR ? (rp & 255) : rp;
    brow1[q] = PAIR ? (rp >> 8) : rp;
  }
  double av[LG_AV], bv[LG_BV];
  // A at clamped indices, used as loaded: rows past M only feed outputs that
  // are not stored, and x past I meets a zero of B
  auto load = [&](int x0) {
#pragma unroll
    for (int q = 0; q < LG_AV; ++q) {
      if (WIDE) {
        const int x = x0 + (tid >> 6) + 4 * q;
        av[q] = a.in[wbase + (long long)min(x, a.I - 1) * a.Bn];
      } else {
        const long long m = m0 + (tid >> 6) + 4 * q;
        const int x = x0 + (tid & 63);
        av[q] = a.in[min(m, M - 1) * a.I + min(x, a.I - 1)];
      }
    }
    const int xc = min(x0 + bx, a.I - 1);
    double b1[LG_BV];
#pragma unroll
    for (int q = 0; q < LG_BV; ++q) {
      bv[q] = a.Bm[(long long)brow0[q] * a.ldb + xc];
      if (PAIR) b1[q] = a.Bm[(long long)brow1[q] * a.ldb + xc];
    }
    const bool xin = x0 + bx < a.I;
#pragma unroll
    for (int q = 0; q < LG_BV; ++q) {
      double v = pin(bv[q]);
      if (PAIR) v *= pin(b1[q]);
      bv[q] = xin ? v : 0.0;
    }
  };
  const int mm = tid & 63, ng = tid >> 6;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  load(0);
  for (int x0 = 0; x0 < a.I; x0 += LG_TK) {
#pragma unroll
    for (int q = 0; q < LG_AV; ++q) {
      if (WIDE)
        As[(tid >> 6) + 4 * q][tid & 63] = av[q];
      else
        As[tid & 63][(tid >> 6) + 4 * q] = av[q];
    }
#pragma unroll
    for (int q = 0; q < LG_BV; ++q) Bs[bx][bn + 4 * q] = bv[q];
    __syncthreads();
    if (x0 + LG_TK < a.I) load(x0 + LG_TK);
    // B zero past I: whole chunks, four x per step with every LDS read of the
    // step issued before its multiply-adds
    for (int xx = 0; xx < LG_TK; xx += 4) {
      double va[4];
      double2 vb[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        va[u] = As[xx + u][mm];
        const double2* br = reinterpret_cast<const double2*>(&Bs[xx + u][ng * 8]);
#pragma unroll
        for (int h = 0; h < 4; ++h) vb[u][h] = br[h];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          acc[2 * h] += va[u] * vb[u][h].x;
          acc[2 * h + 1] += va[u] * vb[u][h].y;
        }
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
// c(j, y) = sum_x A(j, x) B(y, x) over the flat index x of the other modes,
// A(j, x) = prod_p W_kp(j, x_p)^2 prod_{p<q} W_pq(x_p, x_q)^2 and
// B(y, x) = prod_p W_ip(y, x_p)^2.  One workgroup per (j, 64 values of y):
// A(j, .) is staged in LDS in chunks; thread (y, s) sums x = s, s + ks, ...
// of each chunk with its loads issued eight at a time, and the ks slices of
// each y are added in order.
// --------------------------------------------------------------------------
constexpr int LC_CH = 2048, LC_NY = 64;

// NR = N - 2 other modes (a template parameter, so every load below is
// unconditional and a batch of them is in flight together)
template <int NR>
__device__ __forceinline__ void lr_decode(const LrCArgs& a, long long x, int* xp) {
#pragma unroll
  for (int p = NR - 1; p >= 0; --p) {
    xp[p] = (int)(x % a.rdim[p]);
    x /= a.rdim[p];
  }
}

template <int NR>
__global__ __launch_bounds__(NT) void k_lr_c(LrCArgs a) {
  if (a.stop && *a.stop) return;
  __shared__ double Ash[LC_CH];
  __shared__ double part[NT];
  const int tid = threadIdx.x;
  const int j = blockIdx.x;
  const int ny = min(a.Ii, LC_NY), ks = NT / ny;
  const int yl = tid % ny, s = tid / ny;
  const int y = blockIdx.y * LC_NY + yl;
  const bool live = s < ks && y < a.Ii;
  const int yc = min(y, a.Ii - 1);
  constexpr int NPR = NR * (NR - 1) / 2;
  long long K = 1;
#pragma unroll
  for (int p = 0; p < NR; ++p) K *= a.rdim[p];
  double sum = 0.0;
  for (long long x0 = 0; x0 < K; x0 += LC_CH) {
    const int n = (int)min((long long)LC_CH, K - x0);
    __syncthreads();
    for (int e = tid; e < n; e += NT) {
      int xp[NR > 0 ? NR : 1];
      lr_decode<NR>(a, x0 + e, xp);
      double f[NR + NPR > 0 ? NR + NPR : 1];
#pragma unroll
      for (int p = 0; p < NR; ++p) f[p] = w_at(a.W64, a.ek[p], j, xp[p]);
#pragma unroll
      for (int t = 0; t < NPR; ++t) f[NR + t] = w_at(a.W64, a.ep[t], xp[a.pa[t]], xp[a.pb[t]]);
      double v = 1.0;
#pragma unroll
      for (int q = 0; q < NR + NPR; ++q) v *= f[q] * f[q];
      Ash[e] = v;
    }
    __syncthreads();
    if (live) {
      for (int e0 = s; e0 < n; e0 += 8 * ks) {
        double bv[8][NR > 0 ? NR : 1];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          int xp[NR > 0 ? NR : 1];
          lr_decode<NR>(a, x0 + min(e0 + u * ks, n - 1), xp);
#pragma unroll
          for (int p = 0; p < NR; ++p) bv[u][p] = w_at(a.W64, a.ei[p], yc, xp[p]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          double b = 1.0;
#pragma unroll
          for (int p = 0; p < NR; ++p) {
            const double f = pin(bv[u][p]);
            b *= f * f;
          }
          if (e0 + u * ks < n) sum += Ash[e0 + u * ks] * b;
        }
      }
    }
  }
  part[tid] = sum;
  __syncthreads();
  if (live && s == 0) {
    double t = 0.0;
    for (int q = 0; q < ks; ++q) t += part[q * ny + yl];
    a.c[(long long)j * a.Ii + y] = t;
  }
}

// --------------------------------------------------------------------------
// Solve of one column j (one wave): b_j and H_j + rho I in LDS, Cholesky
// H = L L^T in place, L y = b and L^T g = y with lane r holding entry r of
// the right-hand side (pivots broadcast with readlane); finally G_{k,i}
// column j and ||g - g_old||^2 (W_{k,i} is refreshed by the edge kernel).
// --------------------------------------------------------------------------
constexpr int LS_NT = 64;

__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__global__ __launch_bounds__(LS_NT) void k_lr_solve(LrSolveArgs a) {
  if (a.stop && *a.stop) return;
  __shared__ double Hs[LR_MAXR][LR_MAXR + 1];
  __shared__ double gl[MAXN][LR_MAXR];
  __shared__ double gold[LR_MAXR];
  __shared__ double vs[LR_MAXR];
  __shared__ double dinv[LR_MAXR];       // 1 / L(c, c)
  __shared__ double red[LS_NT];
  const int lane = threadIdx.x;
  const int j = blockIdx.x;
  const int R = a.R, Ik = a.Ik;
  {
    // the other g columns (ranks <= 36 < 64: one entry per lane and mode) and
    // the old column, loaded together
    double gv[MAXN - 1];
#pragma unroll
    for (int p = 0; p < MAXN - 2; ++p) {
      // modes past nr (none at all for N = 2) re-read a valid entry, unused
      const int pc = min(p, max(a.nr - 1, 0));
      const long long base = a.nr > 0 ? a.goff_o[pc] : a.goff_ki;
      const int rmax = a.nr > 0 ? a.urank[pc] : R;
      gv[p] = a.G[base + (long long)min(lane, rmax - 1) * Ik + j];
    }
    gv[MAXN - 2] = a.G[a.goff_ki + (long long)min(lane, R - 1) * Ik + j];
#pragma unroll
    for (int p = 0; p < MAXN - 2; ++p) {
      const double v = pin(gv[p]);
      if (p < a.nr && lane < a.urank[p]) gl[p][lane] = v;
    }
    const double v = pin(gv[MAXN - 2]);
    if (lane < R) gold[lane] = v;
  }
  // H_j + rho I from the packed pairs p(r, r') = r R - r (r - 1) / 2 + (r' - r)
  const int P = R * (R + 1) / 2;
  const double* Hj = a.H + (long long)j * P;
  for (int e0 = lane; e0 < P; e0 += 8 * LS_NT) {
    double hv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) hv[u] = Hj[min(e0 + u * LS_NT, P - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) hv[u] = pin(hv[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      int pp = e0 + u * LS_NT;
      if (pp < P) {
        int r = 0;
        while (pp >= R - r) {
          pp -= R - r;
          ++r;
        }
        const int rr = r + pp;
        Hs[r][rr] = hv[u] + (r == rr ? a.rho : 0.0);
        Hs[rr][r] = hv[u] + (r == rr ? a.rho : 0.0);
      }
    }
  }
  __syncthreads();
  // b_j(r) + rho g_old(r): lane r sums U_k(j, r, .) against the other g
  // columns, eight loads of U in flight at a time
  double v = 0.0;
  if (lane < R) {
    long long total = 1;
    for (int p = 0; p < a.nr; ++p) total *= a.urank[p];
    const double* Ur = a.U + (long long)j * a.ustr_j + (long long)lane * a.ustr_i;
    for (long long q0 = 0; q0 < total; q0 += 8) {
      double uv[8], wv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        long long q = min(q0 + u, total - 1), off = 0;
        double w = q0 + u < total ? 1.0 : 0.0;
#pragma unroll
        for (int p = MAXN - 3; p >= 0; --p)
          if (p < a.nr) {
            const int x = (int)(q % a.urank[p]);
            q /= a.urank[p];
            w *= gl[p][x];
            off += (long long)x * a.ustr[p];
          }
        uv[u] = Ur[off];
        wv[u] = w;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) v += uv[u] * wv[u];
    }
    v += a.rho * gold[lane];
  }
  // Cholesky H = L L^T, left-looking, L over the lower triangle of Hs: at
  // step c lane r >= c forms H(r, c) - sum_{q<c} L(r, q) L(c, q) (four partial
  // sums over q mod 4, added in a fixed order: a quarter of the dependent
  // chain), lane c's value gives L(c, c).  One wave: its LDS accesses complete
  // in issue order, so the column written at step c is what every lane reads
  // at step c + 1.
  for (int c = 0; c < R; ++c) {
    double t = 0.0;
    if (lane >= c && lane < R) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int q = 0;
      for (; q + 4 <= c; q += 4) {
        s0 += Hs[lane][q] * Hs[c][q];
        s1 += Hs[lane][q + 1] * Hs[c][q + 1];
        s2 += Hs[lane][q + 2] * Hs[c][q + 2];
        s3 += Hs[lane][q + 3] * Hs[c][q + 3];
      }
      for (; q < c; ++q) s0 += Hs[lane][q] * Hs[c][q];
      t = Hs[lane][c] - ((s0 + s1) + (s2 + s3));
    }
    const double d = sqrt(lane_bcast(t, c));
    const double id = 1.0 / d;
    if (lane > c && lane < R) Hs[lane][c] = t * id;
    if (lane == c) {
      Hs[c][c] = d;
      dinv[c] = id;
    }
  }
  // L y = b: y_c = v_c / L(c, c), then lanes r > c subtract L(r, c) y_c
  for (int c = 0; c < R; ++c) {
    const double lrc = lane > c && lane < R ? Hs[lane][c] : 0.0;
    const double yc = lane_bcast(v, c) * dinv[c];
    if (lane == c) v = yc;
    if (lane > c) v -= lrc * yc;
  }
  // L^T g = y: g_c = v_c / L(c, c), then lanes r < c subtract L(c, r) g_c
  for (int c = R - 1; c >= 0; --c) {
    const double lcr = lane < c ? Hs[c][lane] : 0.0;
    const double gc = lane_bcast(v, c) * dinv[c];
    if (lane == c) v = gc;
    if (lane < c) v -= lcr * gc;
  }
  if (lane < R) vs[lane] = v;
  __syncthreads();
  double dg = 0.0;
  if (lane < R) {
    a.G[a.goff_ki + (long long)lane * Ik + j] = v;
    const double d = v - gold[lane];
    dg = d * d;
  }
  red[lane] = dg;
  __syncthreads();
  if (lane == 0) {
    double t = 0.0;
    for (int r = 0; r < R; ++r) t += red[r];
    a.dgpart[j] = t;
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
    unsigned t = (unsigned)L;                // nX < 2^31
    for (int m = a.N - 1; m >= 0; --m) {
      const unsigned d = (unsigned)a.dims[m], q = t / d;
      idx[m] = (int)(t - q * d);
      t = q;
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
    IFCTN_GO(k_lr_y<double>, dim3(cdivu(a.nX, NT)), dim3(NT), 0, s, a);
  else
    IFCTN_GO(k_lr_y<float>, dim3(cdivu(a.nX, NT)), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lr_gemm(const LrGemmArgs& a, hipStream_t s) {
  const long long M = a.A * a.Bn;
  if (M <= 0 || a.Nn <= 0) return hipSuccess;
  const dim3 grid(cdivu(M, LG_TM), cdivu(a.Nn, LG_TN));
  if (a.Bn > 1) {
    if (a.pairR > 0)
      IFCTN_GO((k_lr_gemm<true, true>), grid, dim3(NT), 0, s, a);
    else
      IFCTN_GO((k_lr_gemm<true, false>), grid, dim3(NT), 0, s, a);
  } else {
    if (a.pairR > 0)
      IFCTN_GO((k_lr_gemm<false, true>), grid, dim3(NT), 0, s, a);
    else
      IFCTN_GO((k_lr_gemm<false, false>), grid, dim3(NT), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_lr_c(const LrCArgs& a, hipStream_t s) {
  if ((long long)a.Ik * a.Ii <= 0) return hipSuccess;
  const dim3 grid((unsigned)a.Ik, cdivu(a.Ii, LC_NY));
  switch (a.nr) {
    case 0: IFCTN_GO(k_lr_c<0>, grid, dim3(NT), 0, s, a); break;
    case 1: IFCTN_GO(k_lr_c<1>, grid, dim3(NT), 0, s, a); break;
    case 2: IFCTN_GO(k_lr_c<2>, grid, dim3(NT), 0, s, a); break;
    default: IFCTN_GO(k_lr_c<3>, grid, dim3(NT), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_lr_solve(const LrSolveArgs& a, hipStream_t s) {
  if (a.Ik <= 0) return hipSuccess;
  IFCTN_GO(k_lr_solve, dim3((unsigned)a.Ik), dim3(LS_NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_lr_x(int dtype, const LrXArgs& a, int nblk, hipStream_t s) {
  if (dtype)
    IFCTN_GO(k_lr_x<double>, dim3((unsigned)nblk), dim3(NT), 0, s, a);
  else
    IFCTN_GO(k_lr_x<float>, dim3((unsigned)nblk), dim3(NT), 0, s, a);
  return hipGetLastError();
}

}  // namespace ifctn
