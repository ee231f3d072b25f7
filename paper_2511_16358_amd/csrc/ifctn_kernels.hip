// HIP kernels of the iFCTN-TC PAM sweep for gfx950 (CDNA4, wave64).
//
// Paper: "iFCTN: an intra-block Fully-Connected Tensor Network Decomposition
// for Tensor Completion" (arXiv 2511.16358).  The kernels evaluate
//   - the edge matrices G_{a,b}^T G_{b,a} from which Prop. 1 builds S_k,
//   - the mode-k contraction of X against the cherry sub-network Z_k
//     (Prop. 1: X_(k)^T = Z_k G_(k)^T), which supplies the right-hand sides
//     of eq. (updateG) for every i != k at once,
//   - the Gram weights and the FP64 Cholesky solves of eq. (updateG),
//   - the reconstruction of eq. (iFCTN) fused with the X step eq. (updateX)
//     and the reductions of the stop test of Algorithm 1.
// Reductions are fixed-order (no floating-point atomics), so every launch is
// bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ifctn_internal.h"

namespace ifctn {

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  // fixed butterfly order: every run adds the same operands in the same order
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T ld(const T* p, long long i) {
  return p[i];
}

__device__ __forceinline__ long long eaddr(const EdgeRef& e, long long a, long long b) {
  return e.off + a * e.s1 + b * e.s2;
}

// --------------------------------------------------------------------------
// K1: X^0 = P_Omega(O), packed mask bits, finiteness check of observed data
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_init_x(const T* __restrict__ O, const uint8_t* __restrict__ mask,
                                               T* __restrict__ X, uint32_t* __restrict__ bits,
                                               int* __restrict__ bad, long long nX) {
  const long long L = (long long)blockIdx.x * NT + threadIdx.x;
  bool obs = false;
  if (L < nX) {
    obs = mask[L] != 0;
    T v = O[L];
    if (obs && !isfinite((double)v)) atomicOr(bad, 1);   // integer flag, order-free
    X[L] = obs ? v : T(0);
  }
  const unsigned long long b = __ballot(obs);
  const int lane = threadIdx.x & 63;
  const long long w0 = (L - lane) >> 5;          // wave covers 64 aligned entries = 2 words
  const long long nw = (nX + 31) >> 5;
  if (lane == 0 && w0 < nw) bits[w0] = (uint32_t)(b & 0xffffffffu);
  if (lane == 0 && w0 + 1 < nw) bits[w0 + 1] = (uint32_t)(b >> 32);
}

// --------------------------------------------------------------------------
// K2: edge matrix W_ab(x, y) = sum_r G_ab(r, x) G_ba(r, y)   (a < b)
// --------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(NT) void k_edge(const double* __restrict__ Gab, const double* __restrict__ Gba,
                                             int R, int Ia, int Ib, double* __restrict__ W64,
                                             TC* __restrict__ Wc) {
  const long long e = (long long)blockIdx.x * NT + threadIdx.x;
  if (e >= (long long)Ia * Ib) return;
  const int x = (int)(e / Ib), y = (int)(e - (long long)x * Ib);
  double s = 0.0;
  for (int r = 0; r < R; ++r) s += Gab[(long long)r * Ia + x] * Gba[(long long)r * Ib + y];
  W64[e] = s;
  Wc[e] = (TC)s;
}

// --------------------------------------------------------------------------
// K3 (+ K6): mode-k contraction, optionally fused with the X step of the
// previous sweep.
//
// A workgroup owns j-tile [j0, j0+jn) of mode k and a range of planes.  Per
// batch of PB planes it
//   (a) decodes the planes, forms S_k's plane-constant part and the
//       Kronecker coefficients a_c(r_c) = prod_{m in c} G_{m,k}(r_m, i_m),
//   (b) streams the X elements of the batch from HBM (optionally applying
//       eq. (updateX) first and writing X back), multiplies by S_k and
//       stages Y = X * S_k in LDS,
//   (c) contracts the fibre mode: T(j, r_f) = sum_{i_f} Y(j, i_f) G_{f,k}(r_f, i_f),
//   (d) accumulates U(j, r_c, r_f) += a_c(r_c) T(j, r_f) into float64
//       registers; each (j, r) slot is owned by one thread.
// The Khatri-Rao / Kronecker expansion of Z_k is never materialised.
// --------------------------------------------------------------------------
struct CLayout {
  size_t pbase, pidx, acoef, scc, scf, t0, tile, T, gf, red, total;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline CLayout clayout(int tcsz, const ContractArgs& a) {
  CLayout L;
  size_t o = 0;
  L.pbase = o; o = al16(o + (size_t)a.PB * 8);
  L.pidx = o;  o = al16(o + (size_t)a.PB * MAXC * 4);
  L.acoef = o; o = al16(o + (size_t)a.PB * a.Rc * 8);
  L.scc = o;   o = al16(o + (size_t)a.PB * tcsz);
  L.scf = o;   o = al16(o + (size_t)a.PB * a.LDF * tcsz);
  L.t0 = o;    o = al16(o + (size_t)a.PB * a.jn * tcsz);
  L.tile = o;  o = al16(o + (size_t)a.PB * a.jn * a.LDF * tcsz);
  L.T = o;     o = al16(o + (size_t)a.PB * a.jn * a.Rf * tcsz);
  L.gf = o;    o = al16(o + (size_t)a.If * a.Rf * tcsz);
  L.red = o;   o = al16(o + 4 * 3 * 8);
  L.total = o;
  return L;
}

template <typename TX, typename TC, bool UPD, bool CON, int SPT>
__global__ __launch_bounds__(NT) void k_contract(ContractArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const CLayout Ly = clayout((int)sizeof(TC), a);
  long long* pbase = (long long*)(smem + Ly.pbase);
  int* pidx = (int*)(smem + Ly.pidx);
  double* acoef = (double*)(smem + Ly.acoef);
  TC* sccl = (TC*)(smem + Ly.scc);
  TC* scf = (TC*)(smem + Ly.scf);
  TC* t0 = (TC*)(smem + Ly.t0);
  TC* tile = (TC*)(smem + Ly.tile);
  TC* Tl = (TC*)(smem + Ly.T);
  TC* gf = (TC*)(smem + Ly.gf);
  double* red = (double*)(smem + Ly.red);

  const int tid = threadIdx.x;
  const int jt = blockIdx.x % a.JT;
  const int sp = blockIdx.x / a.JT;
  const int j0 = jt * a.jn;
  const int jcnt = min(a.jn, a.Ik - j0);
  const long long p_begin = (long long)sp * a.PPW;
  const long long p_end = min(a.nplanes, p_begin + a.PPW);
  const TC* __restrict__ Wc = (const TC*)a.Wc;
  TX* __restrict__ X = (TX*)a.X;
  const double* __restrict__ G = a.G;
  const int If = a.If, Rf = a.Rf, Rc = a.Rc, Rprod = a.Rprod, nc = a.nc, jn = a.jn;

  double acc[SPT];
  int aoff[SPT], toff[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    acc[q] = 0.0;
    aoff[q] = -1;
    toff[q] = 0;
    if (CON) {
      const int s = q * NT + tid;
      if (s < jcnt * Rprod) {
        const int jl = s / Rprod, col = s - jl * Rprod;
        aoff[q] = col / Rf;
        toff[q] = jl * Rf + (col - (col / Rf) * Rf);
      }
    }
  }
  if (CON) {
    for (int e = tid; e < Rf * If; e += NT) {
      const int r = e / If, ff = e - r * If;
      gf[ff * Rf + r] = (TC)G[a.gfoff + e];
    }
  }
  double dx2 = 0.0, x2 = 0.0, f2 = 0.0;
  const TC rx = (TC)a.rho_x;
  const TC inv1 = (TC)1 / ((TC)1 + rx);

  for (long long pb0 = p_begin; pb0 < p_end; pb0 += a.PB) {
    const int np = (int)min((long long)a.PB, p_end - pb0);
    // (a) planes
    for (int e = tid; e < np; e += NT) {
      long long p = pb0 + e, base = 0;
      int ic[MAXC];
      for (int c = nc - 1; c >= 0; --c) {
        ic[c] = (int)(p % a.cdim[c]);
        p /= a.cdim[c];
        base += (long long)ic[c] * a.cstride[c];
      }
      TC s = (TC)1;
      for (int q = 0; q < a.ncc; ++q) s *= Wc[eaddr(a.ecc[q], ic[a.cc_a[q]], ic[a.cc_b[q]])];
      pbase[e] = base;
      sccl[e] = s;
      for (int c = 0; c < MAXC; ++c) pidx[e * MAXC + c] = c < nc ? ic[c] : 0;
    }
    __syncthreads();
    for (int e = tid; e < np * If; e += NT) {
      const int pl = e / If, ff = e - pl * If;
      TC s = sccl[pl];
      for (int c = 0; c < nc; ++c) s *= Wc[eaddr(a.ecf[c], pidx[pl * MAXC + c], ff)];
      scf[pl * a.LDF + ff] = s;
    }
    if (CON) {
      for (int e = tid; e < np * Rc; e += NT) {
        const int pl = e / Rc;
        int rr = e - pl * Rc;
        double v = 1.0;
        for (int c = nc - 1; c >= 0; --c) {
          const int r = rr % a.crank[c];
          rr /= a.crank[c];
          v *= G[a.gcoff[c] + (long long)r * a.cdim[c] + pidx[pl * MAXC + c]];
        }
        acoef[e] = v;
      }
    }
    if (UPD) {
      for (int e = tid; e < np * jcnt; e += NT) {
        const int pl = e / jcnt, jl = e - pl * jcnt;
        TC v = (TC)1;
        for (int c = 0; c < nc; ++c) v *= Wc[eaddr(a.e0c[c], j0 + jl, pidx[pl * MAXC + c])];
        t0[pl * jn + jl] = v;
      }
    }
    __syncthreads();

    // (b) stream X: the batch is enumerated over (D0, D1, D2) = extents of the
    // axes ord[0..2]; a carried mixed-radix counter avoids divisions
    {
      const int o0 = a.ord[0], o1 = a.ord[1], o2 = a.ord[2];
      const int D0 = o0 == 0 ? jcnt : (o0 == 1 ? np : If);
      const int D1 = o1 == 0 ? jcnt : (o1 == 1 ? np : If);
      const int D2 = o2 == 0 ? jcnt : (o2 == 1 ? np : If);
      const long long total = (long long)D0 * D1 * D2;
      const int s2 = NT % D2, s1 = (NT / D2) % D1, s0 = NT / (D1 * D2);
      int i2 = tid % D2, i1 = (tid / D2) % D1, i0 = tid / (D1 * D2);
      for (long long e = tid; e < total; e += NT) {
        const int jl = o0 == 0 ? i0 : (o1 == 0 ? i1 : i2);
        const int pl = o0 == 1 ? i0 : (o1 == 1 ? i1 : i2);
        const int ff = o0 == 2 ? i0 : (o1 == 2 ? i1 : i2);
        const long long L = pbase[pl] + (long long)(j0 + jl) * a.stride_k + (long long)ff * a.stride_f;
        TC x = (TC)X[L];
        const TC sk = scf[pl * a.LDF + ff];
        if (UPD) {
          const TC xh = sk * t0[pl * jn + jl] * Wc[eaddr(a.e0f, j0 + jl, ff)];
          const bool obs = (a.maskbits[L >> 5] >> (L & 31)) & 1u;
          const TC xn = obs ? x : (xh + rx * x) * inv1;
          if (!obs) X[L] = (TX)xn;
          const double d = (double)xn - (double)x;
          dx2 += d * d;
          x2 += (double)x * (double)x;
          const double rr = (double)xn - (double)xh;
          f2 += rr * rr;
          x = xn;
        }
        if (CON) tile[(pl * jn + jl) * a.LDF + ff] = x * sk;
        i2 += s2;
        if (i2 >= D2) { i2 -= D2; ++i1; }
        i1 += s1;
        if (i1 >= D1) { i1 -= D1; ++i0; }
        i0 += s0;
      }
    }
    __syncthreads();

    if (CON) {
      // (c) fibre contraction
      const int rows = np * jcnt;
      for (int row = tid; row < rows; row += NT) {
        const int pl = row / jcnt, jl = row - pl * jcnt;
        TC t[MAXR];
#pragma unroll
        for (int r = 0; r < MAXR; ++r) t[r] = (TC)0;
        const TC* trow = tile + (pl * jn + jl) * a.LDF;
        for (int ff = 0; ff < If; ++ff) {
          const TC v = trow[ff];
          const TC* g = gf + ff * Rf;
#pragma unroll
          for (int r = 0; r < MAXR; ++r)
            if (r < Rf) t[r] += v * g[r];
        }
#pragma unroll
        for (int r = 0; r < MAXR; ++r)
          if (r < Rf) Tl[(pl * jn + jl) * Rf + r] = t[r];
      }
      __syncthreads();
      // (d) Kronecker accumulation into owned slots
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        if (aoff[q] >= 0) {
          double s = acc[q];
          for (int pl = 0; pl < np; ++pl)
            s += acoef[pl * Rc + aoff[q]] * (double)Tl[pl * jn * Rf + toff[q]];
          acc[q] = s;
        }
      }
    }
    __syncthreads();
  }

  if (CON) {
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      if (aoff[q] >= 0) {
        const int s = q * NT + tid;
        const int jl = s / Rprod, sl = s - jl * Rprod;
        // slot (r_c, r_f) -> canonical U column (modes != k ascending, row-major)
        int rc = sl / Rf;
        long long col = (long long)(sl - rc * Rf) * a.ustf;
        for (int c = nc - 1; c >= 0; --c) {
          const int r = rc % a.crank[c];
          rc /= a.crank[c];
          col += (long long)r * a.ustc[c];
        }
        a.Upart[((long long)sp * a.Ik + j0 + jl) * Rprod + col] = acc[q];
      }
    }
  }
  if (UPD) {
    const double v0 = wave_sum(dx2), v1 = wave_sum(x2), v2 = wave_sum(f2);
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
      red[w * 3 + 0] = v0;
      red[w * 3 + 1] = v1;
      red[w * 3 + 2] = v2;
    }
    __syncthreads();
    if (tid < 3) {
      double s = 0.0;
      for (int q = 0; q < NT / 64; ++q) s += red[q * 3 + tid];
      a.normpart[(long long)blockIdx.x * 3 + tid] = s;
    }
  }
}

// --------------------------------------------------------------------------
// K4: Gram weights Q_{k,i} for every i != k of block k (float64).
// Work item = (d, fibre chunk); the lanes of one d are adjacent in a wave and
// reduce with a fixed butterfly.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_gram_q(QArgs a) {
  int ii = 0;
  while (ii + 1 < a.ni && (long long)blockIdx.x >= a.blk0[ii + 1]) ++ii;
  const long long item = ((long long)blockIdx.x - a.blk0[ii]) * NT + threadIdx.x;
  const int lg = a.lg2P[ii];
  const long long dd = item >> lg;
  const int ch = (int)(item & ((1 << lg) - 1));
  const int R = a.R[ii], np = a.np[ii], Ii = a.Ii[ii];
  const bool valid = dd < a.D[ii];
  double acc[MAXP];
#pragma unroll
  for (int p = 0; p < MAXP; ++p) acc[p] = 0.0;
  if (valid) {
    int im[MAXC];
    long long t = dd;
    for (int c = a.nd - 1; c >= 0; --c) {
      im[c] = (int)(t % a.ddim[ii][c]);
      t /= a.ddim[ii][c];
    }
    double sdd = 1.0;
    for (int q = 0; q < a.ndd; ++q) {
      const double w = a.W64[eaddr(a.edd[ii][q], im[a.dd_a[ii][q]], im[a.dd_b[ii][q]])];
      sdd *= w * w;
    }
    const int lo = ch * a.CH[ii], hi = min(Ii, lo + a.CH[ii]);
    const double* Gik = a.G + a.gik[ii];
    for (int x = lo; x < hi; ++x) {
      double w = sdd;
      for (int c = 0; c < a.nd; ++c) {
        const double v = a.W64[eaddr(a.edi[ii][c], im[c], x)];
        w *= v * v;
      }
      double g[MAXR];
#pragma unroll
      for (int r = 0; r < MAXR; ++r) g[r] = r < R ? Gik[(long long)r * Ii + x] : 0.0;
      // acc holds the upper triangle in a fixed MAXR layout (compile-time slots)
#pragma unroll
      for (int r = 0; r < MAXR; ++r) {
#pragma unroll
        for (int s = r; s < MAXR; ++s) acc[r * MAXR - r * (r - 1) / 2 + (s - r)] += w * g[r] * g[s];
      }
    }
  }
  for (int o = 1; o < (1 << lg); o <<= 1) {
#pragma unroll
    for (int p = 0; p < MAXP; ++p) acc[p] += __shfl_xor(acc[p], o, 64);
  }
  if (valid && ch == 0) {
    // packed upper triangle for the runtime rank: p(r, s) = r R - r (r - 1) / 2 + (s - r)
    double* q = a.Q + a.qoff[ii] + dd * np;
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
#pragma unroll
      for (int s = r; s < MAXR; ++s)
        if (s < R) q[r * R - r * (r - 1) / 2 + (s - r)] = acc[r * MAXR - r * (r - 1) / 2 + (s - r)];
    }
  }
}

// --------------------------------------------------------------------------
// K5: one factor block G_{k,i}, one workgroup per column j.
// --------------------------------------------------------------------------
constexpr int TD = 512;   // d-tile staged in LDS

__host__ __device__ inline size_t solve_layout(const SolveArgs& a, size_t* o_u, size_t* o_w, size_t* o_part,
                                               size_t* o_gk, size_t* o_misc) {
  size_t o = 0;
  *o_u = o;    o = al16(o + (size_t)a.Rprod * 8);
  *o_w = o;    o = al16(o + (size_t)TD * 8);
  *o_part = o; o = al16(o + (size_t)NT * 8);
  *o_gk = o;   o = al16(o + (size_t)(MAXN - 1) * MAXR * 8);
  *o_misc = o; o = al16(o + (size_t)(MAXP + 3 * MAXR + 8) * 8);
  return o;
}

template <typename TC>
__global__ __launch_bounds__(NT) void k_solve(SolveArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  size_t ou, ow, op, og, om;
  solve_layout(a, &ou, &ow, &op, &og, &om);
  double* u = (double*)(smem + ou);
  double* wl = (double*)(smem + ow);
  double* part = (double*)(smem + op);
  double* gk = (double*)(smem + og);
  double* Hs = (double*)(smem + om);
  double* bs = Hs + MAXP;
  double* gold = bs + MAXR;
  double* gnew = gold + MAXR;

  const int tid = threadIdx.x;
  const int j = blockIdx.x;
  const int R = a.R, np = a.np, Ik = a.Ik;
  double* G = a.G;

  // U_k row j: reduce the split partials in fixed order (first block of k)
  for (int col = tid; col < a.Rprod; col += NT) {
    double s;
    if (a.first) {
      s = 0.0;
      for (int q = 0; q < a.S; ++q) s += a.Upart[((long long)q * Ik + j) * a.Rprod + col];
      a.Ufin[(long long)j * a.Rprod + col] = s;
    } else {
      s = a.Ufin[(long long)j * a.Rprod + col];
    }
    u[col] = s;
  }
  // own-side factor columns G_{k,m}(:, j) for the U modes, and g_old
  for (int e = tid; e < a.nu * MAXR; e += NT) {
    const int t = e / MAXR, r = e - t * MAXR;
    gk[e] = (t != a.upos_i && r < a.urank[t]) ? G[a.ugoff[t] + (long long)r * Ik + j] : 0.0;
  }
  if (tid < R) gold[tid] = G[a.goff_ki + (long long)tid * Ik + j];

  // H_j = sum_d w_j(d) Q(d) over d-tiles; thread (p, c) sums d = c mod cpp
  const int cpp = NT / np;
  const int p_me = tid % np, c_me = tid / np;
  double hacc = 0.0;
  for (long long d0 = 0; d0 < a.D; d0 += TD) {
    const int nd_t = (int)min((long long)TD, a.D - d0);
    __syncthreads();
    for (int e = tid; e < nd_t; e += NT) {
      long long t = d0 + e;
      double w = 1.0;
      for (int c = a.nd - 1; c >= 0; --c) {
        const int im = (int)(t % a.ddim[c]);
        t /= a.ddim[c];
        const double v = a.W64[eaddr(a.ekd[c], j, im)];
        w *= v * v;
      }
      wl[e] = w;
    }
    __syncthreads();
    if (c_me < cpp) {
      for (int e = c_me; e < nd_t; e += cpp) hacc += wl[e] * a.Q[(d0 + e) * np + p_me];
    }
  }
  __syncthreads();
  part[tid] = (c_me < cpp) ? hacc : 0.0;
  __syncthreads();
  if (tid < np) {
    double s = 0.0;
    for (int c = 0; c < cpp; ++c) s += part[c * np + tid];
    Hs[tid] = s;
  }
  __syncthreads();

  // b_j(r_i) = sum over the other U indices of prod_{m != k,i} G_{k,m}(r_m, j) U(j, r)
  const int cpr = NT / R;
  const int r_me = tid % R, cb = tid / R;
  const int nother = a.Rprod / a.urank[a.upos_i];
  double bacc = 0.0;
  if (cb < cpr) {
    for (int o = cb; o < nother; o += cpr) {
      int rem = o;
      long long col = (long long)r_me * a.ustride[a.upos_i];
      double coef = 1.0;
      for (int t = a.nu - 1; t >= 0; --t) {
        if (t == a.upos_i) continue;
        const int r = rem % a.urank[t];
        rem /= a.urank[t];
        col += (long long)r * a.ustride[t];
        coef *= gk[t * MAXR + r];
      }
      bacc += coef * u[col];
    }
  }
  part[tid] = (cb < cpr) ? bacc : 0.0;
  __syncthreads();
  if (tid < R) {
    double s = 0.0;
    for (int c = 0; c < cpr; ++c) s += part[c * R + tid];
    bs[tid] = s + a.rho * gold[tid];
  }
  __syncthreads();

  // Cholesky solve of (H + rho I) g = b (R <= 8, one lane; unrolled over the
  // maximal rank so that the factor stays in registers)
  if (tid == 0) {
    double L[MAXR][MAXR];
#pragma unroll
    for (int r = 0; r < MAXR; ++r)
#pragma unroll
      for (int s = 0; s < MAXR; ++s) L[r][s] = 0.0;
#pragma unroll
    for (int r = 0; r < MAXR; ++r)
#pragma unroll
      for (int s = r; s < MAXR; ++s)
        if (s < R) L[s][r] = Hs[r * R - r * (r - 1) / 2 + (s - r)] + (r == s ? a.rho : 0.0);
#pragma unroll
    for (int c = 0; c < MAXR; ++c) {
      if (c < R) {
        double d = L[c][c];
#pragma unroll
        for (int q = 0; q < c; ++q) d -= L[c][q] * L[c][q];
        d = sqrt(d);
        L[c][c] = d;
#pragma unroll
        for (int r = c + 1; r < MAXR; ++r) {
          double v = L[r][c];
#pragma unroll
          for (int q = 0; q < c; ++q) v -= L[r][q] * L[c][q];
          L[r][c] = v / d;
        }
      }
    }
    double y[MAXR], x[MAXR];
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
      double v = r < R ? bs[r] : 0.0;
#pragma unroll
      for (int q = 0; q < r; ++q) v -= L[r][q] * y[q];
      y[r] = r < R ? v / L[r][r] : 0.0;
    }
#pragma unroll
    for (int r = MAXR - 1; r >= 0; --r) {
      double v = y[r];
#pragma unroll
      for (int q = r + 1; q < MAXR; ++q) v -= L[q][r] * x[q];
      x[r] = r < R ? v / L[r][r] : 0.0;
    }
    double dg = 0.0;
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
      if (r < R) {
        gnew[r] = x[r];
        const double dd = x[r] - gold[r];
        dg += dd * dd;
        G[a.goff_ki + (long long)r * Ik + j] = x[r];
      }
    }
    a.dgpart[j] = dg;
  }
  __syncthreads();

  // refresh the edge matrix of {k, i} for this column of G_{k,i}
  TC* Wc = (TC*)a.Wc;
  const double* Gik = G + a.goff_ik;
  for (int y = tid; y < a.Ii; y += NT) {
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += gnew[r] * Gik[(long long)r * a.Ii + y];
    const long long ad = a.w_off + (long long)j * a.w_sj + (long long)y * a.w_sy;
    a.W64[ad] = s;
    Wc[ad] = (TC)s;
  }
}

// --------------------------------------------------------------------------
// K8: dense reconstruction eq. (iFCTN) = product of all edge matrices
// --------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(NT) void k_reconstruct(ReconArgs a) {
  const long long L = (long long)blockIdx.x * NT + threadIdx.x;
  if (L >= a.nX) return;
  int idx[MAXN];
  long long t = L;
  for (int m = a.N - 1; m >= 0; --m) {
    idx[m] = (int)(t % a.dims[m]);
    t /= a.dims[m];
  }
  const TC* W = (const TC*)a.Wc;
  TC v = (TC)1;
  for (int e = 0; e < a.ne; ++e) v *= W[a.woff[e] + (long long)idx[a.ea[e]] * a.dims[a.eb[e]] + idx[a.eb[e]]];
  ((TC*)a.out)[L] = v;
}

// --------------------------------------------------------------------------
// K7: fixed-order finalisation of the sweep statistics
// out5 = {||dX||^2, ||X^s||^2, ||X^{s+1} - Xhat||^2, sum ||dG||^2, 0}
// --------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_finalize(const double* __restrict__ normpart, int nnorm,
                                                 const double* __restrict__ dgpart, int ndg,
                                                 double* __restrict__ out5) {
  __shared__ double s[4][NT];
  const int tid = threadIdx.x;
  double v[4] = {0, 0, 0, 0};
  for (int b = tid; b < nnorm; b += NT)
    for (int c = 0; c < 3; ++c) v[c] += normpart[(long long)b * 3 + c];
  for (int b = tid; b < ndg; b += NT) v[3] += dgpart[b];
  for (int c = 0; c < 4; ++c) s[c][tid] = v[c];
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int c = 0; c < 4; ++c) s[c][tid] += s[c][tid + w];
    __syncthreads();
  }
  if (tid < 4) out5[tid] = s[tid][0];
  if (tid == 4) out5[4] = 0.0;
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
static inline unsigned nblk(long long n) { return (unsigned)((n + NT - 1) / NT); }

hipError_t launch_init_x(int dtype, const void* O, const uint8_t* mask, void* X, uint32_t* bits, int* bad,
                         long long nX, hipStream_t s) {
  if (nX == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_init_x<float>, dim3(nblk(nX)), dim3(NT), 0, s, (const float*)O, mask, (float*)X,
                       bits, bad, nX);
  else
    hipLaunchKernelGGL(k_init_x<double>, dim3(nblk(nX)), dim3(NT), 0, s, (const double*)O, mask,
                       (double*)X, bits, bad, nX);
  return hipGetLastError();
}

hipError_t launch_edge(int dtype, const double* Gab, const double* Gba, int R, int Ia, int Ib, double* W64,
                       void* Wc, hipStream_t s) {
  const long long n = (long long)Ia * Ib;
  if (dtype == 0)
    hipLaunchKernelGGL(k_edge<float>, dim3(nblk(n)), dim3(NT), 0, s, Gab, Gba, R, Ia, Ib, W64, (float*)Wc);
  else
    hipLaunchKernelGGL(k_edge<double>, dim3(nblk(n)), dim3(NT), 0, s, Gab, Gba, R, Ia, Ib, W64, (double*)Wc);
  return hipGetLastError();
}

size_t contract_smem_bytes(int dtype, const ContractArgs& a) {
  return clayout(dtype == 0 ? 4 : 8, a).total;
}

template <typename TX, typename TC>
static hipError_t contract_dispatch(bool upd, bool con, int spt, const ContractArgs& a, size_t smem,
                                    hipStream_t s) {
  const dim3 grid((unsigned)(a.JT * a.S)), blk(NT);
#define IFCTN_CASE(U, C, P)                                                      \
  if (upd == U && con == C && spt == P) {                                        \
    hipLaunchKernelGGL((k_contract<TX, TC, U, C, P>), grid, blk, smem, s, a);    \
    return hipGetLastError();                                                    \
  }
  IFCTN_CASE(true, false, 1)
  IFCTN_CASE(false, true, 1) IFCTN_CASE(false, true, 2) IFCTN_CASE(false, true, 4)
  IFCTN_CASE(false, true, 8) IFCTN_CASE(false, true, 16) IFCTN_CASE(false, true, 32)
  IFCTN_CASE(true, true, 1) IFCTN_CASE(true, true, 2) IFCTN_CASE(true, true, 4)
  IFCTN_CASE(true, true, 8) IFCTN_CASE(true, true, 16) IFCTN_CASE(true, true, 32)
#undef IFCTN_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_contract(int dtype, bool upd, bool con, int spt, const ContractArgs& a, size_t smem,
                           hipStream_t s) {
  if (dtype == 0) return contract_dispatch<float, float>(upd, con, spt, a, smem, s);
  return contract_dispatch<double, double>(upd, con, spt, a, smem, s);
}

hipError_t launch_q(const QArgs& a, hipStream_t s) {
  if (a.blk0[a.ni] == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_q, dim3((unsigned)a.blk0[a.ni]), dim3(NT), 0, s, a);
  return hipGetLastError();
}

size_t solve_smem_bytes(const SolveArgs& a) {
  size_t o1, o2, o3, o4, o5;
  return solve_layout(a, &o1, &o2, &o3, &o4, &o5);
}

hipError_t launch_solve(int dtype, const SolveArgs& a, hipStream_t s) {
  const size_t smem = solve_smem_bytes(a);
  if (dtype == 0)
    hipLaunchKernelGGL(k_solve<float>, dim3((unsigned)a.Ik), dim3(NT), smem, s, a);
  else
    hipLaunchKernelGGL(k_solve<double>, dim3((unsigned)a.Ik), dim3(NT), smem, s, a);
  return hipGetLastError();
}

hipError_t launch_reconstruct(int dtype, const ReconArgs& a, hipStream_t s) {
  if (a.nX == 0) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_reconstruct<float>, dim3(nblk(a.nX)), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL(k_reconstruct<double>, dim3(nblk(a.nX)), dim3(NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* normpart, int nnorm, const double* dgpart, int ndg, double* out5,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(NT), 0, s, normpart, nnorm, dgpart, ndg, out5);
  return hipGetLastError();
}

}  // namespace ifctn
