// Device code shared by the translation units of libifctn.so: small helpers,
// the mode-k contraction kernels (templates over the X storage type and the
// streaming arithmetic type) and their launch dispatch.  Each contraction
// translation unit instantiates one type pair, so the library compiles in
// parallel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "ifctn_internal.h"

namespace ifctn {

// An empty register pin: the value counts as used where the pin stands, so
// the compiler cannot sink the load that produced it into a later
// conditional use (which would make each load of a batch wait for the
// previous one).  The loads of a batch are all issued before the first pin.
template <typename T>
__device__ __forceinline__ T pin(T v) {
  asm volatile("" : "+v"(v));
  return v;
}

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

__device__ __forceinline__ long long eaddr(const EdgeRef e, long long a, long long b) {
  return e.off + a * e.s1 + b * e.s2;
}

// --------------------------------------------------------------------------
// Gram weights Q_{k,i} (see k_gram_q)
// --------------------------------------------------------------------------
// Rows [R0, R1) of the packed upper triangle of Q(dd) for one d: every lane of
// a group of 2^lg lanes sums a chunk of the far-side mode x, the group adds its
// chunks by a fixed butterfly, and lane 0 of the group stores the entries.
// Splitting the rows over passes keeps the accumulators few, so that the
// contraction launch these workgroups ride in keeps its occupancy.
template <int R, int R0, int R1, int XU>
__device__ __forceinline__ void gram_rows(const double* __restrict__ W64, const double* __restrict__ Gik,
                                          double* __restrict__ q, int nd, const QItem& it, const int* im,
                                          double sdd, bool valid, int lo, int hi, int lg, int Ii, bool store) {
  constexpr int P0 = R0 * R - R0 * (R0 - 1) / 2;      // packed index of (R0, R0)
  constexpr int P1 = R1 * R - R1 * (R1 - 1) / 2;
  constexpr int NQ = P1 - P0;
  double acc[NQ];
#pragma unroll
  for (int p = 0; p < NQ; ++p) acc[p] = 0.0;
  if (valid) {
    for (int x0 = lo; x0 < hi; x0 += XU) {
      double wv[XU][MAXC], g[XU][R];
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        const int x = min(x0 + u, hi - 1);
        // every load unconditional: unused edge records are zero (offset
        // and strides), so they read W64[0]; their factor is replaced by 1
#pragma unroll
        for (int c = 0; c < MAXC; ++c) wv[u][c] = W64[eaddr(it.edi[c], im[c], x)];
#pragma unroll
        for (int r = R0; r < R; ++r) g[u][r] = Gik[(long long)r * Ii + x];
      }
#pragma unroll
      for (int u = 0; u < XU; ++u) {
#pragma unroll
        for (int c = 0; c < MAXC; ++c) wv[u][c] = pin(wv[u][c]);
      }
#pragma unroll
      for (int u = 0; u < XU; ++u) {
        const double live = (x0 + u < hi) ? 1.0 : 0.0;
        double w = sdd * live;
#pragma unroll
        for (int c = 0; c < MAXC; ++c) w *= c < nd ? wv[u][c] * wv[u][c] : 1.0;
        int p = 0;
#pragma unroll
        for (int r = R0; r < R1; ++r) {
          const double wr = w * g[u][r];
#pragma unroll
          for (int s2 = r; s2 < R; ++s2) acc[p++] += wr * g[u][s2];
        }
      }
    }
  }
  for (int o = 1; o < (1 << lg); o <<= 1) {
#pragma unroll
    for (int p = 0; p < NQ; ++p) acc[p] += __shfl_xor(acc[p], o, 64);
  }
  if (store) {
#pragma unroll
    for (int p = 0; p < NQ; ++p) q[P0 + p] = acc[p];
  }
}

template <int R>
__device__ __forceinline__ void gram_work(const double* __restrict__ W64, const double* __restrict__ Gp,
                                          double* __restrict__ Qp, int nd, int ndd, const QItem it,
                                          long long item) {
  constexpr int NP = R * (R + 1) / 2;
  const int lg = it.lg2P;
  const long long dd = item >> lg;
  const int ch = (int)(item & ((1 << lg) - 1));
  const int Ii = it.Ii;
  const bool valid = dd < it.D;
  int im[MAXC];
  double sdd = 1.0;
  if (valid) {
    long long t = dd;
#pragma unroll
    for (int c = MAXC - 1; c >= 0; --c) {
      im[c] = 0;
      if (c < nd) {
        im[c] = (int)(t % it.ddim[c]);
        t /= it.ddim[c];
      }
    }
    double wd[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {   // unused records are zero: they read W64[0]
      const int xa = it.dd_a[q], xb = it.dd_b[q];
      const int ia = xa == 0 ? im[0] : (xa == 1 ? im[1] : im[2]);
      const int ib = xb == 0 ? im[0] : (xb == 1 ? im[1] : im[2]);
      wd[q] = W64[eaddr(it.edd[q], ia, ib)];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) wd[q] = pin(wd[q]);
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (q < ndd) sdd *= wd[q] * wd[q];
  } else {
#pragma unroll
    for (int c = 0; c < MAXC; ++c) im[c] = 0;
  }
  const int lo = ch * it.CH, hi = min(Ii, lo + it.CH);
  const double* Gik = Gp + it.gik;
  double* q = Qp + it.qoff + (valid ? dd : 0) * NP;
  const bool store = valid && ch == 0;
  if constexpr (R <= 4) {
    gram_rows<R, 0, R, 4>(W64, Gik, q, nd, it, im, sdd, valid, lo, hi, lg, Ii, store);
  } else if constexpr (R <= 6) {
    gram_rows<R, 0, R, 2>(W64, Gik, q, nd, it, im, sdd, valid, lo, hi, lg, Ii, store);
  } else {
    gram_rows<R, 0, 2, 2>(W64, Gik, q, nd, it, im, sdd, valid, lo, hi, lg, Ii, store);
    gram_rows<R, 2, R, 2>(W64, Gik, q, nd, it, im, sdd, valid, lo, hi, lg, Ii, store);
  }
}

// One workgroup of Gram weights: block bid of the items of every i != k
// (constant indices into the records; they come from device memory, a
// runtime index into the argument block would force a scratch copy).
__device__ __forceinline__ void gram_block(const GramRef& a, long long bid) {
  int ii = 0;
  if (a.ni > 1 && bid >= a.blk0[1]) ii = 1;
  if (a.ni > 2 && bid >= a.blk0[2]) ii = 2;
  if (a.ni > 3 && bid >= a.blk0[3]) ii = 3;
  const long long b0 = ii == 0 ? a.blk0[0] : ii == 1 ? a.blk0[1] : ii == 2 ? a.blk0[2] : a.blk0[3];
  const long long item = (bid - b0) * NT + threadIdx.x;
  const QItem it = a.dit[ii];
  switch (it.R) {   // uniform per workgroup
    case 1: gram_work<1>(a.W64, a.G, a.Q, a.nd, a.ndd, it, item); break;
    case 2: gram_work<2>(a.W64, a.G, a.Q, a.nd, a.ndd, it, item); break;
    case 3: gram_work<3>(a.W64, a.G, a.Q, a.nd, a.ndd, it, item); break;
    case 4: gram_work<4>(a.W64, a.G, a.Q, a.nd, a.ndd, it, item); break;
    case 5: gram_work<5>(a.W64, a.G, a.Q, a.nd, a.ndd, it, item); break;
    case 6: gram_work<6>(a.W64, a.G, a.Q, a.nd, a.ndd, it, item); break;
    case 7: gram_work<7>(a.W64, a.G, a.Q, a.nd, a.ndd, it, item); break;
    default: gram_work<8>(a.W64, a.G, a.Q, a.nd, a.ndd, it, item); break;
  }
}

// Division by a loop-invariant divisor through a float reciprocal: for
// 0 <= n < 2^22 the estimate trunc(n * (1/d)) is within one of n / d (the two
// roundings are below 2^-23 relative), and one correction step makes it exact.
struct FDiv {
  int d;
  float r;
};

__device__ __forceinline__ FDiv mkdiv(int d) { return FDiv{d, 1.0f / (float)d}; }

__device__ __forceinline__ int fdiv(int n, const FDiv f) {
  int q = (int)((float)n * f.r);
  const int rem = n - q * f.d;
  q += (rem >= f.d ? 1 : 0) - (rem < 0 ? 1 : 0);
  return q;
}

// quotient and remainder; n may exceed the fast range (rare: falls back)
__device__ __forceinline__ int fdivmod(int n, const FDiv f, int* rem) {
  const int q = n < (1 << 22) ? fdiv(n, f) : n / f.d;
  *rem = n - q * f.d;
  return q;
}

// s + term(0, load(0)) + ... + term(n-1, load(n-1)), added in ascending u, with
// the loads issued U at a time: a batch's loads are all in flight before its
// first term is added, and a short last batch clamps its indices (in bounds,
// results unused), so n loads take ceil(n / U) round trips, not a serial tail.
template <int U, typename Load, typename Term>
__device__ __forceinline__ double ordered_sum(double s, int n, Load load, Term term) {
  for (int u0 = 0; u0 < n; u0 += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load(min(u0 + u, n - 1));
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = pin(v[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u0 + u < n) s += term(u0 + u, v[u]);
  }
  return s;
}

// for (e = tid; e < n; e += NT) use(e, load(e)), with the loads of U
// consecutive iterations issued before any of them is consumed (the index is
// clamped so that every load is in bounds and the body has no branches)
template <int U, typename Load, typename Use>
__device__ __forceinline__ void for_batched(int n, Load load, Use use) {
  for (int eb = threadIdx.x; eb < n; eb += NT * U) {
    decltype(load(0)) v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load(min(eb + u * NT, n - 1));
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = pin(v[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (eb + u * NT < n) use(eb + u * NT, v[u]);
  }
}

// for_batched from element threadIdx.x + e0 on (e0 a multiple of NT): the rest
// of an array whose first elements were loaded together with other arrays
template <int U, typename Load, typename Use>
__device__ __forceinline__ void for_batched_from(int e0, int n, Load load, Use use) {
  for (int eb = threadIdx.x + e0; eb < n; eb += NT * U) {
    decltype(load(0)) v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = load(min(eb + u * NT, n - 1));
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = pin(v[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (eb + u * NT < n) use(eb + u * NT, v[u]);
  }
}
// Grouped reduction of the partial slots (ContractArgs::ugrp): called by every
// contraction workgroup after its partial slot is written.  The workgroup
// releases its writes and counts itself in; the last of the group's
// workgroups to arrive -- every slot of the group is then written and
// visible -- adds the group's slots in slot order.  No workgroup waits for
// another.  Workgroup-uniform: every thread returns together.
__device__ __forceinline__ void group_partials(const ContractArgs& a, int jt, int slot, int j0, int jcnt) {
  __shared__ int last;
  const int St = a.S * a.FS;
  const int g = slot / a.ugrp, lo = g * a.ugrp, hi = min(St, lo + a.ugrp);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&a.ucnt[jt * a.ngrp + g], 1) == hi - lo - 1 ? 1 : 0;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int Rprod = a.Rprod, n = jcnt * Rprod;
  const long long stride = (long long)a.Ik * Rprod;
  for (int e = threadIdx.x; e < n; e += NT) {
    const int jl = e / Rprod, c = e - jl * Rprod;
    const double* up = a.Upart + ((long long)lo * a.Ik + j0 + jl) * Rprod + c;
    a.Ugrp[((long long)g * a.Ik + j0 + jl) * Rprod + c] = ordered_sum<16>(
        0.0, hi - lo, [&](int q) { return up[(long long)q * stride]; }, [](int, double x) { return x; });
  }
  if (threadIdx.x == 0) a.ucnt[jt * a.ngrp + g] = 0;   // ready for the next launch (stream order)
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
  L.tile = o;  o = al16(o + std::max((size_t)a.PB * a.jn * a.LDF * tcsz, (size_t)NT * 8));
  L.T = o;     o = al16(o + (size_t)a.PB * a.jn * a.Rf * tcsz);
  L.gf = o;    o = al16(o + (size_t)a.If * a.Rf * tcsz);
  L.red = o;   o = al16(o + 4 * 3 * 8);
  L.total = o;
  return L;
}

constexpr int UNR = 8;   // X elements in flight per thread in the streaming stage

template <typename TX, typename TC, bool UPD, bool CON, int SPT>
__global__ __launch_bounds__(NT) void k_contract(ContractArgs a) {
  if (a.stop && *a.stop) return;
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

  const int bid = (int)blockIdx.x;
  const int tid = threadIdx.x;
  const int jt = bid % a.JT;
  const int sp = bid / a.JT;
  const int j0 = jt * a.jn;
  const int jcnt = min(a.jn, a.Ik - j0);
  const long long p_begin = (long long)sp * a.PPW;
  const long long p_end = min(a.nplanes, p_begin + a.PPW);
  const TC* __restrict__ Wc = (const TC*)a.Wc;
  TX* __restrict__ X = (TX*)a.X;
  const double* __restrict__ G = a.G;
  const int If = a.If, Rf = a.Rf, Rc = a.Rc, Rprod = a.Rprod, nc = a.nc, jn = a.jn, LDF = a.LDF;
  const int psplit = a.psplit;

  // accumulator slots: slot s -> (j, r_c, r_f) and a plane residue class
  double acc[SPT];
  int aoff[SPT], toff[SPT], psub[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) {
    acc[q] = 0.0;
    aoff[q] = -1;
    toff[q] = 0;
    psub[q] = 0;
    if (CON) {
      const int s = q * NT + tid;
      if (s < jcnt * Rprod * psplit) {
        const int b = s / psplit;
        const int jl = b / Rprod, sl = b - jl * Rprod;
        psub[q] = s - b * psplit;
        aoff[q] = sl / Rf;
        toff[q] = jl * Rf + (sl - (sl / Rf) * Rf);
      }
    }
  }
  if (CON) {
    for_batched<4>(
        Rf * If, [&](int e) { return G[a.gfoff + e]; },
        [&](int e, double v) {
          const int r = e / If, ff = e - r * If;
          gf[ff * Rf + r] = (TC)v;
        });
  }
  double dx2 = 0.0, x2 = 0.0, f2 = 0.0;
  const TC rx = (TC)a.rho_x;
  const TC inv1 = (TC)1 / ((TC)1 + rx);

  for (long long pb0 = p_begin; pb0 < p_end; pb0 += a.PB) {
    const int np = (int)min((long long)a.PB, p_end - pb0);
    // (a) planes: base offsets, S_k factors, Kronecker coefficients
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
    for_batched<4>(
        np * If,
        [&](int e) {
          const int pl = e / If, ff = e - pl * If;
          TC s = sccl[pl];
#pragma unroll
          for (int c = 0; c < MAXC; ++c)
            if (c < nc) s *= Wc[eaddr(a.ecf[c], pidx[pl * MAXC + c], ff)];
          return s;
        },
        [&](int e, TC v) {
          const int pl = e / If;
          scf[pl * LDF + (e - pl * If)] = v;
        });
    if (CON) {
      for_batched<4>(
          np * Rc,
          [&](int e) {
            const int pl = e / Rc;
            int rr = e - pl * Rc;
            double v = 1.0;
#pragma unroll
            for (int c = MAXC - 1; c >= 0; --c) {
              if (c < nc) {
                const int r = rr % a.crank[c];
                rr /= a.crank[c];
                v *= G[a.gcoff[c] + (long long)r * a.cdim[c] + pidx[pl * MAXC + c]];
              }
            }
            return v;
          },
          [&](int e, double v) { acoef[e] = v; });
    }
    if (UPD) {
      for_batched<4>(
          np * jcnt,
          [&](int e) {
            const int pl = e / jcnt, jl = e - pl * jcnt;
            TC v = (TC)1;
#pragma unroll
            for (int c = 0; c < MAXC; ++c)
              if (c < nc) v *= Wc[eaddr(a.e0c[c], j0 + jl, pidx[pl * MAXC + c])];
            return v;
          },
          [&](int e, TC v) {
            const int pl = e / jcnt;
            t0[pl * jn + (e - pl * jcnt)] = v;
          });
    }
    __syncthreads();

    // (b) stream X.  The batch is enumerated over the extents of the axes
    // ord[0..2] (slowest memory stride first); a carried mixed-radix counter
    // replaces divisions, and UNR loads are issued before any is consumed.
    {
      const int o0 = a.ord[0], o1 = a.ord[1];
      const int D0 = o0 == 0 ? jcnt : (o0 == 1 ? np : If);
      const int D1 = o1 == 0 ? jcnt : (o1 == 1 ? np : If);
      const int D2 = (o0 != 0 && o1 != 0) ? jcnt : ((o0 != 1 && o1 != 1) ? np : If);
      const int total = D0 * D1 * D2;
      const int s2 = NT % D2, s1 = (NT / D2) % D1, s0 = NT / (D1 * D2);
      int i2 = tid % D2, i1 = (tid / D2) % D1, i0 = tid / (D1 * D2);
      for (int eb = tid; eb < total; eb += NT * UNR) {
        long long Lv[UNR];
        int pv[UNR], jv[UNR], fv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const bool ok = eb + u * NT < total;
          const int jl = o0 == 0 ? i0 : (o1 == 0 ? i1 : i2);
          const int pl = o0 == 1 ? i0 : (o1 == 1 ? i1 : i2);
          const int ff = (o0 != 2 && o1 != 2) ? i2 : (o0 == 2 ? i0 : i1);
          jv[u] = ok ? jl : 0;
          pv[u] = ok ? pl : 0;
          fv[u] = ok ? ff : 0;
          // out-of-range lanes load element (0, 0, 0) of the batch and drop it
          Lv[u] = pbase[pv[u]] + (long long)(j0 + jv[u]) * a.stride_k + (long long)fv[u] * a.stride_f;
          if (!ok) Lv[u] = -1 - Lv[u];
          i2 += s2;
          if (i2 >= D2) { i2 -= D2; ++i1; }
          i1 += s1;
          if (i1 >= D1) { i1 -= D1; ++i0; }
          i0 += s0;
        }
        TX xr[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) xr[u] = X[Lv[u] >= 0 ? Lv[u] : -1 - Lv[u]];
        uint32_t mw[UNR];
        TC w0[UNR];
        if (UPD) {
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            mw[u] = a.maskbits[(Lv[u] >= 0 ? Lv[u] : -1 - Lv[u]) >> 5];
            w0[u] = Wc[eaddr(a.e0f, j0 + jv[u], fv[u])];
          }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          if (Lv[u] < 0) continue;
          TC x = (TC)xr[u];
          const TC sk = scf[pv[u] * LDF + fv[u]];
          if (UPD) {
            const TC xh = sk * t0[pv[u] * jn + jv[u]] * w0[u];
            const bool obs = (mw[u] >> (Lv[u] & 31)) & 1u;
            // the new value as stored (rounded to the storage type)
            const TC xn = obs ? x : (TC)(TX)((xh + rx * x) * inv1);
            if (!obs) X[Lv[u]] = (TX)xn;
            const double d = (double)xn - (double)x;
            dx2 += d * d;
            x2 += (double)x * (double)x;
            const double rr = (double)xn - (double)xh;
            f2 += rr * rr;
            x = xn;
          }
          if (CON) tile[(pv[u] * jn + jv[u]) * LDF + fv[u]] = x * sk;
        }
      }
    }
    __syncthreads();

    if (CON) {
      // (c) fibre contraction T(row, r_f), each row shared by fch adjacent lanes
      const int rows = np * jcnt;
      const int fch = a.fch;
      const int rpp = NT / fch;
      const int chunk = (If + fch - 1) / fch;
      const int ch = tid & (fch - 1);
      const int passes = (rows + rpp - 1) / rpp;
      for (int ps = 0; ps < passes; ++ps) {
        const int row = ps * rpp + tid / fch;
        TC t[MAXR];
#pragma unroll
        for (int r = 0; r < MAXR; ++r) t[r] = (TC)0;
        if (row < rows) {
          const int pl = row / jcnt, jl = row - pl * jcnt;
          const TC* trow = tile + (pl * jn + jl) * LDF;
          const int lo = ch * chunk, hi = min(If, lo + chunk);
          for (int ff = lo; ff < hi; ++ff) {
            const TC v = trow[ff];
            const TC* g = gf + ff * Rf;
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
              if (r < Rf) t[r] += v * g[r];
          }
        }
        for (int o = 1; o < fch; o <<= 1) {
#pragma unroll
          for (int r = 0; r < MAXR; ++r) t[r] += __shfl_xor(t[r], o, 64);
        }
        if (row < rows && ch == 0) {
          const int pl = row / jcnt, jl = row - pl * jcnt;
#pragma unroll
          for (int r = 0; r < MAXR; ++r)
            if (r < Rf) Tl[(pl * jn + jl) * Rf + r] = t[r];
        }
      }
      __syncthreads();
      // (d) Kronecker accumulation into owned slots (planes split round-robin)
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        if (aoff[q] >= 0) {
          double sum = acc[q];
          for (int pl = psub[q]; pl < np; pl += psplit)
            sum += acoef[pl * Rc + aoff[q]] * (double)Tl[pl * jn * Rf + toff[q]];
          acc[q] = sum;
        }
      }
    }
    __syncthreads();
  }

  if (CON) {
    // combine the plane residue classes in a fixed order, then write the
    // slot's canonical U column (modes != k ascending, row-major)
    double* comb = (double*)(smem + Ly.tile);   // tile is free now; psplit > 1 implies <= NT slots
    if (psplit > 1) {
#pragma unroll
      for (int q = 0; q < SPT; ++q)
        if (aoff[q] >= 0) comb[q * NT + tid] = acc[q];
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      if (aoff[q] >= 0 && psub[q] == 0) {
        const int s = q * NT + tid;
        double v = acc[q];
        for (int t = 1; t < psplit; ++t) v += comb[s + t];
        const int b = s / psplit;
        const int jl = b / Rprod, sl = b - jl * Rprod;
        int rc = sl / Rf;
        long long col = (long long)(sl - rc * Rf) * a.ustf;
        for (int c = nc - 1; c >= 0; --c) {
          const int r = rc % a.crank[c];
          rc /= a.crank[c];
          col += (long long)r * a.ustc[c];
        }
        a.Upart[((long long)sp * a.Ik + j0 + jl) * Rprod + col] = v;
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
      double sum = 0.0;
      for (int q = 0; q < NT / 64; ++q) sum += red[q * 3 + tid];
      a.normpart[(long long)bid * 3 + tid] = sum;
    }
  }
  if (CON && a.ugrp) group_partials(a, jt, sp, j0, jcnt);
}

// --------------------------------------------------------------------------
// K3 fast paths.  Same contraction as k_contract, for the two layouts every
// tensor of this library's workloads uses, with X read from HBM straight into
// registers (no LDS tile):
//   rows:    the fibre mode f is the contiguous last mode; each fibre (plane,
//            j) is split over `fch` adjacent lanes that reduce with a fixed
//            butterfly;
//   columns: mode k is the contiguous last mode; lanes run along j (coalesced)
//            and loop over the fibre, fibre chunks reduced through LDS in a
//            fixed order.
// Both finish like k_contract: T(plane, j, r_f) in LDS, then the Kronecker
// accumulation into float64 slots and the split partials of U_k.
// --------------------------------------------------------------------------
struct FLayout {
  size_t pbase, pidx, acoef, scc, scf, t0, w0f, gf, T, tpart, red, T2, gl, total;
};

// fibre entries per workgroup: the fibre range is split into FS chunks
__host__ __device__ inline int fibre_chunk(const ContractArgs& a) { return a.FS == 1 ? a.If : (a.If + a.FS - 1) / a.FS; }

__host__ __device__ inline FLayout flayout(int tcsz, const ContractArgs& a) {
  FLayout L;
  size_t o = 0;
  const size_t fcs = (size_t)fibre_chunk(a);
  L.pbase = o; o = al16(o + (size_t)a.PB * 8);
  L.pidx = o;  o = al16(o + (size_t)a.PB * MAXC * 4);
  L.acoef = o; o = al16(o + (size_t)a.PB * a.Rc * 8);
  L.scc = o;   o = al16(o + (size_t)a.PB * tcsz);
  L.scf = o;   o = al16(o + (size_t)a.PB * fcs * tcsz);
  L.t0 = o;    o = al16(o + (size_t)a.PB * a.jn * tcsz);
  L.w0f = o;   o = al16(o + (size_t)(a.k == 0 ? a.jn * fcs : 0) * tcsz);
  L.gf = o;    o = al16(o + fcs * MAXR * tcsz);               // zero-padded to MAXR ranks
  L.T = o;     o = al16(o + std::max((size_t)a.PB * a.jn * a.Rf * tcsz, (size_t)NT * 8));
  L.tpart = o; o = al16(o + (a.kind == 2 ? (size_t)NT * a.Rf * tcsz : 0));
  L.red = o;   o = al16(o + 4 * 3 * 8);
  // staged accumulation: partial contraction over the last c-mode, its factor
  L.T2 = o;    o = al16(o + (a.stage ? (size_t)(a.PB / a.cdl) * a.jn * a.Rl * a.Rf * 8 : 0));
  L.gl = o;    o = al16(o + (a.stage ? (size_t)a.cdl * MAXR * 8 : 0));
  L.total = o;
  return L;
}

// shared pieces of the fast kernels (NC = number of modes other than k and f,
// a compile-time constant so that no load sits behind a per-mode branch) -----
template <typename TC, int NC>
__device__ __forceinline__ void plane_setup(const ContractArgs& a, long long pb0, int np, int jcnt, int j0,
                                            long long* pbase, int* pidx, TC* sccl, TC* scf, double* acoef,
                                            TC* t0, bool con, bool upd, int flo, int fcn, int fcs) {
  const TC* __restrict__ Wc = (const TC*)a.Wc;
  const int tid = threadIdx.x, Rc = a.Rc, jn = a.jn;
  FDiv fcd[NC > 0 ? NC : 1];
#pragma unroll
  for (int c = 0; c < NC; ++c) fcd[c] = mkdiv(a.cdim[c]);
  const FDiv fIf = mkdiv(fcn);
  for (int e = tid; e < np; e += NT) {
    long long base = 0;
    int p = (int)(pb0 + e);          // plane index (< 2^31: the plane count is checked on the host)
    int ic[MAXC > 0 ? MAXC : 1];
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
      p = fdivmod(p, fcd[c], &ic[c]);
      base += (long long)ic[c] * a.cstride[c];
    }
    TC sv = (TC)1;
#pragma unroll
    for (int x = 0; x < NC; ++x)
#pragma unroll
      for (int y = x + 1; y < NC; ++y) sv *= Wc[eaddr(a.ecc[x * (2 * NC - x - 1) / 2 + (y - x - 1)], ic[x], ic[y])];
    pbase[e] = base;
    sccl[e] = sv;
#pragma unroll
    for (int c = 0; c < NC; ++c) pidx[e * MAXC + c] = ic[c];
  }
  __syncthreads();
  // scf(pl, f) for the fibre chunk: row pl at pl * fcs
  for_batched<4>(
      np * fcn,
      [&](int e) {
        int ff;
        const int pl = fdivmod(e, fIf, &ff);
        TC v = sccl[pl];
#pragma unroll
        for (int c = 0; c < NC; ++c) v *= Wc[eaddr(a.ecf[c], pidx[pl * MAXC + c], flo + ff)];
        return v;
      },
      [&](int e, TC v) {
        int ff = e, pl = 0;
        if (fcn != fcs) pl = fdivmod(e, fIf, &ff);   // a short last chunk: rows keep stride fcs
        scf[pl * fcs + ff] = v;
      });
  if (con && a.stage) {
    // per group of cdl planes: product over the c-modes but the last
    const int ng = np / a.cdl, Rc2 = a.Rc2;
    for_batched<4>(
        ng * Rc2,
        [&](int e) {
          int rr;
          const int g = fdivmod(e, mkdiv(Rc2), &rr);
          const int pl = g * a.cdl;
          double v = 1.0;
#pragma unroll
          for (int c = NC - 2; c >= 0; --c) {
            int r;
            rr = fdivmod(rr, mkdiv(a.crank[c]), &r);
            v *= a.G[a.gcoff[c] + (long long)r * a.cdim[c] + pidx[pl * MAXC + c]];
          }
          return v;
        },
        [&](int e, double v) { acoef[e] = v; });
  } else if (con) {
    for_batched<4>(
        np * Rc,
        [&](int e) {
          int rr;
          const int pl = fdivmod(e, mkdiv(Rc), &rr);
          double v = 1.0;
#pragma unroll
          for (int c = NC - 1; c >= 0; --c) {
            int r;
            rr = fdivmod(rr, mkdiv(a.crank[c]), &r);
            v *= a.G[a.gcoff[c] + (long long)r * a.cdim[c] + pidx[pl * MAXC + c]];
          }
          return v;
        },
        [&](int e, double v) { acoef[e] = v; });
  }
  if (upd) {
    for_batched<4>(
        np * jcnt,
        [&](int e) {
          int jl;
          const int pl = fdivmod(e, mkdiv(jcnt), &jl);
          TC v = (TC)1;
#pragma unroll
          for (int c = 0; c < NC; ++c) v *= Wc[eaddr(a.e0c[c], j0 + jl, pidx[pl * MAXC + c])];
          return v;
        },
        [&](int e, TC v) {
          int jl;
          const int pl = fdivmod(e, mkdiv(jcnt), &jl);
          t0[pl * jn + jl] = v;
        });
  }
  __syncthreads();
}

// G_{f,k} as gf[f][r] zero-padded to MAXR ranks (unconditional FMAs later)
template <typename TC>
__device__ __forceinline__ void load_gf(const ContractArgs& a, TC* gf, int flo, int fcn) {
  const int If = a.If, Rf = a.Rf;
  for_batched<4>(
      fcn * MAXR,
      [&](int e) {
        const int ff = e / MAXR, r = e - ff * MAXR;
        return a.G[a.gfoff + (long long)min(r, Rf - 1) * If + flo + ff];   // in bounds; padding zeroed below
      },
      [&](int e, double v) { gf[e] = (e % MAXR) < Rf ? (TC)v : (TC)0; });
}

template <int SPT>
struct Slots {
  double acc[SPT];
  int aoff[SPT], toff[SPT];
  int jls[SPT], cols[SPT];     // row of U and canonical U column of each slot
  int psub;
  template <int NC>
  __device__ __forceinline__ void init(const ContractArgs& a, int jcnt) {
    const int tid = threadIdx.x, Rprod = a.Rprod, Rf = a.Rf, psplit = a.psplit;
    const int lgp = __ffs(psplit) - 1;   // psplit is a power of two
    psub = tid & (psplit - 1);           // NT is a multiple of psplit: the same for every slot
    const FDiv fR = mkdiv(Rprod), fRf = mkdiv(Rf);
    FDiv fcr[NC > 0 ? NC : 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) fcr[c] = mkdiv(a.crank[c]);
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      acc[q] = 0.0;
      aoff[q] = -1;
      toff[q] = 0;
      jls[q] = 0;
      cols[q] = 0;
      const int s = q * NT + tid;
      if (s < jcnt * Rprod * psplit) {
        const int b = s >> lgp;
        int sl, rf;
        const int jl = fdivmod(b, fR, &sl);
        const int rc = fdivmod(sl, fRf, &rf);
        if (a.stage) {
          // rc = rc2 * Rl + rl (the last c-mode is the fastest digit)
          int rl;
          const int rc2 = fdivmod(rc, mkdiv(a.Rl), &rl);
          aoff[q] = rc2;
          toff[q] = (jl * a.Rl + rl) * Rf + rf;
        } else {
          aoff[q] = rc;
          toff[q] = jl * Rf + rf;
        }
        jls[q] = jl;
        long long col = (long long)rf * a.ustf;
        int rr = rc;
#pragma unroll
        for (int c = NC - 1; c >= 0; --c) {
          int r;
          rr = fdivmod(rr, fcr[c], &r);
          col += (long long)r * a.ustc[c];
        }
        cols[q] = (int)col;
      }
    }
  }
  // planes outer, slots inner: the 2 SPT LDS reads of a plane are issued together
  template <typename TC>
  __device__ __forceinline__ void accumulate(const double* acoef, const TC* Tl, int np, int jn, int Rc, int Rf,
                                             int psplit) {
    int ao[SPT], to[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      ao[q] = aoff[q] >= 0 ? aoff[q] : 0;
      to[q] = toff[q];
    }
    for (int pl = psub; pl < np; pl += psplit) {
      double av[SPT], tv[SPT];
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        av[q] = acoef[pl * Rc + ao[q]];
        tv[q] = (double)Tl[pl * jn * Rf + to[q]];
      }
#pragma unroll
      for (int q = 0; q < SPT; ++q) acc[q] += av[q] * tv[q];
    }
  }
  // combine the plane residue classes in a fixed order and write the slot's
  // canonical U column (modes != k ascending, row-major)
  template <int NC>
  __device__ __forceinline__ void write(const ContractArgs& a, double* comb, int sp, int j0) {
    const int tid = threadIdx.x, psplit = a.psplit, Rprod = a.Rprod;
    if (psplit > 1) {
#pragma unroll
      for (int q = 0; q < SPT; ++q)
        if (aoff[q] >= 0) comb[q * NT + tid] = acc[q];
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      if (aoff[q] >= 0 && psub == 0) {
        const int s = q * NT + tid;
        double v = acc[q];
        for (int t = 1; t < psplit; ++t) v += comb[s + t];
        a.Upart[((long long)sp * a.Ik + j0 + jls[q]) * Rprod + cols[q]] = v;
      }
    }
  }
};

// Staged accumulation of a batch: T2(g, j, r_l, r_f) = sum over the last
// c-mode index i of G_{m_last,k}(r_l, i) T(g cdl + i, j, r_f) in float64, then
// the slots accumulate over the groups g.
template <int SPT, typename TC>
__device__ __forceinline__ void staged_accumulate(const ContractArgs& a, Slots<SPT>& sl, const double* acoef,
                                                  const TC* Tl, double* T2, const double* gl, int np, int jcnt) {
  const int tid = threadIdx.x, jn = a.jn, Rf = a.Rf, Rl = a.Rl, cdl = a.cdl;
  const int ng = np / cdl;
  const int per = jcnt * Rl * Rf;
  const FDiv fper = mkdiv(per), fRf = mkdiv(Rf), fRl = mkdiv(Rl);
  for (int e = tid; e < ng * per; e += NT) {
    int rem, rf, rl;
    const int g = fdivmod(e, fper, &rem);
    const int t = fdivmod(rem, fRf, &rf);
    const int jl = fdivmod(t, fRl, &rl);
    const TC* tp = Tl + ((long long)g * cdl * jn + jl) * Rf + rf;
    double v = 0.0;
    for (int i = 0; i < cdl; ++i) v += gl[i * MAXR + rl] * (double)tp[(long long)i * jn * Rf];
    T2[((g * jn + jl) * Rl + rl) * Rf + rf] = v;
  }
  __syncthreads();
  sl.accumulate(acoef, (const double*)T2, ng, jn, a.Rc2, Rl * Rf, a.psplit);
}

// G_{m_last,k} as gl[i][r] (float64, zero-padded to MAXR ranks)
__device__ __forceinline__ void load_gl(const ContractArgs& a, double* gl) {
  const int cdl = a.cdl, Rl = a.Rl;
  for_batched<4>(
      cdl * MAXR,
      [&](int e) {
        const int i = e / MAXR, r = e - i * MAXR;
        return a.G[a.gloff + (long long)min(r, Rl - 1) * cdl + i];   // in bounds; padding zeroed below
      },
      [&](int e, double v) { gl[e] = (e % MAXR) < Rl ? v : 0.0; });
}

__device__ __forceinline__ void block_norms(double dx2, double x2, double f2, double* red, double* out) {
  const int tid = threadIdx.x;
  const double v0 = wave_sum(dx2), v1 = wave_sum(x2), v2 = wave_sum(f2);
  const int w = tid >> 6;
  if ((tid & 63) == 0) {
    red[w * 3 + 0] = v0;
    red[w * 3 + 1] = v1;
    red[w * 3 + 2] = v2;
  }
  __syncthreads();
  if (tid < 3) {
    double sum = 0.0;
    for (int q = 0; q < NT / 64; ++q) sum += red[q * 3 + tid];
    out[tid] = sum;
  }
}

// Workgroups are dispatched to the 8 XCDs in turn (launch index mod 8), each
// XCD with its own L2. Logical index L = (A mod 8) * q + A / 8 over the first
// 8q launch indices (identity after them) puts logical neighbours -- j-tiles
// that share cache lines of X, consecutive plane ranges -- on the same XCD.
// A bijection on [0, total), so every logical workgroup runs exactly once.
// Applied to the contraction workgroups only: the Gram workgroups keep the
// first launch indices, spread over all XCDs (grouped on one XCD they would
// become the launch's critical path).
__device__ __forceinline__ int xcd_local(int A, int total) {
  const int q = total >> 3;
  return A < (q << 3) ? (A & 7) * q + (A >> 3) : A;
}

// rows variant (fibre mode contiguous) ---------------------------------------
template <typename TX, typename TC, int NC, bool UPD, bool CON, int SPT>
__global__ __launch_bounds__(NT) void k_contract_rows(ContractArgs a) {
  if (a.stop && *a.stop) return;
  if (blockIdx.x < a.gblocks) {           // Gram weights of the same block
    gram_block(a.gr, blockIdx.x);
    return;
  }
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const FLayout Ly = flayout((int)sizeof(TC), a);
  long long* pbase = (long long*)(smem + Ly.pbase);
  int* pidx = (int*)(smem + Ly.pidx);
  double* acoef = (double*)(smem + Ly.acoef);
  TC* sccl = (TC*)(smem + Ly.scc);
  TC* scf = (TC*)(smem + Ly.scf);
  TC* t0 = (TC*)(smem + Ly.t0);
  TC* w0f = (TC*)(smem + Ly.w0f);
  TC* gf = (TC*)(smem + Ly.gf);
  TC* Tl = (TC*)(smem + Ly.T);
  double* red = (double*)(smem + Ly.red);

  // contraction workgroup index, XCD-local among the contraction workgroups
  const int tid = threadIdx.x, bid = xcd_local((int)blockIdx.x - a.gblocks, (int)gridDim.x - a.gblocks);
  const int jt = bid % a.JT, spf = bid / a.JT;          // partial index = plane split * FS + fibre split
  const int sp = a.FS == 1 ? spf : spf / a.FS, fs = spf - sp * a.FS;
  const int j0 = jt * a.jn, jcnt = min(a.jn, a.Ik - j0);
  const long long p_begin = (long long)sp * a.PPW, p_end = min(a.nplanes, p_begin + a.PPW);
  const TC* __restrict__ Wc = (const TC*)a.Wc;
  TX* __restrict__ X = (TX*)a.X;
  const int Rf = a.Rf, jn = a.jn;
  // this workgroup's fibre chunk [flo, fhi); the fibre tables hold it with row stride fcs
  const int fcs = fibre_chunk(a), flo = fs * fcs, fhi = min(a.If, flo + fcs), fcn = fhi - flo;

  Slots<SPT> sl;
  double* T2 = (double*)(smem + Ly.T2);
  double* gl = (double*)(smem + Ly.gl);
  if (CON) {
    sl.template init<NC>(a, jcnt);
    load_gf<TC>(a, gf, flo, fcn);
    if (NC >= 2 && a.stage) load_gl(a, gl);
  }
  if (UPD)
    for_batched<4>(
        jcnt * fcn,
        [&](int e) {
          int ff;
          const int jl = fdivmod(e, mkdiv(fcn), &ff);
          return Wc[eaddr(a.e0f, j0 + jl, flo + ff)];
        },
        [&](int e, TC v) {
          int ff = e, jl = 0;
          if (fcn != fcs) jl = fdivmod(e, mkdiv(fcn), &ff);
          w0f[jl * fcs + ff] = v;
        });
  double dx2 = 0.0, x2 = 0.0, f2 = 0.0;
  const TC rx = (TC)a.rho_x, inv1 = (TC)1 / ((TC)1 + rx);
  const int fch = a.fch, rpp = NT / fch, chunk = (fcn + fch - 1) / fch, ch = tid & (fch - 1);

  for (long long pb0 = p_begin; pb0 < p_end; pb0 += a.PB) {
    const int np = (int)min((long long)a.PB, p_end - pb0);
    plane_setup<TC, NC>(a, pb0, np, jcnt, j0, pbase, pidx, sccl, scf, acoef, t0, CON, UPD, flo, fcn, fcs);
    const int rows = np * jcnt;
    const int passes = (rows + rpp - 1) / rpp;
    const FDiv frow = mkdiv(a.plfast ? np : jcnt);
    for (int ps = 0; ps < passes; ++ps) {
      const int row = ps * rpp + tid / fch;
      TC t[MAXR];
#pragma unroll
      for (int r = 0; r < MAXR; ++r) t[r] = (TC)0;
      const bool rok = row < rows;
      const int rowc = rok ? row : rows - 1;
      int rq;
      const int rd = fdivmod(rowc, frow, &rq);
      const int pl = a.plfast ? rq : rd;
      const int jl = a.plfast ? rd : rq;
      const long long base = pbase[pl] + (long long)(j0 + jl) * a.stride_k;
      // chunk-relative fibre tables: entry f of the tensor sits at f - flo
      // of its row (the offsets fold the chunk start; every index is >= 0)
      const int sro = pl * fcs - flo, wro = jl * fcs - flo, gfo = -flo * MAXR;
      const TC tt = UPD ? t0[pl * jn + jl] : (TC)0;
      const int lo = flo + ch * chunk, hi = rok ? min(fhi, lo + chunk) : lo;
      for (int f0 = lo; f0 < hi; f0 += 4) {
        TX xv[4];
        uint32_t mw[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const long long L = base + min(f0 + u, hi - 1);
          xv[u] = X[L];
          if (UPD) mw[u] = a.maskbits[L >> 5];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ff = min(f0 + u, hi - 1);
          const bool live = f0 + u < hi;
          TC x = (TC)xv[u];
          const TC sk = scf[sro + ff];
          if (UPD) {
            const long long L = base + ff;
            const TC xh = sk * tt * w0f[wro + ff];
            const bool obs = (mw[u] >> (L & 31)) & 1u;
            const TC xn = obs ? x : (TC)(TX)((xh + rx * x) * inv1);   // as stored
            if (live && !obs) X[L] = (TX)xn;
            const double lv = live ? 1.0 : 0.0;
            const double d = (double)xn - (double)x;
            dx2 += lv * d * d;
            x2 += lv * (double)x * (double)x;
            const double rr = (double)xn - (double)xh;
            f2 += lv * rr * rr;
            x = xn;
          }
          if (CON) {
            const TC y = live ? x * sk : (TC)0;
            const TC* g = gf + (gfo + ff * MAXR);
#pragma unroll
            for (int r = 0; r < MAXR; ++r) t[r] += y * g[r];
          }
        }
      }
      if (CON) {
        for (int o = 1; o < fch; o <<= 1) {
#pragma unroll
          for (int r = 0; r < MAXR; ++r) t[r] += __shfl_xor(t[r], o, 64);
        }
        if (rok && ch == 0) {
#pragma unroll
          for (int r = 0; r < MAXR; ++r)
            if (r < Rf) Tl[(pl * jn + jl) * Rf + r] = t[r];
        }
      }
    }
    __syncthreads();
    if (CON) {
      if (NC >= 2 && a.stage)
        staged_accumulate(a, sl, acoef, Tl, T2, gl, np, jcnt);
      else
        sl.accumulate(acoef, Tl, np, jn, a.Rc, Rf, a.psplit);
    }
    __syncthreads();
  }
  if (CON) sl.template write<NC>(a, (double*)(smem + Ly.T), spf, j0);
  if (UPD) block_norms(dx2, x2, f2, red, a.normpart + (long long)bid * 3);
  if (CON && a.ugrp) group_partials(a, jt, spf, j0, jcnt);
}

// columns variant (mode k contiguous) ----------------------------------------
template <typename TX, typename TC, int NC, int SPT>
__global__ __launch_bounds__(NT) void k_contract_cols(ContractArgs a) {
  if (a.stop && *a.stop) return;
  if (blockIdx.x < a.gblocks) {
    gram_block(a.gr, blockIdx.x);
    return;
  }
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const FLayout Ly = flayout((int)sizeof(TC), a);
  long long* pbase = (long long*)(smem + Ly.pbase);
  int* pidx = (int*)(smem + Ly.pidx);
  double* acoef = (double*)(smem + Ly.acoef);
  TC* sccl = (TC*)(smem + Ly.scc);
  TC* scf = (TC*)(smem + Ly.scf);
  TC* t0 = (TC*)(smem + Ly.t0);
  TC* gf = (TC*)(smem + Ly.gf);
  TC* Tl = (TC*)(smem + Ly.T);
  TC* tpart = (TC*)(smem + Ly.tpart);

  // contraction workgroup index, XCD-local among the contraction workgroups
  const int tid = threadIdx.x, bid = xcd_local((int)blockIdx.x - a.gblocks, (int)gridDim.x - a.gblocks);
  const int jt = bid % a.JT, spf = bid / a.JT;          // partial index = plane split * FS + fibre split
  const int sp = spf / a.FS, fs = spf - sp * a.FS;
  const int j0 = jt * a.jn, jcnt = min(a.jn, a.Ik - j0);
  const long long p_begin = (long long)sp * a.PPW, p_end = min(a.nplanes, p_begin + a.PPW);
  const TX* __restrict__ X = (const TX*)a.X;
  const int If = a.If, Rf = a.Rf, jn = a.jn;
  const int fcs = fibre_chunk(a), flo = fs * fcs, fhi = min(If, flo + fcs), fcn = fhi - flo;
  const long long sf = a.stride_f;

  Slots<SPT> sl;
  double* T2 = (double*)(smem + Ly.T2);
  double* gl = (double*)(smem + Ly.gl);
  sl.template init<NC>(a, jcnt);
  load_gf<TC>(a, gf, flo, fcn);
  if (NC >= 2 && a.stage) load_gl(a, gl);

  for (long long pb0 = p_begin; pb0 < p_end; pb0 += a.PB) {
    const int np = (int)min((long long)a.PB, p_end - pb0);
    plane_setup<TC, NC>(a, pb0, np, jcnt, j0, pbase, pidx, sccl, scf, acoef, t0, true, false, flo, fcn, fcs);
    const int NI = np * jcnt;                     // (plane, j) columns of this batch
    const int fg = NI >= NT ? 1 : NT / NI;        // fibre groups within the workgroup
    const int fchunk = (fhi - flo + fg - 1) / fg;
    const int npass = fg > 1 ? 1 : (NI + NT - 1) / NT;
    for (int ps = 0; ps < npass; ++ps) {
      const int g = fg > 1 ? fdiv(tid, mkdiv(NI)) : 0;
      const int it = fg > 1 ? tid - g * NI : ps * NT + tid;
      const bool ok = g < fg && it < NI;
      const int itc = ok ? it : NI - 1;
      TC t[MAXR];
#pragma unroll
      for (int r = 0; r < MAXR; ++r) t[r] = (TC)0;
      int jl;
      const int pl = fdivmod(itc, mkdiv(jcnt), &jl);
      const int sro = pl * fcs - flo, gfo = -flo * MAXR;   // chunk-relative, as in the rows kernel
      const long long base = pbase[pl] + j0 + jl;
      const int lo = flo + (ok ? g : 0) * fchunk, hi = ok ? min(fhi, lo + fchunk) : lo;
      for (int f0 = lo; f0 < hi; f0 += 4) {
        TX xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = X[base + (long long)min(f0 + u, hi - 1) * sf];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ff = min(f0 + u, hi - 1);
          const TC y = (f0 + u < hi) ? (TC)xv[u] * scf[sro + ff] : (TC)0;
          const TC* gg = gf + (gfo + ff * MAXR);
#pragma unroll
          for (int r = 0; r < MAXR; ++r) t[r] += y * gg[r];
        }
      }
      if (fg > 1) {
        if (ok) {
#pragma unroll
          for (int r = 0; r < MAXR; ++r)
            if (r < Rf) tpart[(g * NI + it) * Rf + r] = t[r];
        }
        __syncthreads();
        for (int e = tid; e < NI * Rf; e += NT) {
          TC v = (TC)0;
          for (int q = 0; q < fg; ++q) v += tpart[q * NI * Rf + e];
          int r, j2;
          const int i2 = fdivmod(e, mkdiv(Rf), &r);
          const int p2 = fdivmod(i2, mkdiv(jcnt), &j2);
          Tl[(p2 * jn + j2) * Rf + r] = v;
        }
      } else if (ok) {
#pragma unroll
        for (int r = 0; r < MAXR; ++r)
          if (r < Rf) Tl[(pl * jn + jl) * Rf + r] = t[r];
      }
    }
    __syncthreads();
    if (NC >= 2 && a.stage)
      staged_accumulate(a, sl, acoef, Tl, T2, gl, np, jcnt);
    else
      sl.accumulate(acoef, Tl, np, jn, a.Rc, Rf, a.psplit);
    __syncthreads();
  }
  sl.template write<NC>(a, (double*)(smem + Ly.T), spf, j0);
  if (a.ugrp) group_partials(a, jt, spf, j0, jcnt);
}

template <typename TX, typename TC>
static hipError_t contract_dispatch(bool upd, bool con, int spt, const ContractArgs& a, size_t smem,
                                    hipStream_t s) {
  const dim3 grid((unsigned)(a.JT * a.S)), blk(NT);
#define IFCTN_CASE(U, C, P)                                                      \
  if (upd == U && con == C && spt == P) {                                        \
    IFCTN_GO((k_contract<TX, TC, U, C, P>), grid, blk, smem, s, a);             \
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

template <typename TX, typename TC, int NC>
static hipError_t fast_dispatch_nc(bool upd, bool con, int spt, const ContractArgs& a, size_t smem, hipStream_t s) {
  const dim3 grid((unsigned)(a.JT * a.S * a.FS + a.gblocks)), blk(NT);
  if (a.kind == 1) {
#define IFCTN_ROWS(U, C, P)                                                              \
  if (upd == U && con == C && spt == P) {                                                \
    IFCTN_GO((k_contract_rows<TX, TC, NC, U, C, P>), grid, blk, smem, s, a);             \
    return hipGetLastError();                                                            \
  }
    IFCTN_ROWS(true, false, 1)
    IFCTN_ROWS(false, true, 1) IFCTN_ROWS(false, true, 2) IFCTN_ROWS(false, true, 4) IFCTN_ROWS(false, true, 8)
    IFCTN_ROWS(true, true, 1) IFCTN_ROWS(true, true, 2) IFCTN_ROWS(true, true, 4) IFCTN_ROWS(true, true, 8)
#undef IFCTN_ROWS
  } else if (a.kind == 2 && con && !upd) {
#define IFCTN_COLS(P)                                                              \
  if (spt == P) {                                                                  \
    IFCTN_GO((k_contract_cols<TX, TC, NC, P>), grid, blk, smem, s, a);             \
    return hipGetLastError();                                                      \
  }
    IFCTN_COLS(1) IFCTN_COLS(2) IFCTN_COLS(4) IFCTN_COLS(8)
#undef IFCTN_COLS
  }
  return hipErrorInvalidValue;
}

template <typename TX, typename TC>
static hipError_t fast_dispatch(bool upd, bool con, int spt, const ContractArgs& a, size_t smem, hipStream_t s) {
  switch (a.nc) {
    case 0: return fast_dispatch_nc<TX, TC, 0>(upd, con, spt, a, smem, s);
    case 1: return fast_dispatch_nc<TX, TC, 1>(upd, con, spt, a, smem, s);
    case 2: return fast_dispatch_nc<TX, TC, 2>(upd, con, spt, a, smem, s);
    default: return fast_dispatch_nc<TX, TC, 3>(upd, con, spt, a, smem, s);
  }
}

}  // namespace ifctn
