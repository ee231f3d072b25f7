// Gram matrix of the mode-k cherry sub-network, Gamma_k = Z_k^T Z_k (Prop. 1;
// the Gram term of eq. (updateG) for every column and every sub-block of
// factor block k at once), built by a launch of its own between the
// contraction and the solve of the block; the same launch reduces the
// contraction's partial slots into the U rows.
//
// With the modes other than k in Gamma order (prefix modes, then x, then y)
// and GG_m(i, p) = G_{m,k}(r, i) G_{m,k}(r', i) for the pair p = {r, r'}:
//   Gamma(p_pre, p_x, p_y) = sum_{prefix tuples q} cP_q(p_pre) Y_q(p_x, p_y)
//   Y_q(p_x, p_y)  = sum_x wB_q(x) GG_x(x, p_x) T_q(x, p_y)                 (stage B)
//   T_q(x, p_y)    = sum_y W_xy(x, y)^2 c_q(y) GG_y(y, p_y)                  (stage A)
// where c_q(y), wB_q(x) are the squared edges between the prefix modes (at
// tuple q) and y, x, and cP_q(p_pre) = prod over prefix edges W^2 times
// prod over prefix modes GG.  Stage A holds almost all of the arithmetic: it
// is a dense product, (I_x x I_y) . (I_y x chunk * np_y), run on the FP64
// matrix cores (v_mfma_f64_16x16x4f64) with its operands formed on the fly.
// Workgroups split the y pair index and the prefix tuples; a workgroup sums
// its tuples into partial Gamma entries (registers), and the last of a y
// group's workgroups adds that group's partial sums in a fixed order, so
// Gamma is bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

#include "ifctn_device.h"
#include "ifctn_internal.h"

namespace ifctn {

typedef double gm_d4 __attribute__((ext_vector_type(4)));

constexpr int GM_VPT = 8;              // 16 x 16 accumulation tiles per wave (planned to fit)
constexpr int GM_KB = 16;              // stage-A steps whose operand loads are issued together

__device__ __forceinline__ double gm_sq(double v) { return v * v; }

// Operand layouts of v_mfma_f64_16x16x4f64 (one wave, lane l):
//   A (16 x 4): A[l % 16][l / 16];  B (4 x 16): B[l / 16][l % 16];
//   D (16 x 16): lane l holds D[l / 16 + 4 v][l % 16], v = 0..3.
__device__ __forceinline__ gm_d4 gm_mfma(double a, double b, gm_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// U rows of block k from the contraction's partial slots: UO outputs per
// workgroup, each summed by US slices of the slots (slot order within a
// slice), then the slices in slice order (a fixed order: bitwise
// reproducible).
// Gamma_k(e) = sum over the nqg prefix ranges of their partial rows, in range
// order (the order of the in-launch last-workgroup sum), four entries per
// thread with all their loads in flight; workgroup b covers 4 NT entries.
__device__ __forceinline__ void gamma_reduce_block(const GammaPlan* __restrict__ gp, int b) {
  const int P = gp->P, nqg = gp->nqg;
  const double* part = gp->part;
  const int e0 = b * 4 * NT + (int)threadIdx.x;
  double vv[4][GM_QG];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int e = min(e0 + h * NT, P - 1);
#pragma unroll
    for (int q = 0; q < GM_QG; ++q) vv[h][q] = part[(long long)min(q, nqg - 1) * P + e];
  }
#pragma unroll
  for (int h = 0; h < 4; ++h)
#pragma unroll
    for (int q = 0; q < GM_QG; ++q) vv[h][q] = pin(vv[h][q]);
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < GM_QG; ++q)
      if (q < nqg) s += vv[h][q];
    if (e0 + h * NT < P) gp->gamma[e0 + h * NT] = s;
  }
}

__device__ __forceinline__ void urow_block(const GammaPlan* __restrict__ gp, int b) {
  __shared__ double ured[NT];
  const int tid = threadIdx.x, US = gp->us, UO = NT / US;
  const int ol = tid % UO, sl = tid / UO;
  const long long o = (long long)b * UO + ol;
  const long long nout = gp->nout;
  const long long oc = min(o, nout - 1);
  const double* up = gp->Upart + oc;
  const int S = gp->S;
  const double v = ordered_sum<8>(
      0.0, S > sl ? (S - sl + US - 1) / US : 0, [&](int u) { return up[(long long)(sl + US * u) * nout]; },
      [](int, double x) { return x; });
  ured[tid] = v;
  __syncthreads();
  if (tid < UO && o < nout) {
    double s = 0.0;
    for (int q = 0; q < US; ++q) s += ured[q * UO + tid];
    gp->Ufin[o] = s;
  }
}

template <int VPT>
__device__ __forceinline__ void gamma_block(const GammaPlan* __restrict__ gp, int w) {
  extern __shared__ __attribute__((aligned(16))) unsigned char gm_smem[];
  double* sm = (double*)gm_smem;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = gp->n, npre = gp->npre, hasx = gp->hasx;
  const int npp = gp->npp, nqc = gp->nqc;
  const int py = n - 1, px = n - 2;
  const int Ky = n >= 2 ? gp->dim[py] : 0, npy = n >= 2 ? gp->np[py] : 1;
  const int Kx = hasx ? gp->dim[px] : 0, npx = hasx ? gp->np[px] : 1;
  const int yg = w % gp->nyg, qg = w / gp->nyg;
  const int py0 = yg * gp->pyw, npyw = min(gp->pyw, npy - py0);   // this workgroup's y pairs
  const double* __restrict__ W64 = gp->W64;
  const double* __restrict__ G = gp->G;
  double* gy = sm + gp->o_gy;
  double* gx = sm + gp->o_gx;
  double* wa = sm + gp->o_wa;           // stage-A rows: W_xy^2 (x mode) or W_{0y}^2 of the tuples (n == 2)
  double* cq = sm + gp->o_cq;
  double* wb = sm + gp->o_wb;
  double* T = sm + gp->o_t;
  double* Y = sm + gp->o_y;
  double* cp = sm + gp->o_cp;
  int* pr = (int*)(sm + gp->o_pr);      // [n][MAXP]: r | r' << 8
  const int qa = qg * gp->qpw;
  const int nqw = (int)min((long long)gp->qpw, gp->nq - qa);   // prefix tuples of this workgroup

  // ---- everything the chunks read, gathered into LDS once (wide batches) ----
  for (int e = tid; e < n * MAXP; e += NT) {
    const int pos = e / MAXP, p = e - pos * MAXP;
    const int R = gp->rank[pos];
    int r = 0;
    while (r + 1 < R && (r + 1) * R - (r + 1) * r / 2 <= p) ++r;
    const int rr = min(R - 1, r + (p - (r * R - r * (r - 1) / 2)));
    pr[e] = r | (rr << 8);
  }
  // prefix index of mode s (s < npre) for tuple q (row-major over the prefix modes)
  const int d1 = npre == 2 ? gp->dim[1] : 1;
  auto pidx = [&](int q, int s) { return s == 0 ? q / d1 : q % d1; };
  if (hasx) {
    // the y and x factors, the squared x-y edge and the squared prefix edges
    // towards y and x per tuple: the first round of all five (4 + 4 + 24 +
    // 2 x 8 + 2 x 4 loads per thread) in flight together, the rest in batches
    const double* srcy = G + gp->goff[py];
    const double* srcx = G + gp->goff[px];
    const int ny = gp->rank[py] * Ky, nx = gp->rank[px] * Kx, nxy = Kx * Ky, ncq = nqw * Ky, nwb = nqw * Kx;
    const EdgeRef exy = gp->e[px][py];
    const EdgeRef e0y = gp->e[0][py], e1y = gp->e[npre == 2 ? 1 : 0][py];
    const EdgeRef e0x = gp->e[0][px], e1x = gp->e[npre == 2 ? 1 : 0][px];
    const int s1 = npre == 2 ? 1 : 0;   // without a second prefix mode the b loads repeat the a address
    auto axy = [&](int e) {
      const int x = e / Ky, y = e - x * Ky;
      return W64 + exy.off + (long long)x * exy.s1 + (long long)y * exy.s2;
    };
    auto acq = [&](int e, int s) {
      const int qq = e / Ky, y = e - qq * Ky, q = qa + qq;
      const EdgeRef& ed = s ? e1y : e0y;
      return W64 + ed.off + (long long)pidx(q, s) * ed.s1 + (long long)y * ed.s2;
    };
    auto awb = [&](int e, int s) {
      const int qq = e / Kx, x = e - qq * Kx, q = qa + qq;
      const EdgeRef& ed = s ? e1x : e0x;
      return W64 + ed.off + (long long)pidx(q, s) * ed.s1 + (long long)x * ed.s2;
    };
    double vy[4], vx[4], va[24], vq[8], vq2[8], vb[4], vb2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) vy[u] = srcy[min(tid + u * NT, ny - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) vx[u] = srcx[min(tid + u * NT, nx - 1)];
#pragma unroll
    for (int u = 0; u < 24; ++u) va[u] = *axy(min(tid + u * NT, nxy - 1));
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      vq[u] = *acq(min(tid + u * NT, ncq - 1), 0);
      vq2[u] = *acq(min(tid + u * NT, ncq - 1), s1);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      vb[u] = *awb(min(tid + u * NT, nwb - 1), 0);
      vb2[u] = *awb(min(tid + u * NT, nwb - 1), s1);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      vy[u] = pin(vy[u]);
      vx[u] = pin(vx[u]);
      vb[u] = pin(vb[u]);
      vb2[u] = pin(vb2[u]);
    }
#pragma unroll
    for (int u = 0; u < 24; ++u) va[u] = pin(va[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      vq[u] = pin(vq[u]);
      vq2[u] = pin(vq2[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + u * NT;
      if (e < ny) gy[e] = vy[u];
      if (e < nx) gx[e] = vx[u];
      if (e < nwb) wb[e] = gm_sq(vb[u]) * (s1 ? gm_sq(vb2[u]) : 1.0);
    }
#pragma unroll
    for (int u = 0; u < 24; ++u)
      if (tid + u * NT < nxy) wa[tid + u * NT] = gm_sq(va[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (tid + u * NT < ncq) cq[tid + u * NT] = gm_sq(vq[u]) * (s1 ? gm_sq(vq2[u]) : 1.0);
    for_batched_from<16>(4 * NT, ny, [&](int e) { return srcy[e]; }, [&](int e, double v) { gy[e] = v; });
    for_batched_from<16>(4 * NT, nx, [&](int e) { return srcx[e]; }, [&](int e, double v) { gx[e] = v; });
    for_batched_from<16>(24 * NT, nxy, [&](int e) { return *axy(e); }, [&](int e, double v) { wa[e] = gm_sq(v); });
    for_batched_from<16>(
        8 * NT, ncq, [&](int e) { return gm_sq(*acq(e, 0)) * (s1 ? gm_sq(*acq(e, 1)) : 1.0); },
        [&](int e, double v) { cq[e] = v; });
    for_batched_from<16>(
        4 * NT, nwb, [&](int e) { return gm_sq(*awb(e, 0)) * (s1 ? gm_sq(*awb(e, 1)) : 1.0); },
        [&](int e, double v) { wb[e] = v; });
  } else if (n == 2) {
    const double* src = G + gp->goff[py];
    for_batched<16>(gp->rank[py] * Ky, [&](int e) { return src[e]; }, [&](int e, double v) { gy[e] = v; });
    const EdgeRef e0y = gp->e[0][py];
    for_batched<16>(
        nqw * Ky,
        [&](int e) {
          const int qq = e / Ky, y = e - qq * Ky;
          return W64[e0y.off + (long long)(qa + qq) * e0y.s1 + (long long)y * e0y.s2];
        },
        [&](int e, double v) { wa[e] = gm_sq(v); });
  }
  __syncthreads();                      // pr is complete
  {
    const EdgeRef e01 = gp->e[0][npre == 2 ? 1 : 0];
    const double* G0 = G + gp->goff[0];
    const double* G1 = G + gp->goff[npre == 2 ? 1 : 0];
    const int I0 = gp->dim[0], I1 = npre == 2 ? gp->dim[1] : 1, np1 = npre == 2 ? gp->np[1] : 1;
    for_batched<8>(
        nqw * npp,
        [&](int e) {
          const int qq = e / npp, pp = e - qq * npp, q = qa + qq;
          const int i0 = pidx(q, 0), i1 = npre == 2 ? pidx(q, 1) : 0;
          const int p0 = npre == 2 ? pp / np1 : pp, p1 = npre == 2 ? pp - p0 * np1 : 0;
          const int rp0 = pr[p0], rp1 = npre == 2 ? pr[MAXP + p1] : 0;
          double c = G0[(long long)(rp0 & 255) * I0 + i0] * G0[(long long)(rp0 >> 8) * I0 + i0];
          if (npre == 2)
            c *= gm_sq(W64[e01.off + (long long)i0 * e01.s1 + (long long)i1 * e01.s2]) *
                 G1[(long long)(rp1 & 255) * I1 + i1] * G1[(long long)(rp1 >> 8) * I1 + i1];
          return c;
        },
        [&](int e, double v) { cp[e] = v; });
  }

  // this workgroup's Gamma entries: (p_pre, p_x, p_y in the y group), row-major;
  // accumulated as the product cP^T Y over the tuples on the matrix cores:
  // wave wv owns the 16 x 16 tiles wv, wv + 4, ... of the npp x NYw result
  const int NYw = hasx ? npx * npyw : npyw;    // Y entries per tuple (n == 1: one)
  const int Pw = npp * NYw;
  const int AMT = (npp + 15) >> 4, ANT = (NYw + 15) >> 4;
  gm_d4 V[VPT];
#pragma unroll
  for (int v = 0; v < VPT; ++v) V[v] = gm_d4{0.0, 0.0, 0.0, 0.0};

  for (int q0 = 0; q0 < nqw; q0 += nqc) {
    const int nc = min(nqc, nqw - q0);
    __syncthreads();                      // tables complete / the previous chunk's T and Y are free
    // stage A on the matrix cores, operands from LDS: columns (tuple, y pair)
    if (n >= 2) {
      const int M = hasx ? Kx : nc;
      const int Ncol = hasx ? nqc * npyw : npyw;
      const int MT = (M + 15) >> 4, NTL = (Ncol + 15) >> 4;
      for (int tile = wv; tile < MT * NTL; tile += NT / 64) {
        const int mt = tile / NTL, nt = tile - mt * NTL;
        const int row = mt * 16 + (lane & 15);
        const int col = nt * 16 + (lane & 15);
        const bool aok = row < M;
        const double* arow = wa + (long long)(hasx ? min(row, M - 1) : q0 + min(row, M - 1)) * Ky;
        int qq = 0, pl = col;
        if (hasx) {
          qq = col / npyw;
          pl = col - qq * npyw;
        }
        const bool bok = col < Ncol && qq < nc;
        const int rp = pr[py * MAXP + py0 + (bok ? pl : 0)], r = rp & 255, rr = rp >> 8;
        const double* g1 = gy + r * Ky;
        const double* g2 = gy + rr * Ky;
        const double* cqr = cq + (hasx ? (q0 + min(qq, nc - 1)) * Ky : 0);
        gm_d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < Ky; k0 += 16) {
          // operands read at clamped indices, every read of the step issued
          // before the first use; out-of-range terms are zeroed afterwards
          double av[4], bv[4], b1v[4], b2v[4], b3v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int yc = min(k0 + 4 * u + (lane >> 4), Ky - 1);
            av[u] = arow[yc];
            b1v[u] = g1[yc];
            b2v[u] = g2[yc];
            b3v[u] = hasx ? cqr[yc] : 1.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            av[u] = pin(av[u]);
            b1v[u] = pin(b1v[u]);
            b2v[u] = pin(b2v[u]);
            b3v[u] = pin(b3v[u]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int y = k0 + 4 * u + (lane >> 4);
            av[u] = (aok && y < Ky) ? av[u] : 0.0;
            bv[u] = (bok && y < Ky) ? b1v[u] * b2v[u] * b3v[u] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc = gm_mfma(av[u], bv[u], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int orow = mt * 16 + (lane >> 4) + 4 * v, ocol = nt * 16 + (lane & 15);
          if (orow < M && ocol < Ncol) T[orow * Ncol + ocol] = acc[v];
        }
      }
      __syncthreads();
    }
    // stage B (x mode): Y_q(p_x, p_y) = sum_x wB_q(x) GG_x(x, p_x) T_q(x, p_y)
    if (hasx) {
      const int Ncol = nqc * npyw;
      for (int e = tid; e < nc * NYw; e += NT) {
        const int qq = e / NYw, t = e - qq * NYw;
        const int pxi = t / npyw, pyl = t - pxi * npyw;
        const int rp = pr[px * MAXP + pxi], r = rp & 255, rr = rp >> 8;
        const double* g1 = gx + r * Kx;
        const double* g2 = gx + rr * Kx;
        const double* wq = wb + (q0 + qq) * Kx;
        const double* tc = T + qq * npyw + pyl;
        double s = 0.0;
        for (int x0 = 0; x0 < Kx; x0 += 4) {     // four x at a time, loads first
          double a[4], b[4], c[4], d[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int x = min(x0 + u, Kx - 1);
            a[u] = wq[x];
            b[u] = g1[x];
            c[u] = g2[x];
            d[u] = tc[x * Ncol];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a[u] = pin(a[u]);
            b[u] = pin(b[u]);
            c[u] = pin(c[u]);
            d[u] = pin(d[u]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (x0 + u < Kx) s += a[u] * b[u] * c[u] * d[u];
        }
        Y[e] = s;
      }
      __syncthreads();
    }
    // partial Gamma entries += cP^T Y over this chunk's tuples (K = nc)
    const double* Ys = hasx ? Y : T;
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
      const int tile = wv + 4 * v;
      if (tile < AMT * ANT) {
        const int mt = tile / ANT, nt = tile - mt * ANT;
        const int row = mt * 16 + (lane & 15), col = nt * 16 + (lane & 15);
        const int rowc = min(row, npp - 1), colc = min(col, NYw - 1);
        // four matrix-core steps per batch of operand reads (clamped
        // indices, all reads in flight before the first step; terms out of
        // range zeroed), k in the same order as one step at a time
        for (int k0 = 0; k0 < nc; k0 += 16) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kc = min(k0 + 4 * u + (lane >> 4), nc - 1);
            av[u] = cp[(q0 + kc) * npp + rowc];
            bv[u] = n >= 2 ? Ys[kc * NYw + colc] : 1.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            av[u] = pin(av[u]);
            bv[u] = pin(bv[u]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = k0 + 4 * u + (lane >> 4);
            if (k0 + 4 * u < nc) {        // uniform: the step has at least one k in range
              const bool kok = k < nc;
              const double a = (kok && row < npp) ? av[u] : 0.0;
              const double b = (kok && col < NYw) ? bv[u] : 0.0;
              V[v] = gm_mfma(a, b, V[v]);
            }
          }
        }
      }
    }
  }

  // global index of local entry (pp, t): ((p_pre * npx + p_x) * npy + py0 + p_y local)
  auto gidx = [&](int e) {
    const int row = e / npyw, pl = e - row * npyw;
    return row * npy + py0 + pl;
  };
  const int P = gp->P, nqg = gp->nqg;
  double* dstv = nqg == 1 ? gp->gamma : gp->part + (long long)qg * P;   // one prefix range: final
#pragma unroll
  for (int v = 0; v < VPT; ++v) {
    const int tile = wv + 4 * v;
    if (tile < AMT * ANT) {
      const int mt = tile / ANT, nt = tile - mt * ANT;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int pp = mt * 16 + (lane >> 4) + 4 * c, t = nt * 16 + (lane & 15);
        if (pp < npp && t < NYw) dstv[gidx(pp * NYw + t)] = V[v][c];
      }
    }
  }
  // with nqg > 1 the partial rows are summed by gamma_reduce_block in the next launch
}

}  // namespace ifctn
