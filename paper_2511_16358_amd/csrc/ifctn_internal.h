// Internal declarations shared by the HIP kernels and the host orchestration
// of the iFCTN-TC library.  Not part of the public ABI (include/ifctn.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ifctn {

constexpr int MAXN = 5;              // tensor order
constexpr int MAXR = 8;              // edge rank
constexpr int MAXC = MAXN - 2;       // modes other than k and the fibre mode
constexpr int MAXP = MAXR * (MAXR + 1) / 2;  // distinct entries of an R x R Gram matrix
constexpr int NT = 256;              // threads per workgroup (4 wavefronts of 64)

// bfloat16 storage of X: the upper half of an IEEE binary32.  Narrowing rounds
// to nearest, ties to even (add 0x7fff plus the lowest kept bit, truncate);
// NaN stays NaN.  Widening is exact.
struct bf16x {
  uint16_t v;
  bf16x() = default;
  __device__ explicit bf16x(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u)
      v = (uint16_t)((u >> 16) | 0x40u);
    else
      v = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
  __device__ explicit operator float() const { return __uint_as_float((uint32_t)v << 16); }
};

// kernel data types: X storage / streaming arithmetic
enum KType { KT_F32 = 0, KT_F64 = 1, KT_BF16 = 2 };  // KT_BF16: bf16 X, float arithmetic

// Oriented reference to an edge matrix: W(i_first, i_second) lives at
// base[off + i_first * s1 + i_second * s2].  Edge {a,b}, a < b, is stored
// row-major I_a x I_b, so the reversed orientation just swaps the strides.
struct EdgeRef {
  long long off;
  int s1, s2;
};

// Q_{k,i}(d; r, r') = sum_{i_i} S_k(i_{-k})^2 G_{i,k}(r, i_i) G_{i,k}(r', i_i),
// d = index over the modes other than k and i; constant during block k.
struct QItem {               // one i != k
  int Ii, R, lg2P, CH;        // lanes per d = 2^lg2P (<= 64), fibre chunk per lane
  long long D, qoff, gik;     // d count, offset of Q_{k,i}, offset of G_{i,k}
  int ddim[MAXC];
  EdgeRef edi[MAXC];          // W(i_m, i_i), m in d
  int dd_a[3], dd_b[3];
  EdgeRef edd[3];             // W(i_a, i_b), a, b in d
};

// What a workgroup of Gram weights needs (device records and buffers)
struct GramRef {
  const QItem* dit;
  int ni, nd, ndd;
  long long blk0[MAXN];
  const double* W64;
  const double* G;
  double* Q;
};

struct QArgs {
  int ni, nd, ndd;
  long long blk0[MAXN];       // first workgroup of each i; blk0[ni] = total
  QItem it[MAXN - 1];         // host copy (plans, sizes)
  const QItem* dit;           // device copy read by the kernel
  const double* W64;
  const double* G;
  double* Q;
  const int* stop;            // device stop flag: nonzero = the job has met its stop test
};

// Gram matrix of the mode-k cherry sub-network (Prop. 1), Gamma_k = Z_k^T Z_k:
//   Gamma_k(r, r') = sum_{i_{-k}} S_k(i_{-k})^2 prod_{m != k} G_{m,k}(r_m, i_m) G_{m,k}(r'_m, i_m).
// It depends on every mode m != k only through the unordered pair {r_m, r'_m},
// so it is stored with one packed pair index per mode (np = R (R + 1) / 2
// values, p(r, r') = r R - r (r - 1) / 2 + (r' - r) for r <= r'), row-major
// over the modes in "Gamma order": the prefix modes, then x (orders >= 4),
// then y (orders >= 3).  Gamma_k needs no X and no factor owned by mode k, so
// one Gamma_k serves every column and every sub-block of factor block k:
//   H_j = (I (x) c_j)^T Gamma_k (I (x) c_j),  c_j = Kronecker product of the
// own-side columns G_{k,m}(:, j), m != k, i -- the Gram term of eq. (updateG).
constexpr int GM_PMAX = 6144;   // entries of Gamma_k (kept in LDS by the solve)
constexpr int GM_QG = 8;        // prefix ranges (partial sums per Gamma entry), at most
constexpr int GM_MAXW = 128;    // workgroups that build one Gamma_k

struct GammaPlan {
  int n;                        // modes other than k (N - 1)
  int npre;                     // prefix modes: Gamma positions 0 .. npre-1
  int hasx;                     // position n - 2 is the x mode (n >= 3)
  int mode[MAXN - 1], dim[MAXN - 1], rank[MAXN - 1], np[MAXN - 1];
  long long goff[MAXN - 1];     // G_{m,k} (R x I, row-major) in the packed factors
  int st[MAXN - 1];             // stride of each position's pair index in Gamma
  EdgeRef e[MAXN - 1][MAXN - 1];// W(i_a, i_b) for positions a != b
  int P;                        // entries of Gamma
  int npp;                      // pair tuples of the prefix modes
  long long nq;                 // index tuples of the prefix modes
  int qpw, nqc;                 // prefix tuples per workgroup, per LDS chunk
  // workgroup w = (y group w % nyg, prefix range w / nyg): the y pair
  // indices [yg * pyw, +pyw) of Gamma over prefix tuples [qg * qpw, +qpw);
  // with nqg > 1 the partial rows are summed by the next launch
  int nyg, pyw, nqg;
  int nw;                       // nyg * nqg
  double fma;                   // multiply-adds of the build (stage A + B + accumulation)
  int smem;                     // LDS bytes of a workgroup
  // LDS offsets (doubles)
  int o_gy, o_gx, o_wa, o_cq, o_wb, o_t, o_y, o_cp, o_pr;
  const double* W64;
  const double* G;
  double* part;                 // [nqg][P] partial sums (each y group writes its entries)
  double* gamma;                // [P]
  // the launch after Gamma_k's (and after the contraction of block k): nuw
  // workgroups reduce the contraction's partial slots into the U rows (NT / us
  // outputs each, every output summed in us slices of the S slots), then nred
  // workgroups sum the nqg partial rows of Gamma_k
  int nuw, S, us;
  int nred;
  long long nout;               // I_k * Rprod
  const double* Upart;          // [S][nout]
  double* Ufin;                 // [nout]
};

// Factor block k by the Gamma route: one workgroup per column j; per sub-block (i ascending) H_j from Gamma_k and the current
// own-side columns (a chain of small contractions in LDS), b_j from the U
// row, LDL^T, then rows j of every W_{k,m} refreshed at the end of the block.
struct GSolve {
  int k, Ik, n, P, Rprod, S;
  double rho;
  int R[MAXN - 1], np[MAXN - 1], dim[MAXN - 1];
  int gst[MAXN - 1];             // Gamma stride of U position t's pair index
  int ust[MAXN - 1];             // canonical U column stride of U position t
  int ord[MAXN - 1][MAXN - 2];   // sub-block t: U positions contracted, in order
  long long goff_ki[MAXN - 1], goff_ik[MAXN - 1];
  long long w_off[MAXN - 1];
  int w_sj[MAXN - 1], w_sy[MAXN - 1];
  int scr;                       // doubles of each per-wave contraction scratch buffer
  // the contraction chains of sub-block t: for H (c = 0 .. n-2, over Gamma
  // with the pair weights) and for b (over the U row with the own-side
  // columns): stage c contracts U position hord/bord[t][c]; its output o
  // reads the input at tab[hoff/boff[t][c] + o] + q * stride, q < extent
  int bord[MAXN - 1][MAXN - 2];
  int hoff[MAXN - 1][MAXN - 2], hnout[MAXN - 1][MAXN - 2], hsc[MAXN - 1][MAXN - 2];
  int boff[MAXN - 1][MAXN - 2], bnout[MAXN - 1][MAXN - 2], bsc[MAXN - 1][MAXN - 2];
  int tabtot;                    // ints of all offset tables (LDS copy of tab)
  const int* tab;                // offset tables, built on the host
  int gik_lds;                   // 1: the far-side factors G_{i,k} are staged in LDS for the row refresh
  int gik_off[MAXN - 1];         // their offsets in that LDS region (doubles)
  int gik_tot;
  int smem;                      // LDS bytes
  const double* gamma;
  const double* Upart;
  double* W64;
  void* Wc;
  double* G;
  double* dgpart;                // [n][Ik]
  const int* stop;
};

// LDS of the Gamma-route solve (one column per workgroup): Gamma_k and the
// pair tables, the U row, own-side columns, pair weights, four contraction
// buffers (two for H, two for b), H, b; the far-side factors; the offset
// tables.
__host__ __device__ inline int gsolve_wave_doubles(int n, int Rprod, int scr) {
  const int v = Rprod + n * MAXR + n * MAXP + 4 * scr + MAXP + 3 * MAXR;
  return (v + 1) & ~1;
}

__host__ __device__ inline int gsolve_smem(int n, int P, int Rprod, int scr, int gik, int tabtot) {
  const int prd = (n * MAXP + 1) / 2;
  return 8 * (P + prd + gsolve_wave_doubles(n, Rprod, scr) + gik + (tabtot + 1) / 2);
}

// Mode-k contraction U_k(j, r_{-k}) = sum_{i_{-k}} X(i) S_k(i_{-k}) prod_{m != k}
// G_{m,k}(r_m, i_m), organised by "planes": for a fixed index c of the modes
// other than k and the fibre mode f, the plane is the I_k x I_f slice of X.
// Optionally fused with the X step of the previous sweep (k == 0).
struct ContractArgs {
  int k, f, nc;
  int Ik, If, LDF;
  long long stride_k, stride_f;
  int cdim[MAXC];
  long long cstride[MAXC];
  int crank[MAXC];       // R_{m,k} of each c-mode
  long long gcoff[MAXC]; // offset of G_{m,k} (R_{m,k} x I_m) in the packed factors
  long long gfoff;       // offset of G_{f,k} (R_{f,k} x I_f)
  int Rf, Rc, Rprod;
  EdgeRef ecf[MAXC];     // W(i_m, i_f) for each c-mode m
  int ncc;               // edges among c-modes
  int cc_a[3], cc_b[3];
  EdgeRef ecc[3];
  long long ustc[MAXC];   // canonical U column stride of each c-mode
  long long ustf;         // canonical U column stride of the fibre mode
  // tiling: the X elements of a batch are enumerated over three axes
  // (0 = j, 1 = plane, 2 = fibre) in the order ord[0] (outer) .. ord[2]
  // (inner), i.e. by decreasing memory stride, so that consecutive lanes
  // touch consecutive addresses
  int ord[3];
  int jn, PB, JT, S;
  int fch;               // lanes sharing one fibre dot product (power of two <= 64)
  int psplit;            // threads sharing one accumulator slot (planes split round-robin)
  // kernel variant: 0 = generic LDS tile, 1 = rows (fibre mode contiguous,
  // lanes split each fibre), 2 = columns (mode k contiguous, lanes along j)
  int kind;
  int plfast;            // rows: consecutive planes are closer in memory than consecutive j
  int FS;                // columns: fibre range split over FS workgroups (partials S * FS)
  long long PPW, nplanes;
  // staged accumulation (two or more c-modes): the planes of a batch come in
  // whole groups of the last c-mode (size cdl, rank Rl); that mode is
  // contracted first, U then accumulates over the groups with the product of
  // the other c-modes' factors (Rc2 = Rc / Rl terms) instead of over planes
  int stage, cdl, Rl, Rc2;
  long long gloff;       // offset of G_{m_last,k} (Rl x cdl)
  // fused X step (k == 0 only)
  EdgeRef e0c[MAXC];     // W(i_0, i_m) for the c-modes
  EdgeRef e0f;           // W(i_0, i_f)
  double rho_x;
  // buffers
  void* X;
  const uint32_t* maskbits;
  const void* Wc;        // edge matrices in the streaming precision
  const double* G;       // packed float64 factors
  double* Upart;         // [S][I_k][Rprod] split partial sums
  double* normpart;      // [blocks][3]: ||dX||^2, ||X||^2, ||X_new - Xhat||^2
  const int* stop;       // device stop flag (every launch of a stopped job is a no-op)
  // the Gram weights of the same block, computed by gblocks extra workgroups
  // of the launch (they depend on the same inputs as the contraction)
  int gblocks;
  GramRef gr;
  // grouped partial sums: with ugrp > 0 the last workgroup of each group of
  // ugrp consecutive partial slots of a j-tile to finish (arrival counter
  // ucnt[jt * ngrp + g]) adds the group's slots in slot order into Ugrp[g];
  // the solve then reduces ngrp slots instead of S * FS
  int ugrp, ngrp;
  double* Ugrp;          // [ngrp][I_k][Rprod]
  int* ucnt;             // [JT][ngrp], zero between launches
};

// Factor block k (all G_{k,i}, i != k, in ascending i), one workgroup per
// column j.  Column j of every G_{k,i} depends only on row j of the edge
// matrices of mode k (plus factors owned by other modes, fixed during block
// k), so the Gauss-Seidel chain over i runs inside the workgroup.
struct SubBlock {
  int i, Ii, R, np, upos;
  int nd;
  long long D;
  int ddim[MAXC];
  int dt[MAXC];          // U-mode index of each d-mode
  const double* Q;       // Q_{k,i}: [D][np]
  long long goff_ki, goff_ik;
  long long w_off;
  int w_sj, w_sy;        // W_{k,i}(j, y) at w_off + j * w_sj + y * w_sy
};

struct SolveArgs {
  int k, Ik, nsub;
  double rho;
  SubBlock sb[MAXN - 1];
  int Rprod, nu;
  int udim[MAXN - 1];
  int urank[MAXN - 1];
  long long ustride[MAXN - 1];
  long long ugoff[MAXN - 1];     // G_{k,m} for each U mode m (modes != k ascending)
  int rowoff[MAXN - 1];          // LDS offset of the row W_{k,m}(j, :)
  int rowtot;
  EdgeRef ekm[MAXN - 1];         // W(j, i_m) for each U mode (float64 edge matrices)
  int S;
  const double* Upart;
  double* W64;
  void* Wc;
  double* G;
  double* dgpart;                // [nsub][Ik]
  const int* stop;               // device stop flag
};

// Phased factor block, for blocks whose Gram weight sets are large (many d):
// per sub-block, k_hpart forms partial H_j over ranges of d for a tile of
// columns (the Q range and the weights staged in LDS, Q read once per tile),
// then k_solve_col reduces the partials of column j in a fixed order, forms
// b_j, solves and refreshes row j of W_{k,i}.  The Gauss-Seidel order over i
// is kept by launching the sub-blocks one after another.
constexpr int HP_JW = 16;     // max columns per k_hpart workgroup (power of two)
constexpr int HS_JW = 4;      // columns per workgroup of the one-launch form (one wave each)
constexpr int HP_DC = 28;     // d per k_hpart workgroup (many short workgroups: measured best on the served mix)

struct PhaseArgs {
  SubBlock B;
  int t;                      // sub-block index (row of the block's dgpart)
  int k, Ik, nu, Rprod;
  double rho;
  int urank[MAXN - 1];
  long long ustride[MAXN - 1];
  long long ugoff[MAXN - 1];
  EdgeRef edm[MAXC];          // W_{k,m}(j, i_m) for the d-modes of this sub-block
  int JW, JT, KS;             // column tile, column tiles, d ranges
  const double* Ufin;         // [Ik][Rprod]
  double* Hpart;              // [KS][Ik][np]
  int* cnt;                   // [JT] arrival counters of the one-launch form (zero between launches)
  double* W64;
  void* Wc;
  double* G;
  double* dgpart;             // the block's [nsub][Ik]
  const int* stop;
};

struct ReconArgs {
  int N;
  int dims[MAXN];
  long long nX;
  int ne;
  int ea[10], eb[10];
  long long woff[10];
  const void* Wc;
  void* out;
};

// --------------------------------------------------------------------------
// Large-rank route: the factor blocks of a job with any edge rank above MAXR
// (up to LR_MAXR).  Every quantity of eq. (updateG) is formed explicitly in
// float64 with rank-generic kernels:
//   Y   = X o D_{-k}                 (D_{-k}: the edge factors not touching k)
//   U_k = Y x_{a != k} G_{a,k}       (one mode product per mode a != k)
//   c_j(y) = sum over the other modes of the squared edge factors, so that
//   H_j = G_{i,k} diag(c_j) G_{i,k}^T + rho I,  b_j = U_k(j) . (g_{k,a})_{a != k,i} + rho g_j
// and one Cholesky factorisation per column.
// --------------------------------------------------------------------------
constexpr int LR_MAXR = 36;                              // IFCTN_MAX_RANK
constexpr int LR_MAXP = LR_MAXR * (LR_MAXR + 1) / 2;     // distinct entries of a 36 x 36 Gram matrix

struct LrEdge {          // W(x, y) = W64[off + x * s1 + y * s2], either orientation of a stored W_ab
  long long off, s1, s2;
};

// Y = X o D_{-k}: X times every edge factor W_ab(i_a, i_b) with a, b != k
struct LrYArgs {
  int N;
  int dims[MAXN];
  long long nX;
  int ne;
  int ea[10], eb[10];
  long long woff[10];
  const void* X;
  const double* W64;
  double* Y;
  const int* stop;
};

// out[a][n][b] = sum_x in[a][x][b] * B(n, x) for a < A, n < Nn, b < Bn, x < I,
// with B(n, x) = Bm[n * ldb + x], or for pairR > 0 the packed Gram pair
// n = (r, r'), r <= r' < pairR: B(n, x) = Bm[r * ldb + x] * Bm[r' * ldb + x]
struct LrGemmArgs {
  long long A, Bn;
  int I, Nn, pairR;
  long long ldb;
  const double* in;
  const double* Bm;
  double* out;
  const int* stop;
};

// c(j, y) for j < Ik (mode k), y < Ii (mode i): over the nr = N - 2 other
// modes a, the sum of prod_a W_ka(j, x_a)^2 W_ia(y, x_a)^2 times
// prod_{pairs a < b} W_ab(x_a, x_b)^2
struct LrCArgs {
  int Ik, Ii, nr;
  int rdim[MAXN];
  LrEdge ek[MAXN], ei[MAXN];
  int npr;
  int pa[10], pb[10];       // positions in rdim
  LrEdge ep[10];
  const double* W64;
  double* c;
  const int* stop;
};

// one column j of G_{k,i} per workgroup: b_j from U_k, H_j from the packed
// Gram rows, Cholesky, the new column and its ||dg||^2
struct LrSolveArgs {
  int Ik, R, nr;
  double rho;
  const double* U;
  long long ustr_j, ustr_i;
  long long ustr[MAXN];     // the other modes a != k, i
  int urank[MAXN];
  long long goff_o[MAXN];   // G_{k,a} of those modes
  long long goff_ki;
  const double* H;          // [Ik][R (R + 1) / 2]
  double* G;
  double* dgpart;           // [Ik] of this sub-block
  const int* stop;
};

// eq. (updateX) with the reconstruction of eq. (iFCTN) from W64 and the
// partial norms {||dX||^2, ||X||^2, ||X_new - Xhat||^2} of each workgroup
struct LrXArgs {
  int N;
  int dims[MAXN];
  long long nX;
  int ne;
  int ea[10], eb[10];
  long long woff[10];
  void* X;
  const uint32_t* bits;
  const double* W64;
  double rx, inv1;
  double* normpart;
  const int* stop;
};

// Per-launch timing (events set by set_kernel_events; see ifctn_kernels.hip):
// with events set, a launcher goes through hipExtLaunchKernel, which stamps
// the start event with its first kernel's start and the stop event with the
// last kernel's end.
extern thread_local hipEvent_t tl_ev_start, tl_ev_stop;
extern thread_local bool tl_ev_used;

#define IFCTN_GO(kern, grid, blk, smem, s, ...)                                                   \
  do {                                                                                            \
    if (tl_ev_start) {                                                                            \
      hipExtLaunchKernelGGL(kern, grid, blk, smem, s, tl_ev_used ? nullptr : tl_ev_start,          \
                            tl_ev_stop, 0u, __VA_ARGS__);                                          \
      tl_ev_used = true;                                                                          \
    } else {                                                                                      \
      hipLaunchKernelGGL(kern, grid, blk, smem, s, __VA_ARGS__);                                  \
    }                                                                                             \
  } while (0)

hipError_t launch_lr_y(int dtype, const LrYArgs& a, hipStream_t s);
hipError_t launch_lr_gemm(const LrGemmArgs& a, hipStream_t s);
hipError_t launch_lr_c(const LrCArgs& a, hipStream_t s);
hipError_t launch_lr_solve(const LrSolveArgs& a, hipStream_t s);
hipError_t launch_lr_x(int dtype, const LrXArgs& a, int nblk, hipStream_t s);

// kernel classes for timing
enum KernelClass { KC_CONTRACT = 0, KC_SOLVE = 1, KC_UPDATE = 2, KC_GRAM = 3, KC_UROW = 4, KC_COUNT = 5 };

// ---- launchers (ifctn_kernels.hip) ----------------------------------------
// dtype: 0 = float32 streaming data, 1 = float64
hipError_t launch_init_x(int dtype, const void* O, const uint8_t* mask, void* X, uint32_t* maskbits,
                         int* bad_flag, long long nX, hipStream_t s);
// part[b], cnt[b]: sum of O^2 and count over the observed entries seen by
// workgroup b of nblocks (grid-stride)
hipError_t launch_obs_sumsq(int dtype, const void* O, const uint8_t* mask, long long nX, double* part,
                           unsigned long long* cnt, int nblocks, hipStream_t s);
// X_bf16 = bf16(X32) / out = observed ? X32 : float(X_bf16) (exact widening)
hipError_t launch_narrow(const float* X32, bf16x* Xb, long long nX, hipStream_t s);
hipError_t launch_widen(const bf16x* Xb, const uint32_t* maskbits, const float* X32, float* out, long long nX,
                        hipStream_t s);
hipError_t launch_edge(int dtype, const double* Gab, const double* Gba, int R, int Ia, int Ib,
                       double* W64, void* Wc, hipStream_t s);
// one per X storage type (ifctn_contract_*.hip)
hipError_t launch_contract_f32(bool upd, bool con, int spt, const ContractArgs& a, size_t smem, hipStream_t s);
hipError_t launch_contract_f64(bool upd, bool con, int spt, const ContractArgs& a, size_t smem, hipStream_t s);
hipError_t launch_contract_bf16(bool upd, bool con, int spt, const ContractArgs& a, size_t smem, hipStream_t s);
hipError_t launch_contract(int dtype, bool upd, bool con, int spt, const ContractArgs& a,
                           size_t smem, hipStream_t s);
size_t contract_smem_bytes(int dtype, const ContractArgs& a);
hipError_t launch_q(const QArgs& a, hipStream_t s);
// events stamped with the next hot-path kernel's start and end (nullptr = off)
void set_kernel_events(hipEvent_t start, hipEvent_t stop);
bool kernel_events_used();
hipError_t launch_solve(int dtype, const SolveArgs& a, hipStream_t s);
// Gamma route: Gamma_k in a launch of its own (gm: device copy of hp), and the solve
// part 1: Gamma_k (no dependence on X or U_k); part 2, after it and after the
// contraction of block k: the U rows and the sum of Gamma_k's partial rows;
// part 3: the U rows alone (after the contraction); part 4: the partial-row
// sum alone (after Gamma_k)
hipError_t launch_gamma(const GammaPlan& hp, const GammaPlan* gm, const int* stop, hipStream_t s, int part);
hipError_t launch_solve_gamma(int dtype, const GSolve& hs, const GSolve* gs, hipStream_t s);
size_t solve_smem_bytes(const SolveArgs& a);
// phased factor block: U rows into Ufin, then per sub-block k_hpart + k_solve_col
hipError_t launch_urow(const SolveArgs& a, double* Ufin, hipStream_t s);
hipError_t launch_hpart(const PhaseArgs& a, hipStream_t s);
hipError_t launch_solve_col(int dtype, const PhaseArgs& a, hipStream_t s);
// one launch per sub-block: partial H as k_hpart, then the last workgroup of
// each column tile (a.JW <= 4) reduces and solves its columns, one wave each
hipError_t launch_hsolve(int dtype, const PhaseArgs& a, hipStream_t s);
hipError_t launch_reconstruct(int dtype, const ReconArgs& a, hipStream_t s);
// Stop test of Algorithm 1 on the device, after an X step: reduces the
// partial norms like launch_finalize and, unless state[0] (stop flag) is
// already set, counts the sweep in state[1] and sets state[0] when
// ||dX|| / ||X|| < eps.
hipError_t launch_stop_test(const double* normpart, int nnorm, double eps, int* state, hipStream_t s);
hipError_t launch_finalize(const double* normpart, int nnorm, const double* dgpart, int ndg,
                           double* out5, hipStream_t s);

}  // namespace ifctn
