// Host side of the iFCTN-TC library: the C ABI of include/ifctn.h, job state,
// work plans for the kernels and the order of the PAM sweep (Algorithm 1 of
// arXiv 2511.16358: factor blocks k ascending, i ascending, then the X step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ifctn.h"
#include "ifctn_host.h"
#include "ifctn_internal.h"

using namespace ifctn;

namespace {

thread_local std::string g_err;

ifctn_status fail(ifctn_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPTRY(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(e_ == hipErrorOutOfMemory ? IFCTN_E_NOMEM : IFCTN_E_HIP, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                        \
  } while (0)

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct Geo {
  int N = 0;
  int dims[MAXN] = {};
  long long strides[MAXN] = {};
  long long nX = 0;
  int R[MAXN][MAXN] = {};
  int dtype = 0;       // streaming arithmetic and master X: 0 float32, 1 float64
  size_t esz = 4;
  bool bf16 = false;   // BF16_REFINE: X streamed as bfloat16 until the job is promoted
  int refine = 0;      // float32 sweeps that end ifctn_complete in BF16_REFINE mode
  double rho = 0.1, rho_x = 0.1;
  long long goff[MAXN][MAXN] = {};
  long long nG = 0;
  int eid[MAXN][MAXN] = {};
  int ne = 0;
  int ea[10] = {}, eb[10] = {};
  long long woff[10] = {};
  long long nW = 0;
};

constexpr long long kMaxEntries = IFCTN_MAX_ENTRIES;
static_assert(IFCTN_MAX_RANK == LR_MAXR, "the large-rank kernels size their LDS for the largest rank");

ifctn_status make_geo(const ifctn_params* p, Geo* g) {
  if (!p) return fail(IFCTN_E_INVAL, "params is NULL");
  const int N = p->order;
  if (N < 2 || N > IFCTN_MAX_ORDER) return fail(IFCTN_E_INVAL, "order %d outside 2..%d", N, IFCTN_MAX_ORDER);
  if (!(p->rho > 0.0) || !std::isfinite(p->rho)) return fail(IFCTN_E_INVAL, "rho must be > 0");
  if (p->rho_x < 0.0 || !std::isfinite(p->rho_x)) return fail(IFCTN_E_INVAL, "rho_x must be >= 0 (0 = rho)");
  if (p->precision != IFCTN_FP32 && p->precision != IFCTN_FP64 && p->precision != IFCTN_BF16_REFINE)
    return fail(IFCTN_E_INVAL, "unknown precision %d", p->precision);
  if (p->precision == IFCTN_BF16_REFINE ? p->refine_sweeps < 0 : p->refine_sweeps != 0)
    return fail(IFCTN_E_INVAL, "refine_sweeps must be >= 0 for BF16_REFINE and 0 otherwise");
  g->N = N;
  long long nX = 1;
  for (int m = 0; m < N; ++m) {
    if (p->dims[m] < 1) return fail(IFCTN_E_INVAL, "dims[%d] = %lld < 1", m, (long long)p->dims[m]);
    if (p->dims[m] > (1LL << 30)) return fail(IFCTN_E_INVAL, "dims[%d] too large", m);
    if (nX > (1LL << 40) / p->dims[m]) return fail(IFCTN_E_INVAL, "tensor has too many entries");
    nX *= p->dims[m];
    g->dims[m] = (int)p->dims[m];
  }
  // the streaming kernels run one work-item per entry on a 1-D grid, whose
  // work-item count is a 32-bit quantity
  if (nX > kMaxEntries)
    return fail(IFCTN_E_UNSUPPORTED, "tensor has %lld entries; at most %lld are supported", nX, kMaxEntries);
  g->nX = nX;
  long long st = 1;
  for (int m = N - 1; m >= 0; --m) {
    g->strides[m] = st;
    st *= g->dims[m];
  }
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      if (a == b) continue;
      const int r = p->ranks[a][b];
      if (r != p->ranks[b][a]) return fail(IFCTN_E_INVAL, "rank matrix not symmetric at (%d,%d)", a, b);
      if (r < 1) return fail(IFCTN_E_INVAL, "rank R[%d][%d] = %d < 1", a, b, r);
      if (r > IFCTN_MAX_RANK) return fail(IFCTN_E_UNSUPPORTED, "rank %d > %d", r, IFCTN_MAX_RANK);
      g->R[a][b] = r;
    }
  g->dtype = p->precision == IFCTN_FP64 ? 1 : 0;
  g->esz = g->dtype ? 8 : 4;
  g->bf16 = p->precision == IFCTN_BF16_REFINE;
  g->refine = g->bf16 ? p->refine_sweeps : 0;
  g->rho = p->rho;
  g->rho_x = p->rho_x > 0.0 ? p->rho_x : p->rho;
  long long off = 0;
  for (int k = 0; k < N; ++k)
    for (int i = 0; i < N; ++i) {
      if (i == k) continue;
      g->goff[k][i] = off;
      off += (long long)g->R[k][i] * g->dims[k];
    }
  g->nG = off;
  off = 0;
  int e = 0;
  for (int a = 0; a < N; ++a)
    for (int b = a + 1; b < N; ++b) {
      g->eid[a][b] = g->eid[b][a] = e;
      g->ea[e] = a;
      g->eb[e] = b;
      g->woff[e] = off;
      off += (long long)g->dims[a] * g->dims[b];
      ++e;
    }
  g->ne = e;
  g->nW = off;
  return IFCTN_OK;
}

// W(i_a, i_b) for an ordered pair of modes
EdgeRef edge_ref(const Geo& g, int a, int b) {
  EdgeRef r;
  if (a < b) {
    r.off = g.woff[g.eid[a][b]];
    r.s1 = g.dims[b];
    r.s2 = 1;
  } else {
    r.off = g.woff[g.eid[b][a]];
    r.s1 = 1;
    r.s2 = g.dims[a];
  }
  return r;
}

long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// work plans
// ---------------------------------------------------------------------------
struct ContractPlan {
  ContractArgs a;
  int spt;
  size_t smem;
};

constexpr int kTargetBlocks = 1024;

// tuning options (ifctn_set_option): < 0 = default
std::atomic<long long> g_contract_div{-1}, g_contract_emin{-1}, g_merge_gram{-1}, g_onelaunch{-1}, g_contract_jmax{-1},
    g_ugroup{-1}, g_gamma{-1}, g_overlap{-1};
// A factor block takes the phased form when one of its Gram weight sets is
// large: the one-workgroup-per-column kernel would stream all of Q_{k,i}
// through each of only I_k workgroups.
constexpr long long kPhasedMinDefault = 16384;
std::atomic<long long> g_phased_min{-1};

}  // namespace

namespace ifctn {
// The options as they stand now; a job is planned with one snapshot from
// sizing to creation (a server takes it at submit).
PlanOpts current_opts() {
  PlanOpts o;
  long long v;
  v = g_phased_min.load();
  o.phased_min = v >= 0 ? v : kPhasedMinDefault;
  o.onelaunch = g_onelaunch.load() > 0;                  // off by default: measured slower
  o.overlap = g_overlap.load() != 0;
  o.merge_gram = g_merge_gram.load() != 0;
  v = g_contract_div.load();
  o.contract_div = v > 0 ? v : 1280;
  v = g_contract_emin.load();
  o.contract_emin = v > 0 ? v : 4096;
  // at most 8 indices of mode k per workgroup: more, shorter workgroups (each
  // runs its X passes as a chain of dependent loads; with XCD-local numbering
  // neighbouring tiles share their XCD's L2); measured best on the
  // 256 x 256 x 31 workload and on order-4/5 served tensors
  v = g_contract_jmax.load();
  o.contract_jmax = v > 0 ? v : 8;
  // grouped reduction of the contraction's partial slots: off by default --
  // every workgroup's device-scope release (an L2 write-back on this chip,
  // whose L2 is per XCD) made the grouped launches about three times slower;
  // the Gamma route reduces the partials in parallel in its own launch instead
  v = g_ugroup.load();
  o.ugroup = v >= 0 ? v : 0;
  // Gamma route for the blocks whose Gram weight sets are large (where the
  // per-column route would take the phased form); with small sets the
  // per-column route merges its Gram weights into the contraction launch and
  // needs no launch of its own
  v = g_gamma.load();
  o.gamma = v < 0 ? 1 : (int)std::min<long long>(v, 2);
  return o;
}
std::atomic<long long> g_inject_admit{0};

bool take_injected_admit_failure() {
  long long v = g_inject_admit.load();
  while (v > 0)
    if (g_inject_admit.compare_exchange_weak(v, v - 1)) return true;
  return false;
}
}  // namespace ifctn

namespace {

constexpr size_t kMaxLds = 64 << 10;
// the Gamma-route kernels run few workgroups: they may take most of a
// compute unit's 160 KB of LDS (their launchers raise the kernel's limit)
constexpr size_t kMaxLdsGamma = 144 << 10;
constexpr int GM_VPT_HOST = 8;   // accumulation tiles per wave of the Gamma kernel

// fibre mode f: the contiguous last mode when it is long enough, otherwise
// the longest mode != k (the Kronecker accumulation costs Rprod / I_f per element)
int preferred_fibre(const Geo& g, int k) {
  const int N = g.N;
  int f = -1;
  if (k != N - 1 && g.dims[N - 1] >= 16) {
    f = N - 1;
  } else {
    for (int m = 0; m < N; ++m)
      if (m != k && (f < 0 || g.dims[m] >= g.dims[f])) f = m;
  }
  return f;
}

ContractPlan plan_contract_f(const Geo& g, int k, int f, const PlanOpts& o) {
  ContractPlan P;
  ContractArgs& a = P.a;
  std::memset(&a, 0, sizeof(a));
  const int N = g.N;
  a.k = k;
  a.f = f;
  a.Ik = g.dims[k];
  a.If = g.dims[f];
  a.LDF = (a.If % 2 == 0) ? a.If + 1 : a.If;
  a.stride_k = g.strides[k];
  a.stride_f = g.strides[f];
  int cm[MAXC], nc = 0;
  for (int m = 0; m < N; ++m)
    if (m != k && m != f) cm[nc++] = m;
  a.nc = nc;
  // canonical U column strides over the modes != k (ascending, row-major)
  long long ust[MAXN];
  {
    long long s = 1;
    for (int m = N - 1; m >= 0; --m) {
      if (m == k) continue;
      ust[m] = s;
      s *= g.R[k][m];
    }
  }
  a.Rf = g.R[f][k];
  a.ustf = ust[f];
  a.Rc = 1;
  for (int c = 0; c < nc; ++c) {
    const int m = cm[c];
    a.cdim[c] = g.dims[m];
    a.cstride[c] = g.strides[m];
    a.crank[c] = g.R[m][k];
    a.gcoff[c] = g.goff[m][k];
    a.ecf[c] = edge_ref(g, m, f);
    a.ustc[c] = ust[m];
    a.Rc *= a.crank[c];
    if (k == 0) a.e0c[c] = edge_ref(g, 0, m);
  }
  a.gfoff = g.goff[f][k];
  a.Rprod = a.Rc * a.Rf;
  a.ncc = 0;
  for (int x = 0; x < nc; ++x)
    for (int y = x + 1; y < nc; ++y) {
      a.cc_a[a.ncc] = x;
      a.cc_b[a.ncc] = y;
      a.ecc[a.ncc] = edge_ref(g, cm[x], cm[y]);
      ++a.ncc;
    }
  if (k == 0) a.e0f = edge_ref(g, 0, f);
  a.rho_x = g.rho_x;
  a.nplanes = g.nX / ((long long)a.Ik * a.If);
  // enumeration order: axes by decreasing memory stride (j, plane, fibre)
  long long st[3] = {a.stride_k, nc > 0 ? a.cstride[nc - 1] : (long long)1 << 62, a.stride_f};
  int ord[3] = {0, 1, 2};
  std::sort(ord, ord + 3, [&](int x, int y) { return st[x] > st[y]; });
  for (int t = 0; t < 3; ++t) a.ord[t] = ord[t];
  int jpos = 0;
  for (int t = 0; t < 3; ++t)
    if (ord[t] == 0) jpos = t;

  const long long budget0 = std::max<long long>(g.nX * (long long)g.esz / 2, 256 << 10);
  // fast layouts: fibre mode contiguous (rows) or mode k contiguous (columns)
  if (a.stride_f == 1 || a.stride_k == 1) {
    a.kind = a.stride_f == 1 ? 1 : 2;
    a.plfast = (nc > 0 && a.cstride[nc - 1] < a.stride_k) ? 1 : 0;
    const long long jcapf = std::max<long long>(1, (long long)NT * 8 / a.Rprod);   // <= 8 slots per thread
    // workgroups of a few thousand elements: enough work to amortise the
    // per-plane set-up, several hundred workgroups over the chip (nX / 1280,
    // at least 4096 entries: measured best on the 256 x 256 x 31 workload
    // and on order-4/5 served tensors)
    const long long E = std::min<long long>(65536, std::max<long long>(o.contract_emin, g.nX / o.contract_div));
    long long jn = (a.kind == 1 && a.plfast) ? std::min<long long>({(long long)a.Ik, jcapf, 8})
                                             : std::min<long long>({(long long)a.Ik, jcapf, o.contract_jmax});
    long long JT = cdiv(a.Ik, jn);
    jn = cdiv(a.Ik, JT);
    long long PPW = std::max<long long>(1, std::min<long long>(a.nplanes, E / std::max<long long>(1, jn * a.If)));
    long long S = cdiv(a.nplanes, PPW);
    while (S * a.Ik * a.Rprod * 8 > budget0 && PPW < a.nplanes) {
      PPW = std::min<long long>(a.nplanes, PPW * 2);
      S = cdiv(a.nplanes, PPW);
    }
    // columns: split the fibre range too when plane splits alone leave the chip idle
    long long FS = 1;
    if (a.kind == 2 && JT * S < 240)
      FS = std::max<long long>(1, std::min<long long>(cdiv(240, JT * S), a.If / 16));
    while (FS > 1 && S * FS * a.Ik * a.Rprod * 8 > budget0) --FS;
    a.FS = (int)FS;
    a.jn = (int)jn;
    a.JT = (int)JT;
    a.S = (int)S;
    a.PPW = PPW;
    a.PB = (int)std::min<long long>(PPW, a.kind == 1 ? 64 : 32);
    a.fch = 1;
    // two or more c-modes: contract the last one first (staged accumulation)
    // when the batches and workgroups can hold whole groups of its planes
    a.stage = 0;
    if (nc >= 2 && a.crank[nc - 1] >= 2) {
      const int cdl = a.cdim[nc - 1];
      const int pbmax = a.kind == 1 ? 64 : 32;
      if (cdl <= pbmax) {
        a.PPW = cdiv(a.PPW, cdl) * cdl;
        a.S = (int)cdiv(a.nplanes, a.PPW);
        a.stage = 1;
        a.cdl = cdl;
        a.Rl = a.crank[nc - 1];
        a.Rc2 = a.Rc / a.Rl;
        a.gloff = a.gcoff[nc - 1];
        a.PB = (int)std::max<long long>(cdl, (std::min<long long>(a.PPW, pbmax) / cdl) * cdl);
        while (a.PB > cdl && contract_smem_bytes(g.dtype, a) > kMaxLds) a.PB -= cdl;
        if (contract_smem_bytes(g.dtype, a) > kMaxLds) a.stage = 0;   // plain accumulation
      }
    }
    while (a.PB > 1 && contract_smem_bytes(g.dtype, a) > kMaxLds) a.PB = std::max(1, a.PB * 3 / 4);
    // a fibre too long for the LDS tables (fibre factor, per-plane scales):
    // split it into chunks over workgroups, each with a partial slot of its
    // own; chunks are re-balanced so that none is empty
    {
      long long fcs = cdiv(a.If, a.FS);
      while (fcs > 1 && contract_smem_bytes(g.dtype, a) > kMaxLds) {
        fcs = cdiv(fcs, 2);
        a.FS = (int)cdiv(a.If, fcs);
      }
    }
    if (a.kind == 1) {   // lanes per fibre row: at least 4 entries of the chunk each
      const int fc = (a.If + a.FS - 1) / a.FS;
      int fch = 1;
      while (fch < 64 && fc / (2 * fch) >= 4) fch *= 2;
      a.fch = fch;
    }
    int ps = 1;
    const int units = a.stage ? a.PB / a.cdl : a.PB;   // what the split threads share: planes or groups
    while (ps < 16 && jn * a.Rprod * ps * 2 <= NT && units >= 2 * ps) ps *= 2;
    a.psplit = ps;
    const long long slots = jn * a.Rprod * a.psplit;
    int spt = 1;
    while ((long long)spt * NT < slots) spt *= 2;
    P.spt = spt;
    P.smem = contract_smem_bytes(g.dtype, a);
    if (spt <= 8) return P;
    // more than 8 accumulator slots per thread (very large Rprod): the
    // layout-specialised kernels are built for at most 8; plan the generic one
    a.kind = 0;
    a.plfast = 0;
    a.FS = 1;
    a.fch = 1;
    a.psplit = 1;
    a.stage = 0;
    a.cdl = a.Rl = a.Rc2 = 0;
    a.gloff = 0;
  }

  // generic layout: an LDS tile of at most `tile` streaming elements, at
  // most 32 float64 accumulators per thread, split partials bounded by half of X
  const long long tile = g.dtype ? 4096 : 8192;
  const long long budget = std::max<long long>(g.nX * (long long)g.esz / 2, 256 << 10);
  const long long smax = std::max<long long>(1, budget / ((long long)a.Ik * a.Rprod * 8));
  const long long jcap = std::max<long long>(1, std::min<long long>((long long)NT * 32 / a.Rprod, tile / a.LDF));
  long long JT, S;
  if (jpos == 0) {
    // j is the slowest axis: a few j per workgroup (the per-plane set-up is
    // shared by the j of a tile), planes split to fill the chip
    const long long jw = std::min<long long>({(long long)a.Ik, jcap, 8});
    JT = cdiv(a.Ik, jw);
    S = std::max<long long>(1, std::min<long long>(std::min(smax, a.nplanes), cdiv(kTargetBlocks, JT)));
  } else {
    S = std::max<long long>(1, std::min(smax, a.nplanes));
    const long long jt_min = cdiv(a.Ik, jcap);
    long long jt_max = a.Ik;
    // j innermost: keep the whole j range (contiguous runs, no cache line
    // shared by workgroups on different XCDs) unless the slots do not fit
    if (jpos == 2) jt_max = jt_min;
    JT = std::min(jt_max, std::max(jt_min, cdiv(kTargetBlocks, S)));
  }
  long long jn = cdiv(a.Ik, JT);
  jn = std::min(jn, jcap);
  JT = cdiv(a.Ik, jn);
  const long long PPW = cdiv(a.nplanes, S);
  S = cdiv(a.nplanes, PPW);
  long long PB = std::max<long long>(1, std::min<long long>({tile / (jn * a.LDF), 256, PPW}));
  a.jn = (int)jn;
  a.JT = (int)JT;
  a.S = (int)S;
  a.FS = 1;
  a.PPW = PPW;
  a.PB = (int)PB;
  // shrink the plane batch until the LDS layout fits
  while (a.PB > 1 && contract_smem_bytes(g.dtype, a) > kMaxLds) a.PB = std::max(1, a.PB * 3 / 4);
  // lanes per fibre dot product: enough rows x lanes to cover the workgroup,
  // at least 4 fibre elements per lane
  {
    const long long rows = (long long)a.PB * jn;
    int fch = 1;
    while (fch < 64 && rows * fch * 2 <= NT && (a.If + 2 * fch - 1) / (2 * fch) >= 4) fch *= 2;
    a.fch = fch;
  }
  // threads per accumulator slot when there are few slots
  {
    int ps = 1;
    while (ps < 16 && jn * a.Rprod * ps * 2 <= NT && PPW >= 2 * ps) ps *= 2;
    a.psplit = ps;
  }
  const long long slots = jn * a.Rprod * a.psplit;
  int spt = 1;
  while ((long long)spt * NT < slots) spt *= 2;
  P.spt = spt;
  P.smem = contract_smem_bytes(g.dtype, a);
  return P;
}


// Invariants every launch relies on (indices stay inside X, the LDS layout
// and the partial buffers).  A plan that breaks one is rejected before any
// kernel runs.
bool plan_ok(const Geo& g, const ContractPlan& P, const char** why) {
  if (P.a.stage && (P.a.cdl < 1 || P.a.PB % P.a.cdl || P.a.PPW % P.a.cdl || P.a.nplanes % P.a.cdl ||
                    P.a.Rl * P.a.Rc2 != P.a.Rc || P.a.kind == 0)) {
    *why = "staged accumulation groups";
    return false;
  }
  if (P.a.nplanes >= (1LL << 31)) {
    *why = "more than 2^31 planes";
    return false;
  }
  const ContractArgs& a = P.a;
  if ((long long)a.JT * a.jn < a.Ik || (long long)(a.JT - 1) * a.jn >= a.Ik) { *why = "j tiling"; return false; }
  if ((long long)a.S * a.PPW < a.nplanes || (long long)(a.S - 1) * a.PPW >= a.nplanes) { *why = "plane split"; return false; }
  if (a.FS < 1 || (a.FS > 1 && a.kind == 0) || (long long)(a.FS - 1) * ((a.If + a.FS - 1) / a.FS) >= a.If) { *why = "fibre split"; return false; }
  if ((long long)a.nplanes * a.Ik * a.If != g.nX) { *why = "plane count"; return false; }
  if ((long long)a.jn * a.Rprod * a.psplit > (long long)P.spt * NT || P.spt > 32) { *why = "accumulator slots"; return false; }
  if (a.psplit > 1 && (long long)a.jn * a.Rprod * a.psplit > NT) { *why = "split slots"; return false; }
  if (a.fch < 1 || a.fch > 64 || (a.fch & (a.fch - 1)) != 0) { *why = "fibre lanes"; return false; }
  if (a.kind == 1 && a.stride_f != 1) { *why = "rows layout"; return false; }
  if (a.kind == 2 && a.stride_k != 1) { *why = "columns layout"; return false; }
  if (a.kind != 0 && (long long)a.PB * a.jn * a.Rf * 0 + (long long)a.psplit * a.jn * a.Rprod > (long long)P.spt * NT) { *why = "fast slots"; return false; }
  if (a.PB < 1 || a.PB > 256 || a.jn < 1) { *why = "batch"; return false; }
  if (P.smem > kMaxLds) { *why = "LDS size"; return false; }
  if (a.Rf > MAXR || a.Rc > 4096) { *why = "rank product"; return false; }
  return true;
}

// The preferred fibre mode's plan, or, when that one breaks an invariant (a
// long fibre that only the generic layout could take, whose LDS tables would
// not fit), the first valid plan over the other modes: the contiguous last
// mode first, then by decreasing length.
ContractPlan plan_contract(const Geo& g, int k, const PlanOpts& o) {
  const int f0 = preferred_fibre(g, k);
  ContractPlan P = plan_contract_f(g, k, f0, o);
  const char* why = nullptr;
  if (plan_ok(g, P, &why)) return P;
  int order[MAXN], n = 0;
  if (g.N - 1 != k && g.N - 1 != f0) order[n++] = g.N - 1;
  for (int m = 0; m < g.N; ++m)
    if (m != k && m != f0 && m != g.N - 1) order[n++] = m;
  std::stable_sort(order + (n > 0 && order[0] == g.N - 1 ? 1 : 0), order + n,
                   [&](int x, int y) { return g.dims[x] > g.dims[y]; });
  for (int q = 0; q < n; ++q) {
    ContractPlan Q = plan_contract_f(g, k, order[q], o);
    if (plan_ok(g, Q, &why)) return Q;
  }
  return P;   // the caller reports why it is invalid
}

QArgs plan_q(const Geo& g, int k, long long* qsize) {
  QArgs a;
  std::memset(&a, 0, sizeof(a));
  const int N = g.N;
  a.ni = N - 1;
  a.nd = N - 2;
  a.ndd = (N - 2) * (N - 3) / 2;
  long long blk = 0, qo = 0;
  int t = 0;
  for (int i = 0; i < N; ++i) {
    if (i == k) continue;
    QItem& it = a.it[t];
    it.Ii = g.dims[i];
    it.R = g.R[k][i];
    const int np = it.R * (it.R + 1) / 2;
    int dm[MAXC], nd = 0;
    long long D = 1;
    for (int m = 0; m < N; ++m)
      if (m != k && m != i) dm[nd++] = m;
    for (int c = 0; c < nd; ++c) {
      it.ddim[c] = g.dims[dm[c]];
      it.edi[c] = edge_ref(g, dm[c], i);
      D *= g.dims[dm[c]];
    }
    int q = 0;
    for (int x = 0; x < nd; ++x)
      for (int y = x + 1; y < nd; ++y) {
        it.dd_a[q] = x;
        it.dd_b[q] = y;
        it.edd[q] = edge_ref(g, dm[x], dm[y]);
        ++q;
      }
    it.D = D;
    int lanes = (int)std::min<long long>(64, cdiv(it.Ii, 4));   // about 4 fibre entries per lane
    int lg = 0;
    while ((1 << lg) < lanes) ++lg;
    it.lg2P = lg;
    it.CH = (int)cdiv(it.Ii, 1 << lg);
    a.blk0[t] = blk;
    blk += cdiv(D << lg, NT);
    it.qoff = qo;
    qo += D * np;
    it.gik = g.goff[i][k];
    ++t;
  }
  a.blk0[t] = blk;
  *qsize = qo;
  return a;
}

// Gamma route of factor block k (see GammaPlan): the modes other than k in
// Gamma order, the prefix split over workgroups and the LDS layout of one
// workgroup.  Returns false when Gamma_k or a workgroup's tables are too large.
bool plan_gamma(const Geo& g, int k, GammaPlan* gp) {
  std::memset(gp, 0, sizeof(*gp));
  const int N = g.N, n = N - 1;
  int srt[MAXN - 1], c = 0;
  for (int q = 0; q < N; ++q)
    if (q != k) srt[c++] = q;
  std::stable_sort(srt, srt + n, [&](int x, int y) { return g.dims[x] < g.dims[y]; });
  int om[MAXN - 1];
  if (n == 1) {
    om[0] = srt[0];
  } else if (n == 2) {            // prefix: the shorter mode; y: the longer
    om[0] = srt[0];
    om[1] = srt[1];
  } else if (n == 3) {            // prefix: middle; x: shortest; y: longest
    om[0] = srt[1];
    om[1] = srt[0];
    om[2] = srt[2];
  } else {                        // prefix: the two middle modes
    om[0] = srt[1];
    om[1] = srt[2];
    om[2] = srt[0];
    om[3] = srt[3];
  }
  gp->n = n;
  gp->npre = n >= 3 ? n - 2 : 1;
  gp->hasx = n >= 3 ? 1 : 0;
  long long P = 1;
  for (int u = 0; u < n; ++u) {
    const int m = om[u];
    gp->mode[u] = m;
    gp->dim[u] = g.dims[m];
    gp->rank[u] = g.R[m][k];
    gp->np[u] = gp->rank[u] * (gp->rank[u] + 1) / 2;
    gp->goff[u] = g.goff[m][k];
    P *= gp->np[u];
  }
  if (P > GM_PMAX) return false;
  gp->P = (int)P;
  int sacc = 1;
  for (int u = n - 1; u >= 0; --u) {
    gp->st[u] = sacc;
    sacc *= gp->np[u];
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (a != b) gp->e[a][b] = edge_ref(g, om[a], om[b]);
  gp->nq = 1;
  gp->npp = 1;
  for (int u = 0; u < gp->npre; ++u) {
    gp->nq *= gp->dim[u];
    gp->npp *= gp->np[u];
  }
  const int py = n - 1, px = n - 2;
  // LDS of a workgroup with qpw prefix tuples (nqc per chunk) and pyw y pairs
  auto lds = [&](int qpw, int nqc, int pyw, GammaPlan* o) {
    int at = 0;
    o->o_gy = at; at += n >= 2 ? gp->rank[py] * gp->dim[py] : 0;
    o->o_gx = at; at += gp->hasx ? gp->rank[px] * gp->dim[px] : 0;
    o->o_wa = at; at += gp->hasx ? gp->dim[px] * gp->dim[py] : (n == 2 ? qpw * gp->dim[py] : 0);
    o->o_cq = at; at += n >= 3 ? qpw * gp->dim[py] : 0;
    o->o_wb = at; at += gp->hasx ? qpw * gp->dim[px] : 0;
    o->o_t = at;  at += gp->hasx ? gp->dim[px] * nqc * pyw : (n == 2 ? nqc * pyw : 0);
    o->o_y = at;  at += gp->hasx ? nqc * gp->np[px] * pyw : 0;
    o->o_cp = at; at += qpw * gp->npp;
    o->o_pr = at; at += (n * MAXP + 1) / 2;
    return (size_t)at * 8;
  };
  // work per prefix tuple (multiply-adds): stage A, stage B, accumulation;
  // about 2^18 per workgroup: the y pairs split first (no partial sums), then
  // the prefix tuples (at most GM_QG partial sums per entry)
  const int npy = n >= 2 ? gp->np[py] : 1;
  const double costA = n >= 2 ? (gp->hasx ? (double)gp->dim[px] : 1.0) * gp->dim[py] * gp->np[py] : 0.0;
  const double costB = gp->hasx ? (double)gp->dim[px] * gp->np[px] * gp->np[py] : 0.0;
  const double total = (double)gp->nq * (costA + costB + (double)P);
  gp->fma = total;
  long long nwt = (long long)std::ceil(total / 32768.0);
  nwt = std::max<long long>(1, std::min<long long>(nwt, GM_MAXW));
  int nyg = (int)std::min<long long>(npy, nwt);
  int pyw = (int)cdiv(npy, nyg);
  // the accumulation tiles of a workgroup (npp x np_x pyw entries) over its
  // four waves: at most GM_VPT per wave
  const int nppx = gp->npp * (gp->hasx ? gp->np[px] : 1);
  auto tiles = [&](int w) { return (int)(cdiv(gp->npp, 16) * cdiv((long long)nppx / gp->npp * w, 16)); };
  while (pyw > 1 && tiles(pyw) > 4 * GM_VPT_HOST) pyw = (int)cdiv(pyw, 2);
  if (tiles(pyw) > 4 * GM_VPT_HOST) return false;
  nyg = (int)cdiv(npy, pyw);
  long long nqg = std::max<long long>(1, std::min<long long>({cdiv(nwt, nyg), (long long)GM_QG, gp->nq}));
  long long qpw = cdiv(gp->nq, nqg);
  int nqc = 16;
  for (;;) {
    nqc = (int)std::min<long long>(16, qpw);
    while (nqc > 1 && lds((int)qpw, nqc, pyw, gp) > kMaxLdsGamma) --nqc;
    if (lds((int)qpw, nqc, pyw, gp) <= kMaxLdsGamma) break;
    if (nqg >= std::min<long long>(GM_QG, gp->nq)) return false;
    nqg = std::min<long long>({nqg * 2, (long long)GM_QG, gp->nq});
    qpw = cdiv(gp->nq, nqg);
  }
  gp->nqc = nqc;
  gp->smem = (int)lds((int)qpw, nqc, pyw, gp);
  gp->qpw = (int)qpw;
  gp->nqg = (int)cdiv(gp->nq, qpw);
  gp->nyg = nyg;
  gp->nred = gp->nqg > 1 ? (int)cdiv(gp->P, 4 * NT) : 0;
  gp->pyw = pyw;
  gp->nw = gp->nyg * gp->nqg;
  return true;
}

// The Gamma-route solve of block k (see GSolve); false when its LDS does not fit.
bool plan_gsolve(const Geo& g, int k, const GammaPlan& gp, GSolve* gs, std::vector<int>* tabv = nullptr) {
  std::memset(gs, 0, sizeof(*gs));
  const int N = g.N, n = N - 1;
  gs->k = k;
  gs->Ik = g.dims[k];
  gs->n = n;
  gs->P = gp.P;
  gs->rho = g.rho;
  int um[MAXN - 1], c = 0;
  for (int q = 0; q < N; ++q)
    if (q != k) um[c++] = q;
  int Rprod = 1;
  for (int t = n - 1; t >= 0; --t) {
    gs->ust[t] = Rprod;
    Rprod *= g.R[k][um[t]];
  }
  gs->Rprod = Rprod;
  for (int t = 0; t < n; ++t) {
    const int m = um[t];
    gs->R[t] = g.R[k][m];
    gs->np[t] = gs->R[t] * (gs->R[t] + 1) / 2;
    gs->dim[t] = g.dims[m];
    for (int u = 0; u < n; ++u)
      if (gp.mode[u] == m) gs->gst[t] = gp.st[u];
    gs->goff_ki[t] = g.goff[k][m];
    gs->goff_ik[t] = g.goff[m][k];
    const EdgeRef w = edge_ref(g, k, m);
    gs->w_off[t] = w.off;
    gs->w_sj[t] = w.s1;
    gs->w_sy[t] = w.s2;
  }
  int scr = 1, tab = 0;
  for (int t = 0; t < n; ++t) {
    int o[MAXN - 1], ob[MAXN - 1], no = 0;
    for (int u = 0; u < n; ++u)
      if (u != t) o[no++] = u;
    for (int q = 0; q < no; ++q) ob[q] = o[q];
    // largest extent first: the first (largest) intermediate is smallest
    std::stable_sort(o, o + no, [&](int x, int y) { return gs->np[x] > gs->np[y]; });
    std::stable_sort(ob, ob + no, [&](int x, int y) { return gs->R[x] > gs->R[y]; });
    long long hn = gp.P, bn = Rprod;
    for (int q = 0; q < no; ++q) {
      (void)0;
      gs->ord[t][q] = o[q];
      gs->bord[t][q] = ob[q];
      hn /= gs->np[o[q]];
      bn /= gs->R[ob[q]];
      gs->hnout[t][q] = (int)hn;
      gs->bnout[t][q] = (int)bn;
      gs->hoff[t][q] = tab;
      tab += (int)hn;
      gs->boff[t][q] = tab;
      tab += (int)bn;
      if (q == 0) scr = std::max<long long>({(long long)scr, hn, bn});
    }
  }
  gs->tabtot = tab;
  gs->scr = (scr + 1) & ~1;
  // the offset tables: replay each chain's dims and strides
  std::vector<int> scratch_tab;
  if (!tabv) tabv = &scratch_tab;
  {
    tabv->assign(tab, 0);
    for (int t = 0; t < n; ++t)
      for (int which = 0; which < 2; ++which) {
        int d[MAXN - 1], st[MAXN - 1], alive[MAXN - 1];
        for (int u = 0; u < n; ++u) {
          d[u] = which ? gs->R[u] : gs->np[u];
          st[u] = which ? gs->ust[u] : gs->gst[u];
          alive[u] = 1;
        }
        for (int c = 0; c < n - 1; ++c) {
          const int uc = which ? gs->bord[t][c] : gs->ord[t][c];
          (which ? gs->bsc : gs->hsc)[t][c] = st[uc];
          alive[uc] = 0;
          const int nout = (which ? gs->bnout : gs->hnout)[t][c];
          int* out = tabv->data() + (which ? gs->boff : gs->hoff)[t][c];
          for (int o = 0; o < nout; ++o) {
            int rem = o, off = 0;
            for (int u = n - 1; u >= 0; --u)
              if (alive[u]) {
                off += (rem % d[u]) * st[u];
                rem /= d[u];
              }
            out[o] = off;
          }
          int sacc = 1;
          for (int u = n - 1; u >= 0; --u)
            if (alive[u]) {
              st[u] = sacc;
              sacc *= d[u];
            }
        }
      }
  }
  int gik = 0;
  for (int t = 0; t < n; ++t) {
    gs->gik_off[t] = gik;
    gik += gs->R[t] * gs->dim[t];
  }
  gs->gik_tot = gik;
  gs->gik_lds = (size_t)gsolve_smem(n, gp.P, Rprod, gs->scr, gik, tab) <= kMaxLdsGamma ? 1 : 0;
  gs->smem = gsolve_smem(n, gp.P, Rprod, gs->scr, gs->gik_lds ? gik : 0, tab);
  return (size_t)gs->smem <= kMaxLdsGamma;
}

}  // namespace

// ---------------------------------------------------------------------------
// job
// ---------------------------------------------------------------------------
size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// large-rank route (any edge rank above MAXR): plan of its launches
// ---------------------------------------------------------------------------
bool large_ranks(const Geo& g) {
  for (int a = 0; a < g.N; ++a)
    for (int b = 0; b < g.N; ++b)
      if (a != b && g.R[a][b] > MAXR) return true;
  return false;
}

// W_uv(x_u, x_v) in the stored edge matrix of {u, v}
LrEdge lr_edge(const Geo& g, int u, int v) {
  LrEdge r;
  r.off = g.woff[g.eid[u][v]];
  if (u < v) {
    r.s1 = g.dims[v];
    r.s2 = 1;
  } else {
    r.s1 = 1;
    r.s2 = g.dims[u];
  }
  return r;
}

struct LrBlock {
  int nst;
  LrYArgs y;
  LrGemmArgs st[MAXN - 1];     // mode products, the last one leaves U_k
  bool st_out1[MAXN - 1];      // stage output in buffer 1 (else 0)
  LrCArgs c[MAXN - 1];
  LrGemmArgs h[MAXN - 1];
  LrSolveArgs s[MAXN - 1];
};

struct LrPlan {
  LrBlock b[MAXN];
  long long n0 = 0, n1 = 0, nc = 0, nh = 0;   // doubles in buffer 0 / 1, c, H
  int xblk = 1;
  LrXArgs x;
};

// Geometry of every launch (pointers are filled in by lr_bind).  Stage t of
// block k contracts the last not yet contracted mode m != k, so its input is
// [A][I_m][B] with the contracted modes (ranks) after m; buffer 0 holds Y,
// the stages alternate 0 -> 1 -> 0 ...  Returns false when an intermediate
// exceeds 2^31 entries.
bool plan_lr(const Geo& g, LrPlan* P) {
  const int N = g.N;
  P->n0 = g.nX;
  for (int k = 0; k < N; ++k) {
    LrBlock& B = P->b[k];
    std::memset(&B, 0, sizeof(B));
    LrYArgs& y = B.y;
    y.N = N;
    for (int m = 0; m < N; ++m) y.dims[m] = g.dims[m];
    y.nX = g.nX;
    for (int e = 0; e < g.ne; ++e)
      if (g.ea[e] != k && g.eb[e] != k) {
        y.ea[y.ne] = g.ea[e];
        y.eb[y.ne] = g.eb[e];
        y.woff[y.ne] = g.woff[e];
        ++y.ne;
      }
    long long cur[MAXN];
    for (int m = 0; m < N; ++m) cur[m] = g.dims[m];
    int t = 0;
    for (int m = N - 1; m >= 0; --m) {
      if (m == k) continue;
      LrGemmArgs& a = B.st[t];
      a.A = 1;
      for (int q = 0; q < m; ++q) a.A *= cur[q];
      a.Bn = 1;
      for (int q = m + 1; q < N; ++q) a.Bn *= cur[q];
      a.I = g.dims[m];
      a.Nn = g.R[k][m];
      a.ldb = g.dims[m];
      cur[m] = g.R[k][m];
      const long long out = a.A * a.Nn * a.Bn;
      if (out > (1LL << 31)) return false;
      B.st_out1[t] = (t % 2) == 0;
      if (B.st_out1[t])
        P->n1 = std::max(P->n1, out);
      else
        P->n0 = std::max(P->n0, out);
      ++t;
    }
    B.nst = t;
    long long ustr[MAXN];
    {
      long long st = 1;
      for (int q = N - 1; q >= 0; --q) {
        ustr[q] = st;
        st *= cur[q];
      }
    }
    int sb = 0;
    for (int i = 0; i < N; ++i) {
      if (i == k) continue;
      int o[MAXN], nr = 0;
      for (int m = 0; m < N; ++m)
        if (m != k && m != i) o[nr++] = m;
      const int R = g.R[k][i];
      LrCArgs& c = B.c[sb];
      c.Ik = g.dims[k];
      c.Ii = g.dims[i];
      c.nr = nr;
      for (int p = 0; p < nr; ++p) {
        c.rdim[p] = g.dims[o[p]];
        c.ek[p] = lr_edge(g, k, o[p]);
        c.ei[p] = lr_edge(g, i, o[p]);
      }
      for (int p = 0; p < nr; ++p)
        for (int q = p + 1; q < nr; ++q) {
          c.pa[c.npr] = p;
          c.pb[c.npr] = q;
          c.ep[c.npr] = lr_edge(g, o[p], o[q]);
          ++c.npr;
        }
      LrGemmArgs& h = B.h[sb];
      h.A = g.dims[k];
      h.Bn = 1;
      h.I = g.dims[i];
      h.Nn = R * (R + 1) / 2;
      h.pairR = R;
      h.ldb = g.dims[i];
      LrSolveArgs& v = B.s[sb];
      v.Ik = g.dims[k];
      v.R = R;
      v.nr = nr;
      v.rho = g.rho;
      v.ustr_j = ustr[k];
      v.ustr_i = ustr[i];
      for (int p = 0; p < nr; ++p) {
        v.ustr[p] = ustr[o[p]];
        v.urank[p] = g.R[k][o[p]];
        v.goff_o[p] = g.goff[k][o[p]];
      }
      v.goff_ki = g.goff[k][i];
      P->nc = std::max(P->nc, (long long)g.dims[k] * g.dims[i]);
      P->nh = std::max(P->nh, (long long)g.dims[k] * h.Nn);
      ++sb;
    }
  }
  LrXArgs& x = P->x;
  std::memset(&x, 0, sizeof(x));
  x.N = N;
  for (int m = 0; m < N; ++m) x.dims[m] = g.dims[m];
  x.nX = g.nX;
  x.ne = g.ne;
  for (int e = 0; e < g.ne; ++e) {
    x.ea[e] = g.ea[e];
    x.eb[e] = g.eb[e];
    x.woff[e] = g.woff[e];
  }
  x.rx = g.rho_x;
  x.inv1 = 1.0 / (1.0 + g.rho_x);
  P->xblk = (int)std::min<long long>(1024, std::max<long long>(1, (g.nX + NT - 1) / NT));
  return true;
}

// Device pointers of every launch; buf0/buf1 the mode-product buffers.
void lr_bind(LrPlan* P, const Geo& g, const void* X, const uint32_t* bits, double* G, double* W64, void* Wc,
             double* buf0, double* buf1, double* cbuf, double* hbuf, double* normpart, double* dgpart,
             const int* stop) {
  long long dgo = 0;
  for (int k = 0; k < g.N; ++k) {
    LrBlock& B = P->b[k];
    B.y.X = X;
    B.y.W64 = W64;
    B.y.Y = buf0;
    B.y.stop = stop;
    const double* in = buf0;
    for (int t = 0; t < B.nst; ++t) {
      LrGemmArgs& a = B.st[t];
      double* out = B.st_out1[t] ? buf1 : buf0;
      a.in = in;
      a.out = out;
      int m = -1;                      // the mode of stage t: modes != k from the last down
      for (int q = g.N - 1, n = 0; q >= 0; --q) {
        if (q == k) continue;
        if (n++ == t) {
          m = q;
          break;
        }
      }
      a.Bm = G + g.goff[m][k];
      a.stop = stop;
      in = out;
    }
    for (int t = 0; t < g.N - 1; ++t) {
      B.c[t].W64 = W64;
      B.c[t].c = cbuf;
      B.c[t].stop = stop;
      int i = -1;
      for (int q = 0, n = 0; q < g.N; ++q) {
        if (q == k) continue;
        if (n++ == t) {
          i = q;
          break;
        }
      }
      B.h[t].in = cbuf;
      B.h[t].Bm = G + g.goff[i][k];
      B.h[t].out = hbuf;
      B.h[t].stop = stop;
      LrSolveArgs& v = B.s[t];
      v.U = in;
      v.H = hbuf;
      v.G = G;
      v.dgpart = dgpart + dgo + (long long)t * g.dims[k];
      v.stop = stop;
    }
    dgo += (long long)(g.N - 1) * g.dims[k];
  }
  P->x.X = (void*)X;
  P->x.bits = bits;
  P->x.W64 = W64;
  P->x.normpart = normpart;
  P->x.stop = stop;
}

struct ifctn_job {
  Geo g;
  PlanOpts opts;              // tuning options the job was planned with
  hipStream_t stream = nullptr;
  unsigned char* arena = nullptr;
  size_t arena_bytes = 0;
  bool own_arena = true;      // false: the arena is a slice of a server's pool
  void* X = nullptr;          // master X (float32 / float64)
  bf16x* Xb = nullptr;        // bfloat16 X of the BF16 phase (BF16_REFINE jobs)
  bool bf16_phase = false;
  uint32_t* bits = nullptr;
  double* G = nullptr;
  double* W64 = nullptr;
  void* Wc = nullptr;
  double* Q = nullptr;
  double* Upart = nullptr;
  double* Ugrp = nullptr;     // group sums of the partial slots (grouped reduction)
  int* ucnt = nullptr;
  double* Ufin = nullptr;
  double* Hpart = nullptr;
  int* hcnt = nullptr;
  bool onelaunch = true;       // phased blocks: one launch per sub-block
  double* normpart = nullptr;
  double* dgpart = nullptr;
  double* stats5 = nullptr;
  int* flag = nullptr;
  ContractPlan cplan[MAXN];
  QArgs qplan[MAXN];
  SolveArgs splan[MAXN];
  bool phased[MAXN] = {};
  bool groute[MAXN] = {};      // factor block by the Gamma route
  GammaPlan gplan[MAXN];       // host copies (device copies at dgp / dgs)
  GSolve gsol[MAXN];
  GammaPlan* dgp = nullptr;
  GSolve* dgs = nullptr;
  std::vector<int> htab;       // host copy of the Gamma-route offset tables (source of an async copy)
  double* gamma = nullptr;
  double* gmpart = nullptr;
  bool merge[MAXN] = {};       // Gram weights inside the contraction launch
  PhaseArgs pplan[MAXN][MAXN - 1];
  int nnorm = 0, ndg = 0;
  // Gamma route with overlap: the mode-k contraction runs on `side`, forked
  // from and joined back into `stream` (where Gamma_k is built) by the events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool lr = false;             // large-rank route for every block (an edge rank above MAXR)
  LrPlan lp;
  bool pending = false;
  int sweeps_done = 0;
  // device-side stop test (Algorithm 1) after every X step: flag[1] = stop,
  // flag[2] = sweeps completed before the stop
  bool dev_stop = false;
  double stop_eps = 0.0;
  bool timing = false;
  std::vector<hipEvent_t> ev[KC_COUNT];
  size_t evn[KC_COUNT] = {};
};

namespace {

struct Sizes {
  size_t x, xb, bits, G, W64, Wc, Q, Upart, Ugrp, ucnt, Ufin, Hpart, hcnt, normpart, dgpart, stats, flag, qitems;
  size_t gamma, gmpart, grec, gtab;
  size_t lr0, lr1, lrc, lrh;   // large-rank route: Y / mode-product buffers, c weights, packed H rows
  size_t total;
};

size_t sizes_total(const Sizes& s) {
  return s.x + s.xb + s.bits + s.G + s.W64 + s.Wc + s.Q + s.Upart + s.Ugrp + s.ucnt + s.Ufin + s.Hpart + s.hcnt +
         s.normpart + s.dgpart + s.stats + s.flag + s.qitems + s.gamma + s.gmpart + s.grec + s.gtab +
         s.lr0 + s.lr1 + s.lrc + s.lrh;
}

// arena of a large-rank job: X, mask bits, factors, edges, statistics and the
// route's own buffers (none of the fused route's)
Sizes lr_sizes(const Geo& g, const LrPlan& P) {
  Sizes s{};
  s.x = al256(g.nX * g.esz);
  s.bits = al256(((g.nX + 63) / 64) * 8);
  s.G = al256(g.nG * 8);
  s.W64 = al256(g.nW * 8);
  s.Wc = al256(g.nW * g.esz);
  long long ndg = 0;
  for (int k = 0; k < g.N; ++k) ndg += (long long)(g.N - 1) * g.dims[k];
  s.normpart = al256((size_t)P.xblk * 3 * 8);
  s.dgpart = al256(ndg * 8);
  s.stats = al256(8 * 8);
  s.flag = al256(16);
  s.qitems = al256(sizeof(QItem) * MAXN * (MAXN - 1));
  s.grec = al256(sizeof(GammaPlan) * MAXN) + al256(sizeof(GSolve) * MAXN);
  s.lr0 = al256(P.n0 * 8);
  s.lr1 = al256(P.n1 * 8);
  s.lrc = al256(P.nc * 8);
  s.lrh = al256(P.nh * 8);
  s.total = sizes_total(s);
  return s;
}

bool use_phased(const Geo& g, const QArgs& Q, int k, const PlanOpts& o) {
  long long m = 0;
  for (int t = 0; t < g.N - 1; ++t) m = std::max(m, Q.it[t].D * (long long)(Q.it[t].R * (Q.it[t].R + 1) / 2));
  if (m >= o.phased_min) return true;
  // the per-column kernel keeps the column's edge rows of every other mode in
  // LDS; when a long mode makes them too large, the phased form (which reads
  // them from HBM) takes the block
  SolveArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.Rprod = 1;
  for (int q = 0; q < g.N; ++q)
    if (q != k) {
      sa.Rprod *= g.R[k][q];
      sa.rowtot += (int)g.dims[q];
    }
  return solve_smem_bytes(sa) > kMaxLds;
}

int hp_width(int Ik) {
  int w = 1;
  while (w < Ik && w < HP_JW) w <<= 1;
  return w;
}


Sizes job_sizes(const Geo& g, ContractPlan* cp, QArgs* qp, const PlanOpts& o, GammaPlan* gpl = nullptr,
                GSolve* gsl = nullptr, bool* groute = nullptr) {
  Sizes s{};
  s.x = al256(g.nX * g.esz);
  s.xb = g.bf16 ? al256(g.nX * 2) : 0;
  s.bits = al256(((g.nX + 63) / 64) * 8);
  s.G = al256(g.nG * 8);
  s.W64 = al256(g.nW * 8);
  s.Wc = al256(g.nW * g.esz);
  long long qmax = 0, upmax = 0, ugmax = 0, ucmax = 0, ufmax = 0, hmax = 0, nnorm = 0, ndg = 0;
  long long gmP = 0, gmpart = 0, gtab = 0;
  const bool dbg = std::getenv("IFCTN_DEBUG_PLAN") != nullptr;
  for (int k = 0; k < g.N; ++k) {
    ContractPlan P = plan_contract(g, k, o);
    {
      const long long St = (long long)P.a.S * P.a.FS;
      if (o.ugroup > 1 && St > o.ugroup) {
        P.a.ugrp = (int)o.ugroup;
        P.a.ngrp = (int)cdiv(St, o.ugroup);
      }
    }
    long long qs = 0;
    QArgs Q = plan_q(g, k, &qs);
    if (dbg) {
      const ContractArgs& a = P.a;
      std::fprintf(stderr,
                   "[ifctn plan] k=%d f=%d kind=%d plfast=%d ord=%d%d%d Ik=%d If=%d LDF=%d nc=%d Rf=%d Rc=%d Rprod=%d jn=%d JT=%d S=%d "
                   "PPW=%lld PB=%d FS=%d nplanes=%lld spt=%d fch=%d psplit=%d smem=%zu blocks=%lld upart=%lld stage=%d cdl=%d Rl=%d | Q blocks=%lld size=%lld\n",
                   k, a.f, a.kind, a.plfast, a.ord[0], a.ord[1], a.ord[2], a.Ik, a.If, a.LDF, a.nc, a.Rf, a.Rc, a.Rprod, a.jn, a.JT, a.S, a.PPW, a.PB,
                   a.FS, a.nplanes, P.spt, a.fch, a.psplit, P.smem, (long long)a.JT * a.S * a.FS,
                   (long long)a.S * a.FS * a.Ik * a.Rprod, a.stage, a.cdl, a.Rl,
                   Q.blk0[Q.ni], qs);
    }
    if (cp) cp[k] = P;
    if (qp) qp[k] = Q;
    GammaPlan gpk;
    GSolve gsk;
    const bool gr = o.gamma > 0 && (o.gamma == 2 || use_phased(g, Q, k, o)) && plan_gamma(g, k, &gpk) &&
                    plan_gsolve(g, k, gpk, &gsk);
    if (groute) groute[k] = gr;
    if (gr) {
      if (gpl) gpl[k] = gpk;
      if (gsl) gsl[k] = gsk;
      gmP = std::max<long long>(gmP, gpk.P);
      gmpart = std::max<long long>(gmpart, (long long)gpk.nqg * gpk.P);
      gtab += gsk.tabtot;
      qs = 0;                        // no Gram weight sets for this block
    }
    qmax = std::max(qmax, qs);
    upmax = std::max(upmax, (long long)P.a.S * P.a.FS * P.a.Ik * P.a.Rprod);
    ugmax = std::max(ugmax, (long long)P.a.ngrp * P.a.Ik * P.a.Rprod);
    ucmax = std::max(ucmax, (long long)P.a.ngrp * P.a.JT);
    ufmax = std::max(ufmax, (long long)P.a.Ik * P.a.Rprod);
    if (!gr && use_phased(g, Q, k, o))
      for (int t = 0; t < g.N - 1; ++t) {
        const long long ks = (Q.it[t].D + HP_DC - 1) / HP_DC;
        hmax = std::max(hmax, ks * g.dims[k] * (long long)(Q.it[t].R * (Q.it[t].R + 1) / 2));
      }
    if (k == 0) nnorm = (long long)P.a.JT * P.a.S * P.a.FS;
    ndg += (long long)(g.N - 1) * g.dims[k];
  }
  s.Q = al256(qmax * 8);
  s.Upart = al256(upmax * 8);
  s.Ugrp = al256(ugmax * 8);
  s.ucnt = al256(ucmax * 4);
  s.Ufin = al256(ufmax * 8);
  s.Hpart = al256(hmax * 8);
  long long ikmax = 1;
  for (int k = 0; k < g.N; ++k) ikmax = std::max<long long>(ikmax, g.dims[k]);
  s.hcnt = al256(ikmax * 4);              // one arrival counter per column tile
  s.normpart = al256(nnorm * 3 * 8);
  s.dgpart = al256(ndg * 8);
  s.stats = al256(8 * 8);
  s.flag = al256(16);
  s.qitems = al256(sizeof(QItem) * MAXN * (MAXN - 1));
  s.gamma = al256(gmP * 8);
  s.gmpart = al256(gmpart * 8);
  s.grec = al256(sizeof(GammaPlan) * MAXN) + al256(sizeof(GSolve) * MAXN);
  s.gtab = al256(gtab * 4);
  s.total = sizes_total(s);
  return s;
}

void build_solve_plans(ifctn_job* J) {
  const Geo& g = J->g;
  const int N = g.N;
  long long dgo = 0;
  for (int k = 0; k < N; ++k) {
    const ContractPlan& P = J->cplan[k];
    const QArgs& Q = J->qplan[k];
    SolveArgs& a = J->splan[k];
    std::memset(&a, 0, sizeof(a));
    a.k = k;
    a.Ik = g.dims[k];
    a.nsub = N - 1;
    a.rho = g.rho;
    int umodes[MAXN - 1], nu = 0;
    for (int m = 0; m < N; ++m)
      if (m != k) umodes[nu++] = m;
    a.nu = nu;
    long long st = 1;
    for (int t = nu - 1; t >= 0; --t) {
      a.ustride[t] = st;
      st *= g.R[k][umodes[t]];
    }
    int ro = 0;
    for (int t = 0; t < nu; ++t) {
      const int m = umodes[t];
      a.udim[t] = g.dims[m];
      a.urank[t] = g.R[k][m];
      a.ugoff[t] = g.goff[k][m];
      a.rowoff[t] = ro;
      ro += g.dims[m];
      a.ekm[t] = edge_ref(g, k, m);
    }
    a.rowtot = ro;
    a.Rprod = P.a.Rprod;
    a.S = P.a.ugrp ? P.a.ngrp : P.a.S * P.a.FS;
    a.Upart = P.a.ugrp ? J->Ugrp : J->Upart;
    a.W64 = J->W64;
    a.Wc = J->Wc;
    a.G = J->G;
    a.dgpart = J->dgpart + dgo;
    dgo += (long long)(N - 1) * a.Ik;
    int t = 0;
    for (int i = 0; i < N; ++i) {
      if (i == k) continue;
      SubBlock& B = a.sb[t];
      B.i = i;
      B.Ii = g.dims[i];
      B.R = g.R[k][i];
      B.np = B.R * (B.R + 1) / 2;
      for (int u = 0; u < nu; ++u)
        if (umodes[u] == i) B.upos = u;
      int nd = 0;
      for (int u = 0; u < nu; ++u) {
        const int m = umodes[u];
        if (m == i) continue;
        B.ddim[nd] = g.dims[m];
        B.dt[nd] = u;
        ++nd;
      }
      B.nd = nd;
      B.D = Q.it[t].D;
      B.Q = J->Q + Q.it[t].qoff;
      B.goff_ki = g.goff[k][i];
      B.goff_ik = g.goff[i][k];
      const EdgeRef w = edge_ref(g, k, i);
      B.w_off = w.off;
      B.w_sj = w.s1;
      B.w_sy = w.s2;
      ++t;
    }
    J->phased[k] = use_phased(g, Q, k, J->opts);
    for (int t2 = 0; t2 < a.nsub; ++t2) {
      PhaseArgs& h = J->pplan[k][t2];
      std::memset(&h, 0, sizeof(h));
      h.B = a.sb[t2];
      h.t = t2;
      h.k = k;
      h.Ik = a.Ik;
      h.nu = a.nu;
      h.Rprod = a.Rprod;
      h.rho = a.rho;
      for (int u = 0; u < a.nu; ++u) {
        h.urank[u] = a.urank[u];
        h.ustride[u] = a.ustride[u];
        h.ugoff[u] = a.ugoff[u];
      }
      for (int c = 0; c < h.B.nd; ++c) h.edm[c] = a.ekm[h.B.dt[c]];
      h.JW = hp_width(a.Ik);
      h.JT = (a.Ik + h.JW - 1) / h.JW;
      h.KS = (int)((h.B.D + HP_DC - 1) / HP_DC);
      h.Ufin = J->Ufin;
      h.Hpart = J->Hpart;
      h.cnt = J->hcnt;
      h.W64 = J->W64;
      h.Wc = J->Wc;
      h.G = J->G;
      h.dgpart = a.dgpart;
    }
  }
  J->ndg = (int)dgo;
}

hipError_t timed(ifctn_job* J, int cls, hipError_t (*fn)(ifctn_job*, const void*), const void* ctx) {
  if (!J->timing) return fn(J, ctx);
  auto& v = J->ev[cls];
  size_t n = J->evn[cls];
  while (v.size() < 2 * (n + 1)) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    v.push_back(e);
  }
  // the launch itself stamps the pair with the kernel's start and end
  set_kernel_events(v[2 * n], v[2 * n + 1]);
  hipError_t err = fn(J, ctx);
  const bool used = kernel_events_used();
  set_kernel_events(nullptr, nullptr);
  if (err != hipSuccess) return err;
  if (!used) {  // nothing was launched: an empty interval
    err = hipEventRecord(v[2 * n], J->stream);
    if (err == hipSuccess) err = hipEventRecord(v[2 * n + 1], J->stream);
  }
  J->evn[cls] = n + 1;
  return err;
}

struct ContractCall {
  int k;
  bool upd, con;
};

// The Gram weights of block k ride along as extra workgroups of the
// contraction launch (same inputs, no ordering between them), for the
// layout-specialised contraction kernels.
bool gram_merged(const ifctn_job* J, int k) {
  return !J->groute[k] && J->cplan[k].a.kind != 0 && J->qplan[k].blk0[J->qplan[k].ni] > 0 && J->merge[k];
}


hipError_t do_contract(ifctn_job* J, const void* c) {
  const ContractCall* cc = (const ContractCall*)c;
  const ContractPlan& P = J->cplan[cc->k];
  const int kt = J->bf16_phase ? KT_BF16 : (J->g.dtype ? KT_F64 : KT_F32);
  if (cc->con && gram_merged(J, cc->k)) {
    ContractArgs a = P.a;
    const QArgs& q = J->qplan[cc->k];
    a.gblocks = (int)q.blk0[q.ni];
    a.gr.dit = q.dit;
    a.gr.ni = q.ni;
    a.gr.nd = q.nd;
    a.gr.ndd = q.ndd;
    for (int t = 0; t < MAXN; ++t) a.gr.blk0[t] = q.blk0[t];
    a.gr.W64 = q.W64;
    a.gr.G = q.G;
    a.gr.Q = q.Q;
    return launch_contract(kt, cc->upd, cc->con, P.spt, a, P.smem, J->stream);
  }
  return launch_contract(kt, cc->upd, cc->con, cc->con ? P.spt : 1, P.a, P.smem, J->stream);
}

hipError_t do_gram(ifctn_job* J, const void* c) { return launch_q(*(const QArgs*)c, J->stream); }

hipError_t do_gamma(ifctn_job* J, const void* c) {
  const int k = *(const int*)c;
  const GammaPlan& gp = J->gplan[k];
  // Gamma_k, then the U rows and the sum of its partial rows
  hipError_t e = launch_gamma(gp, J->dgp + k, J->flag + 1, J->stream, 1);
  if (e == hipSuccess) e = launch_gamma(gp, J->dgp + k, J->flag + 1, J->stream, 2);
  return e;
}

// Gamma_k, then the sum of its partial rows, on the job's stream (the
// contraction runs on the second one)
hipError_t do_gamma_main(ifctn_job* J, const void* c) {
  const int k = *(const int*)c;
  return launch_gamma(J->gplan[k], J->dgp + k, J->flag + 1, J->stream, 1);
}

hipError_t do_gsum_main(ifctn_job* J, const void* c) {
  const int k = *(const int*)c;
  return launch_gamma(J->gplan[k], J->dgp + k, J->flag + 1, J->stream, 4);
}

// the U rows of block k on the second stream, after its contraction
hipError_t do_urow_side(ifctn_job* J, const void* c) {
  const int k = *(const int*)c;
  return launch_gamma(J->gplan[k], J->dgp + k, J->flag + 1, J->side, 3);
}

hipError_t do_solve(ifctn_job* J, const void* c) {
  const SolveArgs* a = (const SolveArgs*)c;
  const int k = a->k;
  if (J->groute[k]) return launch_solve_gamma(J->g.dtype, J->gsol[k], J->dgs + k, J->stream);
  if (!J->phased[k]) return launch_solve(J->g.dtype, *a, J->stream);
  hipError_t e = launch_urow(*a, J->Ufin, J->stream);
  for (int t = 0; t < a->nsub && e == hipSuccess; ++t) {
    if (J->onelaunch) {
      PhaseArgs h = J->pplan[k][t];
      h.JW = std::min(h.JW, HS_JW);
      h.JT = (h.Ik + h.JW - 1) / h.JW;
      e = launch_hsolve(J->g.dtype, h, J->stream);
    } else {
      e = launch_hpart(J->pplan[k][t], J->stream);
      if (e == hipSuccess) e = launch_solve_col(J->g.dtype, J->pplan[k][t], J->stream);
    }
  }
  return e;
}

hipError_t do_lr_x(ifctn_job* J, const void*) {
  return launch_lr_x(J->g.dtype, J->lp.x, J->lp.xblk, J->stream);
}

hipError_t do_lr_contract(ifctn_job* J, const void* c) {
  const LrBlock& B = J->lp.b[*(const int*)c];
  hipError_t e = launch_lr_y(J->g.dtype, B.y, J->stream);
  for (int t = 0; t < B.nst && e == hipSuccess; ++t) e = launch_lr_gemm(B.st[t], J->stream);
  return e;
}

struct LrSub {
  int k, t;
};

hipError_t do_lr_gram(ifctn_job* J, const void* c) {
  const LrSub* q = (const LrSub*)c;
  const LrBlock& B = J->lp.b[q->k];
  hipError_t e = launch_lr_c(B.c[q->t], J->stream);
  if (e == hipSuccess) e = launch_lr_gemm(B.h[q->t], J->stream);
  return e;
}

// the column solves, then W_{k,i} from the new G_{k,i}
hipError_t do_lr_solve(ifctn_job* J, const void* c) {
  const LrSub* q = (const LrSub*)c;
  hipError_t e = launch_lr_solve(J->lp.b[q->k].s[q->t], J->stream);
  if (e != hipSuccess) return e;
  const Geo& g = J->g;
  int i = -1;
  for (int m = 0, n = 0; m < g.N; ++m) {
    if (m == q->k) continue;
    if (n++ == q->t) {
      i = m;
      break;
    }
  }
  const int a = std::min(q->k, i), b = std::max(q->k, i), x = g.eid[a][b];
  return launch_edge(g.dtype, J->G + g.goff[a][b], J->G + g.goff[b][a], g.R[a][b], g.dims[a], g.dims[b],
                     J->W64 + g.woff[x], (unsigned char*)J->Wc + g.woff[x] * g.esz, J->stream);
}

// one sweep of the large-rank route: the pending X step (and stop test),
// then for every k: Y and the mode products into U_k, and per sub-block the
// weights, H rows and the column solves
hipError_t lr_sweep(ifctn_job* J) {
  hipError_t e;
  if (J->pending) {
    e = timed(J, KC_UPDATE, do_lr_x, nullptr);
    if (e == hipSuccess && J->dev_stop) e = launch_stop_test(J->normpart, J->nnorm, J->stop_eps, J->flag + 1, J->stream);
    if (e != hipSuccess) return e;
  }
  for (int k = 0; k < J->g.N; ++k) {
    e = timed(J, KC_CONTRACT, do_lr_contract, &k);
    if (e != hipSuccess) return e;
    for (int t = 0; t < J->g.N - 1; ++t) {
      const LrSub q{k, t};
      e = timed(J, KC_GRAM, do_lr_gram, &q);
      if (e == hipSuccess) e = timed(J, KC_SOLVE, do_lr_solve, &q);
      if (e != hipSuccess) return e;
    }
  }
  J->pending = true;
  J->sweeps_done++;
  return hipSuccess;
}

hipError_t run_sweep(ifctn_job* J) {
  if (J->lr) return lr_sweep(J);
  const int N = J->g.N;
  hipError_t e;
  for (int k = 0; k < N; ++k) {
    if (!J->groute[k] && !gram_merged(J, k)) {
      e = timed(J, KC_GRAM, do_gram, &J->qplan[k]);
      if (e != hipSuccess) return e;
    }
    // Gamma route with overlap: the contraction (and stop test) forked onto
    // the job's second stream, Gamma_k launched on the job's stream right
    // after it -- launched first on its own queue, Gamma_k's few workgroups
    // take their CUs before the contraction's fill the rest
    const bool swap = J->groute[k] && J->side;
    ContractCall cc{k, k == 0 && J->pending, true};
    if (swap) {
      e = hipEventRecord(J->ev_fork, J->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(J->side, J->ev_fork, 0);
      if (e != hipSuccess) return e;
      std::swap(J->stream, J->side);
    }
    e = timed(J, KC_CONTRACT, do_contract, &cc);
    if (e == hipSuccess && cc.upd && J->dev_stop)
      e = launch_stop_test(J->normpart, J->nnorm, J->stop_eps, J->flag + 1, J->stream);
    if (swap) {
      std::swap(J->stream, J->side);
      // the U rows follow the contraction there; Gamma_k and the sum of its
      // partial rows run here; the solve waits for both
      if (e == hipSuccess) e = timed(J, KC_UROW, do_urow_side, &k);
      if (e == hipSuccess) e = hipEventRecord(J->ev_join, J->side);
      if (e == hipSuccess) e = timed(J, KC_GRAM, do_gamma_main, &k);
      if (e == hipSuccess) e = timed(J, KC_UROW, do_gsum_main, &k);
      if (e == hipSuccess) e = hipStreamWaitEvent(J->stream, J->ev_join, 0);
    }
    if (e != hipSuccess) return e;
    if (J->groute[k] && !swap) {     // Gamma_k, the U rows and the partial-row sum, then the solve
      e = timed(J, KC_GRAM, do_gamma, &k);
      if (e != hipSuccess) return e;
    }
    e = timed(J, KC_SOLVE, do_solve, &J->splan[k]);
    if (e != hipSuccess) return e;
  }
  J->pending = true;
  J->sweeps_done++;
  return hipSuccess;
}

hipError_t flush_update(ifctn_job* J) {
  if (!J->pending) return hipSuccess;
  ContractCall cc{0, true, false};
  hipError_t e = J->lr ? timed(J, KC_UPDATE, do_lr_x, nullptr) : timed(J, KC_UPDATE, do_contract, &cc);
  J->pending = false;
  if (e == hipSuccess && J->dev_stop) e = launch_stop_test(J->normpart, J->nnorm, J->stop_eps, J->flag + 1, J->stream);
  return e;
}

// Algorithm 1's loop for an initialised job.  With eps > 0 the stop test runs
// on the device after every X step (k_stop_test); once it is met every later
// launch of the job is a no-op, so the host issues sweeps in chunks and reads
// the flag once per chunk instead of once per sweep.
constexpr int kStopChunk = 8;

ifctn_status run_complete(ifctn_job* J, int t_max, double eps, void* X_out_dev, ifctn_stats* out);

// End the bfloat16 phase: the float32 master takes the widened bf16 values off
// Omega (it holds O on Omega), and every later pass streams float32.
hipError_t promote(ifctn_job* J) {
  if (!J->bf16_phase) return hipSuccess;
  hipError_t e = flush_update(J);
  if (e != hipSuccess) return e;
  e = launch_widen(J->Xb, J->bits, (const float*)J->X, (float*)J->X, J->g.nX, J->stream);
  if (e != hipSuccess) return e;
  J->bf16_phase = false;
  for (int k = 0; k < J->g.N; ++k) J->cplan[k].a.X = J->X;
  return hipSuccess;
}

}  // namespace

extern "C" ifctn_status ifctn_sweep(ifctn_job* J, int32_t nsweeps, ifctn_stats* stats);
extern "C" ifctn_status ifctn_reconstruct(ifctn_job* J, void* out_dev, int32_t which);

namespace {

ifctn_status run_complete(ifctn_job* J, int t_max, double eps, void* X_out_dev, ifctn_stats* out) {
  ifctn_stats s;
  std::memset(&s, 0, sizeof(s));
  // BF16_REFINE: the last `refine` sweeps stream float32 (after promotion)
  const int refine = std::min(J->g.refine, t_max);
  const int t_main = t_max - refine;
  int state[2] = {0, 0};
  int done_main = t_main;
  if (eps > 0.0 && t_main > 0) {
    J->dev_stop = true;
    J->stop_eps = eps;
    HIPTRY(hipMemsetAsync(J->flag + 1, 0, 2 * sizeof(int), J->stream));
    for (int t = 0; t < t_main; t += kStopChunk) {
      const int n = std::min(kStopChunk, t_main - t);
      for (int q = 0; q < n; ++q) HIPTRY(run_sweep(J));
      if (t + n >= t_main) HIPTRY(flush_update(J));   // X step (and stop test) of the last sweep
      HIPTRY(hipMemcpyAsync(state, J->flag + 1, sizeof(state), hipMemcpyDeviceToHost, J->stream));
      HIPTRY(hipStreamSynchronize(J->stream));
      if (state[0]) break;
    }
    if (state[0]) HIPTRY(flush_update(J));              // a no-op on the device: the job has stopped
    done_main = state[1];
    J->dev_stop = false;
  } else if (t_main > 0) {
    for (int q = 0; q < t_main; ++q) HIPTRY(run_sweep(J));
    HIPTRY(flush_update(J));
  }
  ifctn_status st = IFCTN_OK;
  if (J->g.bf16) {
    HIPTRY(promote(J));
    if (refine > 0) {
      HIPTRY(hipMemsetAsync(J->flag + 1, 0, 2 * sizeof(int), J->stream));   // the refinement always runs
      for (int q = 0; q < refine; ++q) HIPTRY(run_sweep(J));
      HIPTRY(flush_update(J));
    }
  }
  st = ifctn_sweep(J, 0, &s);                            // statistics of the last sweep run
  if (st != IFCTN_OK) return st;
  s.sweeps_done = done_main + refine;
  s.converged = state[0];
  st = ifctn_reconstruct(J, X_out_dev, 1);
  if (st != IFCTN_OK) return st;
  HIPTRY(hipStreamSynchronize(J->stream));
  if (out) *out = s;
  return IFCTN_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* ifctn_last_error(void) { return g_err.c_str(); }

size_t ifctn_num_factor_entries(const ifctn_params* params) {
  Geo g;
  if (make_geo(params, &g) != IFCTN_OK) return 0;
  return (size_t)g.nG;
}

size_t ifctn_workspace_bytes(const ifctn_params* params) { return job_bytes(params, current_opts()); }

}  // extern "C"

namespace ifctn {

ifctn_status lr_check(const Geo& g, LrPlan* P) {
  if (g.bf16) return fail(IFCTN_E_UNSUPPORTED, "BF16_REFINE supports edge ranks up to %d", MAXR);
  if (!plan_lr(g, P)) return fail(IFCTN_E_UNSUPPORTED, "a mode product of the large-rank route exceeds 2^31 entries");
  return IFCTN_OK;
}

size_t job_bytes(const ifctn_params* params, const PlanOpts& o) {
  Geo g;
  if (make_geo(params, &g) != IFCTN_OK) return 0;
  if (large_ranks(g)) {
    LrPlan P;
    if (lr_check(g, &P) != IFCTN_OK) return 0;
    return lr_sizes(g, P).total;
  }
  ContractPlan cp[MAXN];
  const Sizes s = job_sizes(g, cp, nullptr, o);
  const char* why = "";
  for (int k = 0; k < g.N; ++k)
    if (!plan_ok(g, cp[k], &why)) {
      fail(IFCTN_E_UNSUPPORTED, "no valid work plan for mode %d (%s)", k, why);
      return 0;
    }
  return s.total;
}

}  // namespace ifctn

extern "C" {

ifctn_status ifctn_destroy(ifctn_job* job) {
  if (!job) return IFCTN_OK;
  for (int c = 0; c < KC_COUNT; ++c)
    for (hipEvent_t e : job->ev[c]) (void)hipEventDestroy(e);
  if (job->side) {
    (void)hipStreamSynchronize(job->side);
    (void)hipStreamDestroy(job->side);
  }
  if (job->ev_fork) (void)hipEventDestroy(job->ev_fork);
  if (job->ev_join) (void)hipEventDestroy(job->ev_join);
  if (job->arena && job->own_arena) (void)hipFree(job->arena);
  delete job;
  return IFCTN_OK;
}

}  // extern "C"

namespace ifctn {

// Output n of SplitMix64 started from `seed` (Steele, Lea and Flood, "Fast
// splittable pseudorandom number generators", OOPSLA 2014): the state after n + 1
// steps is seed + (n + 1) gamma, mixed by two xor-shift-multiply rounds.
uint64_t splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Seeded default G^0 (Algorithm 1 takes G^0 as an input and the paper draws
// it without saying how): packed entry n is s u_n, u_n the 53 high bits of
// SplitMix64 output n as a fraction in [0, 1).  With every factor entry of
// mean s/2, E[W_ab] = R_ab s^2 / 4, and the edge matrices are built from
// disjoint factors, so E[Xhat] = prod_{a<b} R_ab s^2 / 4; s is chosen to make
// that the root mean square m of the observed entries (m = 1 when nothing is
// observed or m is 0).  m is reduced on the device in a fixed order.
ifctn_status default_factors(const Geo& g, const void* O_dev, const uint8_t* mask_dev, uint64_t seed,
                             hipStream_t s, double* G) {
  const int nb = (int)std::min<long long>(1024, std::max<long long>(1, (g.nX + NT - 1) / NT));
  // a stream-ordered buffer: unlike hipFree, hipFreeAsync does not wait for
  // the other streams of the device (jobs a server may be running meanwhile)
  void* buf = nullptr;
  HIPTRY(hipMallocAsync(&buf, (size_t)nb * 16, s));
  double* part = (double*)buf;
  unsigned long long* cnt = (unsigned long long*)(part + nb);
  std::vector<double> hp(nb);
  std::vector<unsigned long long> hc(nb);
  hipError_t e = launch_obs_sumsq(g.dtype, O_dev, mask_dev, g.nX, part, cnt, nb, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, (size_t)nb * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), cnt, (size_t)nb * 8, hipMemcpyDeviceToHost, s);
  const hipError_t ef = hipFreeAsync(buf, s);
  if (e == hipSuccess) e = ef;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  HIPTRY(e);
  double sum = 0.0;
  unsigned long long c = 0;
  for (int b = 0; b < nb; ++b) {
    sum += hp[b];
    c += hc[b];
  }
  double m = c > 0 ? std::sqrt(sum / (double)c) : 0.0;
  if (!(m > 0.0) || !std::isfinite(m)) m = 1.0;
  double prodR = 1.0;
  for (int a = 0; a < g.N; ++a)
    for (int b = a + 1; b < g.N; ++b) prodR *= g.R[a][b];
  const double sc = 2.0 * std::pow(m / prodR, 1.0 / (2.0 * g.ne));
  for (long long n = 0; n < g.nG; ++n)
    G[n] = sc * ((double)(splitmix64(seed, (uint64_t)n) >> 11) * 0x1.0p-53);
  return IFCTN_OK;
}

ifctn_status job_open(const ifctn_params* params, const void* O_dev, const uint8_t* mask_dev,
                      const double* G0_host, hipStream_t stream, unsigned char* pool, size_t pool_bytes,
                      bool check_now, const PlanOpts& opts, ifctn_job** out) {
  if (!out) return fail(IFCTN_E_INVAL, "out is NULL");
  *out = nullptr;
  Geo g;
  ifctn_status st = make_geo(params, &g);
  if (st != IFCTN_OK) return st;
  if (!O_dev || !mask_dev) return fail(IFCTN_E_INVAL, "O_dev and mask_dev are required");
  if (!G0_host) return fail(IFCTN_E_INVAL, "G0_host (initial factors) is required");
  ifctn_job* J = new ifctn_job();
  J->g = g;
  J->stream = (hipStream_t)stream;
  J->opts = opts;
  J->lr = large_ranks(g);
  if (J->lr) {
    st = lr_check(g, &J->lp);
    if (st != IFCTN_OK) {
      delete J;
      return st;
    }
  }
  const Sizes s = J->lr ? lr_sizes(g, J->lp) : job_sizes(g, J->cplan, J->qplan, opts, J->gplan, J->gsol, J->groute);
  for (int k = 0; k < g.N && !J->lr; ++k) {
    const char* why = "";
    if (!plan_ok(g, J->cplan[k], &why)) {
      delete J;
      return fail(IFCTN_E_UNSUPPORTED, "no valid work plan for mode %d (%s)", k, why);
    }
  }
  if (pool) {
    if (pool_bytes < s.total) {
      delete J;
      return fail(IFCTN_E_NOMEM, "pool slice of %zu bytes < %zu needed", pool_bytes, s.total);
    }
    J->arena = pool;
    J->own_arena = false;
  } else {
    hipError_t e = hipMalloc((void**)&J->arena, s.total);
    if (e != hipSuccess) {
      delete J;
      (void)hipGetLastError();
      return fail(e == hipErrorOutOfMemory ? IFCTN_E_NOMEM : IFCTN_E_HIP, "hipMalloc(%zu): %s", s.total,
                  hipGetErrorString(e));
    }
  }
  J->arena_bytes = s.total;
  unsigned char* p = J->arena;
  J->X = p;                      p += s.x;
  J->Xb = (bf16x*)p;             p += s.xb;
  J->bits = (uint32_t*)p;        p += s.bits;
  J->G = (double*)p;             p += s.G;
  J->W64 = (double*)p;           p += s.W64;
  J->Wc = p;                     p += s.Wc;
  J->Q = (double*)p;             p += s.Q;
  J->Upart = (double*)p;         p += s.Upart;
  J->Ugrp = (double*)p;          p += s.Ugrp;
  J->ucnt = (int*)p;             p += s.ucnt;
  J->Ufin = (double*)p;          p += s.Ufin;
  J->Hpart = (double*)p;         p += s.Hpart;
  J->hcnt = (int*)p;             p += s.hcnt;
  J->normpart = (double*)p;      p += s.normpart;
  J->dgpart = (double*)p;        p += s.dgpart;
  J->stats5 = (double*)p;        p += s.stats;
  J->flag = (int*)p;             p += s.flag;
  QItem* dq = (QItem*)p;         p += s.qitems;
  J->gamma = (double*)p;         p += s.gamma;
  J->gmpart = (double*)p;        p += s.gmpart;
  J->dgp = (GammaPlan*)p;        p += al256(sizeof(GammaPlan) * MAXN);
  J->dgs = (GSolve*)p;           p += al256(sizeof(GSolve) * MAXN);
  int* dtab = (int*)p;           p += s.gtab;
  double* lrb0 = (double*)p;     p += s.lr0;
  double* lrb1 = (double*)p;     p += s.lr1;
  double* lrc = (double*)p;      p += s.lrc;
  double* lrh = (double*)p;      p += s.lrh;
  std::vector<int>& htab = J->htab;
  J->bf16_phase = g.bf16;
  if (J->lr) {
    lr_bind(&J->lp, g, J->X, J->bits, J->G, J->W64, J->Wc, lrb0, lrb1, lrc, lrh, J->normpart, J->dgpart,
            J->flag + 1);
    J->nnorm = J->lp.xblk;
    long long ndg = 0;
    for (int k = 0; k < g.N; ++k) ndg += (long long)(g.N - 1) * g.dims[k];
    J->ndg = (int)ndg;
  }
  for (int k = 0; k < g.N && !J->lr; ++k) {
    ContractArgs& a = J->cplan[k].a;
    a.X = g.bf16 ? (void*)J->Xb : J->X;
    a.maskbits = J->bits;
    a.Wc = J->Wc;
    a.G = J->G;
    a.Upart = J->Upart;
    a.Ugrp = J->Ugrp;
    a.ucnt = J->ucnt;
    a.normpart = J->normpart;
    J->qplan[k].W64 = J->W64;
    J->qplan[k].G = J->G;
    J->qplan[k].Q = J->Q;
    J->qplan[k].dit = dq + (size_t)k * (MAXN - 1);
    a.stop = J->flag + 1;
    J->qplan[k].stop = J->flag + 1;
  }
  if (!J->lr) {
    J->nnorm = J->cplan[0].a.JT * J->cplan[0].a.S * J->cplan[0].a.FS;
    build_solve_plans(J);
  }
  for (int k = 0; k < g.N && !J->lr; ++k) {
    if (!J->groute[k]) continue;
    GammaPlan& gp = J->gplan[k];
    gp.W64 = J->W64;
    gp.G = J->G;
    gp.part = J->gmpart;
    gp.gamma = J->gamma;
    const ContractArgs& ca = J->cplan[k].a;
    gp.S = ca.ugrp ? ca.ngrp : ca.S * ca.FS;
    gp.Upart = ca.ugrp ? J->Ugrp : J->Upart;
    gp.nout = (long long)ca.Ik * ca.Rprod;
    // slices of about 8 slots (one batch of loads each), 4..64 per output
    gp.us = 4;
    while (gp.us < 64 && (long long)gp.us * 8 < gp.S) gp.us *= 2;
    gp.nuw = (int)cdiv(gp.nout, NT / gp.us);
    gp.Ufin = J->Ufin;
    GSolve& gs = J->gsol[k];
    gs.S = 1;                        // the U rows arrive reduced (Ufin)
    gs.Upart = J->Ufin;
    gs.gamma = J->gamma;
    gs.W64 = J->W64;
    gs.Wc = J->Wc;
    gs.G = J->G;
    gs.dgpart = J->splan[k].dgpart;
    gs.stop = J->flag + 1;
    J->phased[k] = false;
    std::vector<int> tk;
    GSolve again;
    plan_gsolve(g, k, gp, &again, &tk);          // the same plan, with its offset tables
    for (int t = 0; t < g.N - 1; ++t)
      for (int c = 0; c < g.N - 2; ++c) {
        gs.hsc[t][c] = again.hsc[t][c];
        gs.bsc[t][c] = again.bsc[t][c];
      }
    gs.tab = dtab + htab.size();
    htab.insert(htab.end(), tk.begin(), tk.end());
  }
  J->onelaunch = opts.onelaunch;
  for (int k = 0; k < g.N; ++k) {
    J->merge[k] = opts.merge_gram;
    J->splan[k].stop = J->flag + 1;
    for (int t = 0; t < g.N - 1; ++t) J->pplan[k][t].stop = J->flag + 1;
  }
  for (int k = 0; k < g.N && !J->lr; ++k) {
    const bool too_big = !J->groute[k] && (J->phased[k] ? (size_t)J->splan[k].Rprod * 8 > kMaxLds
                                                        : solve_smem_bytes(J->splan[k]) > kMaxLds);
    if (too_big) {
      if (J->own_arena) (void)hipFree(J->arena);
      delete J;
      return fail(IFCTN_E_UNSUPPORTED, "mode sizes too large for the factor-block kernel (mode %d)", k);
    }
  }
  auto bail = [&](ifctn_status code, const char* what, hipError_t err) {
    ifctn_status r = fail(code, "%s: %s", what, hipGetErrorString(err));
    ifctn_destroy(J);
    return r;
  };
  bool any_gamma = false;
  for (int k = 0; k < g.N && !J->lr; ++k) any_gamma = any_gamma || J->groute[k];
  if (any_gamma && opts.overlap) {
    // default priority (a non-blocking stream: ordered by the events only)
    hipError_t e = hipStreamCreateWithFlags(&J->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&J->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&J->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return bail(IFCTN_E_HIP, "side stream", e);
  }
#define INIT_TRY(expr)                                         \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return bail(IFCTN_E_HIP, #expr, e_); \
  } while (0)
  INIT_TRY(hipMemsetAsync(J->normpart, 0, s.normpart, J->stream));
  INIT_TRY(hipMemsetAsync(J->dgpart, 0, s.dgpart, J->stream));
  INIT_TRY(hipMemsetAsync(J->flag, 0, s.flag, J->stream));
  INIT_TRY(hipMemsetAsync(J->hcnt, 0, s.hcnt, J->stream));
  INIT_TRY(hipMemsetAsync(J->ucnt, 0, s.ucnt, J->stream));
  INIT_TRY(hipMemcpyAsync(J->dgp, J->gplan, sizeof(GammaPlan) * MAXN, hipMemcpyHostToDevice, J->stream));
  INIT_TRY(hipMemcpyAsync(J->dgs, J->gsol, sizeof(GSolve) * MAXN, hipMemcpyHostToDevice, J->stream));
  if (!htab.empty())
    INIT_TRY(hipMemcpyAsync(dtab, htab.data(), htab.size() * sizeof(int), hipMemcpyHostToDevice, J->stream));
  INIT_TRY(hipMemcpyAsync(J->G, G0_host, g.nG * 8, hipMemcpyHostToDevice, J->stream));
  for (int k = 0; k < g.N && !J->lr; ++k)
    INIT_TRY(hipMemcpyAsync((void*)J->qplan[k].dit, J->qplan[k].it, sizeof(QItem) * (MAXN - 1),
                            hipMemcpyHostToDevice, J->stream));
  INIT_TRY(launch_init_x(g.dtype, O_dev, mask_dev, J->X, J->bits, J->flag, g.nX, J->stream));
  if (g.bf16) INIT_TRY(launch_narrow((const float*)J->X, J->Xb, g.nX, J->stream));
  for (int e2 = 0; e2 < g.ne; ++e2) {
    const int a = g.ea[e2], b = g.eb[e2];
    INIT_TRY(launch_edge(g.dtype, J->G + g.goff[a][b], J->G + g.goff[b][a], g.R[a][b], g.dims[a], g.dims[b],
                         J->W64 + g.woff[e2], (unsigned char*)J->Wc + g.woff[e2] * g.esz, J->stream));
  }
  if (check_now) {
    int bad = 0;
    INIT_TRY(hipMemcpyAsync(&bad, J->flag, sizeof(int), hipMemcpyDeviceToHost, J->stream));
    INIT_TRY(hipStreamSynchronize(J->stream));
    if (bad) {
      ifctn_destroy(J);
      return fail(IFCTN_E_INVAL, "an observed entry of O is not finite");
    }
  }
#undef INIT_TRY
  *out = J;
  return IFCTN_OK;
}

hipError_t job_sweeps(ifctn_job* J, int n) {
  for (int q = 0; q < n; ++q) {
    hipError_t e = run_sweep(J);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t job_x_step(ifctn_job* J) { return flush_update(J); }

hipError_t job_promote(ifctn_job* J) { return promote(J); }

bool job_is_bf16(const ifctn_job* J) { return J->g.bf16; }

int job_refine_sweeps(const ifctn_job* J) { return J->g.refine; }

void job_set_stop(ifctn_job* J, double eps) {
  J->dev_stop = eps > 0.0;
  J->stop_eps = eps;
}

hipError_t job_reset_flags(ifctn_job* J) { return hipMemsetAsync(J->flag + 1, 0, 2 * sizeof(int), J->stream); }

const int* job_flags(const ifctn_job* J) { return J->flag; }

hipError_t job_finalize(ifctn_job* J) {
  return launch_finalize(J->normpart, J->nnorm, J->dgpart, J->ndg, J->stats5, J->stream);
}

const double* job_stats_dev(const ifctn_job* J) { return J->stats5; }

void stats_from(const double* h, int sweeps_done, ifctn_stats* out) {
  out->dx_norm2 = h[0];
  out->x_norm2 = h[1];
  out->objective = 0.5 * h[2];
  out->dg_norm2 = h[3];
  out->rel_change = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : (h[0] == 0.0 ? 0.0 : INFINITY);
  out->sweeps_done = sweeps_done;
  out->converged = 0;
}

ifctn_status job_close(ifctn_job* J) { return ifctn_destroy(J); }

ifctn_status set_error(ifctn_status st, const char* msg) { return fail(st, "%s", msg); }

}  // namespace ifctn

extern "C" {

ifctn_status ifctn_init(const ifctn_params* params, const void* O_dev, const uint8_t* mask_dev,
                        const double* G0_host, void* stream, ifctn_job** out) {
  std::vector<double> G0;
  if (!G0_host && params && O_dev && mask_dev) {   // the seeded default, seed 0
    Geo g;
    ifctn_status st = make_geo(params, &g);
    if (st != IFCTN_OK) return st;
    G0.resize((size_t)g.nG);
    st = default_factors(g, O_dev, mask_dev, 0, (hipStream_t)stream, G0.data());
    if (st != IFCTN_OK) return st;
    G0_host = G0.data();
  }
  // job_open synchronises the stream before it returns, so G0 outlives the copy
  return job_open(params, O_dev, mask_dev, G0_host, (hipStream_t)stream, nullptr, 0, true, current_opts(), out);
}

ifctn_status ifctn_default_factors(const ifctn_params* params, const void* O_dev, const uint8_t* mask_dev,
                                   uint64_t seed, void* stream, double* G_host) {
  Geo g;
  ifctn_status st = make_geo(params, &g);
  if (st != IFCTN_OK) return st;
  if (!O_dev || !mask_dev || !G_host) return fail(IFCTN_E_INVAL, "O_dev, mask_dev and G_host are required");
  return default_factors(g, O_dev, mask_dev, seed, (hipStream_t)stream, G_host);
}


ifctn_status ifctn_sweep(ifctn_job* J, int32_t nsweeps, ifctn_stats* stats) {
  if (!J) return fail(IFCTN_E_INVAL, "job is NULL");
  if (nsweeps < 0) return fail(IFCTN_E_INVAL, "nsweeps < 0");
  for (int s = 0; s < nsweeps; ++s) HIPTRY(run_sweep(J));
  HIPTRY(flush_update(J));
  if (stats) {
    HIPTRY(launch_finalize(J->normpart, J->nnorm, J->dgpart, J->ndg, J->stats5, J->stream));
    double h[5];
    HIPTRY(hipMemcpyAsync(h, J->stats5, sizeof(h), hipMemcpyDeviceToHost, J->stream));
    HIPTRY(hipStreamSynchronize(J->stream));
    stats_from(h, J->sweeps_done, stats);
  }
  return IFCTN_OK;
}

ifctn_status ifctn_reconstruct(ifctn_job* J, void* out_dev, int32_t which) {
  if (!J || !out_dev) return fail(IFCTN_E_INVAL, "job and out_dev are required");
  if (which == 1) {
    HIPTRY(flush_update(J));
    if (J->bf16_phase)
      HIPTRY(launch_widen(J->Xb, J->bits, (const float*)J->X, (float*)out_dev, J->g.nX, J->stream));
    else
      HIPTRY(hipMemcpyAsync(out_dev, J->X, J->g.nX * J->g.esz, hipMemcpyDeviceToDevice, J->stream));
    return IFCTN_OK;
  }
  if (which != 0) return fail(IFCTN_E_INVAL, "which must be 0 or 1");
  ReconArgs r;
  std::memset(&r, 0, sizeof(r));
  r.N = J->g.N;
  for (int m = 0; m < r.N; ++m) r.dims[m] = J->g.dims[m];
  r.nX = J->g.nX;
  r.ne = J->g.ne;
  for (int e = 0; e < r.ne; ++e) {
    r.ea[e] = J->g.ea[e];
    r.eb[e] = J->g.eb[e];
    r.woff[e] = J->g.woff[e];
  }
  r.Wc = J->Wc;
  r.out = out_dev;
  HIPTRY(launch_reconstruct(J->g.dtype, r, J->stream));
  return IFCTN_OK;
}

ifctn_status ifctn_get_factors(ifctn_job* J, double* G_host) {
  if (!J || !G_host) return fail(IFCTN_E_INVAL, "job and G_host are required");
  HIPTRY(hipMemcpyAsync(G_host, J->G, J->g.nG * 8, hipMemcpyDeviceToHost, J->stream));
  HIPTRY(hipStreamSynchronize(J->stream));
  return IFCTN_OK;
}

ifctn_status ifctn_promote(ifctn_job* J) {
  if (!J) return fail(IFCTN_E_INVAL, "job is NULL");
  if (!J->g.bf16) return fail(IFCTN_E_STATE, "ifctn_promote needs a BF16_REFINE job");
  HIPTRY(promote(J));
  return IFCTN_OK;
}

ifctn_status ifctn_complete(const ifctn_params* params, const void* O_dev, const uint8_t* mask_dev,
                            const double* G0_host, int32_t t_max, double eps, void* X_out_dev,
                            ifctn_stats* stats, void* stream) {
  if (t_max < 0) return fail(IFCTN_E_INVAL, "t_max < 0");
  if (!(eps >= 0.0)) return fail(IFCTN_E_INVAL, "eps < 0");
  if (!X_out_dev) return fail(IFCTN_E_INVAL, "X_out_dev is required");
  ifctn_job* J = nullptr;
  ifctn_status st = ifctn_init(params, O_dev, mask_dev, G0_host, stream, &J);
  if (st != IFCTN_OK) return st;
  st = run_complete(J, t_max, eps, X_out_dev, stats);
  ifctn_destroy(J);
  return st;
}

}  // extern "C"

namespace {

// iFCTN(G) into out_dev with the edge matrices in buf (bG + bW + bWc bytes):
// G to the device, every W_ab = G_{a,b}^T G_{b,a}, then the Hadamard product.
// Synchronises the stream.
hipError_t assemble_into(const Geo& g, const double* G_host, void* out_dev, hipStream_t s, unsigned char* buf) {
  const size_t bG = al256(g.nG * 8), bW = al256(g.nW * 8);
  double* G = (double*)buf;
  double* W64 = (double*)(buf + bG);
  unsigned char* Wc = buf + bG + bW;
  hipError_t e = hipMemcpyAsync(G, G_host, g.nG * 8, hipMemcpyHostToDevice, s);
  for (int x = 0; x < g.ne && e == hipSuccess; ++x) {
    const int a = g.ea[x], b = g.eb[x];
    e = launch_edge(g.dtype, G + g.goff[a][b], G + g.goff[b][a], g.R[a][b], g.dims[a], g.dims[b],
                    W64 + g.woff[x], Wc + g.woff[x] * g.esz, s);
  }
  if (e == hipSuccess) {
    ReconArgs r;
    std::memset(&r, 0, sizeof(r));
    r.N = g.N;
    for (int m = 0; m < g.N; ++m) r.dims[m] = g.dims[m];
    r.nX = g.nX;
    r.ne = g.ne;
    for (int x = 0; x < g.ne; ++x) {
      r.ea[x] = g.ea[x];
      r.eb[x] = g.eb[x];
      r.woff[x] = g.woff[x];
    }
    r.Wc = Wc;
    r.out = out_dev;
    e = launch_reconstruct(g.dtype, r, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

// The allocation-free variant's edge-matrix buffer: a file-scope device array
// of kScratchBytes, one per GPU, held until the process ends.  In host code
// `scratch` is only a symbol: its device address on the current GPU comes
// from hipGetSymbolAddress, fetched once per device on the first call there.
constexpr size_t kScratchBytes = IFCTN_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::atomic<unsigned char*> g_scratch_dev[kMaxDevices];

ifctn_status scratch_address(unsigned char** out) {
  int dev = -1;
  HIPTRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(IFCTN_E_UNSUPPORTED, "device ordinal %d out of range", dev);
  unsigned char* p = g_scratch_dev[dev].load(std::memory_order_acquire);
  if (!p) {
    void* a = nullptr;
    HIPTRY(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
    p = (unsigned char*)a;
    g_scratch_dev[dev].store(p, std::memory_order_release);   // the same address whichever thread stores
  }
  *out = p;
  return IFCTN_OK;
}

}  // namespace

extern "C" {

ifctn_status ifctn_assemble_noalloc(const ifctn_params* params, const double* G_host, void* out_dev,
                                    void* stream) {
  Geo g;
  ifctn_status st = make_geo(params, &g);
  if (st != IFCTN_OK) return st;
  if (!G_host || !out_dev) return fail(IFCTN_E_INVAL, "G_host and out_dev are required");
  const size_t need = al256(g.nG * 8) + al256(g.nW * 8) + al256(g.nW * g.esz);
  if (need > kScratchBytes)
    return fail(IFCTN_E_UNSUPPORTED, "factors and edge matrices need %zu bytes; the allocation-free assemble holds %zu",
                need, kScratchBytes);
  unsigned char* buf = nullptr;
  st = scratch_address(&buf);
  if (st != IFCTN_OK) return st;
  const hipError_t e = assemble_into(g, G_host, out_dev, (hipStream_t)stream, buf);
  if (e != hipSuccess) return fail(IFCTN_E_HIP, "assemble: %s", hipGetErrorString(e));
  return IFCTN_OK;
}

ifctn_status ifctn_assemble(const ifctn_params* params, const double* G_host, void* out_dev, void* stream) {
  Geo g;
  ifctn_status st = make_geo(params, &g);
  if (st != IFCTN_OK) return st;
  if (!G_host || !out_dev) return fail(IFCTN_E_INVAL, "G_host and out_dev are required");
  hipStream_t s = (hipStream_t)stream;
  const size_t bG = al256(g.nG * 8), bW = al256(g.nW * 8), bWc = al256(g.nW * g.esz);
  unsigned char* buf = nullptr;
  HIPTRY(hipMalloc((void**)&buf, bG + bW + bWc));
  const hipError_t e = assemble_into(g, G_host, out_dev, s, buf);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(IFCTN_E_HIP, "assemble: %s", hipGetErrorString(e));
  return IFCTN_OK;
}

ifctn_status ifctn_plan_blocks(const ifctn_params* params, ifctn_block_plan* out) {
  if (!out) return fail(IFCTN_E_INVAL, "out is NULL");
  Geo g;
  ifctn_status st = make_geo(params, &g);
  if (st != IFCTN_OK) return st;
  if (large_ranks(g)) {
    LrPlan P;
    st = lr_check(g, &P);
    if (st != IFCTN_OK) return st;
    for (int k = 0; k < g.N; ++k) {
      out[k].route = 3;
      out[k].reserved = 0;
      out[k].gamma_fma = 0.0;
    }
    return IFCTN_OK;
  }
  const PlanOpts o = current_opts();
  ContractPlan cp[MAXN];
  QArgs qp[MAXN];
  GammaPlan gp[MAXN];
  GSolve gs[MAXN];
  bool gr[MAXN] = {};
  job_sizes(g, cp, qp, o, gp, gs, gr);
  for (int k = 0; k < g.N; ++k) {
    out[k].route = gr[k] ? 2 : (use_phased(g, qp[k], k, o) ? 1 : 0);
    out[k].reserved = 0;
    out[k].gamma_fma = gr[k] ? gp[k].fma : 0.0;
  }
  return IFCTN_OK;
}

ifctn_status ifctn_set_option(const char* name, int64_t value) {
  if (!name) return fail(IFCTN_E_INVAL, "name is NULL");
  if (std::strcmp(name, "phased_min") == 0) {
    g_phased_min.store(value < 0 ? -1 : (long long)value);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "phased_onelaunch") == 0) {
    g_onelaunch.store(value);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "merge_gram") == 0) {
    g_merge_gram.store(value);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "contract_div") == 0) {
    g_contract_div.store(value);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "contract_emin") == 0) {
    g_contract_emin.store(value);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "gamma") == 0) {
    g_gamma.store(value < 0 ? -1 : value);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "overlap") == 0) {
    g_overlap.store(value < 0 ? -1 : value);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "ugroup") == 0) {
    g_ugroup.store(value < 0 ? -1 : value);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "inject_admit_failures") == 0) {
    g_inject_admit.store(value > 0 ? value : 0);
    return IFCTN_OK;
  }
  if (std::strcmp(name, "contract_jmax") == 0) {
    g_contract_jmax.store(value);
    return IFCTN_OK;
  }
  return fail(IFCTN_E_INVAL, "unknown option '%s'", name);
}

ifctn_status ifctn_timing_enable(ifctn_job* J, int32_t enable) {
  if (!J) return fail(IFCTN_E_INVAL, "job is NULL");
  HIPTRY(hipStreamSynchronize(J->stream));
  J->timing = enable != 0;
  for (int c = 0; c < KC_COUNT; ++c) J->evn[c] = 0;
  return IFCTN_OK;
}

ifctn_status ifctn_timing_query(ifctn_job* J, int32_t kernel_class, double* total_ms, int64_t* launches) {
  if (!J || !total_ms || !launches) return fail(IFCTN_E_INVAL, "job, total_ms and launches are required");
  if (kernel_class < 0 || kernel_class >= KC_COUNT) return fail(IFCTN_E_INVAL, "unknown kernel class");
  HIPTRY(hipStreamSynchronize(J->stream));
  double t = 0.0;
  for (size_t n = 0; n < J->evn[kernel_class]; ++n) {
    float ms = 0.f;
    HIPTRY(hipEventElapsedTime(&ms, J->ev[kernel_class][2 * n], J->ev[kernel_class][2 * n + 1]));
    t += ms;
  }
  *total_ms = t;
  *launches = (int64_t)J->evn[kernel_class];
  return IFCTN_OK;
}

}  // extern "C"
