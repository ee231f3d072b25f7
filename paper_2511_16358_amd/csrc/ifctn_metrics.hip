// Image-quality metrics of Sec. 5 for completed image-shaped tensors
// (H x W x B, bands the last mode): MPSNR, the mean over bands of the peak
// signal-to-noise ratio, and MSSIM, the mean over bands of the structural
// similarity index (Wang et al. 2004: 11 x 11 Gaussian window with standard
// deviation 1.5, constants (0.01 L)^2 and (0.03 L)^2 for the dynamic range L,
// mean of the SSIM map over the positions where the window fits).  All sums
// are float64 and reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "ifctn.h"
#include "ifctn_host.h"

namespace ifctn {
namespace {

constexpr int MT = 256;
constexpr int WIN = 11;

__constant__ double c_win[WIN * WIN];

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < MT / 64; ++q) s += red[q];
  return s;
}

// squared error of band b (grid.y) over a range of pixels (grid.x)
template <typename T>
__global__ __launch_bounds__(MT) void k_band_sqerr(const T* __restrict__ X, const T* __restrict__ Y, long long HW,
                                                   int B, double* __restrict__ part) {
  __shared__ double red[MT / 64];
  const int b = blockIdx.y;
  double v = 0.0;
  for (long long p = (long long)blockIdx.x * MT + threadIdx.x; p < HW; p += (long long)gridDim.x * MT) {
    const double d = (double)X[p * B + b] - (double)Y[p * B + b];
    v += d * d;
  }
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = s;
}

// SSIM map of band b (grid.y) over one 16 x 16 tile of window positions
// (grid.x): the 26 x 26 patch of both images is staged in LDS once, then each
// thread forms the weighted moments of its window from LDS.
constexpr int ST = 16;                 // output tile edge
constexpr int SP = ST + WIN - 1;       // staged patch edge

template <typename T>
__global__ __launch_bounds__(MT) void k_band_ssim(const T* __restrict__ X, const T* __restrict__ Y, int H, int W,
                                                  int B, double c1, double c2, double* __restrict__ part) {
  __shared__ double red[MT / 64];
  __shared__ double px[SP * SP], py[SP * SP];
  const int b = blockIdx.y;
  const int Hv = H - WIN + 1, Wv = W - WIN + 1;
  const int tw = (Wv + ST - 1) / ST;
  const int th0 = (int)(blockIdx.x / tw) * ST, tw0 = (int)(blockIdx.x % tw) * ST;
  for (int e = threadIdx.x; e < SP * SP; e += MT) {
    const int y = min(th0 + e / SP, H - 1), x = min(tw0 + e % SP, W - 1);   // clamped: unused past the edge
    const long long o = ((long long)y * W + x) * B + b;
    px[e] = (double)X[o];
    py[e] = (double)Y[o];
  }
  __syncthreads();
  const int ly = threadIdx.x / ST, lx = threadIdx.x % ST;
  double acc = 0.0;
  if (th0 + ly < Hv && tw0 + lx < Wv) {
    double mx = 0.0, my = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
    for (int dy = 0; dy < WIN; ++dy) {
#pragma unroll
      for (int dx = 0; dx < WIN; ++dx) {
        const double g = c_win[dy * WIN + dx];
        const double x = px[(ly + dy) * SP + lx + dx], y = py[(ly + dy) * SP + lx + dx];
        mx += g * x;
        my += g * y;
        sxx += g * x * x;
        syy += g * y * y;
        sxy += g * x * y;
      }
    }
    const double vx = sxx - mx * mx, vy = syy - my * my, cxy = sxy - mx * my;
    acc = ((2.0 * mx * my + c1) * (2.0 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2));
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[(long long)b * gridDim.x + blockIdx.x] = s;
}

// per band: sum of the partials in order
__global__ __launch_bounds__(64) void k_band_total(const double* __restrict__ part, int nblk, int B,
                                                   double* __restrict__ out) {
  for (int b = threadIdx.x; b < B; b += 64) {
    double s = 0.0;
    for (int q = 0; q < nblk; ++q) s += part[(long long)b * nblk + q];
    out[b] = s;
  }
}

}  // namespace
}  // namespace ifctn

using namespace ifctn;

extern "C" ifctn_status ifctn_image_metrics(const void* X_dev, const void* ref_dev, int64_t H, int64_t W, int64_t B,
                                            int32_t precision, double peak, double* psnr_host, double* ssim_host,
                                            double* mpsnr, double* mssim, void* stream) {
  if (!X_dev || !ref_dev || !mpsnr || !mssim) return set_error(IFCTN_E_INVAL, "X_dev, ref_dev, mpsnr, mssim required");
  if (H < WIN || W < WIN || B < 1 || H > (1 << 20) || W > (1 << 20) || B > (1 << 20))
    return set_error(IFCTN_E_INVAL, "image must be at least 11 x 11 with >= 1 band");
  if (!(peak > 0.0)) return set_error(IFCTN_E_INVAL, "peak must be > 0");
  if (precision != IFCTN_FP32 && precision != IFCTN_FP64) return set_error(IFCTN_E_INVAL, "precision must be FP32 or FP64");
  hipStream_t s = (hipStream_t)stream;
  // normalised 11 x 11 Gaussian window, sigma 1.5
  double win[WIN * WIN], tot = 0.0;
  for (int y = 0; y < WIN; ++y)
    for (int x = 0; x < WIN; ++x) {
      const double dy = y - WIN / 2, dx = x - WIN / 2;
      win[y * WIN + x] = std::exp(-(dx * dx + dy * dy) / (2.0 * 1.5 * 1.5));
      tot += win[y * WIN + x];
    }
  for (double& v : win) v /= tot;
  const long long HW = H * W;
  const long long nv = (H - WIN + 1) * (W - WIN + 1);
  const int nb_e = (int)std::min<long long>(64, (HW + MT - 1) / MT);
  const int nb_s = (int)(((H - WIN + 1 + ST - 1) / ST) * ((W - WIN + 1 + ST - 1) / ST));   // output tiles
  double* buf = nullptr;
  const size_t n_part = (size_t)B * (nb_e + nb_s), n_out = 2 * (size_t)B;
  if (hipMalloc((void**)&buf, (n_part + n_out) * sizeof(double)) != hipSuccess)
    return set_error(IFCTN_E_NOMEM, "metrics scratch allocation failed");
  double* pe = buf;
  double* ps = buf + (size_t)B * nb_e;
  double* tot_dev = buf + n_part;
  const double L = peak, c1 = (0.01 * L) * (0.01 * L), c2 = (0.03 * L) * (0.03 * L);
  hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_win), win, sizeof(win), 0, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    const dim3 ge((unsigned)nb_e, (unsigned)B), gs((unsigned)nb_s, (unsigned)B);
    if (precision == IFCTN_FP32) {
      hipLaunchKernelGGL(k_band_sqerr<float>, ge, dim3(MT), 0, s, (const float*)X_dev, (const float*)ref_dev, HW,
                         (int)B, pe);
      hipLaunchKernelGGL(k_band_ssim<float>, gs, dim3(MT), 0, s, (const float*)X_dev, (const float*)ref_dev, (int)H,
                         (int)W, (int)B, c1, c2, ps);
    } else {
      hipLaunchKernelGGL(k_band_sqerr<double>, ge, dim3(MT), 0, s, (const double*)X_dev, (const double*)ref_dev, HW,
                         (int)B, pe);
      hipLaunchKernelGGL(k_band_ssim<double>, gs, dim3(MT), 0, s, (const double*)X_dev, (const double*)ref_dev,
                         (int)H, (int)W, (int)B, c1, c2, ps);
    }
    hipLaunchKernelGGL(k_band_total, dim3(1), dim3(64), 0, s, pe, nb_e, (int)B, tot_dev);
    hipLaunchKernelGGL(k_band_total, dim3(1), dim3(64), 0, s, ps, nb_s, (int)B, tot_dev + B);
    e = hipGetLastError();
  }
  std::vector<double> h(n_out);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), tot_dev, n_out * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) return set_error(IFCTN_E_HIP, hipGetErrorString(e));
  double sp = 0.0, ss = 0.0;
  for (int64_t b = 0; b < B; ++b) {
    const double mse = h[b] / (double)HW;
    const double p = 10.0 * std::log10(peak * peak / mse);   // +inf for identical bands
    const double q = h[B + b] / (double)nv;
    if (psnr_host) psnr_host[b] = p;
    if (ssim_host) ssim_host[b] = q;
    sp += p;
    ss += q;
  }
  *mpsnr = sp / (double)B;
  *mssim = ss / (double)B;
  return IFCTN_OK;
}
