// Backtest metrics of a reward trajectory (the financial metrics the paper evaluates agents with):
// one thread per environment walks its equity curve v_{t+1} = v_t + r_t / scale twice, first for
// the sums, extrema and counts, then for the sample deviation around the mean return.  Loads of
// rew[t][n] are coalesced across the threads of a wavefront.
#include "launch.h"

namespace fm {

namespace {

__global__ void metrics_kernel(const double* __restrict__ rew, int T, int N, double v0_all,
                               const double* __restrict__ v0s, double scale, double P, double rf,
                               double* __restrict__ out) {
#pragma clang fp contract(off)
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double v0 = v0s ? v0s[n] : v0_all;
  const double rfp = rf / P;
  double v = v0, peak = v0, mdd = 0.0, sum = 0.0, up = 0.0, dn = 0.0, down2 = 0.0;
  int wins = 0, losses = 0;
  for (int t = 0; t < T; ++t) {
    const double v_next = v + rew[static_cast<size_t>(t) * N + n] / scale;
    const double rho = v_next / v - 1.0;
    sum += rho;
    if (rho > 0.0) {
      up += rho;
      ++wins;
    } else if (rho < 0.0) {
      dn -= rho;
      ++losses;
    }
    const double ex = rho - rfp;
    if (ex < 0.0) down2 += ex * ex;
    v = v_next;
    peak = fmax(peak, v);
    mdd = fmin(mdd, v / peak - 1.0);
  }
  const double mean = sum / T;
  double ss = 0.0;
  double w = v0;
  for (int t = 0; t < T; ++t) {
    const double w_next = w + rew[static_cast<size_t>(t) * N + n] / scale;
    const double dev = (w_next / w - 1.0) - mean;
    ss += dev * dev;
    w = w_next;
  }
  const double sd = T > 1 ? sqrt(ss / (T - 1)) : __builtin_nan("");
  const double sqp = sqrt(P);
  const double cum = v / v0 - 1.0;
  const double ann = pow(v / v0, P / T) - 1.0;
  const double ex_mean = mean - rfp;
  const double down = sqrt(down2 / T);
  double* o = out + static_cast<size_t>(n) * 10;
  o[0] = cum;
  o[1] = ann;
  o[2] = sd * sqp;
  o[3] = ex_mean / sd * sqp;
  o[4] = mdd;
  o[5] = cum / fabs(mdd);
  o[6] = ex_mean / down * sqp;
  o[7] = ann / fabs(mdd);
  o[8] = up / dn;
  o[9] = static_cast<double>(wins) / static_cast<double>(losses);
}

}  // namespace

hipError_t launch_metrics(const double* rew, int T, int N, double v0, const double* v0s,
                          double reward_scale, double periods_per_year, double risk_free,
                          double* out, hipStream_t stream) {
  hipLaunchKernelGGL(metrics_kernel, dim3((N + 255) / 256), dim3(256), 0, stream, rew, T, N, v0, v0s,
                     reward_scale, periods_per_year, risk_free, out);
  return hipGetLastError();
}

}  // namespace fm
