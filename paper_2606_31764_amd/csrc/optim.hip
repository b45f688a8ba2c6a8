// nsplat_adam_step: one optimiser step on the learnable parameters, as the
// supplementary settings give it: Adam per parameter group with its own
// learning rate, a cosine decay of every rate to final_ratio of itself over
// the run, and the clamps of the rational weights and knot intervals.
//
//   k_step_next  t = *step + 1 (one lane), so that a captured graph advances
//   k_adam       one lane per parameter: moments, bias correction, update,
//                clamp
#include "nsplat_internal.h"

namespace nsp {

namespace {

__global__ void k_step_next(int32_t* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step[0] = step[0] + 1;
}

struct AdamGroups {
  float* x[6];
  const float* g[6];
  int64_t end[6];  // cumulative group sizes (flat index ranges)
};

__global__ __launch_bounds__(256) void k_adam(nsplat_adam cfg, AdamGroups ag, float* __restrict__ m,
                                              float* __restrict__ v, const int32_t* step) {
  const int64_t n = ag.end[5];
  const int t = step[0];
  const double b1t = 1.0 - pow((double)cfg.beta1, (double)t);
  const double b2t = 1.0 - pow((double)cfg.beta2, (double)t);
  double ph = cfg.total_steps > 0 ? (double)(t - 1) / (double)cfg.total_steps : 1.0;
  ph = ph < 0.0 ? 0.0 : (ph > 1.0 ? 1.0 : ph);
  const double decay = (double)cfg.final_ratio + (1.0 - (double)cfg.final_ratio) * 0.5 * (1.0 + cos(M_PI * ph));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int grp = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) grp += i >= ag.end[k] ? 1 : 0;
    const int64_t off = i - (grp ? ag.end[grp - 1] : 0);
    const float g = ag.g[grp][off];
    const float mi = cfg.beta1 * m[i] + (1.0f - cfg.beta1) * g;
    const float vi = cfg.beta2 * v[i] + (1.0f - cfg.beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const double mh = (double)mi / b1t, vh = (double)vi / b2t;
    double x = (double)ag.x[grp][off] - (double)cfg.lr[grp] * decay * mh / (sqrt(vh) + (double)cfg.eps);
    if (grp == 1) x = x < cfg.w_min ? cfg.w_min : (x > cfg.w_max ? cfg.w_max : x);
    if (grp == 3) x = x < cfg.tau_min ? cfg.tau_min : (x > cfg.tau_max ? cfg.tau_max : x);
    ag.x[grp][off] = (float)x;
  }
}

}  // namespace

hipError_t launch_adam(const nsplat_adam* cfg, const nsplat_values* prm, const nsplat_grads* gr, float* m, float* v,
                       int32_t* step_dev, hipStream_t s) {
  AdamGroups ag;
  const int64_t K = prm->n_keys, T = prm->n_taus, N = prm->n_curves, C = prm->channels;
  const int64_t sizes[6] = {2 * K, K, K, T, N * C, N};
  float* xs[6] = {prm->key_xy, prm->key_w, prm->key_s, prm->tau, prm->color, prm->opacity};
  const float* gs[6] = {gr->key_xy, gr->key_w, gr->key_s, gr->tau, gr->color, gr->opacity};
  int64_t acc = 0;
  for (int k = 0; k < 6; ++k) {
    acc += sizes[k];
    ag.end[k] = acc;
    ag.x[k] = xs[k];
    ag.g[k] = gs[k];
  }
  hipLaunchKernelGGL(k_step_next, dim3(1), dim3(64), 0, s, step_dev);
  if (acc > 0)
    hipLaunchKernelGGL(k_adam, dim3(grid_for(acc, 256, 4096)), dim3(256), 0, s, *cfg, ag, m, v, step_dev);
  return hipGetLastError();
}

}  // namespace nsp
