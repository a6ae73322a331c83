// Kick-drift-kick leapfrog on power-of-two time bins around the interaction
// phase: the kernels of one tick (drift, predicted gas velocities and
// internal energies, kicks with the bin rule). The order of the launches of
// a system step is in api.hip (g3_integrate_start, g3_system_step).
//
// The paper's code advances only the particles that are active at a step,
// on adaptive steps, and drifts the tree between rebuilds (section 1, the
// adaptive time-stepping paragraph; section 2.2). The leapfrog is the
// hierarchical kick-drift-kick of Springel (2005, section 5): a system step
// of dt_max is cut into 2^B ticks of tau = dt_max / 2^B; bin k takes steps
// of 2^(B-k) ticks and is active at tick T iff 2^(B-k) divides T.
#include <cmath>

#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {
namespace {

constexpr int kIntBlock = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + kIntBlock - 1) / kIntBlock); }

// x += v tau, in the positions' precision (FP32 positions: one rounding).
template <typename PT>
__global__ void k_drift(PT *__restrict__ pos, const float *__restrict__ vel, int64_t n3,
                        double tau) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  if constexpr (sizeof(PT) == 8)
    pos[i] = fma((double)vel[i], tau, pos[i]);
  else
    pos[i] = fmaf(vel[i], (float)tau, pos[i]);
}

// Gas velocities and internal energies predicted to tick T from the middle
// of each particle's current step [T0, T0 + S], S = 2^(B - bin), where the
// stored half-kicked values belong: q + dq/dt (T - T0 - S/2) tau.
__global__ void k_predict(int64_t n, const uint8_t *__restrict__ type,
                          const float *__restrict__ vel, const float *__restrict__ u,
                          const float *__restrict__ acc, const float *__restrict__ dudt,
                          const int32_t *__restrict__ bin, int32_t depth, int64_t T, double tau,
                          float *__restrict__ vp, float *__restrict__ up) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (type && type[i] != 0)) return;
  const int32_t b = min(max(bin[i], 0), depth);
  const int64_t S = (int64_t)1 << (depth - b);
  const double mid = (double)(S * ((T - 1) / S)) + 0.5 * (double)S;
  const float dt = (float)(((double)T - mid) * tau);
  vp[3 * i] = fmaf(acc[3 * i], dt, vel[3 * i]);
  vp[3 * i + 1] = fmaf(acc[3 * i + 1], dt, vel[3 * i + 1]);
  vp[3 * i + 2] = fmaf(acc[3 * i + 2], dt, vel[3 * i + 2]);
  up[i] = fmaxf(fmaf(dudt[i], dt, u[i]), 0.0f);
}

// One particle's update at a tick. A particle takes part iff every_particle
// or bin >= kmin (the bins before this launch). In this order:
//   sum    acc = acc (gravity, just written) + hydro acceleration (gas);
//   close  v += a dt_bin / 2, u = max(u + du/dt dt_bin / 2, 0) (gas);
//   rebin  bin = max(k, kmin), k the smallest in [0, B] with
//          dt_max / 2^k <= min(sqrt(2 eta eps / |a|), C h / vsig (gas))
//          (Springel 2005, eqs. 34 and 16);
//   open   the half kick of the (new) step, as close.
template <typename HT>
__global__ void k_update(int64_t n, const IntegUpdate up, const uint8_t *__restrict__ type,
                         float *__restrict__ vel, float *__restrict__ u,
                         float *__restrict__ acc, const float *__restrict__ acc_h,
                         const float *__restrict__ dudt, const float *__restrict__ vsig,
                         const HT *__restrict__ h, int32_t *__restrict__ bin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t k = bin[i];
  if (!up.every_particle && k < up.kmin) return;
  const bool gas = !type || type[i] == 0;
  float ax = acc[3 * i], ay = acc[3 * i + 1], az = acc[3 * i + 2];
  if (up.sum) {
    if (gas) {
      ax += acc_h[3 * i];
      ay += acc_h[3 * i + 1];
      az += acc_h[3 * i + 2];
    }
    acc[3 * i] = ax;
    acc[3 * i + 1] = ay;
    acc[3 * i + 2] = az;
  }
  float vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
  float ui = gas ? u[i] : 0.0f;
  const float du = gas ? dudt[i] : 0.0f;
  auto kick = [&](int32_t kb) {
    const float half = (float)ldexp(0.5 * up.dt_max, -kb);
    vx = fmaf(ax, half, vx);
    vy = fmaf(ay, half, vy);
    vz = fmaf(az, half, vz);
    ui = fmaxf(fmaf(du, half, ui), 0.0f);
  };
  if (up.close) kick(k);
  if (up.rebin) {
    // the criterion in FP64 from the FP32 forces
    const double a = sqrt((double)ax * ax + (double)ay * ay + (double)az * az);
    double dt = a > 0.0 ? sqrt(up.eta_eps2 / a) : INFINITY;
    if (gas && vsig[i] > 0.0f) dt = fmin(dt, up.courant * (double)h[i] / (double)vsig[i]);
    int32_t kn = 0;
    if (dt < up.dt_max) {
      const double x = ceil(log2(up.dt_max / dt));
      kn = x >= (double)up.depth ? up.depth : (int32_t)x;
    }
    k = kn > up.kmin ? kn : up.kmin;
    bin[i] = k;
  }
  if (up.open) kick(k);
  if (up.close || up.open) {
    vel[3 * i] = vx;
    vel[3 * i + 1] = vy;
    vel[3 * i + 2] = vz;
    if (gas) u[i] = ui;
  }
}

__global__ void k_store_count(const uint32_t *__restrict__ count, int64_t *__restrict__ out) {
  if (threadIdx.x == 0) *out = count ? (int64_t)*count : 0;
}

}  // namespace

hipError_t launch_drift(void *pos, int f64, const float *vel, int64_t n, double tau,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (f64)
    k_drift<double><<<nblk(3 * n), kIntBlock, 0, s>>>((double *)pos, vel, 3 * n, tau);
  else
    k_drift<float><<<nblk(3 * n), kIntBlock, 0, s>>>((float *)pos, vel, 3 * n, tau);
  return hipGetLastError();
}

hipError_t launch_predict(int64_t n, const uint8_t *type, const float *vel, const float *u,
                          const float *acc, const float *dudt, const int32_t *bin, int depth,
                          int64_t T, double tau, float *vp, float *up, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_predict<<<nblk(n), kIntBlock, 0, s>>>(n, type, vel, u, acc, dudt, bin, depth, T, tau, vp,
                                          up);
  return hipGetLastError();
}

hipError_t launch_update(int64_t n, int f64, const IntegUpdate &up, const uint8_t *type,
                         float *vel, float *u, float *acc, const float *acc_h, const float *dudt,
                         const float *vsig, const void *h, int32_t *bin, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (f64)
    k_update<double><<<nblk(n), kIntBlock, 0, s>>>(n, up, type, vel, u, acc, acc_h, dudt, vsig,
                                                   (const double *)h, bin);
  else
    k_update<float><<<nblk(n), kIntBlock, 0, s>>>(n, up, type, vel, u, acc, acc_h, dudt, vsig,
                                                  (const float *)h, bin);
  return hipGetLastError();
}

hipError_t launch_store_count(const uint32_t *count, int64_t *out, hipStream_t s) {
  k_store_count<<<1, 64, 0, s>>>(count, out);
  return hipGetLastError();
}

}  // namespace g3
