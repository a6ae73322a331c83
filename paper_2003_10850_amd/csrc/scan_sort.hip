// Device-wide exclusive scan and stable LSD radix sort of (u64 key, u32 value)
// pairs: the primitives of the octree build and the active-set compaction.
#include "g3_device.h"
#include "g3_internal.h"

namespace g3 {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanIpt = 8;
constexpr int kScanTile = kScanBlock * kScanIpt;

template <typename T>
__device__ T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, (unsigned)d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive block scan of one value per thread; *total receives the sum.
template <typename T>
__device__ T block_excl_scan(T v, T *total, T *lds /* [kScanBlock/64 + 1] */) {
  const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
  constexpr int kW = kScanBlock / kWave;
  T inc = wave_incl_scan(v);
  if (lane == kWave - 1) lds[w] = inc;
  __syncthreads();
  if (w == 0) {
    T t = lane < kW ? lds[lane] : T(0);
    T ti = wave_incl_scan(t);
    if (lane < kW) lds[lane] = ti - t;
    if (lane == kW - 1) lds[kW] = ti;
  }
  __syncthreads();
  const T res = lds[w] + inc - v;
  *total = lds[kW];
  __syncthreads();
  return res;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const TI *__restrict__ in,
                                                            int64_t n, TO *__restrict__ part) {
  __shared__ TO lds[kScanBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIpt;
  TO s = 0;
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k)
    if (base + k < n) s += (TO)in[base + k];
  TO tot;
  block_excl_scan<TO>(s, &tot, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Scans in[0..n) into out[0..n]; out may alias in (each thread reads its
// items before writing them). part: exclusive per-block offsets or null.
template <typename TI, typename TO>
__global__ __launch_bounds__(kScanBlock) void k_scan_down(const TI *in, int64_t n, TO *out,
                                                          const TO *__restrict__ part) {
  __shared__ TO lds[kScanBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIpt;
  TO v[kScanIpt];
  TO s = 0;
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) {
    v[k] = (base + k < n) ? (TO)in[base + k] : TO(0);
    s += v[k];
  }
  TO tot;
  TO run = block_excl_scan<TO>(s, &tot, lds);
  if (part) run += part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) {
    if (base + k <= n) out[base + k] = run;
    run += v[k];
  }
}

template <typename TI, typename TO>
hipError_t scan_impl(const TI *in, TO *out, int64_t n, TO *tmp, hipStream_t s) {
  const int64_t nb = (n + 1 + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    k_scan_down<TI, TO><<<1, kScanBlock, 0, s>>>(in, n, out, nullptr);
    return hipGetLastError();
  }
  k_scan_reduce<TI, TO><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, tmp);
  hipError_t e = scan_impl<TO, TO>(tmp, tmp, nb, tmp + nb + 1, s);
  if (e != hipSuccess) return e;
  k_scan_down<TI, TO><<<(unsigned)nb, kScanBlock, 0, s>>>(in, n, out, tmp);
  return hipGetLastError();
}

// ------------------------------------------------------------ radix sort

constexpr int kRsBlock = 256;
constexpr int kRsWaves = kRsBlock / kWave;
constexpr int kRsChunks = 8;  // 64-item chunks per wave
constexpr int kRsTile = kRsBlock * kRsChunks;
constexpr int kRsBits = 8;
constexpr int kRsBins = 1 << kRsBits;

__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const uint64_t *__restrict__ keys,
                                                      int64_t n, int shift,
                                                      uint32_t *__restrict__ hist, int nb) {
  __shared__ uint32_t cnt[kRsBins];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int k = threadIdx.x; k < kRsTile; k += kRsBlock) {
    const int64_t i = base + k;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kRsBins - 1)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: wave w ranks its 512 items chunk by chunk (lanes with equal
// digits found by eight ballots), waves are ordered by a per-digit prefix.
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ offs, int nb) {
  __shared__ uint32_t cnt[kRsWaves][kRsBins];
  __shared__ uint32_t base[kRsBins];
  const int w = (int)(threadIdx.x >> 6), lane = lane_id();
  for (int i = threadIdx.x; i < kRsWaves * kRsBins; i += kRsBlock) (&cnt[0][0])[i] = 0;
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kRsTile + (int64_t)w * (kWave * kRsChunks);
  uint64_t key[kRsChunks];
  uint32_t val[kRsChunks], rank[kRsChunks];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int c = 0; c < kRsChunks; ++c) {
    const int64_t i = t0 + (int64_t)c * kWave + lane;
    const bool valid = i < n;
    key[c] = valid ? kin[i] : 0ull;
    val[c] = valid ? vin[i] : 0u;
    const uint32_t d = (uint32_t)(key[c] >> shift) & (kRsBins - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRsBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt);
    const uint32_t prev = cnt[w][d];
    rank[c] = prev + below;
    wave_sync();
    if (valid && below == 0) cnt[w][d] = prev + (uint32_t)__popcll(peers);
    wave_sync();
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < kRsWaves; ++ww) {
      const uint32_t t = cnt[ww][d];
      cnt[ww][d] = run;
      run += t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kRsChunks; ++c) {
    const int64_t i = t0 + (int64_t)c * kWave + lane;
    if (i < n) {
      const uint32_t d = (uint32_t)(key[c] >> shift) & (kRsBins - 1);
      const uint32_t pos = base[d] + cnt[w][d] + rank[c];
      kout[pos] = key[c];
      vout[pos] = val[c];
    }
  }
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) {
  int64_t total = 0;
  int64_t m = n;
  for (;;) {
    const int64_t nb = (m + 1 + kScanTile - 1) / kScanTile;
    if (nb == 1) break;
    total += nb + 1;
    m = nb;
  }
  return total + 1;
}

hipError_t scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp,
                    hipStream_t s) {
  return scan_impl<uint32_t, uint32_t>(in, out, n, tmp, s);
}

hipError_t scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *tmp,
                           hipStream_t s) {
  return scan_impl<int32_t, int64_t>(in, out, n, tmp, s);
}

size_t radix_tmp_bytes(int64_t n) {
  const int64_t nb = (n + kRsTile - 1) / kRsTile;
  const int64_t h = nb * kRsBins;
  return (size_t)(2 * (h + 1) + scan_tmp_elems(h)) * sizeof(uint32_t);
}

hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt,
                            uint32_t *vals_alt, int64_t n, int bits, void *tmp, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  const int64_t nb = (n + kRsTile - 1) / kRsTile;
  const int64_t h = nb * kRsBins;
  uint32_t *hist = (uint32_t *)tmp;
  uint32_t *offs = hist + h + 1;
  uint32_t *stmp = offs + h + 1;
  uint64_t *ka = keys, *kb = keys_alt;
  uint32_t *va = vals, *vb = vals_alt;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += kRsBits, ++passes) {
    k_rs_hist<<<(unsigned)nb, kRsBlock, 0, s>>>(ka, n, shift, hist, (int)nb);
    hipError_t e = scan_u32(hist, offs, h, stmp, s);
    if (e != hipSuccess) return e;
    k_rs_scatter<<<(unsigned)nb, kRsBlock, 0, s>>>(ka, va, kb, vb, n, shift, offs, (int)nb);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (passes & 1) {  // the result is in the alternate buffers: copy it back
    hipError_t e = hipMemcpyAsync(keys, keys_alt, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(vals, vals_alt, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

}  // namespace g3
