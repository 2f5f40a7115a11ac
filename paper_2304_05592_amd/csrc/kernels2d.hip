// 2D time-step kernels for gfx950: forward, adjoint with imaging, Born.
//
// One workgroup (4 x wave64) updates one tile of TZ rows x 64 columns of one shot.  The
// tile of the field at the previous time level plus a 4-cell halo is staged in LDS
// ((TZ + 8) x 72 floats); each wave updates TZ/4 consecutive rows, one column per lane, so
// every global access is a 256-byte coalesced row segment.  Damping is evaluated from the
// grid indices (no array), the source is injected by the threads owning its nodes, the
// receivers whose base node lies in the tile are sampled from LDS, and the adjoint's
// receiver injection is gathered per touched point into LDS (no atomics, fixed order).
//
// Discretisation (row k of A u = s, see awe.h), written in increment form:
//   incr = coef * (L_h u^{k-1} + s^{k-1} - (eta/dt) (u^{k-1} - u^{k-2})),
//   u^k  = 2 u^{k-1} - u^{k-2} + incr,      coef = dt^2 / (m + eta dt / 2),
// with the Laplacian summed as sum_r c_r ((u_{+r} - u) + (u_{-r} - u)) so that a smooth
// field loses few digits to cancellation.  incr equals u^k - 2u^{k-1} + u^{k-2} exactly
// before rounding, which gives the imaging condition and the Born source without the
// cancellation of a second time difference.
#include "awe_internal.h"
#include "codec.h"

namespace awe {

namespace {

__device__ __forceinline__ int xcd_tile(int bid, int n) {
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a contiguous
  // range of tiles so that neighbouring tiles share its L2.
  const int q = n >> 3, r = n & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}

__device__ __forceinline__ int border_dist(int i, int n, int nbl) {
  return max(max(nbl - i, i - (n - 1 - nbl)), 0);
}

template <int TZ>
struct T2 {
  static constexpr int W = kTX + 2 * kHalo;  // 72
  static constexpr int H = TZ + 2 * kHalo;
  static constexpr int RPT = TZ / 4;         // rows per thread
};

template <int TZ>
__device__ __forceinline__ void load_tile(float (*L)[T2<TZ>::W], const float* __restrict__ f,
                                          int nx, int nz, int x0, int z0) {
  constexpr int W = T2<TZ>::W, H = T2<TZ>::H;
  for (int e = threadIdx.x; e < W * H; e += kThreads) {
    const int r = e / W, c = e - r * W;
    const int z = z0 - kHalo + r, x = x0 - kHalo + c;
    float v = 0.f;
    if ((unsigned)z < (unsigned)nz && (unsigned)x < (unsigned)nx) v = f[(long long)z * nx + x];
    L[r][c] = v;
  }
}

// Difference-form Laplacian at tile-local (row lr, column lc) (both without halo offset).
template <int TZ>
__device__ __forceinline__ float lap_at(const float (*L)[T2<TZ>::W], int lr, int lc,
                                        const float* c) {
  const int R = lr + kHalo, C = lc + kHalo;
  const float u = L[R][C];
  float s = 0.f;
#pragma unroll
  for (int r = kHalo; r >= 1; --r) {
    s += c[r] * ((L[R][C - r] - u) + (L[R][C + r] - u));
    s += c[r] * ((L[R - r][C] - u) + (L[R + r][C] - u));
  }
  return s;
}

template <int TZ>
__device__ __forceinline__ float interp_lds(const float (*L)[T2<TZ>::W], int i, int k, int x0,
                                            int z0, const float* w) {
  const int C = i - x0 + kHalo, R = k - z0 + kHalo;
  return w[0] * L[R][C] + w[1] * L[R][C + 1] + w[2] * L[R + 1][C] + w[3] * L[R + 1][C + 1];
}

__device__ __forceinline__ float* fbuf(unsigned char* ws, const ShotDev& S, int b) {
  return reinterpret_cast<float*>(ws + S.fld) + (long long)b * S.npts;
}

// ------------------------------------------------------------------------------ forward
// Produces u^k (k = step - off) for every shot in the tile list; samples d^{k-1}.
template <int TZ, int SK>
__global__ __launch_bounds__(kThreads) void fwd2d_kernel(StepArgs a) {
  constexpr int RPT = T2<TZ>::RPT;
  __shared__ float L[T2<TZ>::H][T2<TZ>::W];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  if (k < 1 || k >= S.nt) return;
  const int nx = S.nx, nz = S.nz;
  const float* __restrict__ u1 = fbuf(a.ws, S, (k - 1) & 1);
  float* __restrict__ u2 = fbuf(a.ws, S, k & 1);
  const float* __restrict__ cf = reinterpret_cast<const float*>(a.ws + S.coef);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = T.x0 + lane;

  float pu2[RPT], pcf[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int z = T.z0 + wv * RPT + i;
    const long long p = (long long)z * nx + x;
    const bool in = x < nx && z < nz;
    pu2[i] = in ? u2[p] : 0.f;
    pcf[i] = in ? cf[p] : 0.f;
  }
  load_tile<TZ>(L, u1, nx, nz, T.x0, T.z0);
  __syncthreads();

  if (a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += kThreads) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] = interp_lds<TZ>(L, R.i, R.k, T.x0, T.z0, R.w);
    }
  }

  const float qk = a.q[S.q + k - 1];
  const int dx = border_dist(x, nx, a.nbl);
  // 16-bit store: u^{k-1} (the centre values read here) is quantised with its finished scale
  float* scl = SK >= kStoreBF16 ? reinterpret_cast<float*>(a.ws + S.scale) : nullptr;
  unsigned short* st16 = SK >= kStoreBF16
      ? reinterpret_cast<unsigned short*>(a.ws + S.store) + (long long)(k - 1) * S.npts : nullptr;
  const float inv_prev = SK >= kStoreBF16 && k >= 2 ? inv_scale(level_scale(scl, k - 1)) : 0.f;
  float lmax = 0.f;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int lr = wv * RPT + i;
    const int z = T.z0 + lr;
    if (x >= nx || z >= nz) continue;
    const float u = L[lr + kHalo][lane + kHalo];
    float lap = lap_at<TZ>(L, lr, lane, a.c);
    const int bx = x - S.src_i, bz = z - S.src_k;
    if ((unsigned)bx < 2u && (unsigned)bz < 2u) lap += S.src_w[bx + 2 * bz] * qk;
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const float incr = pcf[i] * (lap - eta * (u - pu2[i]));
    const float un = (u + u - pu2[i]) + incr;
    const long long p = (long long)z * nx + x;
    u2[p] = un;
    if (SK == kStoreF32) reinterpret_cast<float*>(a.ws + S.store)[(long long)k * S.npts + p] = un;
    if (SK >= kStoreBF16) {
      lmax = fmaxf(lmax, fabsf(un));
      if (k >= 2) st16[p] = enc16(u * inv_prev, SK == kStoreBF16);
    }
  }
  if (SK >= kStoreBF16) block_max_to_slot(lmax, scl, k);
}

// ------------------------------------------------------------------------------ adjoint
// Produces w^j (j = step - off) from w^{j+1} (LDS) and w^{j+2}; injects P_r^T dd^j; samples
// v^j = R(x_s) w^{j+1} / h^ndim; IMG adds u^j * (w^j - 2w^{j+1} + w^{j+2}) into the FP64
// accumulator (u^j from the FULL store or from the recomputed forward buffers).
template <int TZ, int IMG>
__global__ __launch_bounds__(kThreads) void adj2d_kernel(StepArgs a) {
  constexpr int RPT = T2<TZ>::RPT;
  __shared__ float L[T2<TZ>::H][T2<TZ>::W];
  __shared__ float INJ[TZ][kTX];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int j = a.step - S.off;
  if (j < 1 || j >= S.nt) return;
  const int nx = S.nx, nz = S.nz;
  const float* __restrict__ w1 = fbuf(a.ws, S, 2 + ((j + 1) & 1));
  float* __restrict__ w2 = fbuf(a.ws, S, 2 + (j & 1));
  const float* __restrict__ cf = reinterpret_cast<const float*>(a.ws + S.coef);
  const float* __restrict__ uj = nullptr;
  const unsigned short* __restrict__ uj16 = nullptr;
  float usc = 1.f;
  if (IMG == kImgFull32) uj = reinterpret_cast<const float*>(a.ws + S.store) + (long long)j * S.npts;
  if (IMG == kImgBuffers) uj = fbuf(a.ws, S, j & 1);
  if (IMG >= kImgFullBF16) {
    uj16 = reinterpret_cast<const unsigned short*>(a.ws + S.store) + (long long)j * S.npts;
    usc = level_scale(reinterpret_cast<const float*>(a.ws + S.scale), j);
  }
  double* __restrict__ acc = IMG ? reinterpret_cast<double*>(a.ws + S.acc) : nullptr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = T.x0 + lane;
  const bool has_inj = T.inj_count > 0 && a.dd != nullptr;  // no residual: nothing to inject

  float pw2[RPT], pcf[RPT], pu[RPT];
  double pacc[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int z = T.z0 + wv * RPT + i;
    const long long p = (long long)z * nx + x;
    const bool in = x < nx && z < nz;
    pw2[i] = in ? w2[p] : 0.f;
    pcf[i] = in ? cf[p] : 0.f;
    if (IMG) {
      if (IMG >= kImgFullBF16) pu[i] = in ? dec16(uj16[p], IMG == kImgFullBF16) * usc : 0.f;
      else pu[i] = in ? uj[p] : 0.f;
      pacc[i] = in ? acc[p] : 0.0;
    }
    if (has_inj) INJ[wv * RPT + i][lane] = 0.f;
  }
  load_tile<TZ>(L, w1, nx, nz, T.x0, T.z0);
  __syncthreads();

  if (has_inj) {
    const float* ddj = a.dd + S.d + (long long)j * S.nrec;
    for (int t = threadIdx.x; t < T.inj_count; t += kThreads) {
      const InjPoint P = a.t.inj_pts[T.inj_begin + t];
      float s = 0.f;
      for (int e = 0; e < P.e_count; ++e) {
        const InjEntry E = a.t.inj_ent[P.e_begin + e];
        s += E.w * ddj[E.r];
      }
      INJ[P.lz][P.lx] = s;
    }
    __syncthreads();
  }
  if (a.v != nullptr && tid == S.src_tile && threadIdx.x == 0)
    a.v[S.q + j] = interp_lds<TZ>(L, S.src_i, S.src_k, T.x0, T.z0, S.src_w);

  const int dx = border_dist(x, nx, a.nbl);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int lr = wv * RPT + i;
    const int z = T.z0 + lr;
    if (x >= nx || z >= nz) continue;
    const float w = L[lr + kHalo][lane + kHalo];
    float lap = lap_at<TZ>(L, lr, lane, a.c);
    if (has_inj) lap += INJ[lr][lane];
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const float incr = pcf[i] * (lap - eta * (w - pw2[i]));
    const long long p = (long long)z * nx + x;
    w2[p] = (w + w - pw2[i]) + incr;
    if (IMG) acc[p] = pacc[i] + (double)pu[i] * (double)incr;
  }
}

// ------------------------------------------------------------------------------ Born
// Produces u^k and du^k together; samples (J dm)^{k-1} = R du^{k-1}.
template <int TZ>
__global__ __launch_bounds__(kThreads) void born2d_kernel(StepArgs a) {
  constexpr int RPT = T2<TZ>::RPT;
  __shared__ float LU[T2<TZ>::H][T2<TZ>::W];
  __shared__ float LD[T2<TZ>::H][T2<TZ>::W];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  if (k < 1 || k >= S.nt) return;
  const int nx = S.nx, nz = S.nz;
  const float* __restrict__ u1 = fbuf(a.ws, S, (k - 1) & 1);
  float* __restrict__ u2 = fbuf(a.ws, S, k & 1);
  const float* __restrict__ d1 = fbuf(a.ws, S, 2 + ((k - 1) & 1));
  float* __restrict__ d2 = fbuf(a.ws, S, 2 + (k & 1));
  const float* __restrict__ cf = reinterpret_cast<const float*>(a.ws + S.coef);
  const float* __restrict__ dm = a.dm + S.m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = T.x0 + lane;

  float pu2[RPT], pd2[RPT], pcf[RPT], pdm[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int z = T.z0 + wv * RPT + i;
    const long long p = (long long)z * nx + x;
    const bool in = x < nx && z < nz;
    pu2[i] = in ? u2[p] : 0.f;
    pd2[i] = in ? d2[p] : 0.f;
    pcf[i] = in ? cf[p] : 0.f;
    pdm[i] = in ? dm[p] : 0.f;
  }
  load_tile<TZ>(LU, u1, nx, nz, T.x0, T.z0);
  load_tile<TZ>(LD, d1, nx, nz, T.x0, T.z0);
  __syncthreads();

  if (a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += kThreads) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] = interp_lds<TZ>(LD, R.i, R.k, T.x0, T.z0, R.w);
    }
  }

  const float qk = a.q[S.q + k - 1];
  const int dx = border_dist(x, nx, a.nbl);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int lr = wv * RPT + i;
    const int z = T.z0 + lr;
    if (x >= nx || z >= nz) continue;
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const long long p = (long long)z * nx + x;
    // background field
    const float u = LU[lr + kHalo][lane + kHalo];
    float lap = lap_at<TZ>(LU, lr, lane, a.c);
    const int bx = x - S.src_i, bz = z - S.src_k;
    if ((unsigned)bx < 2u && (unsigned)bz < 2u) lap += S.src_w[bx + 2 * bz] * qk;
    const float incr = pcf[i] * (lap - eta * (u - pu2[i]));
    u2[p] = (u + u - pu2[i]) + incr;
    // scattered field, source -dm (u^k - 2u^{k-1} + u^{k-2}) / dt^2 = -dm incr / dt^2
    const float du = LD[lr + kHalo][lane + kHalo];
    const float lapd = lap_at<TZ>(LD, lr, lane, a.c) - pdm[i] * incr * a.inv_dt2;
    const float incd = pcf[i] * (lapd - eta * (du - pd2[i]));
    d2[p] = (du + du - pd2[i]) + incd;
  }
}

template <int TZ>
hipError_t fwd2d_tz(const StepArgs& a, int store, hipStream_t s) {
  switch (store) {
    case kStoreNone: fwd2d_kernel<TZ, kStoreNone><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case kStoreF32: fwd2d_kernel<TZ, kStoreF32><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case kStoreBF16: fwd2d_kernel<TZ, kStoreBF16><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case kStoreFP16: fwd2d_kernel<TZ, kStoreFP16><<<a.ntiles, kThreads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TZ>
hipError_t adj2d_tz(const StepArgs& a, hipStream_t s) {
  switch (a.image_src) {
    case kImgNone: adj2d_kernel<TZ, kImgNone><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case kImgFull32: adj2d_kernel<TZ, kImgFull32><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case kImgBuffers: adj2d_kernel<TZ, kImgBuffers><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case kImgFullBF16: adj2d_kernel<TZ, kImgFullBF16><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case kImgFullFP16: adj2d_kernel<TZ, kImgFullFP16><<<a.ntiles, kThreads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fwd2d(const StepArgs& a, int tz, int store, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: return fwd2d_tz<8>(a, store, s);
    case 16: return fwd2d_tz<16>(a, store, s);
    case 32: return fwd2d_tz<32>(a, store, s);
    case 64: return fwd2d_tz<64>(a, store, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj2d(const StepArgs& a, int tz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: return adj2d_tz<8>(a, s);
    case 16: return adj2d_tz<16>(a, s);
    case 32: return adj2d_tz<32>(a, s);
    case 64: return adj2d_tz<64>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_born2d(const StepArgs& a, int tz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: born2d_kernel<8><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case 16: born2d_kernel<16><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case 32: born2d_kernel<32><<<a.ntiles, kThreads, 0, s>>>(a); break;
    case 64: born2d_kernel<64><<<a.ntiles, kThreads, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace awe
