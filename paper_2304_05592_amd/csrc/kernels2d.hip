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
  static constexpr int NW = TZ >= 32 ? 8 : 4;  // waves per workgroup
  static constexpr int NT = 64 * NW;           // threads per workgroup
  static constexpr int RPT = TZ / NW;          // rows per thread
  static_assert(TZ % NW == 0, "tile rows must split evenly over the waves");
};

// Stage rows z0-4 .. z0+TZ+3 of a field, columns x0-4 .. x0+67, zero outside the grid.  The
// 64-column body of each row is one coalesced row segment per wave (aligned: the row pitch and
// x0 are multiples of 64); the 4 + 4 halo columns of every row follow as one short pass.
// Loads read clamped, always valid addresses (rows past the grid read its last row, columns
// the padded row) and the value is zeroed where the point lies outside: no load sits on a
// branch, so all of a thread's loads are issued before the first wait.
__device__ __forceinline__ long long cidx2(int x, int z, int nz, int px) {
  const int xc = min(max(x, 0), px - 1), zc = min(max(z, 0), nz - 1);
  return (long long)zc * px + xc;
}

// Tile of f (rows z0-4 .. z0+TZ+3, columns x0-4 .. x0+67) into LDS; rows z >= nzv (or < 0)
// and columns outside [0, nx) read as 0.  nzv <= nz: 0 for a level that is zero by definition.
template <int TZ>
__device__ __forceinline__ void load_tile(float (*L)[T2<TZ>::W], const float* __restrict__ f,
                                          int nx, int nzv, int nz, int px, int x0, int z0) {
  constexpr int H = T2<TZ>::H, NW = T2<TZ>::NW, NT = T2<TZ>::NT;
  constexpr int NB = (H + NW - 1) / NW;                      // body rows per thread
  constexpr int NE = H * 2 * kHalo, NH = (NE + NT - 1) / NT; // side-halo cells per thread
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = x0 + lane;
  float vb[NB], vh[NH];
#pragma unroll
  for (int i = 0; i < NB; ++i) vb[i] = f[cidx2(x, z0 - kHalo + wv + i * NW, nz, px)];
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int e = min((int)threadIdx.x + i * NT, NE - 1);
    const int r = e / (2 * kHalo), c8 = e - r * (2 * kHalo);
    const int c = c8 < kHalo ? c8 : kTX + c8;
    vh[i] = f[cidx2(x0 - kHalo + c, z0 - kHalo + r, nz, px)];
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int r = wv + i * NW;
    const int z = z0 - kHalo + r;
    if (r < H) L[r][lane + kHalo] = (x < nx && (unsigned)z < (unsigned)nzv) ? vb[i] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (e < NE) {
      const int r = e / (2 * kHalo), c8 = e - r * (2 * kHalo);
      const int c = c8 < kHalo ? c8 : kTX + c8;
      const int z = z0 - kHalo + r, xx = x0 - kHalo + c;
      L[r][c] = ((unsigned)z < (unsigned)nzv && (unsigned)xx < (unsigned)nx) ? vh[i] : 0.f;
    }
  }
}

// Difference-form Laplacian at *p in an LDS array with row stride `stride` (x neighbours at
// +-1, z neighbours at +-stride); the order of the sum is fixed for every 2D kernel.
__device__ __forceinline__ float lap_ptr(const float* p, int stride, const float* c) {
  const float u = p[0];
  float s = 0.f;
#pragma unroll
  for (int r = kHalo; r >= 1; --r) {
    s += c[r] * ((p[-r] - u) + (p[r] - u));
    s += c[r] * ((p[-r * stride] - u) + (p[r * stride] - u));
  }
  return s;
}

// Increment coef (L u + s - (eta/dt)(u - u_prev)) of one update; the new level is
// (u + u - u_prev) + increment.
__device__ __forceinline__ float step_incr(float u, float um2, float cfv, float lap, float eta) {
  return cfv * (lap - eta * (u - um2));
}

template <int TZ>
__device__ __forceinline__ float lap_at(const float (*L)[T2<TZ>::W], int lr, int lc,
                                        const float* c) {
  return lap_ptr(&L[lr + kHalo][lc + kHalo], T2<TZ>::W, c);
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
__global__ __launch_bounds__(T2<TZ>::NT) void fwd2d_kernel(StepArgs a) {
  constexpr int RPT = T2<TZ>::RPT;
  __shared__ float L[T2<TZ>::H][T2<TZ>::W];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  if (k < 1 || k >= S.nt) return;
  const int nx = S.nx, nz = S.nz, px = S.px;
  const float* __restrict__ u1 = fwd_level(a, S, k - 1);
  const float* __restrict__ u2 = fwd_level(a, S, k - 2);
  float* __restrict__ out = fbuf(a.ws, S, fwd_buf(k));
  const float* __restrict__ cf = reinterpret_cast<const float*>(a.ws + S.coef);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = T.x0 + lane;

  float pu2[RPT], pcf[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int z = T.z0 + wv * RPT + i;
    const long long p = cidx2(x, z, nz, px);
    const bool in = x < nx && z < nz;
    const float v2 = u2[p], vc = cf[p];
    pu2[i] = in && k >= 3 ? v2 : 0.f;
    pcf[i] = in ? vc : 0.f;
  }
  // levels below 1 are zero (initial state); their buffers may hold older levels after a
  // checkpoint restore of a state before this shot's start, so their values are not used
  load_tile<TZ>(L, u1, nx, k >= 2 ? nz : 0, nz, px, T.x0, T.z0);
  __syncthreads();

  if (a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += T2<TZ>::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] = interp_lds<TZ>(L, R.i, R.k, T.x0, T.z0, R.w);
    }
  }

  const float qk = a.q[S.q + k - 1];
  const int dx = border_dist(x, nx, a.nbl);
  // shot fields used in the row loop, in registers: a reload after a store through `out` would
  // wait for every store in flight
  const int src_i = S.src_i, src_k = S.src_k;
  const float sw0 = S.src_w[0], sw1 = S.src_w[1], sw2 = S.src_w[2], sw3 = S.src_w[3];
  float* st32 = SK == kStoreF32 ? reinterpret_cast<float*>(a.ws + S.store) + (long long)k * S.npts : nullptr;
  float* sl = SK == kStoreNone && a.st_slot >= 0
      ? reinterpret_cast<float*>(a.ws + S.store) + (long long)a.st_slot * 2 * S.npts : nullptr;
  const long long npts = S.npts;
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
    const int bx = x - src_i, bz = z - src_k;
    if ((unsigned)bx < 2u && (unsigned)bz < 2u) {
      const int w = bx + 2 * bz;
      lap += (w == 0 ? sw0 : w == 1 ? sw1 : w == 2 ? sw2 : sw3) * qk;
    }
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const float incr = step_incr(u, pu2[i], pcf[i], lap, eta);
    const float un = (u + u - pu2[i]) + incr;
    const long long p = (long long)z * px + x;
    out[p] = un;
    if (SK == kStoreNone && sl != nullptr) {
      // checkpoint store fused into the step that reaches the stored state
      sl[p] = un;
      sl[npts + p] = u;
    }
    if (SK == kStoreF32) __builtin_nontemporal_store(un, st32 + p);
    if (SK >= kStoreBF16) {
      lmax = fmaxf(lmax, fabsf(un));
      if (k >= 2) __builtin_nontemporal_store(enc16(u * inv_prev, SK == kStoreBF16), st16 + p);
    }
  }
  if (SK >= kStoreBF16) block_max_to_slot(lmax, scl, k);
}

// ------------------------------------------------------------------------------ adjoint
// Produces w^j (j = step - off) from w^{j+1} (LDS) and w^{j+2}; injects P_r^T dd^j; samples
// v^j = R(x_s) w^{j+1} / h^ndim; IMG adds u^j * (w^j - 2w^{j+1} + w^{j+2}) into the FP64
// accumulator (u^j from the FULL store or from the recomputed forward buffers).
template <int TZ, int IMG>
__global__ __launch_bounds__(T2<TZ>::NT) void adj2d_kernel(StepArgs a) {
  constexpr int RPT = T2<TZ>::RPT;
  __shared__ float L[T2<TZ>::H][T2<TZ>::W];
  __shared__ float INJ[TZ][kTX];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int j = a.step - S.off;
  if (j < 1 || j >= S.nt) return;
  const int nx = S.nx, nz = S.nz, px = S.px;
  const float* __restrict__ w1 = fbuf(a.ws, S, adj_buf(j + 1));
  const float* __restrict__ w2 = fbuf(a.ws, S, adj_buf(j + 2));
  float* __restrict__ out = fbuf(a.ws, S, adj_buf(j));
  const float* __restrict__ cf = reinterpret_cast<const float*>(a.ws + S.coef);
  const float* __restrict__ uj = nullptr;
  const unsigned short* __restrict__ uj16 = nullptr;
  float usc = 1.f;
  if (IMG == kImgFull32) uj = reinterpret_cast<const float*>(a.ws + S.store) + (long long)j * S.npts;
  if (IMG == kImgBuffers) uj = fwd_level(a, S, j);
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
    const long long p = cidx2(x, z, nz, px);
    const bool in = x < nx && z < nz;
    const float v2 = w2[p], vc = cf[p];
    pw2[i] = in ? v2 : 0.f;
    pcf[i] = in ? vc : 0.f;
    if (IMG) {
      float vu;
      if (IMG >= kImgFullBF16) vu = dec16(__builtin_nontemporal_load(uj16 + p), IMG == kImgFullBF16) * usc;
      else if (IMG == kImgFull32) vu = __builtin_nontemporal_load(uj + p);
      else vu = uj[p];
      const double va = acc[p];
      pu[i] = in ? vu : 0.f;
      pacc[i] = in ? va : 0.0;
    }
    if (has_inj) INJ[wv * RPT + i][lane] = 0.f;
  }
  load_tile<TZ>(L, w1, nx, nz, nz, px, T.x0, T.z0);
  __syncthreads();

  if (has_inj) {
    const float* ddj = a.dd + S.d + (long long)j * S.nrec;
    for (int t = threadIdx.x; t < T.inj_count; t += T2<TZ>::NT) {
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
  if (a.v != nullptr && a.tile_base + tid == S.src_tile && threadIdx.x == 0)
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
    const float incr = step_incr(w, pw2[i], pcf[i], lap, eta);
    const long long p = (long long)z * px + x;
    out[p] = (w + w - pw2[i]) + incr;
    if (IMG) acc[p] = pacc[i] + (double)pu[i] * (double)incr;
  }
}

// ------------------------------------------------------------------------------ Born
// Produces u^k and du^k together; samples (J dm)^{k-1} = R du^{k-1}.
template <int TZ>
__global__ __launch_bounds__(T2<TZ>::NT) void born2d_kernel(StepArgs a) {
  constexpr int RPT = T2<TZ>::RPT;
  __shared__ float LU[T2<TZ>::H][T2<TZ>::W];
  __shared__ float LD[T2<TZ>::H][T2<TZ>::W];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  if (k < 1 || k >= S.nt) return;
  const int nx = S.nx, nz = S.nz, px = S.px;
  const float* __restrict__ u1 = fbuf(a.ws, S, fwd_buf(k - 1));
  const float* __restrict__ u2 = fbuf(a.ws, S, fwd_buf(k - 2));
  float* __restrict__ uout = fbuf(a.ws, S, fwd_buf(k));
  const float* __restrict__ d1 = fbuf(a.ws, S, adj_buf(k - 1));
  const float* __restrict__ d2 = fbuf(a.ws, S, adj_buf(k - 2));
  float* __restrict__ dout = fbuf(a.ws, S, adj_buf(k));
  const float* __restrict__ cf = reinterpret_cast<const float*>(a.ws + S.coef);
  const float* __restrict__ dm = a.dm + S.m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = T.x0 + lane;

  float pu2[RPT], pd2[RPT], pcf[RPT], pdm[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int z = T.z0 + wv * RPT + i;
    const long long p = cidx2(x, z, nz, px);
    const bool in = x < nx && z < nz;
    const float v2 = u2[p], vd = d2[p], vc = cf[p], vm = dm[cidx2(x, z, nz, nx)];
    pu2[i] = in ? v2 : 0.f;
    pd2[i] = in ? vd : 0.f;
    pcf[i] = in ? vc : 0.f;
    pdm[i] = in ? vm : 0.f;
  }
  load_tile<TZ>(LU, u1, nx, nz, nz, px, T.x0, T.z0);
  load_tile<TZ>(LD, d1, nx, nz, nz, px, T.x0, T.z0);
  __syncthreads();

  if (a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += T2<TZ>::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] = interp_lds<TZ>(LD, R.i, R.k, T.x0, T.z0, R.w);
    }
  }

  const int src_i = S.src_i, src_k = S.src_k;   // in registers (see the forward kernel)
  const float sw0 = S.src_w[0], sw1 = S.src_w[1], sw2 = S.src_w[2], sw3 = S.src_w[3];
  const float qk = a.q[S.q + k - 1];
  const int dx = border_dist(x, nx, a.nbl);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int lr = wv * RPT + i;
    const int z = T.z0 + lr;
    if (x >= nx || z >= nz) continue;
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const long long p = (long long)z * px + x;
    // background field
    const float u = LU[lr + kHalo][lane + kHalo];
    float lap = lap_at<TZ>(LU, lr, lane, a.c);
    const int bx = x - src_i, bz = z - src_k;
    if ((unsigned)bx < 2u && (unsigned)bz < 2u) {
      const int w = bx + 2 * bz;
      lap += (w == 0 ? sw0 : w == 1 ? sw1 : w == 2 ? sw2 : sw3) * qk;
    }
    const float incr = pcf[i] * (lap - eta * (u - pu2[i]));
    uout[p] = (u + u - pu2[i]) + incr;
    // scattered field, source -dm (u^k - 2u^{k-1} + u^{k-2}) / dt^2 = -dm incr / dt^2
    const float du = LD[lr + kHalo][lane + kHalo];
    const float lapd = lap_at<TZ>(LD, lr, lane, a.c) - pdm[i] * incr * a.inv_dt2;
    const float incd = pcf[i] * (lapd - eta * (du - pd2[i]));
    dout[p] = (du + du - pd2[i]) + incd;
  }
}

// ------------------------------------------------------------------------------ two steps per launch
// Level n-1 is staged with an 8-cell halo (LDS L1); the first step computes level n on the
// tile plus a 4-cell halo (LDS LE: everything the second step's stencil needs), the second
// step computes level n+1 (forward) or n-1 (adjoint) on the tile.  Both steps do exactly the
// arithmetic of the one-step kernels, in the same order, so results are bitwise identical;
// HBM traffic per two steps falls from 2 x (3 reads + 1 write) to 3 reads + 2 writes.
template <int TZ>
struct F2 {
  static constexpr int W1 = kTX + 4 * kHalo;      // 80: level n-1 with an 8-cell halo
  static constexpr int H1 = TZ + 4 * kHalo;
  static constexpr int WE = kTX + 2 * kHalo;      // 72: first-step level on tile + 4
  static constexpr int HE = TZ + 2 * kHalo;
  static constexpr int NW = TZ >= 16 ? 8 : 4;    // waves per workgroup
  static constexpr int NT = 64 * NW;
  static constexpr int RPT = TZ / NW;                // tile rows per thread
  static_assert(TZ % NW == 0, "tile rows must split evenly over the waves");
  // first-step points of a thread: NB in the 64 body columns (one wave per row, aligned
  // 256-byte rows), NH in the 4 + 4 side columns of every row
  static constexpr int NB = (HE + NW - 1) / NW;
  static constexpr int NH = (2 * kHalo * HE + NT - 1) / NT;
  static constexpr int NS = NB + NH;
};

// Slot i of this thread among the first-step points (row r, column c of the WE x HE region);
// false for an unused slot (its r, c are then a valid point, not to be written).
template <int TZ>
__device__ __forceinline__ bool ext_slot(int i, int* r, int* c) {
  using G = F2<TZ>;
  if (i < G::NB) {
    *r = (int)(threadIdx.x >> 6) + i * G::NW;
    *c = kHalo + (int)(threadIdx.x & 63);
    return *r < G::HE;
  }
  const int e0 = (int)threadIdx.x + (i - G::NB) * G::NT;
  const int e = min(e0, 2 * kHalo * G::HE - 1);
  *r = e / (2 * kHalo);
  const int cc = e - *r * (2 * kHalo);
  *c = cc < kHalo ? cc : kTX + cc;
  return e0 < 2 * kHalo * G::HE;
}

// Level n-1 with an 8-cell halo into LDS: all loads first (clamped addresses, as load_tile),
// then the LDS writes; rows z >= nzv read as 0.
template <int TZ>
__device__ __forceinline__ void load_tile8(float (*L)[F2<TZ>::W1], const float* __restrict__ f,
                                           int nx, int nzv, int nz, int px, int x0, int z0) {
  // body: the tile's 64 columns of every row, one aligned 256-byte load per wave and row;
  // halo: the 8 + 8 side columns of every row
  constexpr int H = F2<TZ>::H1, NW = F2<TZ>::NW, NT = F2<TZ>::NT, HW = 4 * kHalo;  // 16 side cells
  constexpr int NB = (H + NW - 1) / NW, NE = HW * H, NH = (NE + NT - 1) / NT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = x0 + lane;
  float vb[NB], vh[NH];
#pragma unroll
  for (int i = 0; i < NB; ++i) vb[i] = f[cidx2(x, z0 - 2 * kHalo + wv + i * NW, nz, px)];
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int e = min((int)threadIdx.x + i * NT, NE - 1);
    const int r = e / HW, cc = e - r * HW;
    const int c = cc < 2 * kHalo ? cc : kTX + cc;           // columns 0..7 and 72..79
    vh[i] = f[cidx2(x0 - 2 * kHalo + c, z0 - 2 * kHalo + r, nz, px)];
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int r = wv + i * NW;
    const int z = z0 - 2 * kHalo + r;
    if (r < H) L[r][lane + 2 * kHalo] = (x < nx && (unsigned)z < (unsigned)nzv) ? vb[i] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int e = (int)threadIdx.x + i * NT;
    if (e < NE) {
      const int r = e / HW, cc = e - r * HW;
      const int c = cc < 2 * kHalo ? cc : kTX + cc;
      const int z = z0 - 2 * kHalo + r, xx = x0 - 2 * kHalo + c;
      L[r][c] = ((unsigned)z < (unsigned)nzv && (unsigned)xx < (unsigned)nx) ? vh[i] : 0.f;
    }
  }
}

// Forward: levels k and k+1 (k = step - off); SK = kStoreNone or kStoreF32.
template <int TZ, int SK>
__global__ __launch_bounds__(F2<TZ>::NT) void fwd2d2_kernel(StepArgs a) {
  using G = F2<TZ>;
  __shared__ float L1[G::H1][G::W1];
  __shared__ float LE[G::HE][G::WE];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  const bool act1 = k >= 1 && k <= S.nt - 1;
  const bool act2 = k + 1 >= 1 && k + 1 <= S.nt - 1;
  if (!act1 && !act2) return;
  const int nx = S.nx, nz = S.nz, px = S.px;
  const float* __restrict__ u1 = fbuf(a.ws, S, fwd_buf(k - 1));
  const float* __restrict__ u2 = fbuf(a.ws, S, fwd_buf(k - 2));
  float* __restrict__ o1 = fbuf(a.ws, S, fwd_buf(k));
  float* __restrict__ o2 = fbuf(a.ws, S, fwd_buf(k + 1));
  const float* __restrict__ cf = reinterpret_cast<const float*>(a.ws + S.coef);
  float* st = SK == kStoreF32 ? reinterpret_cast<float*>(a.ws + S.store) : nullptr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  // prefetch level k-2 and coef of this thread's extended points, coef of its tile points
  float pm2[G::NS], pcf[G::NS], tcf[G::RPT];
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    int r, c;
    const bool ok = ext_slot<TZ>(i, &r, &c);
    const int z = T.z0 - kHalo + r, x = T.x0 - kHalo + c;
    const bool in = ok && (unsigned)z < (unsigned)nz && (unsigned)x < (unsigned)nx;
    const long long p = cidx2(x, z, nz, px);
    const float v2 = u2[p], vc = cf[p];
    pm2[i] = in && k >= 3 ? v2 : 0.f;  // levels below 1 are zero (see fwd2d_kernel)
    pcf[i] = in ? vc : 0.f;
  }
  {
    const int x = T.x0 + lane;
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int z = T.z0 + wv * G::RPT + i;
      const float vc = cf[cidx2(x, z, nz, px)];
      tcf[i] = x < nx && z < nz ? vc : 0.f;
    }
  }
  load_tile8<TZ>(L1, u1, nx, k >= 2 ? nz : 0, nz, px, T.x0, T.z0);
  __syncthreads();

  if (act1 && a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += G::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      const int C = R.i - T.x0 + 2 * kHalo, Rw = R.k - T.z0 + 2 * kHalo;
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] =
          R.w[0] * L1[Rw][C] + R.w[1] * L1[Rw][C + 1] + R.w[2] * L1[Rw + 1][C] + R.w[3] * L1[Rw + 1][C + 1];
    }
  }
  // shot fields used after stores, in registers (see fwd2d_kernel)
  const int src_i = S.src_i, src_k = S.src_k;
  const float sw0 = S.src_w[0], sw1 = S.src_w[1], sw2 = S.src_w[2], sw3 = S.src_w[3];
  auto src_weight = [&](int w) { return w == 0 ? sw0 : w == 1 ? sw1 : w == 2 ? sw2 : sw3; };
  const long long npts = S.npts;
  // first step: level k on the tile + 4-cell halo (zero outside the grid)
  const float q1 = act1 ? a.q[S.q + k - 1] : 0.f;
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    int r, c;
    if (!ext_slot<TZ>(i, &r, &c)) continue;
    const int z = T.z0 - kHalo + r, x = T.x0 - kHalo + c;
    float v = 0.f;
    if ((unsigned)z < (unsigned)nz && (unsigned)x < (unsigned)nx) {
      const float* pc = &L1[r + kHalo][c + kHalo];
      const float u = pc[0];
      float lap = lap_ptr(pc, G::W1, a.c);
      const int bx = x - src_i, bz = z - src_k;
      if (act1 && (unsigned)bx < 2u && (unsigned)bz < 2u) lap += src_weight(bx + 2 * bz) * q1;
      const int dx = border_dist(x, nx, a.nbl), dz = border_dist(z, nz, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
      const float incr = step_incr(u, pm2[i], pcf[i], lap, eta);
      v = (u + u - pm2[i]) + incr;
      if (act1 && r >= kHalo && r < kHalo + TZ && c >= kHalo && c < kHalo + kTX) {
        const long long p = (long long)z * px + x;
        o1[p] = v;
        if (SK == kStoreF32) st[(long long)k * npts + p] = v;
      }
    }
    LE[r][c] = v;
  }
  __syncthreads();

  if (act2 && a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += G::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      const int C = R.i - T.x0 + kHalo, Rw = R.k - T.z0 + kHalo;
      a.d[S.d + (long long)k * S.nrec + R.r] =
          R.w[0] * LE[Rw][C] + R.w[1] * LE[Rw][C + 1] + R.w[2] * LE[Rw + 1][C] + R.w[3] * LE[Rw + 1][C + 1];
    }
  }
  if (!act2) return;
  // second step: level k+1 on the tile
  const float q2 = a.q[S.q + k];
  const int x = T.x0 + lane;
  const int dx = border_dist(x, nx, a.nbl);
#pragma unroll
  for (int i = 0; i < G::RPT; ++i) {
    const int lr = wv * G::RPT + i;
    const int z = T.z0 + lr;
    if (x >= nx || z >= nz) continue;
    const float* pc = &LE[lr + kHalo][lane + kHalo];
    const float u = pc[0];
    const float um2 = L1[lr + 2 * kHalo][lane + 2 * kHalo];
    float lap = lap_ptr(pc, G::WE, a.c);
    const int bx = x - src_i, bz = z - src_k;
    if ((unsigned)bx < 2u && (unsigned)bz < 2u) lap += src_weight(bx + 2 * bz) * q2;
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const float incr = step_incr(u, um2, tcf[i], lap, eta);
    const float un = (u + u - um2) + incr;
    const long long p = (long long)z * px + x;
    o2[p] = un;
    if (SK == kStoreF32) st[(long long)(k + 1) * npts + p] = un;
  }
}

// Adjoint: levels j and j-1 (j = step - off), receiver residual injected in both steps,
// imaging of both steps accumulated (in step order) into one FP64 read-modify-write.
// IMG = kImgNone or kImgFull32.
template <int TZ, int IMG>
__global__ __launch_bounds__(F2<TZ>::NT) void adj2d2_kernel(StepArgs a) {
  using G = F2<TZ>;
  __shared__ float L1[G::H1][G::W1];
  __shared__ float LE[G::HE][G::WE];
  __shared__ float INJ1[G::HE][G::WE];
  __shared__ float INJ2[TZ][kTX];
  __shared__ float INC1[TZ][kTX];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int j = a.step - S.off;
  const bool act1 = j >= 1 && j <= S.nt - 1;
  const bool act2 = j - 1 >= 1 && j - 1 <= S.nt - 1;
  if (!act1 && !act2) return;
  const int nx = S.nx, nz = S.nz, px = S.px;
  const float* __restrict__ w1 = fbuf(a.ws, S, adj_buf(j + 1));
  const float* __restrict__ w2 = fbuf(a.ws, S, adj_buf(j + 2));
  float* __restrict__ o1 = fbuf(a.ws, S, adj_buf(j));
  float* __restrict__ o2 = fbuf(a.ws, S, adj_buf(j - 1));
  const float* __restrict__ cf = reinterpret_cast<const float*>(a.ws + S.coef);
  const float* __restrict__ ust = IMG == kImgFull32 ? reinterpret_cast<const float*>(a.ws + S.store) : nullptr;
  double* __restrict__ acc = IMG ? reinterpret_cast<double*>(a.ws + S.acc) : nullptr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool inj1 = act1 && a.dd != nullptr && T.ext_count > 0;
  const bool inj2 = act2 && a.dd != nullptr && T.inj_count > 0;

  float pm2[G::NS], pcf[G::NS], tcf[G::RPT], pu1[G::RPT], pu2[G::RPT];
  double pacc[G::RPT];
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    int r, c;
    const bool ok = ext_slot<TZ>(i, &r, &c);
    const int z = T.z0 - kHalo + r, x = T.x0 - kHalo + c;
    const bool in = ok && (unsigned)z < (unsigned)nz && (unsigned)x < (unsigned)nx;
    const long long p = cidx2(x, z, nz, px);
    const float v2 = w2[p], vc = cf[p];
    pm2[i] = in ? v2 : 0.f;
    pcf[i] = in ? vc : 0.f;
    if (inj1 && ok) INJ1[r][c] = 0.f;
  }
  {
    const int x = T.x0 + lane;
    // store levels j and j-1, clamped to the stored range 0..nt-1 (a level outside it belongs
    // to an inactive step and its value is not used)
    const long long lv1 = min(j, S.nt - 1), lv2 = max(j - 1, 0);
#pragma unroll
    for (int i = 0; i < G::RPT; ++i) {
      const int z = T.z0 + wv * G::RPT + i;
      const bool in = x < nx && z < nz;
      const long long p = cidx2(x, z, nz, px);
      const float vc = cf[p];
      tcf[i] = in ? vc : 0.f;
      if (IMG) {
        const float a1 = ust[lv1 * S.npts + p];
        const float a2 = ust[lv2 * S.npts + p];
        const double va = acc[p];
        pu1[i] = in && act1 ? a1 : 0.f;
        pu2[i] = in && act2 ? a2 : 0.f;
        pacc[i] = in ? va : 0.0;
      }
      if (inj2) INJ2[wv * G::RPT + i][lane] = 0.f;
    }
  }
  load_tile8<TZ>(L1, w1, nx, nz, nz, px, T.x0, T.z0);
  __syncthreads();

  if (inj1 || inj2) {
    if (inj1) {
      const float* ddj = a.dd + S.d + (long long)j * S.nrec;
      for (int t = threadIdx.x; t < T.ext_count; t += G::NT) {
        const InjPoint Pt = a.t.ext_pts[T.ext_begin + t];
        float sum = 0.f;
        for (int e = 0; e < Pt.e_count; ++e) {
          const InjEntry E = a.t.inj_ent[Pt.e_begin + e];
          sum += E.w * ddj[E.r];
        }
        INJ1[Pt.lz][Pt.lx] = sum;
      }
    }
    if (inj2) {
      const float* ddj = a.dd + S.d + (long long)(j - 1) * S.nrec;
      for (int t = threadIdx.x; t < T.inj_count; t += G::NT) {
        const InjPoint Pt = a.t.inj_pts[T.inj_begin + t];
        float sum = 0.f;
        for (int e = 0; e < Pt.e_count; ++e) {
          const InjEntry E = a.t.inj_ent[Pt.e_begin + e];
          sum += E.w * ddj[E.r];
        }
        INJ2[Pt.lz][Pt.lx] = sum;
      }
    }
    __syncthreads();
  }
  if (act1 && a.v != nullptr && a.tile_base + tid == S.src_tile && threadIdx.x == 0) {
    const int C = S.src_i - T.x0 + 2 * kHalo, R = S.src_k - T.z0 + 2 * kHalo;
    a.v[S.q + j] = S.src_w[0] * L1[R][C] + S.src_w[1] * L1[R][C + 1] + S.src_w[2] * L1[R + 1][C] +
                   S.src_w[3] * L1[R + 1][C + 1];
  }
  // first step: level j on the tile + 4-cell halo (the loop has no early exit, so it unrolls
  // completely and pm2 / pcf stay in registers)
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    int r, c;
    if (!ext_slot<TZ>(i, &r, &c)) continue;
    const int z = T.z0 - kHalo + r, x = T.x0 - kHalo + c;
    float v = 0.f;
    if ((unsigned)z < (unsigned)nz && (unsigned)x < (unsigned)nx) {
      const float* pc = &L1[r + kHalo][c + kHalo];
      const float w = pc[0];
      float lap = lap_ptr(pc, G::W1, a.c);
      if (inj1) lap += INJ1[r][c];
      const int dx = border_dist(x, nx, a.nbl), dz = border_dist(z, nz, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
      const float incr = step_incr(w, pm2[i], pcf[i], lap, eta);
      v = (w + w - pm2[i]) + incr;
      if (r >= kHalo && r < kHalo + TZ && c >= kHalo && c < kHalo + kTX) {
        if (act1) o1[(long long)z * px + x] = v;
        INC1[r - kHalo][c - kHalo] = incr;
      }
    }
    LE[r][c] = v;
  }
  __syncthreads();

  if (act2 && a.v != nullptr && a.tile_base + tid == S.src_tile && threadIdx.x == 0) {
    const int C = S.src_i - T.x0 + kHalo, R = S.src_k - T.z0 + kHalo;
    a.v[S.q + j - 1] = S.src_w[0] * LE[R][C] + S.src_w[1] * LE[R][C + 1] + S.src_w[2] * LE[R + 1][C] +
                       S.src_w[3] * LE[R + 1][C + 1];
  }
  // second step: level j-1 on the tile; imaging of both steps
  const int x = T.x0 + lane;
  const int dx = border_dist(x, nx, a.nbl);
#pragma unroll
  for (int i = 0; i < G::RPT; ++i) {
    const int lr = wv * G::RPT + i;
    const int z = T.z0 + lr;
    if (x >= nx || z >= nz) continue;
    const long long p = (long long)z * px + x;
    double ac = IMG ? pacc[i] : 0.0;
    if (IMG && act1) ac = ac + (double)pu1[i] * (double)INC1[lr][lane];
    if (act2) {
      const float* pc = &LE[lr + kHalo][lane + kHalo];
      const float w = pc[0];
      const float wm2 = L1[lr + 2 * kHalo][lane + 2 * kHalo];
      float lap = lap_ptr(pc, G::WE, a.c);
      if (inj2) lap += INJ2[lr][lane];
      const int dz = border_dist(z, nz, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
      const float incr = step_incr(w, wm2, tcf[i], lap, eta);
      o2[p] = (w + w - wm2) + incr;
      if (IMG) ac = ac + (double)pu2[i] * (double)incr;
    }
    if (IMG) acc[p] = ac;
  }
}

template <int TZ>
hipError_t fwd2d_tz(const StepArgs& a, int store, hipStream_t s) {
  switch (store) {
    case kStoreNone: fwd2d_kernel<TZ, kStoreNone><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kStoreF32: fwd2d_kernel<TZ, kStoreF32><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kStoreBF16: fwd2d_kernel<TZ, kStoreBF16><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kStoreFP16: fwd2d_kernel<TZ, kStoreFP16><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TZ>
hipError_t adj2d_tz(const StepArgs& a, hipStream_t s) {
  switch (a.image_src) {
    case kImgNone: adj2d_kernel<TZ, kImgNone><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kImgFull32: adj2d_kernel<TZ, kImgFull32><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kImgBuffers: adj2d_kernel<TZ, kImgBuffers><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kImgFullBF16: adj2d_kernel<TZ, kImgFullBF16><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kImgFullFP16: adj2d_kernel<TZ, kImgFullFP16><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TZ>
hipError_t fwd2d2_tz(const StepArgs& a, int store, hipStream_t s) {
  switch (store) {
    case kStoreNone: fwd2d2_kernel<TZ, kStoreNone><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    case kStoreF32: fwd2d2_kernel<TZ, kStoreF32><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TZ>
hipError_t adj2d2_tz(const StepArgs& a, hipStream_t s) {
  switch (a.image_src) {
    case kImgNone: adj2d2_kernel<TZ, kImgNone><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    case kImgFull32: adj2d2_kernel<TZ, kImgFull32><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fwd2d2(const StepArgs& a, int tz, int store, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: return fwd2d2_tz<8>(a, store, s);
    case 16: return fwd2d2_tz<16>(a, store, s);
    case 32: return fwd2d2_tz<32>(a, store, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj2d2(const StepArgs& a, int tz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: return adj2d2_tz<8>(a, s);
    case 16: return adj2d2_tz<16>(a, s);
    case 32: return adj2d2_tz<32>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fwd2d(const StepArgs& a, int tz, int store, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: return fwd2d_tz<8>(a, store, s);
    case 12: return fwd2d_tz<12>(a, store, s);
    case 16: return fwd2d_tz<16>(a, store, s);
    case 20: return fwd2d_tz<20>(a, store, s);
    case 24: return fwd2d_tz<24>(a, store, s);
    case 32: return fwd2d_tz<32>(a, store, s);
    case 64: return fwd2d_tz<64>(a, store, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj2d(const StepArgs& a, int tz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: return adj2d_tz<8>(a, s);
    case 12: return adj2d_tz<12>(a, s);
    case 16: return adj2d_tz<16>(a, s);
    case 20: return adj2d_tz<20>(a, s);
    case 24: return adj2d_tz<24>(a, s);
    case 32: return adj2d_tz<32>(a, s);
    case 64: return adj2d_tz<64>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_born2d(const StepArgs& a, int tz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: born2d_kernel<8><<<a.ntiles, T2<8>::NT, 0, s>>>(a); break;
    case 12: born2d_kernel<12><<<a.ntiles, T2<12>::NT, 0, s>>>(a); break;
    case 16: born2d_kernel<16><<<a.ntiles, T2<16>::NT, 0, s>>>(a); break;
    case 20: born2d_kernel<20><<<a.ntiles, T2<20>::NT, 0, s>>>(a); break;
    case 24: born2d_kernel<24><<<a.ntiles, T2<24>::NT, 0, s>>>(a); break;
    case 32: born2d_kernel<32><<<a.ntiles, T2<32>::NT, 0, s>>>(a); break;
    case 64: born2d_kernel<64><<<a.ntiles, T2<64>::NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace awe
