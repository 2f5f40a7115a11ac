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
//
// Fields are read and written through buffer resources (bufio.h): a lane's byte offset within
// a row is fixed (kOOB for a column outside the grid: its loads read 0, its stores are
// dropped, and it costs no memory traffic) and the row's offset is wave-uniform, so rows cost
// no vector instructions for addresses, clamps or masks.  Rows outside the grid, and levels
// that are zero by definition, are read through a resource of size 0.
#include "awe_internal.h"
#include "bufio.h"
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

// Plane offsets of this thread's side-halo cells of a tile staged with an HW-cell halo: cell e
// of the 2 HW columns left and right of the 64-column body of each of the H rows, starting at
// row z0 - HW (kOOB outside the grid or past the last cell).
template <int NT, int H, int HW>
struct SideHalo {
  static constexpr int NE = H * 2 * HW;
  static constexpr int NH = (NE + NT - 1) / NT;
};

template <int NT, int H, int HW>
__device__ __forceinline__ void side_cell(int i, int* r, int* c) {
  constexpr int NE = SideHalo<NT, H, HW>::NE;
  const int e = min((int)threadIdx.x + i * NT, NE - 1);
  *r = e / (2 * HW);
  const int cc = e - *r * (2 * HW);
  *c = cc < HW ? cc : kTX + cc;          // columns 0 .. HW-1 and 64+HW .. 64+2HW-1
}

template <int NT, int H, int HW>
__device__ __forceinline__ void side_offsets(int (&ho)[(SideHalo<NT, H, HW>::NH)], int nx, int nz, int px,
                                             int x0, int z0) {
#pragma unroll
  for (int i = 0; i < SideHalo<NT, H, HW>::NH; ++i) {
    // a slot past the last side cell takes the last cell (side_cell clamps): it loads and
    // writes the same value as that cell's owner, so the staging needs no condition
    int r, c;
    side_cell<NT, H, HW>(i, &r, &c);
    ho[i] = col_off(x0 - HW + c, z0 - HW + r, nx, nz, px, 4);
  }
}

// Stage rows z0-HW .. z0+TZ+HW-1, columns x0-HW .. x0+63+HW of a field into LDS (W = 64 + 2 HW
// columns, H rows), zero outside the grid: the 64-column body of each row is one aligned
// 256-byte row segment per wave (row offset wave-uniform, column offset cx = 4 x or kOOB), the
// side cells follow from their precomputed offsets.  All loads are issued before the first LDS
// write.
// The staging is split in two: `issue` loads this thread's cells into registers, `commit` writes
// them to LDS.  A kernel issues its tile before its other prefetches: loads complete in issue
// order, so the LDS writes then wait for the tile's loads alone, not for every prefetch.
template <int NT, int NW, int H, int HW>
struct Staged {
  static constexpr int NB = H / NW, NH = SideHalo<NT, H, HW>::NH;
  float vb[NB], vh[NH];
};

template <int NT, int NW, int H, int HW>
__device__ __forceinline__ void stage_issue(Staged<NT, NW, H, HW>& s, const Planes& f, int cx,
                                            const int (&ho)[(SideHalo<NT, H, HW>::NH)], int z0) {
  // every wave stages whole rows: no row condition, so no branch separates the loads from
  // their use (a branch would make the compiler wait for all loads at its start)
  static_assert(H % NW == 0, "staged rows must split evenly over the waves");
  const int wv = wave_id();
#pragma unroll
  for (int i = 0; i < Staged<NT, NW, H, HW>::NB; ++i) s.vb[i] = ldp(f, cx, z0 - HW + wv + i * NW);
#pragma unroll
  for (int i = 0; i < Staged<NT, NW, H, HW>::NH; ++i) s.vh[i] = ldp_at(f, ho[i]);
}

template <int NT, int NW, int H, int HW, int W>
__device__ __forceinline__ void stage_commit(float (*L)[W], const Staged<NT, NW, H, HW>& s) {
  const int lane = threadIdx.x & 63, wv = wave_id();
#pragma unroll
  for (int i = 0; i < Staged<NT, NW, H, HW>::NB; ++i) L[wv + i * NW][lane + HW] = s.vb[i];
  // unconditional: threads past the last side cell write that cell's own value again (a
  // condition here would let the compiler sink the load into it and wait for every load)
#pragma unroll
  for (int i = 0; i < Staged<NT, NW, H, HW>::NH; ++i) {
    int r, c;
    side_cell<NT, H, HW>(i, &r, &c);
    L[r][c] = s.vh[i];
  }
}

template <int TZ>
using Side4 = SideHalo<T2<TZ>::NT, T2<TZ>::H, kHalo>;

// The previous level with a 4-cell halo (one-step kernels): issue, then commit to LDS.
template <int TZ>
using Tile4 = Staged<T2<TZ>::NT, T2<TZ>::NW, T2<TZ>::H, kHalo>;

template <int TZ>
__device__ __forceinline__ void tile_issue(Tile4<TZ>& t, const Planes& f, int cx, const int (&ho)[Side4<TZ>::NH],
                                           int z0) {
  stage_issue<T2<TZ>::NT, T2<TZ>::NW, T2<TZ>::H, kHalo>(t, f, cx, ho, z0);
}

template <int TZ>
__device__ __forceinline__ void tile_commit(float (*L)[T2<TZ>::W], const Tile4<TZ>& t) {
  stage_commit<T2<TZ>::NT, T2<TZ>::NW, T2<TZ>::H, kHalo, T2<TZ>::W>(L, t);
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

// Where a one-level forward step reads level k of shot S.  kStoreF32R: the FULL FP32 store keeps
// every level bit for bit, so the step reads its two previous levels from it (written by the
// launch before, with ordinary stores that leave them in the caches) and the rotating buffers
// are not needed; otherwise the rotating buffers, or a checkpoint slot restored by reference.
template <int SK>
__device__ __forceinline__ const float* fwd_src(const StepArgs& a, const ShotDev& S, int k) {
  if (SK == kStoreF32R) return reinterpret_cast<const float*>(a.ws + S.store) + (long long)k * S.npts;
  return fwd_level(a, S, k);
}

// Bytes of the rotating buffer a one-level forward step writes level k into: with kStoreF32R only
// the last level goes there too (the receivers' last sample is taken from it), so the other
// levels' buffer stores are dropped by the range check.
template <int SK>
__device__ __forceinline__ int fwd_ring_bytes(const ShotDev& S, int k, int bytes) {
  return SK != kStoreF32R || k == S.nt - 1 ? bytes : 0;
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
  const int row4 = 4 * px;
  // levels below 1 are zero (initial state); their buffers may hold older levels after a
  // checkpoint restore of a state before this shot's start, so they are not read
  const Planes u1 = planes(fwd_src<SK>(a, S, k - 1), nz, k >= 2 ? nz : 0, row4);
  const Planes u2 = planes(fwd_src<SK>(a, S, k - 2), nz, k >= 3 ? nz : 0, row4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, row4);
  const brsrc rout = make_rsrc(fbuf(a.ws, S, fwd_buf(k)), fwd_ring_bytes<SK>(S, k, nz * row4));
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int x = T.x0 + lane;
  const int cx = x < nx ? 4 * x : kOOB;

  int ho[Side4<TZ>::NH];
  side_offsets<T2<TZ>::NT, T2<TZ>::H, kHalo>(ho, nx, nz, px, T.x0, T.z0);
  Tile4<TZ> tile;
  tile_issue<TZ>(tile, u1, cx, ho, T.z0);
  float pu2[RPT], pcf[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int z = T.z0 + wv * RPT + i;
    pu2[i] = ldp(u2, cx, z);
    pcf[i] = ldp(cf, cx, z);
  }
  tile_commit<TZ>(L, tile);
  __syncthreads();

  if (a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += T2<TZ>::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] = interp_lds<TZ>(L, R.i, R.k, T.x0, T.z0, R.w);
    }
  }

  const float qk = a.q[S.q + k - 1];
  const int dx = border_dist(x, nx, a.nbl);
  // shot fields used in the row loop, in registers: a reload after a store would wait for every
  // store in flight
  const int src_i = S.src_i, src_k = S.src_k;
  const float sw0 = S.src_w[0], sw1 = S.src_w[1], sw2 = S.src_w[2], sw3 = S.src_w[3];
  const long long npts = S.npts;
  // FULL store: level k (FP32) or level k-1 (16 bits, quantised with its finished scale)
  constexpr bool F32 = SK == kStoreF32 || SK == kStoreF32R;
  const brsrc rst = F32
      ? make_rsrc(reinterpret_cast<float*>(a.ws + S.store) + (long long)k * npts, nz * row4)
      : make_rsrc(reinterpret_cast<unsigned short*>(a.ws + S.store) + (long long)(k - 1) * npts,
                  SK == kStoreBF16 || SK == kStoreFP16 ? nz * row4 / 2 : 0);
  // checkpoint store fused into the step that reaches the stored state: (u^k, u^{k-1}) into slot
  const bool to_slot = SK == kStoreNone && a.st_slot >= 0;
  float* sl = reinterpret_cast<float*>(a.ws + S.store) + (long long)(to_slot ? a.st_slot : 0) * 2 * npts;
  const brsrc rsl0 = make_rsrc(sl, to_slot ? nz * row4 : 0);
  const brsrc rsl1 = make_rsrc(sl + npts, to_slot ? nz * row4 : 0);
  const int cx2 = x < nx ? 2 * x : kOOB;
  constexpr bool S16 = SK == kStoreBF16 || SK == kStoreFP16;
  float* scl = S16 ? reinterpret_cast<float*>(a.ws + S.scale) : nullptr;
  const float inv_prev = S16 && k >= 2 ? inv_scale(level_scale(scl, k - 1)) : 0.f;
  // probed gradient: the r FP64 sums B_j of this shot, and this level's coefficients
  double* pb = SK == kStoreProbe ? reinterpret_cast<double*>(a.ws + S.store) : nullptr;
  const float* pc = SK == kStoreProbe ? a.probe_c + k : nullptr;
  float lmax = 0.f;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    // every lane computes; outside the grid u, u^{k-2} and coef read 0 (so the new value is 0)
    // and the stores are dropped
    const int lr = wv * RPT + i;
    const int z = T.z0 + lr;
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
    const int zo = z * row4;
    stb(rout, un, cx, zo);
    if (to_slot) {
      stb(rsl0, un, cx, zo);
      stb(rsl1, u, cx, zo);
    }
    // a stored level the next launch reads back stays in the caches; otherwise it is written once
    // and read thousands of launches later
    if (SK == kStoreF32) stb_nt(rst, un, cx, zo);
    if (SK == kStoreF32R) stb(rst, un, cx, zo);
    if (S16) {
      lmax = fmaxf(lmax, fabsf(un));
      if (k >= 2) stb16_nt(rst, enc16(u * inv_prev, SK == kStoreBF16), cx2, zo / 2);
    }
    if (SK == kStoreProbe && x < nx && z < nz) {
      // u^k - 2u^{k-1} + u^{k-2} = incr (increment form of the step)
      const long long p = (long long)z * px + x;
      probe_add(probe_sums(pb, p, a.probe_r), a.probe_r, pc, (double)incr, true, nullptr, 0.0, false, a.probe_pitch);
    }
  }
  if (S16) block_max_to_slot(lmax, scl, k);
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
  const int row4 = 4 * px;
  const Planes w1 = planes(fbuf(a.ws, S, adj_buf(j + 1)), nz, nz, row4);
  const Planes w2 = planes(fbuf(a.ws, S, adj_buf(j + 2)), nz, nz, row4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, row4);
  const brsrc rout = make_rsrc(fbuf(a.ws, S, adj_buf(j)), nz * row4);
  // imaging: u^j from the FULL store (FP32, or 16 bits with the level's scale) or the forward
  // buffers, and the FP64 accumulator
  constexpr bool I16 = IMG == kImgFullBF16 || IMG == kImgFullFP16;
  constexpr bool IACC = IMG != kImgNone && IMG != kImgProbe;  // imaging into the FP64 accumulator
  const void* ubase = IMG == kImgBuffers ? (const void*)fwd_level(a, S, j)
                      : IMG == kImgFull32 ? (const void*)(reinterpret_cast<const float*>(a.ws + S.store) + (long long)j * S.npts)
                      : (const void*)(reinterpret_cast<const unsigned short*>(a.ws + S.store) + (long long)j * S.npts);
  const Planes uj = planes(ubase, nz, IACC ? nz : 0, I16 ? row4 / 2 : row4);
  const float usc = I16 ? level_scale(reinterpret_cast<const float*>(a.ws + S.scale), j) : 1.f;
  const Planes acc = planes(a.ws + S.acc, nz, IACC ? nz : 0, 2 * row4);
  const brsrc racc = make_rsrc(a.ws + S.acc, IACC ? 2 * nz * row4 : 0);
  // probed gradient: the r FP64 sums A_j of this shot (after its B_j), and this level's coefficients
  double* pa = IMG == kImgProbe ? reinterpret_cast<double*>(a.ws + S.store) + (long long)a.probe_r * S.npts : nullptr;
  const float* pc = IMG == kImgProbe ? a.probe_c + j : nullptr;
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int x = T.x0 + lane;
  const int cx = x < nx ? 4 * x : kOOB;
  const int cxu = x < nx ? (I16 ? 2 : 4) * x : kOOB;
  const int cx8 = x < nx ? 8 * x : kOOB;
  const bool has_inj = T.inj_count > 0 && a.dd != nullptr;  // no residual: nothing to inject

  int ho[Side4<TZ>::NH];
  side_offsets<T2<TZ>::NT, T2<TZ>::H, kHalo>(ho, nx, nz, px, T.x0, T.z0);
  Tile4<TZ> tile;
  tile_issue<TZ>(tile, w1, cx, ho, T.z0);
  float pw2[RPT], pcf[RPT], pu[RPT];
  double pacc[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int z = T.z0 + wv * RPT + i;
    pw2[i] = ldp(w2, cx, z);
    pcf[i] = ldp(cf, cx, z);
    if (I16) pu[i] = dec16(ldp16_nt(uj, cxu, z), IMG == kImgFullBF16) * usc;
    else if (IMG == kImgFull32) pu[i] = ldp_nt(uj, cxu, z);
    else if (IACC) pu[i] = ldp(uj, cxu, z);
    if (IACC) pacc[i] = ldp64(acc, cx8, z);
    if (has_inj) INJ[wv * RPT + i][lane] = 0.f;
  }
  tile_commit<TZ>(L, tile);
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
    // every lane computes; outside the grid the stores are dropped
    const int lr = wv * RPT + i;
    const int z = T.z0 + lr;
    const float w = L[lr + kHalo][lane + kHalo];
    float lap = lap_at<TZ>(L, lr, lane, a.c);
    if (has_inj) lap += INJ[lr][lane];
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const float incr = step_incr(w, pw2[i], pcf[i], lap, eta);
    const int zo = z * row4;
    const float wn = (w + w - pw2[i]) + incr;
    stb(rout, wn, cx, zo);
    if (IACC) stb64(racc, pacc[i] + (double)pu[i] * (double)incr, cx8, 2 * zo);
    if (IMG == kImgProbe && x < nx && z < nz) {
      const long long p = (long long)z * px + x;
      probe_add(probe_sums(pa, p, a.probe_r), a.probe_r, pc, (double)wn, true, nullptr, 0.0, false, a.probe_pitch);
    }
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
  const int row4 = 4 * px;
  const Planes u1 = planes(fbuf(a.ws, S, fwd_buf(k - 1)), nz, nz, row4);
  const Planes u2 = planes(fbuf(a.ws, S, fwd_buf(k - 2)), nz, nz, row4);
  const Planes d1 = planes(fbuf(a.ws, S, adj_buf(k - 1)), nz, nz, row4);
  const Planes d2 = planes(fbuf(a.ws, S, adj_buf(k - 2)), nz, nz, row4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, row4);
  const Planes dm = planes(a.dm + S.m, nz, nz, 4LL * nx);   // caller's layout: rows of nx
  const brsrc ruo = make_rsrc(fbuf(a.ws, S, fwd_buf(k)), nz * row4);
  const brsrc rdo = make_rsrc(fbuf(a.ws, S, adj_buf(k)), nz * row4);
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int x = T.x0 + lane;
  const int cx = x < nx ? 4 * x : kOOB;

  int ho[Side4<TZ>::NH];
  side_offsets<T2<TZ>::NT, T2<TZ>::H, kHalo>(ho, nx, nz, px, T.x0, T.z0);
  Tile4<TZ> tu, td;
  tile_issue<TZ>(tu, u1, cx, ho, T.z0);
  tile_issue<TZ>(td, d1, cx, ho, T.z0);
  float pu2[RPT], pd2[RPT], pcf[RPT], pdm[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int z = T.z0 + wv * RPT + i;
    pu2[i] = ldp(u2, cx, z);
    pd2[i] = ldp(d2, cx, z);
    pcf[i] = ldp(cf, cx, z);
    pdm[i] = ldp(dm, cx, z);
  }
  tile_commit<TZ>(LU, tu);
  tile_commit<TZ>(LD, td);
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
    // every lane computes; outside the grid the stores are dropped
    const int lr = wv * RPT + i;
    const int z = T.z0 + lr;
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const int zo = z * row4;
    // background field
    const float u = LU[lr + kHalo][lane + kHalo];
    float lap = lap_at<TZ>(LU, lr, lane, a.c);
    const int bx = x - src_i, bz = z - src_k;
    if ((unsigned)bx < 2u && (unsigned)bz < 2u) {
      const int w = bx + 2 * bz;
      lap += (w == 0 ? sw0 : w == 1 ? sw1 : w == 2 ? sw2 : sw3) * qk;
    }
    const float incr = pcf[i] * (lap - eta * (u - pu2[i]));
    stb(ruo, (u + u - pu2[i]) + incr, cx, zo);
    // scattered field, source -dm (u^k - 2u^{k-1} + u^{k-2}) / dt^2 = -dm incr / dt^2
    const float du = LD[lr + kHalo][lane + kHalo];
    const float lapd = lap_at<TZ>(LD, lr, lane, a.c) - pdm[i] * incr * a.inv_dt2;
    const float incd = pcf[i] * (lapd - eta * (du - pd2[i]));
    stb(rdo, (du + du - pd2[i]) + incd, cx, zo);
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
  static constexpr int NB = HE / NW;
  static_assert(HE % NW == 0, "extended rows must split evenly over the waves");
  static constexpr int NH = (2 * kHalo * HE + NT - 1) / NT;
  static constexpr int NS = NB + NH;
};

// Slot i of this thread among the first-step points (row r, column c of the WE x HE region);
// false for an unused slot (its r, c are then a valid point, not to be written).
template <int TZ>
__device__ __forceinline__ bool ext_slot(int i, int* r, int* c) {
  using G = F2<TZ>;
  if (i < G::NB) {       // body slots: every row of the extended region is a whole wave's row
    *r = wave_id() + i * G::NW;
    *c = kHalo + (int)(threadIdx.x & 63);
    return true;
  }
  const int e0 = (int)threadIdx.x + (i - G::NB) * G::NT;
  const int e = min(e0, 2 * kHalo * G::HE - 1);
  *r = e / (2 * kHalo);
  const int cc = e - *r * (2 * kHalo);
  *c = cc < kHalo ? cc : kTX + cc;
  return e0 < 2 * kHalo * G::HE;
}

template <int TZ>
using Side8 = SideHalo<F2<TZ>::NT, F2<TZ>::H1, 2 * kHalo>;

// Level n-1 with an 8-cell halo (two-step kernels): issue, then commit to LDS.
template <int TZ>
using Tile8 = Staged<F2<TZ>::NT, F2<TZ>::NW, F2<TZ>::H1, 2 * kHalo>;

template <int TZ>
__device__ __forceinline__ void tile8_issue(Tile8<TZ>& t, const Planes& f, int cx, const int (&ho)[Side8<TZ>::NH],
                                            int z0) {
  stage_issue<F2<TZ>::NT, F2<TZ>::NW, F2<TZ>::H1, 2 * kHalo>(t, f, cx, ho, z0);
}

template <int TZ>
__device__ __forceinline__ void tile8_commit(float (*L)[F2<TZ>::W1], const Tile8<TZ>& t) {
  stage_commit<F2<TZ>::NT, F2<TZ>::NW, F2<TZ>::H1, 2 * kHalo, F2<TZ>::W1>(L, t);
}

// Plane offsets of this thread's first-step points that lie in the 4 + 4 side columns (the
// extended slots past the NB body slots); kOOB outside the grid or for an unused slot.
template <int TZ>
__device__ __forceinline__ void ext_offsets(int (&eo)[F2<TZ>::NH], int nx, int nz, int px, int x0, int z0) {
  using G = F2<TZ>;
#pragma unroll
  for (int i = 0; i < G::NH; ++i) {
    int r, c;
    const bool ok = ext_slot<TZ>(G::NB + i, &r, &c);
    eo[i] = ok ? col_off(x0 - kHalo + c, z0 - kHalo + r, nx, nz, px, 4) : kOOB;
  }
}

// Load of a first-step point: body slots read the row z0-4+r (wave-uniform) at column offset cx,
// side slots their own offset.
template <int TZ>
__device__ __forceinline__ float ld_ext(const Planes& f, int i, int cx, const int (&eo)[F2<TZ>::NH], int z0) {
  using G = F2<TZ>;
  if (i < G::NB) return ldp(f, cx, z0 - kHalo + wave_id() + i * G::NW);
  return ldp_at(f, eo[i - G::NB]);
}

// Forward: levels k and k+1 (k = step - off); SK = kStoreNone, kStoreF32 or kStoreProbe (both
// levels' increments added to the probe sums in one FP64 read-modify-write, level k first).
template <int TZ, int SK>
__global__ __launch_bounds__(F2<TZ>::NT) void fwd2d2_kernel(StepArgs a) {
  using G = F2<TZ>;
  constexpr bool PRB = SK == kStoreProbe;
  __shared__ float L1[G::H1][G::W1];
  __shared__ float LE[G::HE][G::WE];
  __shared__ float INC1[PRB ? TZ : 1][kTX];  // probe: level k's increment on the tile
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  const bool act1 = k >= 1 && k <= S.nt - 1;
  const bool act2 = k + 1 >= 1 && k + 1 <= S.nt - 1;
  if (!act1 && !act2) return;
  const int nx = S.nx, nz = S.nz, px = S.px;
  const int row4 = 4 * px;
  // levels below 1 are zero (see fwd2d_kernel)
  // (two-level launches never follow a restore by reference: the rotating buffers hold the
  // previous levels)
  const Planes u1 = planes(fbuf(a.ws, S, fwd_buf(k - 1)), nz, k >= 2 ? nz : 0, row4);
  const Planes u2 = planes(fbuf(a.ws, S, fwd_buf(k - 2)), nz, k >= 3 ? nz : 0, row4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, row4);
  const long long npts = S.npts;
  // new levels k and k+1 (a level outside 1..nt-1 belongs to an inactive step: no records)
  const brsrc ro1 = make_rsrc(fbuf(a.ws, S, fwd_buf(k)), act1 ? nz * row4 : 0);
  const brsrc ro2 = make_rsrc(fbuf(a.ws, S, fwd_buf(k + 1)), act2 ? nz * row4 : 0);
  float* st = reinterpret_cast<float*>(a.ws + S.store);
  const brsrc rs1 = make_rsrc(st + (long long)(SK == kStoreF32 ? k : 0) * npts,
                              SK == kStoreF32 && act1 ? nz * row4 : 0);
  const brsrc rs2 = make_rsrc(st + (long long)(SK == kStoreF32 ? k + 1 : 0) * npts,
                              SK == kStoreF32 && act2 ? nz * row4 : 0);
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int x = T.x0 + lane;
  const int cx = x < nx ? 4 * x : kOOB;

  // the level k-1 tile first, then level k-2 and coef of this thread's extended points and coef
  // of its tile points
  int ho[Side8<TZ>::NH];
  side_offsets<G::NT, G::H1, 2 * kHalo>(ho, nx, nz, px, T.x0, T.z0);
  Tile8<TZ> tile;
  tile8_issue<TZ>(tile, u1, cx, ho, T.z0);
  int eo[G::NH];
  ext_offsets<TZ>(eo, nx, nz, px, T.x0, T.z0);
  float pm2[G::NS], pcf[G::NS], tcf[G::RPT];
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    pm2[i] = ld_ext<TZ>(u2, i, cx, eo, T.z0);
    pcf[i] = ld_ext<TZ>(cf, i, cx, eo, T.z0);
  }
#pragma unroll
  for (int i = 0; i < G::RPT; ++i) tcf[i] = ldp(cf, cx, T.z0 + wv * G::RPT + i);
  tile8_commit<TZ>(L1, tile);
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
  // first step: level k on the tile + 4-cell halo (zero outside the grid)
  const float q1 = act1 ? a.q[S.q + k - 1] : 0.f;
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    int r, c;
    if (!ext_slot<TZ>(i, &r, &c)) continue;
    const int z = T.z0 - kHalo + r, xx = T.x0 - kHalo + c;
    float v = 0.f, incr = 0.f;
    if ((unsigned)z < (unsigned)nz && (unsigned)xx < (unsigned)nx) {
      const float* pc = &L1[r + kHalo][c + kHalo];
      const float u = pc[0];
      float lap = lap_ptr(pc, G::W1, a.c);
      const int bx = xx - src_i, bz = z - src_k;
      if (act1 && (unsigned)bx < 2u && (unsigned)bz < 2u) lap += src_weight(bx + 2 * bz) * q1;
      const int dx = border_dist(xx, nx, a.nbl), dz = border_dist(z, nz, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
      incr = step_incr(u, pm2[i], pcf[i], lap, eta);
      v = (u + u - pm2[i]) + incr;
    }
    // body slots on tile rows store level k (wave-uniform condition; columns outside drop)
    if (i < G::NB && r >= kHalo && r < kHalo + TZ) {
      stb(ro1, v, cx, z * row4);
      if (SK == kStoreF32) stb_nt(rs1, v, cx, z * row4);
      if (PRB) INC1[r - kHalo][c - kHalo] = incr;
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
  if (!act2 && !PRB) return;  // probe: level k's increments are still to be added
  // second step: level k+1 on the tile (every lane computes; stores outside the grid drop, as
  // do those of an inactive level k+1)
  const float q2 = act2 ? a.q[S.q + k] : 0.f;
  const int dx = border_dist(x, nx, a.nbl);
  double* pb = PRB ? reinterpret_cast<double*>(a.ws + S.store) : nullptr;
  const float* pc1 = PRB ? a.probe_c + k : nullptr;
  const float* pc2 = PRB ? a.probe_c + k + 1 : nullptr;
#pragma unroll
  for (int i = 0; i < G::RPT; ++i) {
    const int lr = wv * G::RPT + i;
    const int z = T.z0 + lr;
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
    stb(ro2, un, cx, z * row4);
    if (SK == kStoreF32) stb_nt(rs2, un, cx, z * row4);
    if (PRB && x < nx && z < nz) {
      // the same two FP64 additions, in the same order, as two one-level launches
      const long long p = (long long)z * px + x;
      probe_add(probe_sums(pb, p, a.probe_r), a.probe_r, pc1, (double)INC1[lr][lane], act1, pc2, (double)incr, act2,
                a.probe_pitch);
    }
  }
}

// Adjoint: levels j and j-1 (j = step - off), receiver residual injected in both steps,
// imaging of both steps accumulated (in step order) into one FP64 read-modify-write.
// IMG = kImgNone, kImgFull32 or kImgProbe (both levels added to the probe sums A_j in one FP64
// read-modify-write, level j first).
template <int TZ, int IMG>
__global__ __launch_bounds__(F2<TZ>::NT) void adj2d2_kernel(StepArgs a) {
  using G = F2<TZ>;
  // kImgBuffers: the two levels come from the recomputed forward buffers (or the slot restored
  // by reference) instead of the FULL store, as in a checkpointed gradient's paired reversals
  constexpr bool IBUF = IMG == kImgBuffers;
  constexpr bool IACC = IMG == kImgFull32 || IBUF;
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
  const int row4 = 4 * px;
  const Planes w1 = planes(fbuf(a.ws, S, adj_buf(j + 1)), nz, nz, row4);
  const Planes w2 = planes(fbuf(a.ws, S, adj_buf(j + 2)), nz, nz, row4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, row4);
  // new levels j and j-1 (a level of an inactive step gets no records: its stores drop)
  const brsrc ro1 = make_rsrc(fbuf(a.ws, S, adj_buf(j)), act1 ? nz * row4 : 0);
  const brsrc ro2 = make_rsrc(fbuf(a.ws, S, adj_buf(j - 1)), act2 ? nz * row4 : 0);
  // imaging: stored u^j and u^{j-1} (levels of inactive steps read 0) and the FP64 accumulator
  const float* ust = reinterpret_cast<const float*>(a.ws + S.store);
  const Planes us1 = planes(IBUF ? fwd_level(a, S, j) : ust + (long long)(IACC && act1 ? j : 0) * S.npts, nz,
                            IACC && act1 ? nz : 0, row4);
  const Planes us2 = planes(IBUF ? fwd_level(a, S, j - 1) : ust + (long long)(IACC && act2 ? j - 1 : 0) * S.npts, nz,
                            IACC && act2 ? nz : 0, row4);
  const Planes acc = planes(a.ws + S.acc, nz, IACC ? nz : 0, 2 * row4);
  const brsrc racc = make_rsrc(a.ws + S.acc, IACC ? 2 * nz * row4 : 0);
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int x = T.x0 + lane;
  const int cx = x < nx ? 4 * x : kOOB;
  const int cx8 = x < nx ? 8 * x : kOOB;
  const bool inj1 = act1 && a.dd != nullptr && T.ext_count > 0;
  const bool inj2 = act2 && a.dd != nullptr && T.inj_count > 0;

  int ho[Side8<TZ>::NH];
  side_offsets<G::NT, G::H1, 2 * kHalo>(ho, nx, nz, px, T.x0, T.z0);
  Tile8<TZ> tile;
  tile8_issue<TZ>(tile, w1, cx, ho, T.z0);
  int eo[G::NH];
  ext_offsets<TZ>(eo, nx, nz, px, T.x0, T.z0);
  float pm2[G::NS], pcf[G::NS], tcf[G::RPT], pu1[G::RPT], pu2[G::RPT];
  double pacc[G::RPT];
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    pm2[i] = ld_ext<TZ>(w2, i, cx, eo, T.z0);
    pcf[i] = ld_ext<TZ>(cf, i, cx, eo, T.z0);
    int r, c;
    if (inj1 && ext_slot<TZ>(i, &r, &c)) INJ1[r][c] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < G::RPT; ++i) {
    const int z = T.z0 + wv * G::RPT + i;
    tcf[i] = ldp(cf, cx, z);
    if (IACC) {
      pu1[i] = ldp_nt(us1, cx, z);
      pu2[i] = ldp_nt(us2, cx, z);
      pacc[i] = ldp64(acc, cx8, z);
    }
    if (inj2) INJ2[wv * G::RPT + i][lane] = 0.f;
  }
  tile8_commit<TZ>(L1, tile);
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
    const int z = T.z0 - kHalo + r, xx = T.x0 - kHalo + c;
    float v = 0.f, incr = 0.f;
    if ((unsigned)z < (unsigned)nz && (unsigned)xx < (unsigned)nx) {
      const float* pc = &L1[r + kHalo][c + kHalo];
      const float w = pc[0];
      float lap = lap_ptr(pc, G::W1, a.c);
      if (inj1) lap += INJ1[r][c];
      const int dx = border_dist(xx, nx, a.nbl), dz = border_dist(z, nz, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
      incr = step_incr(w, pm2[i], pcf[i], lap, eta);
      v = (w + w - pm2[i]) + incr;
    }
    // body slots on tile rows: level j out, and its increment kept for the imaging
    if (i < G::NB && r >= kHalo && r < kHalo + TZ) {
      stb(ro1, v, cx, z * row4);
      INC1[r - kHalo][c - kHalo] = incr;
    }
    LE[r][c] = v;
  }
  __syncthreads();

  if (act2 && a.v != nullptr && a.tile_base + tid == S.src_tile && threadIdx.x == 0) {
    const int C = S.src_i - T.x0 + kHalo, R = S.src_k - T.z0 + kHalo;
    a.v[S.q + j - 1] = S.src_w[0] * LE[R][C] + S.src_w[1] * LE[R][C + 1] + S.src_w[2] * LE[R + 1][C] +
                       S.src_w[3] * LE[R + 1][C + 1];
  }
  // second step: level j-1 on the tile; imaging of both steps (every lane computes; outside
  // the grid the stores drop)
  const int dx = border_dist(x, nx, a.nbl);
  double* pa = IMG == kImgProbe ? reinterpret_cast<double*>(a.ws + S.store) + (long long)a.probe_r * S.npts
                                : nullptr;
  const float* pc1 = IMG == kImgProbe ? a.probe_c + j : nullptr;
  const float* pc2 = IMG == kImgProbe ? a.probe_c + j - 1 : nullptr;
#pragma unroll
  for (int i = 0; i < G::RPT; ++i) {
    const int lr = wv * G::RPT + i;
    const int z = T.z0 + lr;
    double ac = IACC ? pacc[i] : 0.0;
    if (IACC && act1) ac = ac + (double)pu1[i] * (double)INC1[lr][lane];
    float wj = 0.f, wn = 0.f;  // probe: levels j and j-1 on the tile
    if (act2) {
      const float* pc = &LE[lr + kHalo][lane + kHalo];
      const float w = pc[0];
      const float wm2 = L1[lr + 2 * kHalo][lane + 2 * kHalo];
      float lap = lap_ptr(pc, G::WE, a.c);
      if (inj2) lap += INJ2[lr][lane];
      const int dz = border_dist(z, nz, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
      const float incr = step_incr(w, wm2, tcf[i], lap, eta);
      stb(ro2, (w + w - wm2) + incr, cx, z * row4);
      if (IACC) ac = ac + (double)pu2[i] * (double)incr;
      if (IMG == kImgProbe) {
        wj = w;
        wn = (w + w - wm2) + incr;
      }
    } else if (IMG == kImgProbe) {
      wj = LE[lr + kHalo][lane + kHalo];
    }
    if (IACC) stb64(racc, ac, cx8, 2 * z * row4);
    if (IMG == kImgProbe && x < nx && z < nz) {
      // the same two FP64 additions, in the same order, as two one-level launches
      const long long p = (long long)z * px + x;
      probe_add(probe_sums(pa, p, a.probe_r), a.probe_r, pc1, (double)wj, act1, pc2, (double)wn, act2, a.probe_pitch);
    }
  }
}

// Born, two levels per launch: u and du at levels k and k+1 (k = step - off), each point with
// the arithmetic of born2d_kernel in the same order (so the results are bitwise those of two
// one-level launches); samples (J dm)^{k-1} and (J dm)^k.  Per two levels the launch reads
// u^{k-1}, u^{k-2}, du^{k-1}, du^{k-2}, coef and dm once and writes four levels: 40 B per point
// instead of 2 x 32.
template <int TZ>
__global__ __launch_bounds__(F2<TZ>::NT) void born2d2_kernel(StepArgs a) {
  using G = F2<TZ>;
  __shared__ float L1U[G::H1][G::W1];
  __shared__ float L1D[G::H1][G::W1];
  __shared__ float LEU[G::HE][G::WE];
  __shared__ float LED[G::HE][G::WE];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  const bool act1 = k >= 1 && k <= S.nt - 1;
  const bool act2 = k + 1 >= 1 && k + 1 <= S.nt - 1;
  if (!act1 && !act2) return;
  const int nx = S.nx, nz = S.nz, px = S.px;
  const int row4 = 4 * px;
  // levels below 1 are zero
  const Planes u1 = planes(fbuf(a.ws, S, fwd_buf(k - 1)), nz, k >= 2 ? nz : 0, row4);
  const Planes u2 = planes(fbuf(a.ws, S, fwd_buf(k - 2)), nz, k >= 3 ? nz : 0, row4);
  const Planes d1 = planes(fbuf(a.ws, S, adj_buf(k - 1)), nz, k >= 2 ? nz : 0, row4);
  const Planes d2 = planes(fbuf(a.ws, S, adj_buf(k - 2)), nz, k >= 3 ? nz : 0, row4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, row4);
  const Planes dmp = planes(a.dm + S.m, nz, nz, 4LL * nx);   // caller's layout: rows of nx
  // new levels k and k+1 (a level outside 1..nt-1 belongs to an inactive step: no records)
  const brsrc uo1 = make_rsrc(fbuf(a.ws, S, fwd_buf(k)), act1 ? nz * row4 : 0);
  const brsrc uo2 = make_rsrc(fbuf(a.ws, S, fwd_buf(k + 1)), act2 ? nz * row4 : 0);
  const brsrc do1 = make_rsrc(fbuf(a.ws, S, adj_buf(k)), act1 ? nz * row4 : 0);
  const brsrc do2 = make_rsrc(fbuf(a.ws, S, adj_buf(k + 1)), act2 ? nz * row4 : 0);
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int x = T.x0 + lane;
  const int cx = x < nx ? 4 * x : kOOB;

  // the two level k-1 tiles first, then the first step's other inputs on its extended points
  // (dm in the caller's rows of nx) and coef and dm of the tile points
  int ho[Side8<TZ>::NH];
  side_offsets<G::NT, G::H1, 2 * kHalo>(ho, nx, nz, px, T.x0, T.z0);
  Tile8<TZ> tu, td;
  tile8_issue<TZ>(tu, u1, cx, ho, T.z0);
  tile8_issue<TZ>(td, d1, cx, ho, T.z0);
  int eo[G::NH], eom[G::NH];
  ext_offsets<TZ>(eo, nx, nz, px, T.x0, T.z0);
  ext_offsets<TZ>(eom, nx, nz, nx, T.x0, T.z0);
  float pu2[G::NS], pd2[G::NS], pcf[G::NS], pdm[G::NS], tcf[G::RPT], tdm[G::RPT];
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    pu2[i] = ld_ext<TZ>(u2, i, cx, eo, T.z0);
    pd2[i] = ld_ext<TZ>(d2, i, cx, eo, T.z0);
    pcf[i] = ld_ext<TZ>(cf, i, cx, eo, T.z0);
    pdm[i] = ld_ext<TZ>(dmp, i, cx, eom, T.z0);
  }
#pragma unroll
  for (int i = 0; i < G::RPT; ++i) {
    tcf[i] = ldp(cf, cx, T.z0 + wv * G::RPT + i);
    tdm[i] = ldp(dmp, cx, T.z0 + wv * G::RPT + i);
  }
  tile8_commit<TZ>(L1U, tu);
  tile8_commit<TZ>(L1D, td);
  __syncthreads();

  if (act1 && a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += G::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      const int C = R.i - T.x0 + 2 * kHalo, Rw = R.k - T.z0 + 2 * kHalo;
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] =
          R.w[0] * L1D[Rw][C] + R.w[1] * L1D[Rw][C + 1] + R.w[2] * L1D[Rw + 1][C] + R.w[3] * L1D[Rw + 1][C + 1];
    }
  }
  const int src_i = S.src_i, src_k = S.src_k;   // in registers (see the forward kernel)
  const float sw0 = S.src_w[0], sw1 = S.src_w[1], sw2 = S.src_w[2], sw3 = S.src_w[3];
  auto src_weight = [&](int w) { return w == 0 ? sw0 : w == 1 ? sw1 : w == 2 ? sw2 : sw3; };
  // first step: levels k of u and du on the tile + 4-cell halo (zero outside the grid)
  const float q1 = act1 ? a.q[S.q + k - 1] : 0.f;
#pragma unroll
  for (int i = 0; i < G::NS; ++i) {
    int r, c;
    if (!ext_slot<TZ>(i, &r, &c)) continue;
    const int z = T.z0 - kHalo + r, xx = T.x0 - kHalo + c;
    float v = 0.f, vd = 0.f;
    if ((unsigned)z < (unsigned)nz && (unsigned)xx < (unsigned)nx) {
      const int dx = border_dist(xx, nx, a.nbl), dz = border_dist(z, nz, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
      const float* pc = &L1U[r + kHalo][c + kHalo];
      const float u = pc[0];
      float lap = lap_ptr(pc, G::W1, a.c);
      const int bx = xx - src_i, bz = z - src_k;
      if (act1 && (unsigned)bx < 2u && (unsigned)bz < 2u) lap += src_weight(bx + 2 * bz) * q1;
      const float incr = pcf[i] * (lap - eta * (u - pu2[i]));
      v = (u + u - pu2[i]) + incr;
      const float* pd = &L1D[r + kHalo][c + kHalo];
      const float du = pd[0];
      const float lapd = lap_ptr(pd, G::W1, a.c) - pdm[i] * incr * a.inv_dt2;
      const float incd = pcf[i] * (lapd - eta * (du - pd2[i]));
      vd = (du + du - pd2[i]) + incd;
    }
    // body slots on tile rows store levels k (wave-uniform condition; columns outside drop)
    if (i < G::NB && r >= kHalo && r < kHalo + TZ) {
      stb(uo1, v, cx, z * row4);
      stb(do1, vd, cx, z * row4);
    }
    LEU[r][c] = v;
    LED[r][c] = vd;
  }
  __syncthreads();

  if (act2 && a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += G::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      const int C = R.i - T.x0 + kHalo, Rw = R.k - T.z0 + kHalo;
      a.d[S.d + (long long)k * S.nrec + R.r] =
          R.w[0] * LED[Rw][C] + R.w[1] * LED[Rw][C + 1] + R.w[2] * LED[Rw + 1][C] + R.w[3] * LED[Rw + 1][C + 1];
    }
  }
  if (!act2) return;
  // second step: levels k+1 on the tile (every lane computes; stores outside the grid drop)
  const float q2 = a.q[S.q + k];
  const int dx = border_dist(x, nx, a.nbl);
#pragma unroll
  for (int i = 0; i < G::RPT; ++i) {
    const int lr = wv * G::RPT + i;
    const int z = T.z0 + lr;
    const int dz = border_dist(z, nz, a.nbl);
    const float eta = a.eta_dt * (float)(dx * dx + dz * dz);
    const float* pc = &LEU[lr + kHalo][lane + kHalo];
    const float u = pc[0];
    const float um2 = L1U[lr + 2 * kHalo][lane + 2 * kHalo];
    float lap = lap_ptr(pc, G::WE, a.c);
    const int bx = x - src_i, bz = z - src_k;
    if ((unsigned)bx < 2u && (unsigned)bz < 2u) lap += src_weight(bx + 2 * bz) * q2;
    const float incr = tcf[i] * (lap - eta * (u - um2));
    stb(uo2, (u + u - um2) + incr, cx, z * row4);
    const float* pd = &LED[lr + kHalo][lane + kHalo];
    const float du = pd[0];
    const float dm2 = L1D[lr + 2 * kHalo][lane + 2 * kHalo];
    const float lapd = lap_ptr(pd, G::WE, a.c) - tdm[i] * incr * a.inv_dt2;
    const float incd = tcf[i] * (lapd - eta * (du - dm2));
    stb(do2, (du + du - dm2) + incd, cx, z * row4);
  }
}

template <int TZ>
hipError_t fwd2d_tz(const StepArgs& a, int store, hipStream_t s) {
  switch (store) {
    case kStoreNone: fwd2d_kernel<TZ, kStoreNone><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kStoreF32: fwd2d_kernel<TZ, kStoreF32><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kStoreF32R: fwd2d_kernel<TZ, kStoreF32R><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kStoreBF16: fwd2d_kernel<TZ, kStoreBF16><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kStoreFP16: fwd2d_kernel<TZ, kStoreFP16><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    case kStoreProbe: fwd2d_kernel<TZ, kStoreProbe><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
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
    case kImgProbe: adj2d_kernel<TZ, kImgProbe><<<a.ntiles, T2<TZ>::NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TZ>
hipError_t fwd2d2_tz(const StepArgs& a, int store, hipStream_t s) {
  switch (store) {
    case kStoreNone: fwd2d2_kernel<TZ, kStoreNone><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    case kStoreF32: fwd2d2_kernel<TZ, kStoreF32><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    case kStoreProbe: fwd2d2_kernel<TZ, kStoreProbe><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TZ>
hipError_t adj2d2_tz(const StepArgs& a, hipStream_t s) {
  switch (a.image_src) {
    case kImgNone: adj2d2_kernel<TZ, kImgNone><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    case kImgFull32: adj2d2_kernel<TZ, kImgFull32><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    case kImgBuffers: adj2d2_kernel<TZ, kImgBuffers><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
    case kImgProbe: adj2d2_kernel<TZ, kImgProbe><<<a.ntiles, F2<TZ>::NT, 0, s>>>(a); break;
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
    case 24: return fwd2d2_tz<24>(a, store, s);
    case 32: return fwd2d2_tz<32>(a, store, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj2d2(const StepArgs& a, int tz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: return adj2d2_tz<8>(a, s);
    case 16: return adj2d2_tz<16>(a, s);
    case 24: return adj2d2_tz<24>(a, s);
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

hipError_t launch_born2d2(const StepArgs& a, int tz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (tz) {
    case 8: born2d2_kernel<8><<<a.ntiles, F2<8>::NT, 0, s>>>(a); break;
    case 16: born2d2_kernel<16><<<a.ntiles, F2<16>::NT, 0, s>>>(a); break;
    case 24: born2d2_kernel<24><<<a.ntiles, F2<24>::NT, 0, s>>>(a); break;
    case 32: born2d2_kernel<32><<<a.ntiles, F2<32>::NT, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
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
