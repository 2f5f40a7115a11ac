// 3D time-step kernels for gfx950: forward, adjoint with imaging, Born, and the adjoint's
// receiver injection.
//
// A workgroup (4 x wave64) owns a 64 x TY column block of (x, y) and marches along z over
// [z0, z0 + bz).  Each thread keeps a 9-deep register queue of its columns' values along z
// (one new plane read per step, coalesced 256-byte rows), writes the current plane into a
// double-buffered LDS tile and reads the x/y neighbours (4-cell halo) from there: one
// barrier per plane.  Arithmetic is the increment form of the 2D kernels (see
// kernels2d.hip).  Receivers whose base node lies in the block are sampled from the
// previous level (read-only during the step); the adjoint's receiver injection is a
// separate pass over the touched points (launch_inj3d), applied after the step.
//
// Field planes are read and written through buffer resources (bufio.h): a lane's byte offset
// within a plane is fixed for the whole march (kOOB for a point outside the grid, whose loads
// then read 0 and whose stores are dropped) and the plane's offset is wave-uniform, so the
// march spends no vector instructions on addresses, clamps or masks, and points outside the
// grid cost no memory traffic.  Fields that a block reads only at its own points (u^{k-2},
// coef, the accumulator) and the new level are streamed with nontemporal accesses: a 3D
// step's working set exceeds the last-level cache, and keeping these streams out of the caches
// leaves them to the neighbour planes and halos that are re-read.
#include "awe_internal.h"
#include "bufio.h"
#include "codec.h"

namespace awe {

namespace {

__device__ __forceinline__ int xcd_tile(int bid, int n) {
  const int q = n >> 3, r = n & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}

__device__ __forceinline__ int border_dist(int i, int n, int nbl) {
  return max(max(nbl - i, i - (n - 1 - nbl)), 0);
}

__device__ __forceinline__ float* fbuf(unsigned char* ws, const ShotDev& S, int b) {
  return reinterpret_cast<float*>(ws + S.fld) + (long long)b * S.npts;
}

__device__ __forceinline__ float interp8(const float* f, const ShotDev& S, int i, int j, int k,
                                         const float* w) {
  const long long px = S.px, pxy = (long long)S.px * S.ny;
  const long long p = (long long)k * pxy + (long long)j * px + i;
  return w[0] * f[p] + w[1] * f[p + 1] + w[2] * f[p + px] + w[3] * f[p + px + 1] +
         w[4] * f[p + pxy] + w[5] * f[p + pxy + 1] + w[6] * f[p + pxy + px] +
         w[7] * f[p + pxy + px + 1];
}

// Column block 64 x TY: 4 waves up to TY = 8, 8 waves for TY = 16 (two y-rows per thread).
template <int TY>
struct T3 {
  static constexpr int NW = TY >= 16 ? 8 : 4;  // waves per workgroup
  static constexpr int NT = 64 * NW;           // threads per workgroup
  static constexpr int W = kTX + 2 * kHalo;    // 72
  static constexpr int H = TY + 2 * kHalo;
  static constexpr int NC = TY / NW;           // y-rows per thread
  static_assert(TY % NW == 0, "block rows must split evenly over the waves");
};

// Halo ring of one plane: rows y0-4..y0+TY+3 x columns x0-4..x0+67 minus the 64 x TY
// centre; element e < COUNT maps to one ring position.  Each thread fetches PER elements
// into registers (so the loads can be issued a plane ahead) and later stores them to LDS.
template <int TY>
struct Ring {
  static constexpr int W = T3<TY>::W;
  static constexpr int COUNT = 8 * W + TY * 8;
  static constexpr int PER = (COUNT + T3<TY>::NT - 1) / T3<TY>::NT;
};

template <int TY>
__device__ __forceinline__ void ring_pos(int e, int* r, int* c) {
  constexpr int W = T3<TY>::W;
  if (e < 8 * W) {
    const int band = e / W;
    *c = e - band * W;
    *r = band < 4 ? band : TY + band;          // rows 0..3 and TY+4..TY+7
  } else {
    const int e2 = e - 8 * W;
    const int cc = e2 & 7;
    *r = kHalo + (e2 >> 3);                    // rows 4..TY+3
    *c = cc < 4 ? cc : kTX + cc;               // columns 0..3 and 68..71
  }
}

// Per-lane plane offsets of this thread's ring elements (kOOB outside the grid or past the ring).
template <int TY>
__device__ __forceinline__ void ring_offsets(int (&rv)[Ring<TY>::PER], int nx, int ny, int px, int x0,
                                             int y0) {
#pragma unroll
  for (int i = 0; i < Ring<TY>::PER; ++i) {
    const int e0 = threadIdx.x + i * T3<TY>::NT;
    const int e = e0 < Ring<TY>::COUNT ? e0 : Ring<TY>::COUNT - 1;
    int r, c;
    ring_pos<TY>(e, &r, &c);
    rv[i] = e0 < Ring<TY>::COUNT ? col_off(x0 - kHalo + c, y0 - kHalo + r, nx, ny, px, 4) : kOOB;
  }
}

template <int TY>
__device__ __forceinline__ void ring_fetch(float (&h)[Ring<TY>::PER], const Planes& f,
                                           const int (&rv)[Ring<TY>::PER], int z) {
#pragma unroll
  for (int i = 0; i < Ring<TY>::PER; ++i) h[i] = ldp(f, rv[i], z);
}

template <int TY>
__device__ __forceinline__ void ring_store(float (*P)[T3<TY>::W], const float (&h)[Ring<TY>::PER]) {
#pragma unroll
  for (int i = 0; i < Ring<TY>::PER; ++i) {
    const int e = threadIdx.x + i * T3<TY>::NT;
    if (e < Ring<TY>::COUNT) {
      int r, c;
      ring_pos<TY>(e, &r, &c);
      P[r][c] = h[i];
    }
  }
}

template <int TY>
__device__ __forceinline__ float lap3(const float (*P)[T3<TY>::W], const float* q, int ly, int lx,
                                      const float* c) {
  const int R = ly + kHalo, C = lx + kHalo;
  const float u = q[4];
  float s = 0.f;
#pragma unroll
  for (int r = kHalo; r >= 1; --r) {
    s += c[r] * ((P[R][C - r] - u) + (P[R][C + r] - u));
    s += c[r] * ((P[R - r][C] - u) + (P[R + r][C] - u));
    s += c[r] * ((q[4 - r] - u) + (q[4 + r] - u));
  }
  return s;
}

// ------------------------------------------------------------------------------ forward
// Software-pipelined z-march: after the barrier of plane z each thread issues the global
// loads of plane z+2 (halo ring, next queue value, u^{k-2}, coef), updates plane z from LDS
// buffer b and its register queue, then writes plane z+1 (loaded one plane earlier) into
// buffer 1-b.
template <int TY, int SK>
// Six waves per SIMD (at most 80 VGPRs) for the step and its stores: the z-march is bound by the
// latency of its plane loads, and the register budget costs no spills; the probe kind, with its
// sums in flight, keeps the compiler's own budget.
__global__ __launch_bounds__(T3<TY>::NT) __attribute__((amdgpu_waves_per_eu(SK == kStoreProbe ? 4 : 6, 8)))
void fwd3d_kernel(StepArgs a, int bzlen) {
  constexpr int NC = T3<TY>::NC, HP = Ring<TY>::PER;
  __shared__ float P[2][T3<TY>::H][T3<TY>::W];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  if (k < 1 || k >= S.nt) return;
  const int nx = S.nx, ny = S.ny, nz = S.nz, px = S.px;
  const long long plane4 = 4LL * px * ny;
  // levels below 1 are zero (initial state) and are not read: after a checkpoint restore of a
  // state before this shot's start their buffers may hold older levels
  const float* u1p = fwd_level(a, S, k - 1);
  const Planes u1 = planes(u1p, nz, k >= 2 ? nz : 0, plane4);
  const Planes u2 = planes(fwd_level(a, S, k - 2), nz, k >= 3 ? nz : 0, plane4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, plane4);
  const brsrc rout = make_rsrc(fbuf(a.ws, S, fwd_buf(k)), (int)(nz * plane4));
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int x = T.x0 + lane;
  const int zend = bzlen >= nz - T.z0 ? nz : T.z0 + bzlen;

  if (a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += T3<TY>::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] = k >= 2 ? interp8(u1p, S, R.i, R.j, R.k, R.w) : 0.f;
    }
  }
  const float qk = a.q[S.q + k - 1];
  const int dx = border_dist(x, nx, a.nbl);
  // shot fields used inside the z-march, copied to registers: stores could alias the shot
  // table as far as the compiler knows, and reloading them would wait for every load in flight
  const int src_i = S.src_i, src_j = S.src_j, src_k = S.src_k;
  float srcw[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) srcw[i] = S.src_w[i];
  auto src_weight = [&](int i) {
    float w = srcw[0];
#pragma unroll
    for (int t = 1; t < 8; ++t) w = i == t ? srcw[t] : w;
    return w;
  };
  // FULL store: level k (FP32) or level k-1 (16 bits, quantised once its scale is complete)
  constexpr bool S16 = SK == kStoreBF16 || SK == kStoreFP16;
  const brsrc rst = SK == kStoreF32
      ? make_rsrc(reinterpret_cast<float*>(a.ws + S.store) + (long long)k * S.npts, (int)(nz * plane4))
      : make_rsrc_uniform(reinterpret_cast<unsigned short*>(a.ws + S.store) + (long long)(k - 1) * S.npts,
                          S16 ? (int)(nz * plane4 / 2) : 0);
  float* scl = S16 ? reinterpret_cast<float*>(a.ws + S.scale) : nullptr;
  const float inv_prev = S16 && k >= 2 ? inv_scale(level_scale(scl, k - 1)) : 0.f;
  // probed gradient: the r FP64 sums B_j of this shot, and this level's coefficients
  double* pb = SK == kStoreProbe ? reinterpret_cast<double*>(a.ws + S.store) : nullptr;
  const float* pcol = SK == kStoreProbe ? a.probe_c + k : nullptr;
  const long long plane_pts = (long long)px * ny;
  float lmax = 0.f;

  // per-lane plane offsets (fixed for the march): own columns (4- and 2-byte elements), ring
  int cv[NC], cv2[NC], rv[HP];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int y = T.y0 + g * NC + c;
    cv[c] = col_off(x, y, nx, ny, px, 4);
    cv2[c] = col_off(x, y, nx, ny, px, 2);
  }
  ring_offsets<TY>(rv, nx, ny, px, T.x0, T.y0);

  // Register state of plane z: queue Q (u^{k-1} at z-4..z+4), u^{k-2} and coef.  Set A holds
  // the loads of plane z+1 (issued one plane earlier), set B those of plane z+2 (issued right
  // after the barrier of plane z): two planes of loads are in flight while plane z is updated.
  float Q[NC][9], pu2[NC], pcf[NC];
  float hA[HP] = {}, qA[NC] = {}, u2A[NC] = {}, cfA[NC] = {};
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int t = 0; t < 9; ++t) Q[c][t] = ldp(u1, cv[c], T.z0 - kHalo + t);
    pu2[c] = ldp(u2, cv[c], T.z0);
    pcf[c] = ldp(cf, cv[c], T.z0);
  }
  {
    float h[HP];
    ring_fetch<TY>(h, u1, rv, T.z0);
#pragma unroll
    for (int c = 0; c < NC; ++c) P[0][g * NC + c + kHalo][lane + kHalo] = Q[c][4];
    ring_store<TY>(P[0], h);
  }
  if (T.z0 + 1 < zend) {
    ring_fetch<TY>(hA, u1, rv, T.z0 + 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      qA[c] = ldp(u1, cv[c], T.z0 + 1 + kHalo);
      u2A[c] = ldp_nt(u2, cv[c], T.z0 + 1);
      cfA[c] = ldp_nt(cf, cv[c], T.z0 + 1);
    }
  }
  // One plane: hN.. hold the loads of plane z+1 (issued one plane earlier) and are consumed at
  // the end; hL.. receive the loads of plane z+2.  The loop runs two planes per trip with the
  // two register sets swapping roles, so no register that a load is still filling is copied
  // (a copy would make every plane wait for the loads just issued).
  float hB[HP] = {}, qB[NC] = {}, u2B[NC] = {}, cfB[NC] = {};
  auto plane = [&](int z, float (&hN)[HP], float (&qN)[NC], float (&u2N)[NC], float (&cfN)[NC],
                   float (&hL)[HP], float (&qL)[NC], float (&u2L)[NC], float (&cfL)[NC]) {
    const int b = (z - T.z0) & 1;
    __syncthreads();
    // loads of plane z+2, unconditional (beyond the block they are simply not used)
    ring_fetch<TY>(hL, u1, rv, z + 2);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      qL[c] = ldp(u1, cv[c], z + 2 + kHalo);
      u2L[c] = ldp_nt(u2, cv[c], z + 2);
      cfL[c] = ldp_nt(cf, cv[c], z + 2);
    }
    const int dz = border_dist(z, nz, a.nbl);
    const int zo = z * (int)plane4;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      // every lane computes; the stores of points outside the grid are dropped (offset kOOB)
      const int ly = g * NC + c;
      const int y = T.y0 + ly;
      float lap = lap3<TY>(P[b], Q[c], ly, lane, a.c);
      const int bx = x - src_i, by = y - src_j, bzz = z - src_k;
      if ((unsigned)bx < 2u && (unsigned)by < 2u && (unsigned)bzz < 2u)
        lap += src_weight(bx + 2 * by + 4 * bzz) * qk;
      const int dy = border_dist(y, ny, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dy * dy + dz * dz);
      const float u = Q[c][4];
      const float incr = pcf[c] * (lap - eta * (u - pu2[c]));
      const float un = (u + u - pu2[c]) + incr;
      stb_nt(rout, un, cv[c], zo);
      if (SK == kStoreF32) stb_nt(rst, un, cv[c], zo);
      if (S16) {
        // outside the grid u, u^{k-2} and coef read 0, so un = 0 there
        lmax = fmaxf(lmax, fabsf(un));
        if (k >= 2) stb16_nt(rst, enc16(u * inv_prev, SK == kStoreBF16), cv2[c], zo / 2);
      }
      if (SK == kStoreProbe && cv[c] != kOOB) {
        // u^k - 2u^{k-1} + u^{k-2} = incr (increment form of the step)
        const long long p = z * plane_pts + (cv[c] >> 2);
        probe_add(probe_sums(pb, p, a.probe_r), a.probe_r, pcol, (double)incr, true, nullptr, 0.0, false, a.probe_pitch);
      }
    }
    if (z + 1 < zend) {
      // plane z+1 into the other LDS buffer (every wave has passed the barrier of plane z, so
      // nobody still reads the plane z-1 it held); advance the register state
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        P[1 - b][g * NC + c + kHalo][lane + kHalo] = Q[c][5];
#pragma unroll
        for (int t = 0; t < 8; ++t) Q[c][t] = Q[c][t + 1];
        Q[c][8] = qN[c];
        pu2[c] = u2N[c];
        pcf[c] = cfN[c];
      }
      ring_store<TY>(P[1 - b], hN);
    }
  };
  // the prologue's loads complete before the march, so the loop head only ever sees the loads
  // of the previous trip in flight
  __builtin_amdgcn_s_waitcnt(0);
  for (int z = T.z0; z < zend; z += 2) {
    plane(z, hA, qA, u2A, cfA, hB, qB, u2B, cfB);
    if (z + 1 < zend) plane(z + 1, hB, qB, u2B, cfB, hA, qA, u2A, cfA);
  }
  if (S16) block_max_to_slot(lmax, scl, k);
}

// ------------------------------------------------------------------------------ adjoint
template <int TY, int IMG>
__global__ __launch_bounds__(T3<TY>::NT) void adj3d_kernel(StepArgs a, int bzlen) {
  constexpr int NC = T3<TY>::NC, HP = Ring<TY>::PER;
  __shared__ float P[2][T3<TY>::H][T3<TY>::W];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int j = a.step - S.off;
  if (j < 1 || j >= S.nt) return;
  const int nx = S.nx, ny = S.ny, nz = S.nz, px = S.px;
  const long long plane4 = 4LL * px * ny;
  const float* w1p = fbuf(a.ws, S, adj_buf(j + 1));
  const Planes w1 = planes(w1p, nz, nz, plane4);
  const Planes w2 = planes(fbuf(a.ws, S, adj_buf(j + 2)), nz, nz, plane4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, plane4);
  const brsrc rout = make_rsrc(fbuf(a.ws, S, adj_buf(j)), (int)(nz * plane4));
  // imaging: u^j from the FULL store (FP32, or 16 bits with the level's scale) or the forward
  // buffers, and the FP64 accumulator
  const void* ubase = IMG == kImgBuffers ? (const void*)fwd_level(a, S, j)
                      : IMG == kImgFull32 ? (const void*)(reinterpret_cast<const float*>(a.ws + S.store) + (long long)j * S.npts)
                      : (const void*)(reinterpret_cast<const unsigned short*>(a.ws + S.store) + (long long)j * S.npts);
  constexpr bool I16 = IMG == kImgFullBF16 || IMG == kImgFullFP16;
  constexpr bool IACC = IMG != kImgNone && IMG != kImgProbe;  // imaging into the FP64 accumulator
  const Planes uj = planes(ubase, nz, IACC ? nz : 0, I16 ? plane4 / 2 : plane4);
  const float usc = I16 ? level_scale(reinterpret_cast<const float*>(a.ws + S.scale), j) : 1.f;
  const Planes acc = planes(a.ws + S.acc, nz, IACC ? nz : 0, 2 * plane4);
  const brsrc racc = make_rsrc(a.ws + S.acc, IACC ? (int)(nz * 2 * plane4) : 0);
  // probed gradient: the r FP64 sums A_j of this shot (after its B_j), and this level's
  // coefficients; receiver injection adds its part afterwards (inj3d_kernel)
  double* pa = IMG == kImgProbe ? reinterpret_cast<double*>(a.ws + S.store) + (long long)a.probe_r * S.npts : nullptr;
  const float* pcol = IMG == kImgProbe ? a.probe_c + j : nullptr;
  const long long plane_pts = (long long)px * ny;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int x = T.x0 + lane;
  const int zend = bzlen >= nz - T.z0 ? nz : T.z0 + bzlen;

  if (a.v != nullptr && a.tile_base + tid == S.src_tile && threadIdx.x == 0)
    a.v[S.q + j] = interp8(w1p, S, S.src_i, S.src_j, S.src_k, S.src_w);
  const int dx = border_dist(x, nx, a.nbl);

  // per-lane plane offsets (fixed for the march): own columns for 4-, 2- and 8-byte elements, ring
  int cv[NC], cvu[NC], cv8[NC], rv[HP];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int y = T.y0 + g * NC + c;
    cv[c] = col_off(x, y, nx, ny, px, 4);
    cvu[c] = col_off(x, y, nx, ny, px, I16 ? 2 : 4);
    cv8[c] = col_off(x, y, nx, ny, px, 8);
  }
  ring_offsets<TY>(rv, nx, ny, px, T.x0, T.y0);

  // imaging inputs of one point: u^j and the accumulator (0 outside the grid)
  auto load_img = [&](int c, int z, float* u, double* ac) {
    if (I16) *u = dec16(ldp16_nt(uj, cvu[c], z), IMG == kImgFullBF16) * usc;
    else if (IMG == kImgFull32) *u = ldp_nt(uj, cvu[c], z);
    else if (IACC) *u = ldp(uj, cvu[c], z);
    if (IACC) *ac = ldp64_nt(acc, cv8[c], z);
  };

  // Register state of plane z (queue of w^{j+1}, w^{j+2}, coef, u^j, accumulator); set A holds
  // plane z+1, set B plane z+2 (loads issued right after the barrier of plane z).
  float Q[NC][9], pw2[NC], pcf[NC], pu[NC];
  double pacc[NC];
  float hA[HP] = {}, qA[NC] = {}, w2A[NC] = {}, cfA[NC] = {}, uA[NC] = {};
  double accA[NC] = {};
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int t = 0; t < 9; ++t) Q[c][t] = ldp(w1, cv[c], T.z0 - kHalo + t);
    pw2[c] = ldp(w2, cv[c], T.z0);
    pcf[c] = ldp(cf, cv[c], T.z0);
    pu[c] = 0.f;
    pacc[c] = 0.0;
    load_img(c, T.z0, &pu[c], &pacc[c]);
  }
  {
    float h[HP];
    ring_fetch<TY>(h, w1, rv, T.z0);
#pragma unroll
    for (int c = 0; c < NC; ++c) P[0][g * NC + c + kHalo][lane + kHalo] = Q[c][4];
    ring_store<TY>(P[0], h);
  }
  if (T.z0 + 1 < zend) {
    ring_fetch<TY>(hA, w1, rv, T.z0 + 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      qA[c] = ldp(w1, cv[c], T.z0 + 1 + kHalo);
      w2A[c] = ldp_nt(w2, cv[c], T.z0 + 1);
      cfA[c] = ldp_nt(cf, cv[c], T.z0 + 1);
      load_img(c, T.z0 + 1, &uA[c], &accA[c]);
    }
  }
  // Two planes per trip with the register sets swapping roles (see the forward kernel).
  float hB[HP] = {}, qB[NC] = {}, w2B[NC] = {}, cfB[NC] = {}, uB[NC] = {};
  double accB[NC] = {};
  auto plane = [&](int z, float (&hN)[HP], float (&qN)[NC], float (&w2N)[NC], float (&cfN)[NC],
                   float (&uN)[NC], double (&accN)[NC], float (&hL)[HP], float (&qL)[NC],
                   float (&w2L)[NC], float (&cfL)[NC], float (&uL)[NC], double (&accL)[NC]) {
    const int b = (z - T.z0) & 1;
    __syncthreads();
    ring_fetch<TY>(hL, w1, rv, z + 2);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      qL[c] = ldp(w1, cv[c], z + 2 + kHalo);
      w2L[c] = ldp_nt(w2, cv[c], z + 2);
      cfL[c] = ldp_nt(cf, cv[c], z + 2);
      load_img(c, z + 2, &uL[c], &accL[c]);
    }
    const int dz = border_dist(z, nz, a.nbl);
    const int zo = z * (int)plane4;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      // every lane computes; the stores of points outside the grid are dropped (offset kOOB)
      const int ly = g * NC + c;
      const int y = T.y0 + ly;
      const float lap = lap3<TY>(P[b], Q[c], ly, lane, a.c);
      const int dy = border_dist(y, ny, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dy * dy + dz * dz);
      const float w = Q[c][4];
      const float incr = pcf[c] * (lap - eta * (w - pw2[c]));
      const float wn = (w + w - pw2[c]) + incr;
      stb_nt(rout, wn, cv[c], zo);
      if (IACC) stb64_nt(racc, pacc[c] + (double)pu[c] * (double)incr, cv8[c], 2 * zo);
      if (IMG == kImgProbe && cv[c] != kOOB) {
        const long long p = z * plane_pts + (cv[c] >> 2);
        probe_add(probe_sums(pa, p, a.probe_r), a.probe_r, pcol, (double)wn, true, nullptr, 0.0, false, a.probe_pitch);
      }
    }
    if (z + 1 < zend) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        P[1 - b][g * NC + c + kHalo][lane + kHalo] = Q[c][5];
#pragma unroll
        for (int t = 0; t < 8; ++t) Q[c][t] = Q[c][t + 1];
        Q[c][8] = qN[c];
        pw2[c] = w2N[c];
        pcf[c] = cfN[c];
        pu[c] = uN[c];
        pacc[c] = accN[c];
      }
      ring_store<TY>(P[1 - b], hN);
    }
  };
  __builtin_amdgcn_s_waitcnt(0);   // see the forward kernel
  for (int z = T.z0; z < zend; z += 2) {
    plane(z, hA, qA, w2A, cfA, uA, accA, hB, qB, w2B, cfB, uB, accB);
    if (z + 1 < zend) plane(z + 1, hB, qB, w2B, cfB, uB, accB, hA, qA, w2A, cfA, uA, accA);
  }
}

// Receiver injection after the adjoint step: w^j += coef P_r^T dd^j at the touched points
// (and the matching imaging term).  One thread per touched point, entries in fixed order.
__global__ void inj3d_kernel(StepArgs a, int first, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int t = first + i;
  const InjPoint Pt = a.t.inj_pts[t];
  const ShotDev& S = a.t.shots[Pt.shot];
  const int j = a.step - S.off;
  if (j < 1 || j >= S.nt) return;
  const float* ddj = a.dd + S.d + (long long)j * S.nrec;
  float s = 0.f;
  for (int e = 0; e < Pt.e_count; ++e) {
    const InjEntry E = a.t.inj_ent[Pt.e_begin + e];
    s += E.w * ddj[E.r];
  }
  const float add = reinterpret_cast<const float*>(a.ws + S.coef)[Pt.p] * s;
  float* w = fbuf(a.ws, S, adj_buf(j));
  w[Pt.p] += add;
  if (a.image_src == kImgProbe) {
    // A_j holds C[j][level] times the step's value before injection: add C[j][level] times the
    // injected part (the sums are linear in w^j)
    double* pa = reinterpret_cast<double*>(a.ws + S.store) + (long long)a.probe_r * S.npts;
    probe_add(probe_sums(pa, Pt.p, a.probe_r), a.probe_r, a.probe_c + j, (double)add, true, nullptr, 0.0, false, a.probe_pitch);
  } else if (a.image_src) {
    float u;
    if (a.image_src == kImgFull32)
      u = reinterpret_cast<const float*>(a.ws + S.store)[(long long)j * S.npts + Pt.p];
    else if (a.image_src == kImgBuffers)
      u = fwd_level(a, S, j)[Pt.p];
    else
      u = dec16(reinterpret_cast<const unsigned short*>(a.ws + S.store)[(long long)j * S.npts + Pt.p],
                a.image_src == kImgFullBF16) *
          level_scale(reinterpret_cast<const float*>(a.ws + S.scale), j);
    double* acc = reinterpret_cast<double*>(a.ws + S.acc);
    acc[Pt.p] += (double)u * (double)add;
  }
}

// ------------------------------------------------------------------------------ Born
template <int TY>
__global__ __launch_bounds__(T3<TY>::NT) void born3d_kernel(StepArgs a, int bzlen) {
  constexpr int NC = T3<TY>::NC, HP = Ring<TY>::PER;
  __shared__ float PU[2][T3<TY>::H][T3<TY>::W];
  __shared__ float PD[2][T3<TY>::H][T3<TY>::W];
  const int tid = xcd_tile(blockIdx.x, a.ntiles);
  const TileDev T = a.t.tiles[a.tile_base + tid];
  const ShotDev& S = a.t.shots[T.shot];
  const int k = a.step - S.off;
  if (k < 1 || k >= S.nt) return;
  const int nx = S.nx, ny = S.ny, nz = S.nz, px = S.px;
  const long long plane4 = 4LL * px * ny;
  const Planes u1 = planes(fbuf(a.ws, S, fwd_buf(k - 1)), nz, nz, plane4);
  const Planes u2 = planes(fbuf(a.ws, S, fwd_buf(k - 2)), nz, nz, plane4);
  const float* d1p = fbuf(a.ws, S, adj_buf(k - 1));
  const Planes d1 = planes(d1p, nz, nz, plane4);
  const Planes d2 = planes(fbuf(a.ws, S, adj_buf(k - 2)), nz, nz, plane4);
  const Planes cf = planes(a.ws + S.coef, nz, nz, plane4);
  const Planes dm = planes(a.dm + S.m, nz, nz, 4LL * nx * ny);   // caller's layout: rows of nx
  const brsrc ruo = make_rsrc(fbuf(a.ws, S, fwd_buf(k)), (int)(nz * plane4));
  const brsrc rdo = make_rsrc(fbuf(a.ws, S, adj_buf(k)), (int)(nz * plane4));
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int x = T.x0 + lane;
  const int zend = bzlen >= nz - T.z0 ? nz : T.z0 + bzlen;

  if (a.d != nullptr) {
    for (int t = threadIdx.x; t < T.gat_count; t += T3<TY>::NT) {
      const RecDev R = a.t.recs[T.gat_begin + t];
      a.d[S.d + (long long)(k - 1) * S.nrec + R.r] = interp8(d1p, S, R.i, R.j, R.k, R.w);
    }
  }
  const float qk = a.q[S.q + k - 1];
  const int dx = border_dist(x, nx, a.nbl);
  const int src_i = S.src_i, src_j = S.src_j, src_k = S.src_k;   // kept in registers (see fwd3d)
  const float w0 = S.src_w[0], w1 = S.src_w[1], w2 = S.src_w[2], w3 = S.src_w[3];
  const float w4 = S.src_w[4], w5 = S.src_w[5], w6 = S.src_w[6], w7 = S.src_w[7];
  auto src_weight = [=](int i) {
    return i == 0 ? w0 : i == 1 ? w1 : i == 2 ? w2 : i == 3 ? w3 : i == 4 ? w4 : i == 5 ? w5 : i == 6 ? w6 : w7;
  };
  int cv[NC], cvm[NC], rv[HP];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int y = T.y0 + g * NC + c;
    cv[c] = col_off(x, y, nx, ny, px, 4);
    cvm[c] = col_off(x, y, nx, ny, nx, 4);
  }
  ring_offsets<TY>(rv, nx, ny, px, T.x0, T.y0);

  float QU[NC][9], QD[NC][9], pu2[NC], pd2[NC], pcf[NC], pdm[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      QU[c][t] = ldp(u1, cv[c], T.z0 - kHalo + t);
      QD[c][t] = ldp(d1, cv[c], T.z0 - kHalo + t);
    }
    pu2[c] = ldp(u2, cv[c], T.z0);
    pd2[c] = ldp(d2, cv[c], T.z0);
    pcf[c] = ldp(cf, cv[c], T.z0);
    pdm[c] = ldp(dm, cvm[c], T.z0);
  }
  {
    float hu[HP], hd[HP];
    ring_fetch<TY>(hu, u1, rv, T.z0);
    ring_fetch<TY>(hd, d1, rv, T.z0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      PU[0][g * NC + c + kHalo][lane + kHalo] = QU[c][4];
      PD[0][g * NC + c + kHalo][lane + kHalo] = QD[c][4];
    }
    ring_store<TY>(PU[0], hu);
    ring_store<TY>(PD[0], hd);
  }
  for (int z = T.z0; z < zend; ++z) {
    const int b = (z - T.z0) & 1;
    __syncthreads();
    const bool more = z + 1 < zend;
    float hu[HP], hd[HP], qun[NC], qdn[NC], nu2[NC], nd2[NC], ncf[NC], ndm[NC];
    if (more) {
      ring_fetch<TY>(hu, u1, rv, z + 1);
      ring_fetch<TY>(hd, d1, rv, z + 1);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        qun[c] = ldp(u1, cv[c], z + 1 + kHalo);
        qdn[c] = ldp(d1, cv[c], z + 1 + kHalo);
        nu2[c] = ldp(u2, cv[c], z + 1);
        nd2[c] = ldp(d2, cv[c], z + 1);
        ncf[c] = ldp(cf, cv[c], z + 1);
        ndm[c] = ldp(dm, cvm[c], z + 1);
      }
    }
    const int dz = border_dist(z, nz, a.nbl);
    const int zo = z * (int)plane4;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      // every lane computes; the stores of points outside the grid are dropped (offset kOOB)
      const int y = T.y0 + g * NC + c;
      const int ly = g * NC + c;
      const int dy = border_dist(y, ny, a.nbl);
      const float eta = a.eta_dt * (float)(dx * dx + dy * dy + dz * dz);
      float lap = lap3<TY>(PU[b], QU[c], ly, lane, a.c);
      const int bx = x - src_i, by = y - src_j, bzz = z - src_k;
      if ((unsigned)bx < 2u && (unsigned)by < 2u && (unsigned)bzz < 2u)
        lap += src_weight(bx + 2 * by + 4 * bzz) * qk;
      const float u = QU[c][4];
      const float incr = pcf[c] * (lap - eta * (u - pu2[c]));
      stb(ruo, (u + u - pu2[c]) + incr, cv[c], zo);
      const float du = QD[c][4];
      const float lapd = lap3<TY>(PD[b], QD[c], ly, lane, a.c) - pdm[c] * incr * a.inv_dt2;
      const float incd = pcf[c] * (lapd - eta * (du - pd2[c]));
      stb(rdo, (du + du - pd2[c]) + incd, cv[c], zo);
    }
    if (more) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        PU[1 - b][g * NC + c + kHalo][lane + kHalo] = QU[c][5];
        PD[1 - b][g * NC + c + kHalo][lane + kHalo] = QD[c][5];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          QU[c][t] = QU[c][t + 1];
          QD[c][t] = QD[c][t + 1];
        }
        QU[c][8] = qun[c];
        QD[c][8] = qdn[c];
        pu2[c] = nu2[c];
        pd2[c] = nd2[c];
        pcf[c] = ncf[c];
        pdm[c] = ndm[c];
      }
      ring_store<TY>(PU[1 - b], hu);
      ring_store<TY>(PD[1 - b], hd);
    }
  }
}

template <int TY>
hipError_t fwd3d_ty(const StepArgs& a, int bz, int store, hipStream_t s) {
  switch (store) {
    case kStoreNone: fwd3d_kernel<TY, kStoreNone><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kStoreF32: fwd3d_kernel<TY, kStoreF32><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kStoreBF16: fwd3d_kernel<TY, kStoreBF16><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kStoreFP16: fwd3d_kernel<TY, kStoreFP16><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kStoreProbe: fwd3d_kernel<TY, kStoreProbe><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TY>
hipError_t adj3d_ty(const StepArgs& a, int bz, hipStream_t s) {
  switch (a.image_src) {
    case kImgNone: adj3d_kernel<TY, kImgNone><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kImgFull32: adj3d_kernel<TY, kImgFull32><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kImgBuffers: adj3d_kernel<TY, kImgBuffers><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kImgFullBF16: adj3d_kernel<TY, kImgFullBF16><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kImgFullFP16: adj3d_kernel<TY, kImgFullFP16><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    case kImgProbe: adj3d_kernel<TY, kImgProbe><<<a.ntiles, T3<TY>::NT, 0, s>>>(a, bz); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// bz <= 0 means one block spans the whole depth of every shot.
static int zlen(int bz) { return bz > 0 ? bz : 0x7fffffff; }

hipError_t launch_fwd3d(const StepArgs& a, int ty, int bz, int store, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (ty) {
    case 4: return fwd3d_ty<4>(a, zlen(bz), store, s);
    case 8: return fwd3d_ty<8>(a, zlen(bz), store, s);
    case 16: return fwd3d_ty<16>(a, zlen(bz), store, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adj3d(const StepArgs& a, int ty, int bz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (ty) {
    case 4: return adj3d_ty<4>(a, zlen(bz), s);
    case 8: return adj3d_ty<8>(a, zlen(bz), s);
    case 16: return adj3d_ty<16>(a, zlen(bz), s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_born3d(const StepArgs& a, int ty, int bz, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  switch (ty) {
    case 4: born3d_kernel<4><<<a.ntiles, T3<4>::NT, 0, s>>>(a, zlen(bz)); break;
    case 8: born3d_kernel<8><<<a.ntiles, T3<8>::NT, 0, s>>>(a, zlen(bz)); break;
    case 16: born3d_kernel<16><<<a.ntiles, T3<16>::NT, 0, s>>>(a, zlen(bz)); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_inj3d(const StepArgs& a, int first, int count, hipStream_t s) {
  if (count <= 0 || a.dd == nullptr) return hipSuccess;  // no residual: nothing to inject
  inj3d_kernel<<<(count + kThreads - 1) / kThreads, kThreads, 0, s>>>(a, first, count);
  return hipGetLastError();
}

}  // namespace awe
