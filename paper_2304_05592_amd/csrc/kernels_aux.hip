// Auxiliary gfx950 kernels: coefficients, fills, last-sample gathers, checkpoint slots
// with per-field scaling, the gradient reduction over shots and deterministic FP64
// reductions (residual / misfit, dot products).
#include "awe_internal.h"
#include "codec.h"

#include <cstdint>
#include <initializer_list>
#include <mutex>

namespace awe {

namespace {

__device__ __forceinline__ float* fbuf(unsigned char* ws, const ShotDev& S, int b) {
  return reinterpret_cast<float*>(ws + S.fld) + (long long)b * S.npts;
}

__device__ __forceinline__ float interp_global(const float* f, const ShotDev& S, int ndim, int i,
                                               int j, int k, const float* w) {
  const long long px = S.px, pxy = (long long)S.px * S.ny;
  const long long p = (long long)k * pxy + (long long)j * px + i;
  if (ndim == 2) {
    return w[0] * f[p] + w[1] * f[p + 1] + w[2] * f[p + px] + w[3] * f[p + px + 1];
  }
  return w[0] * f[p] + w[1] * f[p + 1] + w[2] * f[p + px] + w[3] * f[p + px + 1] +
         w[4] * f[p + pxy] + w[5] * f[p + pxy + 1] + w[6] * f[p + pxy + px] +
         w[7] * f[p + pxy + px + 1];
}

// m (rows of nx) -> coef = dt^2 / (m + eta dt / 2) (rows of px, 0 in the padding), computed
// in FP64 and rounded once.
__global__ void coef_kernel(const float* __restrict__ m, float* __restrict__ coef, int nx, int ny,
                            int nz, int px, int nbl, double dt, double amp_nbl2) {
  const long long n = (long long)px * ny * nz;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < n;
       p += (long long)gridDim.x * blockDim.x) {
    const long long row = p / px;
    const int i = (int)(p - row * px);
    if (i >= nx) {
      coef[p] = 0.f;
      continue;
    }
    const int j = (int)(row % ny);
    const int k = (int)(row / ny);
    const int dx = max(max(nbl - i, i - (nx - 1 - nbl)), 0);
    const int dy = ny > 1 ? max(max(nbl - j, j - (ny - 1 - nbl)), 0) : 0;
    const int dz = max(max(nbl - k, k - (nz - 1 - nbl)), 0);
    const double eta = amp_nbl2 * (double)(dx * dx + dy * dy + dz * dz);
    coef[p] = (float)(dt * dt / ((double)m[row * nx + i] + 0.5 * eta * dt));
  }
}

__global__ void fill_kernel(uint4* __restrict__ p, long long n16, unsigned char* tail, int ntail) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n16;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = z;
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ void gather_last_kernel(StepArgs a, int total, int adj) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const RecDev R = a.t.recs[t];
  const ShotDev& S = a.t.shots[R.shot];
  const int k = S.nt - 1;
  const float* f = fbuf(a.ws, S, adj ? adj_buf(k) : fwd_buf(k));
  a.d[S.d + (long long)k * S.nrec + R.r] = interp_global(f, S, a.ndim, R.i, R.j, R.k, R.w);
}

__global__ void src_last_kernel(StepArgs a, int nshot) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshot) return;
  const ShotDev& S = a.t.shots[s];
  const float* w1 = fbuf(a.ws, S, adj_buf(1));
  a.v[S.q] = interp_global(w1, S, a.ndim, S.src_i, S.src_j, S.src_k, S.src_w);
  a.v[S.q + S.nt - 1] = 0.f;
}

// Max |u| of the two fields of a state into scale[slot][0..1] (atomic max on the float bits
// of non-negative values, which is exact and order independent).
__global__ void absmax_kernel(StepArgs a, int slot, int state) {
  const ShotDev& S = a.t.shots[a.t.order[a.shot_base + blockIdx.y]];
  const int ls = state - S.off;
  const float* f = fbuf(a.ws, S, fwd_buf(ls - (int)blockIdx.z));
  float mx = 0.f;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < S.npts;
       p += (long long)gridDim.x * blockDim.x)
    mx = fmaxf(mx, fabsf(f[p]));
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  __shared__ float red[kThreads / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) mx = fmaxf(mx, red[w]);
    unsigned* sc = reinterpret_cast<unsigned*>(a.ws + S.scale) + 2 * slot + blockIdx.z;
    atomicMax(sc, __float_as_uint(mx));
  }
}

// dir 0: slot <- (u^state, u^{state-1}); dir 1: fields <- slot.  blockIdx.y = shot of the
// group (position shot_base + blockIdx.y in t.order), blockIdx.z = which of the two fields.
__global__ void slot_kernel(StepArgs a, int slot, int state, int dir) {
  const ShotDev& S = a.t.shots[a.t.order[a.shot_base + blockIdx.y]];
  const int fz = blockIdx.z;
  const int ls = state - S.off;
  float* f = fwd_level(a, S, ls - fz);  // store: the source may be a slot restored by reference
  const long long base = ((long long)slot * 2 + fz) * S.npts;
  const int prec = a.store_prec;
  float s = 1.f, inv = 1.f;
  if (prec != kFP32) {
    s = reinterpret_cast<const float*>(a.ws + S.scale)[2 * slot + fz];
    if (!(s > 0.f)) s = 1.f;
    inv = 1.f / s;
  }
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < S.npts;
       p += (long long)gridDim.x * blockDim.x) {
    if (prec == kFP32) {
      float* st = reinterpret_cast<float*>(a.ws + S.store) + base;
      if (dir == 0) st[p] = f[p]; else f[p] = st[p];
    } else {
      unsigned short* st = reinterpret_cast<unsigned short*>(a.ws + S.store) + base;
      if (dir == 0) {
        const float y = f[p] * inv;
        st[p] = enc16(y, prec == kBF16);
      } else {
        f[p] = dec16(st[p], prec == kBF16) * s;
      }
    }
  }
}

// u^{nt-1} -> FULL 16-bit store with its scale (the forward steps quantise u^1..u^{nt-2}).
__global__ void store_last_kernel(StepArgs a) {
  const ShotDev& S = a.t.shots[blockIdx.y];
  const int k = S.nt - 1;
  if (k < 1) return;
  const float* f = fbuf(a.ws, S, fwd_buf(k));
  const float inv = inv_scale(level_scale(reinterpret_cast<const float*>(a.ws + S.scale), k));
  unsigned short* st = reinterpret_cast<unsigned short*>(a.ws + S.store) + (long long)k * S.npts;
  const int bf = a.store_prec == kBF16;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < S.npts;
       p += (long long)gridDim.x * blockDim.x)
    st[p] = enc16(f[p] * inv, bf);
}

__global__ void grad_reduce_kernel(Tables t, unsigned char* ws, double* __restrict__ g,
                                   double scale) {
  const WinDev W = t.wins[blockIdx.y];
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < W.npts;
       p += (long long)gridDim.x * blockDim.x) {
    const long long row = p / W.px;
    const int i = (int)(p - row * W.px);
    if (i >= W.nx) continue;
    double s = 0.0;
    for (int k = 0; k < W.scount; ++k) {
      const ShotDev& S = t.shots[t.win_shots[W.sbegin + k]];
      s += reinterpret_cast<const double*>(ws + S.acc)[p];
    }
    g[W.m + row * W.nx + i] = scale * s;
  }
}

// Probed gradient: g = scale * sum over the window's shots (ascending) of sum_j s_j A_j B_j, with
// B_j, A_j the shot's FP64 probe sums [2][r][npts] at S.store.
__global__ void probe_reduce_kernel(Tables t, unsigned char* ws, int r, ProbeWeights w, double* __restrict__ g,
                                    double scale) {
  const WinDev W = t.wins[blockIdx.y];
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < W.npts;
       p += (long long)gridDim.x * blockDim.x) {
    const long long row = p / W.px;
    const int i = (int)(p - row * W.px);
    if (i >= W.nx) continue;
    double s = 0.0;
    for (int k = 0; k < W.scount; ++k) {
      const ShotDev& S = t.shots[t.win_shots[W.sbegin + k]];
      const double* B = reinterpret_cast<const double*>(ws + S.store);
      const double* A = B + (long long)r * S.npts;
      const long long o = ((p >> 6) * r) * 64 + (p & 63);  // sums of p: see probe_sums
      double e = 0.0;
      for (int j = 0; j < r; ++j) e += w.s[j] * (A[o + j * 64] * B[o + j * 64]);
      s += e;
    }
    g[W.m + row * W.nx + i] = scale * s;
  }
}

// Deterministic reduction: block b sums a fixed contiguous chunk in a fixed order, then one
// block sums the kReduceBlocks partials.
__device__ __forceinline__ double block_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __shared__ double red[kThreads / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  return s;
}

template <int KIND>  // 0 residual (r = a - b, sum r^2 / 2), 1 dot float, 2 dot double
__global__ void partial_kernel(const void* a_, const void* b_, float* r, long long n,
                               double* part) {
  const long long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double s = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    if (KIND == 0) {
      const float x = ((const float*)a_)[i] - ((const float*)b_)[i];
      if (r) r[i] = x;
      s += 0.5 * (double)x * (double)x;
    } else if (KIND == 1) {
      s += (double)((const float*)a_)[i] * (double)((const float*)b_)[i];
    } else {
      s += ((const double*)a_)[i] * ((const double*)b_)[i];
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void final_kernel(const double* part, int np, double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) *out = s;
}

// m = 1/v^2 and the chain rule gv = -2 gm / v^3 of the wavespeed parameterisation (FP64
// arithmetic, one rounding).
__global__ void slowness2_kernel(const float* __restrict__ v, float* __restrict__ m, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double x = v[i];
    m[i] = (float)(1.0 / (x * x));
  }
}

__global__ void velocity_grad_kernel(const float* v, const float* gm, float* gv, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double x = v[i];
    gv[i] = (float)(-2.0 * (double)gm[i] / (x * x * x));
  }
}

// Patchy saturation.  With P1 = rho vp^2 (brine rock), mu = P1 / 3, K1 = 5 P1 / 9 and
// r(K) = K / (k_min - K), Gassmann's fluid swap r(K2) = r(K1) + D / phi (D = r(k_co2) - r(k_brine))
// gives, with a = k_min - K1, B = K1 phi + D a and Q = k_min phi + D a:  K2 = k_min B / Q.  The
// CO2 rock's P-wave modulus is P2 = N / Q with N = k_min B + 4/9 P1 Q, the harmonic patchy mix is
// 1/M = Den / (P1 N) with Den = (1 - s) N + s Q P1, and vp_new^2 = M / rho_new, so
//     vp_new = vp sqrt(rho N / (rho_new Den)),
//     dvp_new/ds = -vp_new / 2 (phi drho Den + (Q P1 - N) rho_new) / (rho_new Den),
// one FP64 division and one square root per cell (drho = rho_co2 - rho_brine).
struct PatchyPre {
  double k_min, d, drho;
};

struct PatchyOut {
  double vp_new, rho_new, dvp;
};

template <bool kVjp>
__device__ __forceinline__ PatchyOut patchy_eval(double s, double v, double rho, double phi,
                                                 const PatchyPre& c) {
  const double p1 = 1e6 * rho * v * v;           // vp in km/s -> Pa
  const double a = c.k_min - (5.0 / 9.0) * p1;
  const double b = (5.0 / 9.0) * p1 * phi + c.d * a;
  const double q = c.k_min * phi + c.d * a;
  const double nn = c.k_min * b + (4.0 / 9.0) * p1 * q;
  const double den = (1.0 - s) * nn + s * q * p1;
  PatchyOut o;
  o.rho_new = rho + phi * s * c.drho;
  const double inv = 1.0 / (o.rho_new * den);
  o.vp_new = v * sqrt(rho * nn * inv);
  o.dvp = kVjp ? -0.5 * o.vp_new * (phi * c.drho * den + (q * p1 - nn) * o.rho_new) * inv : 0.0;
  return o;
}

// Streamed once: 16-byte nontemporal loads and stores (the arrays are not reused by the next
// kernel from the cache).
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 ld_nt4(const float* p, long long g) {
  return __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p) + g);
}

__device__ __forceinline__ void st_nt4(float* p, long long g, float a, float b, float c, float d) {
  const f32x4 v = {a, b, c, d};
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p) + g);
}

// Four cells per thread with 16-byte loads when every array is 16-byte aligned (VEC 4), else
// one cell per thread (VEC 1); one group per thread over a grid that covers the array (the
// stride loop only matters past 2^30 workgroups), the last n % VEC cells by the first threads.
template <int VEC>
__global__ void patchy_kernel(const float* __restrict__ s, const float* __restrict__ vp,
                              const float* __restrict__ rho, const float* __restrict__ phi,
                              float* __restrict__ vp_new, float* __restrict__ rho_new, long long n,
                              PatchyPre c) {
  const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long ng = n / VEC;
  for (long long g = tid; g < ng; g += stride) {
    if constexpr (VEC == 4) {
      const f32x4 S = ld_nt4(s, g), V = ld_nt4(vp, g), R = ld_nt4(rho, g), F = ld_nt4(phi, g);
      const PatchyOut o0 = patchy_eval<false>(S.x, V.x, R.x, F.x, c);
      const PatchyOut o1 = patchy_eval<false>(S.y, V.y, R.y, F.y, c);
      const PatchyOut o2 = patchy_eval<false>(S.z, V.z, R.z, F.z, c);
      const PatchyOut o3 = patchy_eval<false>(S.w, V.w, R.w, F.w, c);
      st_nt4(vp_new, g, (float)o0.vp_new, (float)o1.vp_new, (float)o2.vp_new, (float)o3.vp_new);
      if (rho_new)
        st_nt4(rho_new, g, (float)o0.rho_new, (float)o1.rho_new, (float)o2.rho_new, (float)o3.rho_new);
    } else {
      const PatchyOut o = patchy_eval<false>(s[g], vp[g], rho[g], phi[g], c);
      vp_new[g] = (float)o.vp_new;
      if (rho_new) rho_new[g] = (float)o.rho_new;
    }
  }
  const long long i = ng * VEC + tid;
  if (VEC > 1 && i < n) {
    const PatchyOut o = patchy_eval<false>(s[i], vp[i], rho[i], phi[i], c);
    vp_new[i] = (float)o.vp_new;
    if (rho_new) rho_new[i] = (float)o.rho_new;
  }
}

// g_s = g_vp dvp_new/ds + g_rho phi drho (g_rho may be null).
template <int VEC>
__global__ void patchy_vjp_kernel(const float* __restrict__ s, const float* __restrict__ vp,
                                  const float* __restrict__ rho, const float* __restrict__ phi,
                                  const float* __restrict__ g_vp, const float* __restrict__ g_rho,
                                  float* __restrict__ g_s, long long n, PatchyPre c) {
  const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long ng = n / VEC;
  auto one = [&](float sv, float vv, float rv, float fv, float gv, float gr) {
    const PatchyOut o = patchy_eval<true>(sv, vv, rv, fv, c);
    return (float)((double)gv * o.dvp + (double)gr * (double)fv * c.drho);
  };
  for (long long g = tid; g < ng; g += stride) {
    if constexpr (VEC == 4) {
      const f32x4 S = ld_nt4(s, g), V = ld_nt4(vp, g), R = ld_nt4(rho, g), F = ld_nt4(phi, g);
      const f32x4 G = ld_nt4(g_vp, g);
      const f32x4 H = g_rho ? ld_nt4(g_rho, g) : f32x4{0.f, 0.f, 0.f, 0.f};
      st_nt4(g_s, g, one(S.x, V.x, R.x, F.x, G.x, H.x), one(S.y, V.y, R.y, F.y, G.y, H.y),
             one(S.z, V.z, R.z, F.z, G.z, H.z), one(S.w, V.w, R.w, F.w, G.w, H.w));
    } else {
      g_s[g] = one(s[g], vp[g], rho[g], phi[g], g_vp[g], g_rho ? g_rho[g] : 0.f);
    }
  }
  const long long i = ng * VEC + tid;
  if (VEC > 1 && i < n) g_s[i] = one(s[i], vp[i], rho[i], phi[i], g_vp[i], g_rho ? g_rho[i] : 0.f);
}

PatchyPre patchy_pre(const PatchyConsts& c) {
  auto r = [&](double k) { return k / (c.k_min - k); };
  return {c.k_min, r(c.k_co2) - r(c.k_brine), c.rho_co2 - c.rho_brine};
}

// Workgroups covering `units` threads (capped at 2^30; kernels stride beyond that).
int grid_cover(long long units) {
  const long long b = (units + kThreads - 1) / kThreads;
  return (int)(b < 1 ? 1 : (b > (1LL << 30) ? (1LL << 30) : b));
}

bool aligned16(std::initializer_list<const void*> ps) {
  for (const void* p : ps)
    if (p && (reinterpret_cast<uintptr_t>(p) & 15u)) return false;
  return true;
}

int grid_for(long long n) {
  long long b = (n + kThreads - 1) / kThreads;
  return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

// Screening of a caller array: cnt[0] += values that are not finite, cnt[1] += finite values
// below lo.  Integer counts added with one atomic per workgroup, so they do not depend on the
// order in which workgroups run.
template <typename T>
__global__ void __launch_bounds__(kThreads) screen_kernel(const T* __restrict__ x, long long n,
                                                           double lo, unsigned long long* cnt) {
  unsigned long long bad = 0, low = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = (double)x[i];
    if (!__builtin_isfinite(v)) ++bad;
    else if (v < lo) ++low;
  }
  __shared__ unsigned long long red[2][kThreads / 64];
  for (int o = 32; o > 0; o >>= 1) {
    bad += __shfl_xor(bad, o, 64);
    low += __shfl_xor(low, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = bad;
    red[1][threadIdx.x >> 6] = low;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      bad += red[0][w];
      low += red[1][w];
    }
    if (bad) atomicAdd(cnt, bad);
    if (low) atomicAdd(cnt + 1, low);
  }
}

}  // namespace

hipError_t launch_coef(const float* m, unsigned char* ws, long long coef_off, long long m_off,
                       int nx, int ny, int nz, int px, int nbl, double h, double dt, double amp,
                       hipStream_t s) {
  (void)h;
  const long long n = (long long)px * ny * nz;
  const double amp_nbl2 = nbl > 0 ? amp / ((double)nbl * nbl) : 0.0;
  coef_kernel<<<grid_for(n), kThreads, 0, s>>>(m + m_off, reinterpret_cast<float*>(ws + coef_off),
                                                nx, ny, nz, px, nbl, dt, amp_nbl2);
  return hipGetLastError();
}

hipError_t launch_fill(unsigned char* ws, long long off, long long nbytes, hipStream_t s) {
  if (nbytes <= 0) return hipSuccess;
  // off is 16-byte aligned by construction of the workspace layout
  const long long n16 = nbytes / 16;
  const int ntail = (int)(nbytes - n16 * 16);
  fill_kernel<<<grid_for(n16), kThreads, 0, s>>>(reinterpret_cast<uint4*>(ws + off), n16,
                                                 ws + off + n16 * 16, ntail);
  return hipGetLastError();
}

hipError_t launch_screen(const float* x, long long n, double lo, unsigned long long* cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  screen_kernel<float><<<grid_for(n), kThreads, 0, s>>>(x, n, lo, cnt);
  return hipGetLastError();
}

hipError_t launch_screen(const double* x, long long n, double lo, unsigned long long* cnt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  screen_kernel<double><<<grid_for(n), kThreads, 0, s>>>(x, n, lo, cnt);
  return hipGetLastError();
}

hipError_t launch_gather_last(const StepArgs& a, int nshot, int total, int adj, hipStream_t s) {
  (void)nshot;
  if (total <= 0 || a.d == nullptr) return hipSuccess;
  gather_last_kernel<<<(total + kThreads - 1) / kThreads, kThreads, 0, s>>>(a, total, adj);
  return hipGetLastError();
}

hipError_t launch_src_last(const StepArgs& a, int nshot, hipStream_t s) {
  if (a.v == nullptr) return hipSuccess;
  src_last_kernel<<<(nshot + 63) / 64, 64, 0, s>>>(a, nshot);
  return hipGetLastError();
}

hipError_t launch_absmax(const StepArgs& a, int nshot, int slot, int state, hipStream_t s) {
  absmax_kernel<<<dim3(256, nshot, 2), kThreads, 0, s>>>(a, slot, state);
  return hipGetLastError();
}

hipError_t launch_slot(const StepArgs& a, int nshot, int slot, int state, int dir, hipStream_t s) {
  slot_kernel<<<dim3(512, nshot, 2), kThreads, 0, s>>>(a, slot, state, dir);
  return hipGetLastError();
}

hipError_t launch_store_last(const StepArgs& a, int nshot, long long max_npts, hipStream_t s) {
  store_last_kernel<<<dim3(grid_for(max_npts), nshot), kThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const Tables& t, int nwin, long long max_npts, unsigned char* ws,
                              double* g, double scale, hipStream_t s) {
  grad_reduce_kernel<<<dim3(grid_for(max_npts), nwin), kThreads, 0, s>>>(t, ws, g, scale);
  return hipGetLastError();
}

hipError_t launch_probe_reduce(const Tables& t, int nwin, long long max_npts, unsigned char* ws, int r,
                               const ProbeWeights& w, double* g, double scale, hipStream_t s) {
  probe_reduce_kernel<<<dim3(grid_for(max_npts), nwin), kThreads, 0, s>>>(t, ws, r, w, g, scale);
  return hipGetLastError();
}

hipError_t launch_slowness2(const float* v, float* m, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  slowness2_kernel<<<grid_for(n), kThreads, 0, s>>>(v, m, n);
  return hipGetLastError();
}

hipError_t launch_velocity_gradient(const float* v, const float* gm, float* gv, long long n,
                                    hipStream_t s) {
  if (n <= 0) return hipSuccess;
  velocity_grad_kernel<<<grid_for(n), kThreads, 0, s>>>(v, gm, gv, n);
  return hipGetLastError();
}

hipError_t launch_patchy(const float* s, const float* vp, const float* rho, const float* phi,
                         float* vp_new, float* rho_new, long long n, PatchyConsts c, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const PatchyPre pre = patchy_pre(c);
  if (aligned16({s, vp, rho, phi, vp_new, rho_new}))
    patchy_kernel<4><<<grid_cover(n / 4), kThreads, 0, st>>>(s, vp, rho, phi, vp_new, rho_new, n, pre);
  else
    patchy_kernel<1><<<grid_cover(n), kThreads, 0, st>>>(s, vp, rho, phi, vp_new, rho_new, n, pre);
  return hipGetLastError();
}

hipError_t launch_patchy_vjp(const float* s, const float* vp, const float* rho, const float* phi,
                             const float* g_vp, const float* g_rho, float* g_s, long long n,
                             PatchyConsts c, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const PatchyPre pre = patchy_pre(c);
  if (aligned16({s, vp, rho, phi, g_vp, g_rho, g_s}))
    patchy_vjp_kernel<4><<<grid_cover(n / 4), kThreads, 0, st>>>(s, vp, rho, phi, g_vp, g_rho, g_s, n, pre);
  else
    patchy_vjp_kernel<1><<<grid_cover(n), kThreads, 0, st>>>(s, vp, rho, phi, g_vp, g_rho, g_s, n, pre);
  return hipGetLastError();
}

// Scratch of the allocation-free residual entry point: the kReduceBlocks FP64 partial sums of
// the fixed reduction partition (8 KiB, whatever the length reduced).  The array exists once on
// every GPU the library runs on; host code uses the device address hipGetSymbolAddress returns
// for the current device (the array's name is a host-side stand-in), looked up on the first call
// on each device and kept.  Calls that overlap on one GPU share the array and race.
static __device__ __align__(256) double scratch[kScratchDoubles];
static_assert(kScratchDoubles >= kReduceBlocks, "the scratch holds one partial per reduction block");

namespace {
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;
}  // namespace

hipError_t scratch_partials(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_residual(const float* a, const float* b, float* r, long long n, double* loss,
                           unsigned char* ws, hipStream_t s) {
  double* part = reinterpret_cast<double*>(ws);
  partial_kernel<0><<<kReduceBlocks, kThreads, 0, s>>>(a, b, r, n, part);
  if (loss) final_kernel<<<1, kThreads, 0, s>>>(part, kReduceBlocks, loss);
  return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, long long n, double* out, unsigned char* ws,
                      hipStream_t s) {
  double* part = reinterpret_cast<double*>(ws);
  partial_kernel<1><<<kReduceBlocks, kThreads, 0, s>>>(a, b, nullptr, n, part);
  final_kernel<<<1, kThreads, 0, s>>>(part, kReduceBlocks, out);
  return hipGetLastError();
}

hipError_t launch_dotd(const double* a, const double* b, long long n, double* out,
                       unsigned char* ws, hipStream_t s) {
  double* part = reinterpret_cast<double*>(ws);
  partial_kernel<2><<<kReduceBlocks, kThreads, 0, s>>>(a, b, nullptr, n, part);
  final_kernel<<<1, kThreads, 0, s>>>(part, kReduceBlocks, out);
  return hipGetLastError();
}

}  // namespace awe
