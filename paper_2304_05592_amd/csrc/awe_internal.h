// Internal declarations shared by the host library and the gfx950 kernels.
//
// Workspace layout, device tables and kernel argument blocks.  All offsets into the
// caller's workspace are byte offsets; all offsets into caller arrays (m, q, d, ...)
// are element offsets as given in awe_shot.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace awe {

constexpr int kThreads = 256;   // 4 wave64 per workgroup
constexpr int kTX = 64;         // 2D tile width: one wavefront spans the tile row
constexpr int kHalo = 4;        // stencil radius (8th order)
constexpr int kPitch = 64;      // workspace rows are padded to a multiple of 64 elements, so
                                // that every 64-column row segment starts on a 256-byte line
inline int pitch_of(int nx) { return (nx + kPitch - 1) / kPitch * kPitch; }

// Field buffers of a shot: forward level n lives in buffer (n & 3), adjoint / Born-perturbation
// level n in buffer 4 + (n & 3).  A step producing level n reads levels n-1 and n-2 and writes
// a third buffer, so no launch writes a buffer it reads (also for negative n: -1 & 3 = 3).
constexpr int kFieldBufs = 8;
__host__ __device__ inline int fwd_buf(int n) { return n & 3; }
__host__ __device__ inline int adj_buf(int n) { return 4 + (n & 3); }
constexpr int kNoLevel = -(1 << 29);

// Storage precision of a kept wavefield.
enum Prec : int { kFP32 = 0, kBF16 = 1, kFP16 = 2 };

// Where the adjoint's imaging condition reads u^j: nowhere, the FULL store (FP32 / BF16 /
// FP16, the latter two scaled per level) or the recomputed forward buffers.
enum ImageSrc : int { kImgNone = 0, kImgFull32 = 1, kImgBuffers = 2, kImgFullBF16 = 3, kImgFullFP16 = 4,
                      kImgProbe = 5 };  // kImgProbe: A_j += C[j][level] w^level (probed gradient)

// Forward-step storage of each level: none, FP32 copy, or scaled BF16 / FP16 (the level is
// quantised one step later, once its max |u| is complete).
// kStoreProbe: B_j += C[j][level] (u^k - 2u^{k-1} + u^{k-2}) instead of a stored level (probed
// gradient; the second difference is the step's increment).
// kStoreF32R (2D one-level steps of a sweep without two-level launches): FP32 copy as kStoreF32,
// but the step reads its two previous levels back from the store instead of the rotating
// buffers, which then receive only the last level.
enum StoreKind : int { kStoreNone = 0, kStoreF32 = 1, kStoreBF16 = 2, kStoreFP16 = 3, kStoreProbe = 4,
                       kStoreF32R = 5 };

// Probed gradient: at most this many probes; a shot's sums are 2 r FP64 values per point at
// ShotDev::store, B (forward second differences) first, then A (adjoint levels), each in the
// blocked layout of probe_sums.
constexpr int kMaxProbes = 64;

// Per-shot description as the kernels read it.
struct ShotDev {
  int nx, ny, nz;          // computational grid (ny = 1 in 2D)
  int px;                  // row pitch of every workspace field (multiple of kPitch >= nx)
  int nt;                  // local samples
  int off;                 // global state index of the shot's local state 0 (end-aligned)
  int nrec;
  long long npts;          // px * ny * nz (workspace field size, padding included)
  long long coef;          // byte offset of the window's FP32 coefficient array
  long long fld;           // byte offset of field buffer 0; buffer b at fld + b * npts * 4 (b < kFieldBufs)
  long long acc;           // byte offset of the FP64 gradient accumulator (-1: none)
  long long store;         // byte offset of the kept wavefield (FULL: [nt][npts]; CHECKPOINT: [nslots][2][npts])
  long long scale;         // byte offset of FP32 per-field scales (FULL: [nt]; CHECKPOINT: [nslots][2])
  long long m;             // element offset of the window in m, dm, g
  long long q;             // element offset in q and v
  long long d;             // element offset in d and dd
  int src_i, src_j, src_k; // base node of the source (x, y, z indices)
  int src_tile;            // tile index owning the source base node
  float src_w[8];          // interpolation weight / h^ndim; corner = bx + 2 by + 4 bz (2D: bx + 2 bz)
};

// A tile of one shot: 2D = [z0, z0 + TZ) x [x0, x0 + 64); 3D = z-block x xy-tile.
struct TileDev {
  int shot;
  int x0, y0, z0;
  int gat_begin, gat_count;  // receivers whose base node lies in this tile
  int inj_begin, inj_count;  // points of this tile touched by receivers (adjoint injection)
  int ext_begin, ext_count;  // touched points of the tile + 4-cell halo (2D two-step adjoint)
};

// One receiver: column r of the shot's traces, base node and weights.
struct RecDev {
  int shot;
  int r;
  int i, j, k;
  int pad;
  float w[8];                // corner = bx + 2 by + 4 bz (2D: bx + 2 bz)
};

// A grid point touched by receivers: tile-local coordinates and its CSR entry range.
struct InjPoint {
  int shot;
  int lx, ly, lz;
  int e_begin, e_count;
  long long p;               // flat point index in the shot's workspace fields (rows of px)
};

struct InjEntry {
  int r;                     // receiver column within the shot
  float w;                   // interpolation weight
};

// A model window and the shots that run on it (ascending shot order in win_shots).
struct WinDev {
  long long m;               // element offset in m, dm, g (rows of nx)
  long long npts;            // px * ny * nz (coefficient / accumulator layout)
  int nx, px;
  int sbegin, scount;
};

// Device tables of a plan (one allocation, pointers into it).
struct Tables {
  const ShotDev* shots;
  const TileDev* tiles;
  const RecDev* recs;        // all receivers, grouped by gather tile
  const InjPoint* inj_pts;
  const InjPoint* ext_pts;   // per tile: touched points of its 4-cell extended region (2D)
  const InjEntry* inj_ent;
  const WinDev* wins;
  const int* win_shots;
  const int* order;          // shots sorted by time offset; a group is a contiguous range
};

// Arguments of one time-step launch.
struct StepArgs {
  Tables t;
  unsigned char* ws;         // workspace base
  const float* q;            // source wavelets (forward / born)
  float* d;                  // traces out (forward: d; born: J dm); may be null
  const float* dd;           // data residual in (adjoint)
  float* v;                  // F^T dd out (adjoint); may be null
  const float* dm;           // model perturbation (born)
  int ndim;
  int step;                  // global index of the state being produced
  int ntiles;                // tiles in this launch (active prefix of the group's tiles)
  int tile_base;             // first tile of the shot group this launch covers
  int shot_base;             // first position in t.order of the group (per-shot kernels)
  int rs_level;              // global state restored by reference from FP32 slot rs_slot
  int rs_slot;               //   (kNoLevel: none); see fwd_level
  int st_slot;               // 2D forward: also write (u^k, u^{k-1}) into this FP32 slot (-1: no)
  int nbl;
  int store_prec;            // Prec of the kept wavefield (FULL store / checkpoint slots)
  int image_src;             // adjoint imaging source, see ImageSrc
  float c[5];                // stencil weights / h^2
  float eta_dt;              // damping amplitude / (nbl^2 dt): eta/dt = eta_dt * (dx^2 + dy^2 + dz^2)
  float inv_dt2;             // 1 / dt^2 (Born source)
  const float* probe_c;      // probed gradient: coefficients [probe_r][probe_pitch], column = local level
  int probe_r, probe_pitch;
};

// Forward level k (local index) of shot S.  After a checkpoint restore of global state n from
// an FP32 slot, levels n and n - 1 are read from the slot itself until the next restore (no
// copy); every other level lives in the shot's four rotating forward buffers.
__device__ __forceinline__ float* fwd_level(const StepArgs& a, const ShotDev& S, int k) {
  const int d = a.rs_level - (k + S.off);
  if ((unsigned)d < 2u)
    return reinterpret_cast<float*>(a.ws + S.store) + ((long long)a.rs_slot * 2 + d) * S.npts;
  return reinterpret_cast<float*>(a.ws + S.fld) + (long long)fwd_buf(k) * S.npts;
}

// Probed gradient sums, FP64, r per point: blocks of 64 consecutive points (rows are padded to a
// multiple of 64, so a block is the 64 columns a wave updates), each block holding its points'
// sum 0, then sum 1, ...  The sum j of point p lies at ((p / 64) r + j) 64 + p % 64: a wave reads
// sum j of its 64 points as one contiguous 512-byte run, and its r sums as one 512 r-byte range.
static_assert(kPitch % 64 == 0, "probe-sum blocks of 64 points need rows padded to a multiple of 64");
__device__ __forceinline__ double* probe_sums(double* region, long long p, int r) {
  return region + ((p >> 6) * r) * 64 + (p & 63);
}

// For j < r, sum[64 j] += c1[j * pitch] * v1 (when t1), then += c2[j * pitch] * v2 (when t2),
// in FP64 (each product of two floats is exact, so the order of the two additions alone fixes
// the result); sum from probe_sums.  The sums are read in groups of kProbeGroup before any of
// them is written back (the loads of a group are in flight together instead of each waiting for
// the store before it), and since they are read and written once per launch and outgrow the
// caches, both accesses are nontemporal.
constexpr int kProbeGroup = 8;
__device__ __forceinline__ void probe_add(double* sum, int r, const float* c1, double v1, bool t1,
                                          const float* c2, double v2, bool t2, long long pitch) {
  for (int j0 = 0; j0 < r; j0 += kProbeGroup) {
    double t[kProbeGroup];
    const int n = r - j0 < kProbeGroup ? r - j0 : kProbeGroup;
    double* s = sum + j0 * 64;
#pragma unroll
    for (int u = 0; u < kProbeGroup; ++u)
      if (u < n) t[u] = __builtin_nontemporal_load(s + u * 64);
#pragma unroll
    for (int u = 0; u < kProbeGroup; ++u)
      if (u < n) {
        if (t1) t[u] += (double)c1[(j0 + u) * pitch] * v1;
        if (t2) t[u] += (double)c2[(j0 + u) * pitch] * v2;
      }
#pragma unroll
    for (int u = 0; u < kProbeGroup; ++u)
      if (u < n) __builtin_nontemporal_store(t[u], s + u * 64);
  }
}

// Launchers (defined in the .hip files).  All enqueue on `stream`.
hipError_t launch_coef(const float* m, unsigned char* ws, long long coef_off, long long m_off,
                       int nx, int ny, int nz, int px, int nbl, double h, double dt, double amp,
                       hipStream_t stream);
hipError_t launch_fill(unsigned char* ws, long long off, long long nbytes, hipStream_t stream);
// Add to cnt[0] the values of x[0, n) that are not finite and to cnt[1] the finite ones below lo.
hipError_t launch_screen(const float* x, long long n, double lo, unsigned long long* cnt, hipStream_t stream);
hipError_t launch_screen(const double* x, long long n, double lo, unsigned long long* cnt, hipStream_t stream);
hipError_t launch_fwd2d(const StepArgs& a, int tz, int store, hipStream_t stream);
// Quantise the last forward level u^{nt-1} of every shot into the scaled FULL store.
hipError_t launch_store_last(const StepArgs& a, int nshot, long long max_npts, hipStream_t stream);
hipError_t launch_adj2d(const StepArgs& a, int tz, hipStream_t stream);
// Two 2D steps per launch (levels step, step+1 forward; step, step-1 adjoint); tz 8, 16 or 32.
hipError_t launch_fwd2d2(const StepArgs& a, int tz, int store, hipStream_t stream);
hipError_t launch_adj2d2(const StepArgs& a, int tz, hipStream_t stream);
hipError_t launch_born2d(const StepArgs& a, int tz, hipStream_t stream);
// Two Born steps per launch (levels step, step+1); tz 8, 16, 24 or 32.
hipError_t launch_born2d2(const StepArgs& a, int tz, hipStream_t stream);
hipError_t launch_fwd3d(const StepArgs& a, int ty, int bz, int store, hipStream_t stream);
hipError_t launch_adj3d(const StepArgs& a, int ty, int bz, hipStream_t stream);
hipError_t launch_born3d(const StepArgs& a, int ty, int bz, hipStream_t stream);
// Receiver injection over the touched points [first, first + count) (one shot group).
hipError_t launch_inj3d(const StepArgs& a, int first, int count, hipStream_t stream);
// Gather the last sample d^{nt-1} of every shot from the forward (adj = 0) or the
// perturbation (adj = 1, Born) buffers.
hipError_t launch_gather_last(const StepArgs& a, int nshot, int total_recs, int adj, hipStream_t stream);
// v^0 = R(x_s) w^1 / h^ndim and v^{nt-1} = 0 for every shot.
hipError_t launch_src_last(const StepArgs& a, int nshot, hipStream_t stream);
// Checkpoint slot copies: dir 0 = store (fields -> slot), 1 = restore (slot -> fields).
hipError_t launch_slot(const StepArgs& a, int nshot, int slot, int state, int dir, hipStream_t stream);
hipError_t launch_absmax(const StepArgs& a, int nshot, int slot, int state, hipStream_t stream);
// g[window] = scale * sum over the window's shots (ascending) of their FP64 accumulators.
hipError_t launch_grad_reduce(const Tables& t, int nwin, long long max_npts, unsigned char* ws,
                              double* g, double scale, hipStream_t stream);
// Probed gradient: g[window] = scale * sum over the window's shots (ascending) of
// sum_j s[j] A_j B_j, in FP64.
struct ProbeWeights {
  double s[kMaxProbes];
};
hipError_t launch_probe_reduce(const Tables& t, int nwin, long long max_npts, unsigned char* ws, int r,
                               const ProbeWeights& w, double* g, double scale, hipStream_t stream);
hipError_t launch_slowness2(const float* v, float* m, long long n, hipStream_t stream);
hipError_t launch_velocity_gradient(const float* v, const float* gm, float* gv, long long n,
                                    hipStream_t stream);
struct PatchyConsts {
  double k_min, k_brine, k_co2, rho_co2, rho_brine;
};
hipError_t launch_patchy(const float* s, const float* vp, const float* rho, const float* phi,
                         float* vp_new, float* rho_new, long long n, PatchyConsts c, hipStream_t stream);
hipError_t launch_patchy_vjp(const float* s, const float* vp, const float* rho, const float* phi,
                             const float* g_vp, const float* g_rho, float* g_s, long long n,
                             PatchyConsts c, hipStream_t stream);
hipError_t launch_residual(const float* a, const float* b, float* r, long long n, double* loss,
                           unsigned char* ws, hipStream_t stream);
hipError_t launch_dot(const float* a, const float* b, long long n, double* out, unsigned char* ws,
                      hipStream_t stream);
hipError_t launch_dotd(const double* a, const double* b, long long n, double* out,
                       unsigned char* ws, hipStream_t stream);
constexpr int kReduceBlocks = 1024;
// Device address (current GPU) of the library's static reduction scratch of kScratchDoubles
// FP64 values, for the allocation-free residual entry point.
constexpr int kScratchDoubles = 1024;
hipError_t scratch_partials(double** out);

}  // namespace awe
