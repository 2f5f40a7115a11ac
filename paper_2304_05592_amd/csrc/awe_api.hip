// Host side of the awe C ABI: validation, geometry tables, tiling, workspace layout and the
// time loops (forward, reverse sweep with stored or recomputed wavefield, Born).
//
// Time axes of shots with different nt are aligned at their ends: shot s's local state n
// is the global state n + off_s with off_s = max_nt - nt_s.  A launch for global step n
// covers the tiles of the shots with off_s < n, which are a prefix of the tile list
// because shots are ordered by off_s.  Every shot then runs its own nt - 1 steps, and one
// checkpoint schedule over max_nt - 1 global steps serves all shots.
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "awe.h"
#include "awe_internal.h"
#include "codec.h"
#include "schedule.h"

using awe::InjEntry;
using awe::InjPoint;
using awe::RecDev;
using awe::ShotDev;
using awe::TileDev;
using awe::WinDev;
using awe::kHalo;

namespace {

thread_local std::string g_err;

awe_status fail(awe_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

awe_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return AWE_ERR_HIP;
}

#define AWE_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

constexpr double kStencil[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

long long align256(long long x) { return (x + 255) & ~255LL; }

}  // namespace

// Everything that depends on the launch shape: the tile list, the per-tile receiver and
// injection lists, the shot groups' tile ranges and the device tables.  A plan keeps one for its
// forward solves (and Born modelling) and one for its adjoint steps (reverse sweeps and F^T), so
// that each direction runs the tile shape that suits its kernel.
struct Tiling {
  int tz = 32;            // 2D tile rows
  int ty = 8, bz = 0;     // 3D tile rows in y and z-block length
  std::vector<TileDev> tiles;
  std::vector<int> src_tile;        // per shot: tile owning the source base node
  // group g owns tiles [g_tile0[g], g_tile0[g + 1]); g_active[g][n] of them (a prefix) belong
  // to shots with off < n; its touched points are inj_pts[g_inj0[g] .. + g_ninj[g])
  std::vector<int> g_tile0, g_inj0, g_ninj;
  std::vector<std::vector<int>> g_active;
  std::vector<RecDev> recs;
  std::vector<InjPoint> inj_pts;
  std::vector<InjPoint> ext_pts;
  std::vector<InjEntry> inj_ent;
  void* dev = nullptr;
  awe::Tables tab{};
};

struct awe_plan {
  int ndim = 2, nbl = 0;
  double h = 0, dt = 0, vmax = 0, vref = 0, R = 1e-3;
  awe_storage store{};    // the storage in effect (AUTO resolved to FULL or CHECKPOINT)
  awe_storage store_req{};  // the storage asked for
  int checks = 0;         // awe_plan_set_checks flags
  unsigned long long* chk_dev = nullptr;  // screening counters (2 per screened array)
  int nshot = 0, max_nt = 0, nsteps = 0;
  int fuse2 = 0;          // 2D: two time levels per launch where the storage allows
                          // (bit 0: forward solves, bit 1: reverse sweeps)
  Tiling fw, rv;          // launch shapes of forward solves / adjoint steps
  std::vector<awe_shot> shots;
  std::vector<double> rec_pos;    // copy of the problem's receiver rows
  std::vector<ShotDev> sd;
  // Shot groups: consecutive shots of `order` (sorted by time offset) that run their whole
  // time loop before the next group starts, so that a step's working set stays in the
  // last-level cache.
  std::vector<int> order;
  std::vector<int> g_shot0, g_nshot;
  int groups_req = 0;             // 0: automatic
  int cur = 0;                    // group of the launches being issued
  // per group: the state restored by reference (FP32 slots) when its actions stopped
  std::vector<int> g_rs_level, g_rs_slot;
  std::vector<WinDev> wins;
  std::vector<int> win_shots;
  std::vector<int> shot_win;      // window of each shot
  std::vector<long long> win_coef;
  std::vector<int> win_dims;
  long long max_win_npts = 0;
  int total_recs = 0;
  size_t ws_bytes = 0;
  long long fields_off = 0, fields_bytes = 0, acc_off = 0, acc_bytes = 0;
  std::vector<int32_t> sched;
  size_t sched_first_reverse = 0;
  const void* kept_ws = nullptr;
  float c[5] = {0, 0, 0, 0, 0};
  float eta_dt = 0.f;
  double amp = 0.0;
  // kernel timing
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_cls;
  std::vector<long long> prof_cnt;  // launches inside each timed interval
  bool prof_in_run = false;         // inside a timed run of steps (see ProfRun)
  long long prof_run_launches = 0;
  size_t prof_next = 0;
  int prof_stride = 1;
  long long prof_seen = 0;
};

namespace {

// Automatic shot groups: three FP32 fields of every shot of a group (the working set of one
// step) within about 160 MB, well inside the 256 MB last-level cache, and at least 8 M points
// per launch so that a launch still fills the chip.
constexpr long long kGroupBytes = 160LL << 20;
constexpr long long kMinGroupPoints = 8LL << 20;

struct Interp {
  int base[3];     // x, y, z base node
  double w[8];     // corner = bx + 2 by + 4 bz
};

// Bilinear / trilinear weights of a physical position on a window's computational grid.
bool interp(const awe_plan* P, const awe_shot& s, const double* pos, Interp* out) {
  const int n[3] = {s.nx, s.ny, s.nz};
  double f[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) {
    if (a == 1 && P->ndim == 2) {
      out->base[a] = 0;
      continue;
    }
    const double g = pos[a] / P->h + P->nbl;
    const double fl = std::floor(g);
    if (!(fl >= 0.0) || fl > n[a] - 2) return false;
    out->base[a] = (int)fl;
    f[a] = g - fl;
  }
  const int nc = P->ndim == 2 ? 4 : 8;
  for (int c = 0; c < 8; ++c) out->w[c] = 0.0;
  for (int c = 0; c < nc; ++c) {
    const int bx = c & 1;
    const int by = P->ndim == 2 ? 0 : (c >> 1) & 1;
    const int bz = P->ndim == 2 ? (c >> 1) & 1 : (c >> 2) & 1;
    const double w = (bx ? f[0] : 1 - f[0]) * (P->ndim == 3 ? (by ? f[1] : 1 - f[1]) : 1.0) *
                     (bz ? f[2] : 1 - f[2]);
    out->w[c] = w;
  }
  return true;
}

// Corner offsets (dx, dy, dz) of corner c.
void corner(int ndim, int c, int* dx, int* dy, int* dz) {
  *dx = c & 1;
  if (ndim == 2) {
    *dy = 0;
    *dz = (c >> 1) & 1;
  } else {
    *dy = (c >> 1) & 1;
    *dz = (c >> 2) & 1;
  }
}

// Shot order (by time offset, stable) and shot groups balanced by points; source positions.
awe_status build_groups(awe_plan* P) {
  std::vector<int> order(P->nshot);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return P->sd[a].off < P->sd[b].off; });
  P->order = order;
  long long pts = 0;
  for (int s : order) pts += P->sd[s].npts;
  int ng = P->groups_req;
  if (ng <= 0) {
    const long long bytes = 12 * pts;  // three FP32 fields per point touched by every step
    ng = (int)((bytes + kGroupBytes - 1) / kGroupBytes);
    ng = (int)std::min<long long>(ng, std::max<long long>(1, pts / kMinGroupPoints));
  }
  ng = std::max(1, std::min(ng, P->nshot));
  P->g_shot0.assign(1, 0);
  long long acc = 0;
  for (int i = 0; i < P->nshot; ++i) {
    const int g = (int)P->g_shot0.size() - 1;
    acc += P->sd[order[i]].npts;
    // close group g once it holds its share of the points, or when every later group
    // needs one of the remaining shots
    const int later_groups = ng - (g + 1), later_shots = P->nshot - (i + 1);
    if (later_groups > 0 && (later_shots == later_groups ||
                             (acc * ng >= pts * (g + 1) && later_shots >= later_groups)))
      P->g_shot0.push_back(i + 1);
  }
  const int G = (int)P->g_shot0.size();
  P->g_nshot.assign(G, 0);
  for (int g = 0; g < G; ++g) P->g_nshot[g] = (g + 1 < G ? P->g_shot0[g + 1] : P->nshot) - P->g_shot0[g];
  const double hd = std::pow(P->h, P->ndim);
  for (int s = 0; s < P->nshot; ++s) {
    Interp I;
    if (!interp(P, P->shots[s], P->shots[s].src, &I))
      return fail(AWE_ERR_GEOMETRY, "source of shot " + std::to_string(s) +
                                        " lies outside its computational grid");
    ShotDev& d = P->sd[s];
    d.src_i = I.base[0];
    d.src_j = I.base[1];
    d.src_k = I.base[2];
    for (int c = 0; c < 8; ++c) d.src_w[c] = (float)(I.w[c] / hd);
  }
  return AWE_OK;
}

// Tiles of every shot (in shot order) for the launch shape of T, the groups' tile ranges, and
// the per-tile receiver gather lists and injection CSR.
awe_status build_tiling(awe_plan* P, Tiling& T) {
  const int nd = P->ndim;
  const std::vector<int>& order = P->order;
  T.tiles.clear();
  std::vector<int> first_tile(P->nshot), ntx(P->nshot), nty(P->nshot), ntz(P->nshot);
  const int TY = nd == 2 ? 1 : T.ty;
  auto tz_of = [&](int s) { return nd == 2 ? T.tz : (T.bz > 0 ? T.bz : P->shots[s].nz); };
  for (int s : order) {
    const awe_shot& sh = P->shots[s];
    const int TZ = tz_of(s);
    ntx[s] = (sh.nx + awe::kTX - 1) / awe::kTX;
    nty[s] = nd == 2 ? 1 : (sh.ny + TY - 1) / TY;
    ntz[s] = (sh.nz + TZ - 1) / TZ;
    first_tile[s] = (int)T.tiles.size();
    for (int kz = 0; kz < ntz[s]; ++kz)
      for (int ky = 0; ky < nty[s]; ++ky)
        for (int kx = 0; kx < ntx[s]; ++kx) {
          TileDev t{};
          t.shot = s;
          t.x0 = kx * awe::kTX;
          t.y0 = ky * TY;
          t.z0 = kz * TZ;
          T.tiles.push_back(t);
        }
  }
  if (T.tiles.size() > (size_t)0x7fffffff) return fail(AWE_ERR_UNSUPPORTED, "too many tiles");
  auto tile_of = [&](int s, int i, int j, int k) {
    return first_tile[s] + ((k / tz_of(s)) * nty[s] + (j / TY)) * ntx[s] + i / awe::kTX;
  };
  // groups' tile ranges and active prefixes
  const int G = (int)P->g_shot0.size();
  T.g_tile0.assign(G + 1, 0);
  T.g_active.assign(G, std::vector<int>(P->nsteps + 2, 0));
  for (int g = 0; g < G; ++g) {
    const int b = P->g_shot0[g], e = b + P->g_nshot[g];
    T.g_tile0[g] = first_tile[order[b]];
    for (int n = 0; n <= P->nsteps + 1; ++n) {
      int cnt = 0;
      for (int i = b; i < e; ++i)
        if (P->sd[order[i]].off < n) cnt += ntx[order[i]] * nty[order[i]] * ntz[order[i]];
      T.g_active[g][n] = cnt;
    }
  }
  T.g_tile0[G] = (int)T.tiles.size();
  T.src_tile.assign(P->nshot, 0);
  for (int s = 0; s < P->nshot; ++s) T.src_tile[s] = tile_of(s, P->sd[s].src_i, P->sd[s].src_j, P->sd[s].src_k);
  // receivers: gather list grouped by owning tile; injection CSR by touched point
  struct RecTmp { int tile; RecDev r; };
  std::vector<RecTmp> rt;
  struct Touch { int tile; long long p; int shot, lx, ly, lz, r; float w; };
  std::vector<Touch> touches;
  P->total_recs = 0;
  for (int s = 0; s < P->nshot; ++s) {
    const awe_shot& sh = P->shots[s];
    for (int r = 0; r < sh.nrec; ++r) {
      const double* pos = P->rec_pos.data() + 3 * (sh.rec_offset + r);
      Interp I;
      if (!interp(P, sh, pos, &I))
        return fail(AWE_ERR_GEOMETRY, "receiver " + std::to_string(r) + " of shot " +
                                          std::to_string(s) + " lies outside its grid");
      RecDev R{};
      R.shot = s;
      R.r = r;
      R.i = I.base[0];
      R.j = I.base[1];
      R.k = I.base[2];
      for (int c = 0; c < 8; ++c) R.w[c] = (float)I.w[c];
      rt.push_back({tile_of(s, R.i, R.j, R.k), R});
      const int nc = nd == 2 ? 4 : 8;
      for (int c = 0; c < nc; ++c) {
        if (I.w[c] == 0.0) continue;
        int dx, dy, dz;
        corner(nd, c, &dx, &dy, &dz);
        const int i = R.i + dx, j = R.j + dy, k = R.k + dz;
        const int t = tile_of(s, i, j, k);
        const TileDev& Tl = T.tiles[t];
        const long long p = ((long long)k * sh.ny + j) * P->sd[s].px + i;
        touches.push_back({t, p, s, i - Tl.x0, j - Tl.y0, k - Tl.z0, r, (float)I.w[c]});
      }
    }
    P->total_recs += sh.nrec;
  }
  std::stable_sort(rt.begin(), rt.end(), [](const RecTmp& a, const RecTmp& b) { return a.tile < b.tile; });
  T.recs.clear();
  for (size_t i = 0; i < rt.size(); ++i) {
    TileDev& Tl = T.tiles[rt[i].tile];
    if (Tl.gat_count == 0) Tl.gat_begin = (int)i;
    Tl.gat_count++;
    T.recs.push_back(rt[i].r);
  }
  std::stable_sort(touches.begin(), touches.end(), [](const Touch& a, const Touch& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.p != b.p) return a.p < b.p;
    return a.r < b.r;
  });
  T.inj_pts.clear();
  T.inj_ent.clear();
  for (size_t i = 0; i < touches.size();) {
    size_t j = i;
    InjPoint ip{};
    ip.shot = touches[i].shot;
    ip.lx = touches[i].lx;
    ip.ly = touches[i].ly;
    ip.lz = touches[i].lz;
    ip.p = touches[i].p;
    ip.e_begin = (int)T.inj_ent.size();
    while (j < touches.size() && touches[j].tile == touches[i].tile && touches[j].p == touches[i].p) {
      T.inj_ent.push_back({touches[j].r, touches[j].w});
      ++j;
    }
    ip.e_count = (int)(j - i);
    TileDev& Tl = T.tiles[touches[i].tile];
    if (Tl.inj_count == 0) Tl.inj_begin = (int)T.inj_pts.size();
    Tl.inj_count++;
    T.inj_pts.push_back(ip);
    i = j;
  }
  {
    T.g_inj0.assign(G, 0);
    T.g_ninj.assign(G, 0);
    std::vector<int> grp_of(P->nshot, 0);
    for (int g = 0; g < G; ++g)
      for (int i = 0; i < P->g_nshot[g]; ++i) grp_of[order[P->g_shot0[g] + i]] = g;
    for (size_t i = T.inj_pts.size(); i-- > 0;) {
      const int g = grp_of[T.inj_pts[i].shot];
      T.g_inj0[g] = (int)i;
      T.g_ninj[g]++;
    }
  }
  // 2D: every touched point is also listed for each tile whose 4-cell extended region holds
  // it (the two-step adjoint injects on the extended region); same CSR entries
  T.ext_pts.clear();
  if (nd == 2) {
    struct Ext { int tile; long long p; InjPoint ip; };
    std::vector<Ext> ex;
    for (const InjPoint& ip : T.inj_pts) {
      const int px = P->sd[ip.shot].px;
      const int i = (int)(ip.p % px), k = (int)(ip.p / px);
      const int TZ = T.tz;
      for (int kz = std::max(0, (k - TZ - kHalo) / TZ - 1); kz <= (k + kHalo) / TZ; ++kz) {
        for (int kx = std::max(0, (i - awe::kTX - kHalo) / awe::kTX - 1); kx <= (i + kHalo) / awe::kTX; ++kx) {
          if (kz >= ntz[ip.shot] || kx >= ntx[ip.shot]) continue;
          const int x0 = kx * awe::kTX, z0 = kz * TZ;
          const int lx = i - (x0 - kHalo), lz = k - (z0 - kHalo);
          if (lx < 0 || lx >= awe::kTX + 2 * kHalo || lz < 0 || lz >= TZ + 2 * kHalo) continue;
          InjPoint e = ip;
          e.lx = lx;
          e.lz = lz;
          ex.push_back({first_tile[ip.shot] + kz * ntx[ip.shot] + kx, ip.p, e});
        }
      }
    }
    std::stable_sort(ex.begin(), ex.end(), [](const Ext& a, const Ext& b) {
      return a.tile != b.tile ? a.tile < b.tile : a.p < b.p;
    });
    for (size_t q = 0; q < ex.size(); ++q) {
      TileDev& Tl = T.tiles[ex[q].tile];
      if (Tl.ext_count == 0) Tl.ext_begin = (int)T.ext_pts.size();
      Tl.ext_count++;
      T.ext_pts.push_back(ex[q].ip);
    }
  }
  return AWE_OK;
}

awe_status upload_tiling(awe_plan* P, Tiling& T) {
  auto bytes = [](size_t n, size_t e) { return (long long)align256((long long)(n * e)); };
  std::vector<ShotDev> sd = P->sd;
  for (int s = 0; s < P->nshot; ++s) sd[s].src_tile = T.src_tile[s];
  const long long o_sd = 0;
  const long long o_t = o_sd + bytes(sd.size(), sizeof(ShotDev));
  const long long o_r = o_t + bytes(T.tiles.size(), sizeof(TileDev));
  const long long o_ip = o_r + bytes(T.recs.size(), sizeof(RecDev));
  const long long o_xp = o_ip + bytes(T.inj_pts.size(), sizeof(InjPoint));
  const long long o_ie = o_xp + bytes(T.ext_pts.size(), sizeof(InjPoint));
  const long long o_w = o_ie + bytes(T.inj_ent.size(), sizeof(InjEntry));
  const long long o_ws = o_w + bytes(P->wins.size(), sizeof(WinDev));
  const long long o_or = o_ws + bytes(P->win_shots.size(), sizeof(int));
  const long long total = o_or + bytes(P->order.size(), sizeof(int)) + 256;
  std::vector<unsigned char> host(total, 0);
  auto put = [&](long long off, const void* src, size_t n) { if (n) std::memcpy(host.data() + off, src, n); };
  put(o_sd, sd.data(), sd.size() * sizeof(ShotDev));
  put(o_t, T.tiles.data(), T.tiles.size() * sizeof(TileDev));
  put(o_r, T.recs.data(), T.recs.size() * sizeof(RecDev));
  put(o_ip, T.inj_pts.data(), T.inj_pts.size() * sizeof(InjPoint));
  put(o_xp, T.ext_pts.data(), T.ext_pts.size() * sizeof(InjPoint));
  put(o_ie, T.inj_ent.data(), T.inj_ent.size() * sizeof(InjEntry));
  put(o_w, P->wins.data(), P->wins.size() * sizeof(WinDev));
  put(o_ws, P->win_shots.data(), P->win_shots.size() * sizeof(int));
  put(o_or, P->order.data(), P->order.size() * sizeof(int));
  if (T.dev) {
    (void)hipFree(T.dev);
    T.dev = nullptr;
  }
  AWE_HIP(hipMalloc(&T.dev, total));
  AWE_HIP(hipMemcpy(T.dev, host.data(), total, hipMemcpyHostToDevice));
  unsigned char* b = static_cast<unsigned char*>(T.dev);
  T.tab.shots = reinterpret_cast<const ShotDev*>(b + o_sd);
  T.tab.tiles = reinterpret_cast<const TileDev*>(b + o_t);
  T.tab.recs = reinterpret_cast<const RecDev*>(b + o_r);
  T.tab.inj_pts = reinterpret_cast<const InjPoint*>(b + o_ip);
  T.tab.ext_pts = reinterpret_cast<const InjPoint*>(b + o_xp);
  T.tab.inj_ent = reinterpret_cast<const InjEntry*>(b + o_ie);
  T.tab.wins = reinterpret_cast<const WinDev*>(b + o_w);
  T.tab.win_shots = reinterpret_cast<const int*>(b + o_ws);
  T.tab.order = reinterpret_cast<const int*>(b + o_or);
  return AWE_OK;
}

// Shot groups and the tilings of the directions in `dirs` (bit 0 forward, bit 1 adjoint; the
// groups change both, so a change of groups rebuilds both), built and uploaded.
awe_status rebuild(awe_plan* P, int dirs) {
  awe_status st = build_groups(P);
  if (st != AWE_OK) return st;
  for (Tiling* T : {&P->fw, &P->rv}) {
    if (!(dirs & (T == &P->fw ? 1 : 2))) continue;
    if ((st = build_tiling(P, *T)) != AWE_OK) return st;
    if ((st = upload_tiling(P, *T)) != AWE_OK) return st;
  }
  return AWE_OK;
}

// Launch arguments on the tables of tiling T (P->fw for forward solves and Born modelling,
// P->rv for adjoint steps).
awe::StepArgs base_args(const awe_plan* P, const Tiling& T, void* ws) {
  awe::StepArgs a{};
  a.t = T.tab;
  a.ws = static_cast<unsigned char*>(ws);
  a.ndim = P->ndim;
  a.nbl = P->nbl;
  a.store_prec = P->store.prec;
  for (int i = 0; i < 5; ++i) a.c[i] = P->c[i];
  a.eta_dt = P->eta_dt;
  a.inv_dt2 = (float)(1.0 / (P->dt * P->dt));
  a.rs_level = awe::kNoLevel;
  a.rs_slot = 0;
  a.st_slot = -1;
  return a;
}

awe_status check_ws(const awe_plan* P, void* ws, size_t ws_bytes) {
  if (!P) return fail(AWE_ERR_INVALID_ARG, "plan is NULL");
  if (!ws) return fail(AWE_ERR_WORKSPACE, "workspace is NULL");
  if (ws_bytes < P->ws_bytes)
    return fail(AWE_ERR_WORKSPACE, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                       std::to_string(P->ws_bytes));
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(AWE_ERR_WORKSPACE, "workspace not 256-byte aligned");
  return AWE_OK;
}

// ---- host-side launch checks (AWE_CHECK_LAUNCHES): before a launch, the byte ranges and
// indices the host computed for it are checked against the plan's workspace layout and tables.

// [begin, end) of every workspace sub-buffer.
std::vector<std::pair<long long, long long>> sub_buffers(const awe_plan* P) {
  std::vector<std::pair<long long, long long>> r;
  auto add = [&](long long off, long long n) {
    if (off >= 0 && n > 0) r.emplace_back(off, off + n);
  };
  add(0, (long long)awe::kReduceBlocks * 8);
  for (size_t w = 0; w < P->wins.size(); ++w) add(P->win_coef[w], P->wins[w].npts * 4);
  const awe_storage& st = P->store;
  const int esz = st.prec == AWE_PREC_FP32 ? 4 : 2;
  for (const ShotDev& d : P->sd) {
    add(d.fld, (long long)awe::kFieldBufs * d.npts * 4);
    add(d.acc, d.npts * 8);
    if (st.mode == AWE_STORE_FULL) {
      add(d.store, (long long)d.nt * d.npts * esz);
      add(d.scale, (long long)d.nt * awe::kScaleSlots * 4);
    } else if (st.mode == AWE_STORE_CHECKPOINT) {
      add(d.store, (long long)st.nslots * 2 * d.npts * esz);
      add(d.scale, (long long)st.nslots * 2 * 4);
    } else if (st.mode == AWE_STORE_PROBED) {
      add(d.store, (long long)st.nslots * 2 * d.npts * 8);
    }
  }
  return r;
}

awe_status launch_fault(const std::string& what) {
  return fail(AWE_ERR_INTERNAL, "launch check: " + what);
}

// [off, off + n) must lie inside one sub-buffer.
awe_status check_range(const awe_plan* P, long long off, long long n, const char* what) {
  if (!(P->checks & AWE_CHECK_LAUNCHES) || n <= 0) return AWE_OK;
  for (const auto& [b, e] : sub_buffers(P))
    if (off >= b && off + n <= e) return AWE_OK;
  return launch_fault(std::string(what) + ": bytes [" + std::to_string(off) + ", " + std::to_string(off + n) +
                      ") are not inside one workspace sub-buffer");
}

awe_status fill(const awe_plan* P, unsigned char* ws, long long off, long long n, hipStream_t s, const char* what) {
  awe_status st = check_range(P, off, n, what);
  if (st != AWE_OK) return st;
  AWE_HIP(awe::launch_fill(ws, off, n, s));
  return AWE_OK;
}

// A step launch producing levels [lo, hi] of the current group on tiling T.
awe_status check_step(const awe_plan* P, const Tiling& T, const awe::StepArgs& a, int lo, int hi, const char* what) {
  if (!(P->checks & AWE_CHECK_LAUNCHES)) return AWE_OK;
  const std::string id = std::string(what) + " levels " + std::to_string(lo) + ".." + std::to_string(hi);
  if (lo < 1 || hi > P->nsteps || lo > hi) return launch_fault(id + ": outside 1.." + std::to_string(P->nsteps));
  const int g = P->cur;
  if (g < 0 || g >= (int)P->g_nshot.size()) return launch_fault(id + ": no current shot group");
  if (a.tile_base != T.g_tile0[g] || a.ntiles < 0 || a.tile_base + a.ntiles > T.g_tile0[g + 1])
    return launch_fault(id + ": tiles outside the group's range");
  if (a.shot_base != P->g_shot0[g]) return launch_fault(id + ": wrong first shot of the group");
  std::vector<char> in_group(P->nshot, 0);
  for (int i = 0; i < P->g_nshot[g]; ++i) in_group[P->order[P->g_shot0[g] + i]] = 1;
  for (int t = a.tile_base; t < a.tile_base + a.ntiles; ++t) {
    const int sh = T.tiles[t].shot;
    if (sh < 0 || sh >= P->nshot || !in_group[sh]) return launch_fault(id + ": tile of a shot outside the group");
  }
  const bool ckpt = P->store.mode == AWE_STORE_CHECKPOINT;
  if (a.rs_level != awe::kNoLevel && (!ckpt || a.rs_slot < 0 || a.rs_slot >= P->store.nslots))
    return launch_fault(id + ": restore-by-reference slot " + std::to_string(a.rs_slot) + " out of range");
  if (a.st_slot >= 0 && (!ckpt || a.st_slot >= P->store.nslots))
    return launch_fault(id + ": fused store slot " + std::to_string(a.st_slot) + " out of range");
  return AWE_OK;
}

awe_status prepare(awe_plan* P, const float* m, void* ws, bool zero_fwd, bool zero_adj, hipStream_t s) {
  unsigned char* w = static_cast<unsigned char*>(ws);
  for (size_t i = 0; i < P->wins.size(); ++i) {
    AWE_HIP(awe::launch_coef(m, w, P->win_coef[i], P->wins[i].m, P->win_dims[3 * i],
                             P->win_dims[3 * i + 1], P->win_dims[3 * i + 2], P->wins[i].px, P->nbl, P->h, P->dt,
                             P->amp, s));
  }
  for (int i = 0; i < P->nshot; ++i) {
    const ShotDev& d = P->sd[i];
    awe_status st;
    if (zero_fwd && (st = fill(P, w, d.fld, 4 * d.npts * 4, s, "forward buffers")) != AWE_OK) return st;
    if (zero_adj && (st = fill(P, w, d.fld + 4 * d.npts * 4, 4 * d.npts * 4, s, "adjoint buffers")) != AWE_OK)
      return st;
  }
  return AWE_OK;
}

// Kernel timing: an event pair around one launch (class cls) when enabled and not full.
struct ProfScope {
  awe_plan* P;
  hipStream_t s;
  bool on;
  ProfScope(awe_plan* P_, int cls, hipStream_t s_) : P(P_), s(s_) {
    if (P->prof_in_run) {  // counted into the enclosing run's interval
      ++P->prof_run_launches;
      on = false;
      return;
    }
    on = P->prof_next + 2 <= P->prof_ev.size() && (P->prof_seen++ % P->prof_stride) == 0;
    if (on) {
      (void)hipEventRecord(P->prof_ev[P->prof_next], s);
      P->prof_cls.push_back(cls);
      P->prof_cnt.push_back(1);
    }
  }
  ~ProfScope() {
    if (on) {
      (void)hipEventRecord(P->prof_ev[P->prof_next + 1], s);
      P->prof_next += 2;
    }
  }
};

// A run of consecutive time steps of one class (a sweep's step loop, a checkpoint advance)
// timed as one interval: one event pair for the whole run instead of one per launch, whose
// recording would add its dispatch latency to every launch; the run's launches are counted
// into it.
struct ProfRun {
  awe_plan* P;
  hipStream_t s;
  int cls;
  bool on;
  ProfRun(awe_plan* P_, hipStream_t s_, int cls_) : P(P_), s(s_), cls(cls_) {
    on = !P->prof_in_run && P->prof_next + 2 <= P->prof_ev.size() && (P->prof_seen++ % P->prof_stride) == 0;
    if (on) {
      (void)hipEventRecord(P->prof_ev[P->prof_next], s);
      P->prof_in_run = true;
      P->prof_run_launches = 0;
    }
  }
  ~ProfRun() {
    if (on) {
      (void)hipEventRecord(P->prof_ev[P->prof_next + 1], s);
      P->prof_cls.push_back(cls);
      P->prof_cnt.push_back(P->prof_run_launches);
      P->prof_next += 2;
      P->prof_in_run = false;
    }
  }
};

// Launch geometry of the current group at global step n on tiling T.
void set_group(const awe_plan* P, const Tiling& T, awe::StepArgs& a, int n) {
  a.step = n;
  a.ntiles = T.g_active[P->cur][n];
  a.tile_base = T.g_tile0[P->cur];
  a.shot_base = P->g_shot0[P->cur];
}

awe_status step_fwd(awe_plan* P, awe::StepArgs& a, int n, int store, hipStream_t s) {
  set_group(P, P->fw, a, n);
  if (a.ntiles <= 0) return AWE_OK;
  if (awe_status st = check_step(P, P->fw, a, n, n, "forward step")) return st;
  ProfScope ps(P, 0, s);
  if (P->ndim == 2) AWE_HIP(awe::launch_fwd2d(a, P->fw.tz, store, s));
  else AWE_HIP(awe::launch_fwd3d(a, P->fw.ty, P->fw.bz, store, s));
  return AWE_OK;
}

awe_status step_adj(awe_plan* P, awe::StepArgs& a, int n, hipStream_t s) {
  set_group(P, P->rv, a, n);
  if (a.ntiles <= 0) return AWE_OK;
  if (awe_status st = check_step(P, P->rv, a, n, n, "adjoint step")) return st;
  if (P->ndim == 3 && (P->checks & AWE_CHECK_LAUNCHES) &&
      P->rv.g_inj0[P->cur] + P->rv.g_ninj[P->cur] > (int)P->rv.inj_pts.size())
    return launch_fault("receiver injection: touched points outside the table");
  ProfScope ps(P, 1, s);
  if (P->ndim == 2) {
    AWE_HIP(awe::launch_adj2d(a, P->rv.tz, s));
  } else {
    AWE_HIP(awe::launch_adj3d(a, P->rv.ty, P->rv.bz, s));
    AWE_HIP(awe::launch_inj3d(a, P->rv.g_inj0[P->cur], P->rv.g_ninj[P->cur], s));
  }
  return AWE_OK;
}

// Two levels per launch (2D): forward levels n, n+1; adjoint levels n, n-1.
awe_status step_fwd2(awe_plan* P, awe::StepArgs& a, int n, int store, hipStream_t s) {
  set_group(P, P->fw, a, n + 1);
  a.step = n;
  if (a.ntiles <= 0) return AWE_OK;
  if (awe_status st = check_step(P, P->fw, a, n, n + 1, "two-level forward step")) return st;
  ProfScope ps(P, 0, s);
  AWE_HIP(awe::launch_fwd2d2(a, P->fw.tz, store, s));
  return AWE_OK;
}

awe_status step_adj2(awe_plan* P, awe::StepArgs& a, int n, hipStream_t s) {
  set_group(P, P->rv, a, n);
  if (a.ntiles <= 0) return AWE_OK;
  if (awe_status st = check_step(P, P->rv, a, n - 1, n, "two-level adjoint step")) return st;
  ProfScope ps(P, 1, s);
  AWE_HIP(awe::launch_adj2d2(a, P->rv.tz, s));
  return AWE_OK;
}

// Two-level kernels exist for 8, 16, 24 and 32 rows (2D).
bool two_level_rows(int tz) { return tz == 8 || tz == 16 || tz == 24 || tz == 32; }

bool fused_ok(const awe_plan* P, int bit) {
  const int tz = bit == AWE_FUSE_FORWARD ? P->fw.tz : P->rv.tz;
  return P->ndim == 2 && (P->fuse2 & bit) && two_level_rows(tz);
}

// Forward levels 1..nsteps: one single step first when the count is odd, then pairs.
awe_status forward_loop(awe_plan* P, awe::StepArgs& a, int store, hipStream_t s) {
  awe_status st;
  const bool fuse = fused_ok(P, AWE_FUSE_FORWARD) &&
                    (store == awe::kStoreNone || store == awe::kStoreF32 || store == awe::kStoreProbe);
  // a 2D FP32 sweep of one-level steps reads its previous levels back from the store
  if (!fuse && P->ndim == 2 && store == awe::kStoreF32) store = awe::kStoreF32R;
  ProfRun run(P, s, 0);
  int n = 1;
  if (fuse && (P->nsteps & 1)) {
    if ((st = step_fwd(P, a, 1, store, s)) != AWE_OK) return st;
    n = 2;
  }
  for (; n <= P->nsteps; n += fuse ? 2 : 1) {
    st = fuse ? step_fwd2(P, a, n, store, s) : step_fwd(P, a, n, store, s);
    if (st != AWE_OK) return st;
  }
  return AWE_OK;
}

// Adjoint levels nsteps..1 (same pairing, from the top).
awe_status adjoint_loop(awe_plan* P, awe::StepArgs& a, hipStream_t s) {
  awe_status st;
  const bool fuse = fused_ok(P, AWE_FUSE_ADJOINT) &&
                    (a.image_src == awe::kImgNone || a.image_src == awe::kImgFull32 || a.image_src == awe::kImgProbe);
  ProfRun run(P, s, 1);
  int n = P->nsteps;
  if (fuse && (P->nsteps & 1)) {
    if ((st = step_adj(P, a, n, s)) != AWE_OK) return st;
    n -= 1;
  }
  for (; n >= 1; n -= fuse ? 2 : 1) {
    st = fuse ? step_adj2(P, a, n, s) : step_adj(P, a, n, s);
    if (st != AWE_OK) return st;
  }
  return AWE_OK;
}

awe_status run_slot(awe_plan* P, awe::StepArgs& a, int slot, int state, int dir, hipStream_t s) {
  const int g = P->cur, nsh = P->g_nshot[g];
  a.shot_base = P->g_shot0[g];
  if (P->checks & AWE_CHECK_LAUNCHES) {
    if (P->store.mode != AWE_STORE_CHECKPOINT || slot < 0 || slot >= P->store.nslots || state < 0 ||
        state > P->nsteps)
      return launch_fault("slot copy: slot " + std::to_string(slot) + " state " + std::to_string(state) + " out of range");
    const int esz = P->store.prec == AWE_PREC_FP32 ? 4 : 2;
    for (int i = 0; i < nsh; ++i) {
      const ShotDev& d = P->sd[P->order[a.shot_base + i]];
      if (awe_status st = check_range(P, d.store + (long long)slot * 2 * d.npts * esz, 2 * d.npts * esz, "slot copy"))
        return st;
    }
  }
  if (dir == 0 && P->store.prec != AWE_PREC_FP32) {
    for (int i = 0; i < nsh; ++i)
      if (awe_status st = fill(P, a.ws, P->sd[P->order[a.shot_base + i]].scale + 8LL * slot, 8, s, "slot scales"))
        return st;
    AWE_HIP(awe::launch_absmax(a, nsh, slot, state, s));
  }
  AWE_HIP(awe::launch_slot(a, nsh, slot, state, dir, s));
  return AWE_OK;
}

// Execute schedule actions [begin, end).  During the first sweep (gather != 0) traces are
// sampled; REVERSE runs the adjoint step with imaging from the forward buffers.
awe_status run_actions(awe_plan* P, awe::StepArgs& fa, awe::StepArgs& aa, size_t begin, size_t end,
                       hipStream_t s) {
  const int g = P->cur;
  if (P->g_rs_level.size() != P->g_nshot.size()) {
    P->g_rs_level.assign(P->g_nshot.size(), awe::kNoLevel);
    P->g_rs_slot.assign(P->g_nshot.size(), 0);
  }
  if (begin == 0) P->g_rs_level[g] = awe::kNoLevel;  // a new forward sweep of this group
  auto set_rs = [&](int level, int slot) {
    fa.rs_level = aa.rs_level = level;
    fa.rs_slot = aa.rs_slot = slot;
  };
  set_rs(P->g_rs_level[g], P->g_rs_slot[g]);
  const bool by_ref = P->store.prec == AWE_PREC_FP32;
  for (size_t i = begin; i < end; ++i) {
    const int op = P->sched[3 * i], x = P->sched[3 * i + 1], y = P->sched[3 * i + 2];
    switch (op) {
      case awe::kAdvance: {
        // a store of the reached state that follows is fused into the last step (2D, FP32
        // slots, and not into the slot the step may still read by reference)
        int fuse_slot = -1;
        if (by_ref && P->ndim == 2 && i + 1 < end && P->sched[3 * (i + 1)] == awe::kStore &&
            P->sched[3 * (i + 1) + 2] == y &&
            !(fa.rs_level != awe::kNoLevel && fa.rs_slot == P->sched[3 * (i + 1) + 1]))
          fuse_slot = P->sched[3 * (i + 1) + 1];
        ProfRun run(P, s, 0);
        for (int n = x + 1; n <= y; ++n) {
          fa.st_slot = n == y ? fuse_slot : -1;
          awe_status st = step_fwd(P, fa, n, 0, s);
          fa.st_slot = -1;
          if (st != AWE_OK) return st;
        }
        if (fuse_slot >= 0) ++i;  // the store is done
        break;
      }
      case awe::kStore: {
        if (fa.rs_level != awe::kNoLevel && fa.rs_slot == x) {
          // overwriting the slot that is read by reference: copy its state into the
          // buffers first
          awe::StepArgs ca = fa;
          ca.rs_level = awe::kNoLevel;
          awe_status st = run_slot(P, ca, x, fa.rs_level, 1, s);
          if (st != AWE_OK) return st;
          set_rs(awe::kNoLevel, 0);
        }
        awe_status st = run_slot(P, fa, x, y, 0, s);
        if (st != AWE_OK) return st;
        break;
      }
      case awe::kRestore:
        if (x < 0) {
          for (int i = 0; i < P->g_nshot[P->cur]; ++i) {
            const ShotDev& d = P->sd[P->order[P->g_shot0[P->cur] + i]];
            if (awe_status st = fill(P, fa.ws, d.fld, 4 * d.npts * 4, s, "forward buffers (zero state)")) return st;
          }
          set_rs(awe::kNoLevel, 0);
        } else if (by_ref) {
          set_rs(y, x);  // FP32 slot: levels y and y - 1 are read from the slot in place
        } else {
          set_rs(awe::kNoLevel, 0);
          awe_status st = run_slot(P, fa, x, y, 1, s);
          if (st != AWE_OK) return st;
        }
        break;
      case awe::kReverse: {
        // a pair of reversals x, x-1 from one state runs as one two-level launch when the
        // adjoint fusion is on (both levels are read from the current state)
        const bool two = fused_ok(P, AWE_FUSE_ADJOINT) && i + 1 < end && x >= 2 &&
                         P->sched[3 * (i + 1)] == awe::kReverse && P->sched[3 * (i + 1) + 1] == x - 1;
        awe_status st = two ? step_adj2(P, aa, x, s) : step_adj(P, aa, x, s);
        if (st != AWE_OK) return st;
        if (two) ++i;
        break;
      }
    }
  }
  P->g_rs_level[g] = fa.rs_level;
  P->g_rs_slot[g] = fa.rs_slot;
  return AWE_OK;
}

// ---- autotuner result cache: a JSON object of "key": {"fw": [tz, ty, bz], "rv": [...],
// "fusion": f, "ms": t} entries, one per line, in the file named by AWE_TUNE_CACHE.
struct TuneEntry {
  int fw[3], rv[3], fusion;
  double ms;
};

// Device, problem shape, storage, grouping and probe length: what the timing of the candidate
// shapes depends on.  The shots' grids, time axes, receiver counts and windows enter through a
// 64-bit FNV-1a hash.
std::string tune_key(const awe_plan* P, int probe) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char& c : arch)
    if (c == '"' || c == '\\' || c < 32) c = '_';
  unsigned long long h = 1469598103934665603ull;
  auto mix = [&](long long v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (unsigned char)(v >> (8 * i));
      h *= 1099511628211ull;
    }
  };
  for (const awe_shot& sh : P->shots) {
    mix(sh.nx);
    mix(sh.ny);
    mix(sh.nz);
    mix(sh.nt);
    mix(sh.nrec);
    mix(sh.m_offset);
  }
  char buf[512];
  std::snprintf(buf, sizeof buf, "v%d/%s/%dcu/%dd/n%d/st%d.%d.%d/g%zu/p%d/%016llx", AWE_VERSION, arch.c_str(),
                cus, P->ndim, P->nshot, P->store.mode, P->store.nslots, P->store.prec, P->g_nshot.size(),
                probe, h);
  return buf;
}

std::map<std::string, TuneEntry> read_tune_cache(const char* path) {
  std::map<std::string, TuneEntry> out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[2048], key[1024];
  while (std::fgets(line, sizeof line, f)) {
    TuneEntry e{};
    if (std::sscanf(line, " \"%1023[^\"]\": {\"fw\": [%d, %d, %d], \"rv\": [%d, %d, %d], \"fusion\": %d, \"ms\": %lf}",
                    key, &e.fw[0], &e.fw[1], &e.fw[2], &e.rv[0], &e.rv[1], &e.rv[2], &e.fusion, &e.ms) == 9)
      out[key] = e;
  }
  std::fclose(f);
  return out;
}

// Rewrite the cache through a temporary file and a rename, so that a reader never sees half a
// file (concurrent writers: the last rename wins).  Failures leave the cache as it was.
void write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& entries) {
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& [k, e] : entries)
    std::fprintf(f, "  \"%s\": {\"fw\": [%d, %d, %d], \"rv\": [%d, %d, %d], \"fusion\": %d, \"ms\": %.6f}%s\n",
                 k.c_str(), e.fw[0], e.fw[1], e.fw[2], e.rv[0], e.rv[1], e.rv[2], e.fusion, e.ms,
                 ++i < entries.size() ? "," : "");
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}

bool valid_tz(int tz) { return tz == 8 || tz == 12 || tz == 16 || tz == 20 || tz == 24 || tz == 32 || tz == 64; }

// Put a cached result in effect; false (plan unchanged) if the entry is not a valid shape.
bool apply_tune_entry(awe_plan* P, const TuneEntry& e, awe_status* st) {
  for (const int* t : {e.fw, e.rv})
    if (!valid_tz(t[0]) || (t[1] != 4 && t[1] != 8 && t[1] != 16) || t[2] < 0) return false;
  if (e.fusion < 0 || e.fusion > AWE_FUSE_BOTH) return false;
  if ((e.fusion & AWE_FUSE_FORWARD) && !two_level_rows(e.fw[0])) return false;
  if ((e.fusion & AWE_FUSE_ADJOINT) && !two_level_rows(e.rv[0])) return false;
  P->fw.tz = e.fw[0];
  P->fw.ty = e.fw[1];
  P->fw.bz = e.fw[2];
  P->rv.tz = e.rv[0];
  P->rv.ty = e.rv[1];
  P->rv.bz = e.rv[2];
  P->fuse2 = e.fusion;
  P->kept_ws = nullptr;
  *st = rebuild(P, 3);
  return true;
}

// ---- optional screening of caller arrays (awe_plan_set_checks)
enum ArrKind { kPerWindow, kPerShotQ, kPerShotD };
struct Screened {
  const void* p;
  bool f64;
  ArrKind kind;
  const char* name;
  bool vmax_bound;  // also count values below 1/vmax^2 (squared slowness above the velocity bound)
};
constexpr int kMaxScreened = 8;

awe_status screen(awe_plan* P, std::initializer_list<Screened> arrays, hipStream_t s) {
  if (arrays.size() > (size_t)kMaxScreened) return fail(AWE_ERR_INVALID_ARG, "too many screened arrays");
  AWE_HIP(awe::launch_fill(reinterpret_cast<unsigned char*>(P->chk_dev), 0, 2 * kMaxScreened * 8, s));
  int i = 0;
  for (const Screened& a : arrays) {
    unsigned long long* cnt = P->chk_dev + 2 * i++;
    if (!a.p) continue;
    const double lo = a.vmax_bound ? (1.0 - 1e-6) / (P->vmax * P->vmax) : -HUGE_VAL;
    auto run = [&](long long off, long long n) -> hipError_t {
      return a.f64 ? awe::launch_screen(static_cast<const double*>(a.p) + off, n, lo, cnt, s)
                   : awe::launch_screen(static_cast<const float*>(a.p) + off, n, lo, cnt, s);
    };
    if (a.kind == kPerWindow) {
      for (size_t w = 0; w < P->wins.size(); ++w)
        AWE_HIP(run(P->wins[w].m, (long long)P->win_dims[3 * w] * P->win_dims[3 * w + 1] * P->win_dims[3 * w + 2]));
    } else {
      for (const awe_shot& sh : P->shots)
        AWE_HIP(a.kind == kPerShotQ ? run(sh.q_offset, sh.nt) : run(sh.d_offset, (long long)sh.nt * sh.nrec));
    }
  }
  unsigned long long host[2 * kMaxScreened] = {};
  AWE_HIP(hipMemcpyAsync(host, P->chk_dev, sizeof host, hipMemcpyDeviceToHost, s));
  AWE_HIP(hipStreamSynchronize(s));
  i = 0;
  for (const Screened& a : arrays) {
    const unsigned long long bad = host[2 * i], low = host[2 * i + 1];
    ++i;
    if (bad)
      return fail(AWE_ERR_NONFINITE, std::string(a.name) + ": " + std::to_string(bad) + " values are not finite");
    if (low) {
      char buf[200];
      std::snprintf(buf, sizeof buf, "%s: %llu values below 1/vmax^2 = %.6g (velocity above the plan's vmax "
                    "%.6g km/s, the leapfrog may be unstable)", a.name, low, 1.0 / (P->vmax * P->vmax), P->vmax);
      return fail(AWE_ERR_CFL, buf);
    }
  }
  return AWE_OK;
}

}  // namespace

extern "C" {

int awe_version(void) { return AWE_VERSION; }

const char* awe_last_error(void) { return g_err.c_str(); }

const char* awe_status_string(awe_status s) {
  switch (s) {
    case AWE_OK: return "ok";
    case AWE_ERR_INVALID_ARG: return "invalid argument";
    case AWE_ERR_UNSUPPORTED: return "unsupported";
    case AWE_ERR_CFL: return "CFL condition violated";
    case AWE_ERR_GEOMETRY: return "source or receiver outside the grid";
    case AWE_ERR_WORKSPACE: return "workspace too small or misaligned";
    case AWE_ERR_STATE: return "no kept forward wavefield";
    case AWE_ERR_HIP: return "HIP runtime error";
    case AWE_ERR_NONFINITE: return "value not finite";
    case AWE_ERR_INTERNAL: return "internal launch check failed";
  }
  return "unknown status";
}

namespace {

awe_status validate(const awe_problem* prob, const awe_storage* store) {
  if (!prob || !store) return fail(AWE_ERR_INVALID_ARG, "problem or storage is NULL");
  if (prob->ndim != 2 && prob->ndim != 3) return fail(AWE_ERR_INVALID_ARG, "ndim must be 2 or 3");
  if (prob->nshot < 1 || !prob->shots) return fail(AWE_ERR_INVALID_ARG, "need at least one shot");
  if (!(prob->h > 0) || !(prob->dt > 0) || !(prob->vmax > 0) || !(prob->damp_vref > 0))
    return fail(AWE_ERR_INVALID_ARG, "h, dt, vmax and damp_vref must be positive");
  if (!(prob->damp_R > 0) || prob->damp_R > 1) return fail(AWE_ERR_INVALID_ARG, "damp_R must be in (0, 1]");
  if (prob->nbl < 0) return fail(AWE_ERR_INVALID_ARG, "nbl must be >= 0");
  if (store->mode < AWE_STORE_NONE || store->mode > AWE_STORE_PROBED)
    return fail(AWE_ERR_INVALID_ARG, "bad storage mode");
  if (store->mode == AWE_STORE_PROBED && (store->nslots < 1 || store->nslots > awe::kMaxProbes))
    return fail(AWE_ERR_INVALID_ARG, "PROBED storage needs 1 <= nslots <= " + std::to_string(awe::kMaxProbes) + " probes");
  if (store->prec < AWE_PREC_FP32 || store->prec > AWE_PREC_FP16)
    return fail(AWE_ERR_INVALID_ARG, "bad storage precision");
  if (store->mode == AWE_STORE_CHECKPOINT && store->nslots < 1)
    return fail(AWE_ERR_INVALID_ARG, "CHECKPOINT storage needs nslots >= 1");
  if (store->mode == AWE_STORE_AUTO && (store->nslots < 0 || store->budget_mib < 0))
    return fail(AWE_ERR_INVALID_ARG, "AUTO storage needs nslots >= 0 and budget_mib >= 0");
  if (store->mode == AWE_STORE_CHECKPOINT && prob->ndim == 3)
    return fail(AWE_ERR_UNSUPPORTED,
                "CHECKPOINT storage is disabled in 3D: its first GPU run faulted and the cause "
                "is not yet identified; use FULL storage");
  // stability of undamped leapfrog with the 8th-order stencil: v dt / h <= 2 / sqrt(ndim S)
  double S = std::fabs(kStencil[0]);
  for (int r = 1; r <= 4; ++r) S += 2 * std::fabs(kStencil[r]);
  const double limit = 2.0 / std::sqrt(prob->ndim * S);
  const double cfl = prob->vmax * prob->dt / prob->h;
  if (cfl > limit) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "vmax dt / h = %.6f exceeds the stability limit %.6f", cfl, limit);
    return fail(AWE_ERR_CFL, buf);
  }
  return AWE_OK;
}

// Offsets of every workspace sub-buffer for the plan's storage (P->store), and the total size.
void layout_ws(awe_plan* P) {
  long long off = align256((long long)awe::kReduceBlocks * 8);
  P->win_coef.resize(P->wins.size());
  for (size_t w = 0; w < P->wins.size(); ++w) {
    P->win_coef[w] = off;
    off = align256(off + P->wins[w].npts * 4);
  }
  const awe_storage& st = P->store;
  const int esz = st.prec == AWE_PREC_FP32 ? 4 : 2;
  P->fields_off = off;
  for (int s = 0; s < P->nshot; ++s) {
    ShotDev& d = P->sd[s];
    d.coef = P->win_coef[P->shot_win[s]];
    d.fld = off;
    off = align256(off + (long long)awe::kFieldBufs * d.npts * 4);
  }
  P->fields_bytes = off - P->fields_off;
  P->acc_off = off;
  for (int s = 0; s < P->nshot; ++s) {
    ShotDev& d = P->sd[s];
    d.acc = -1;
    d.store = -1;
    d.scale = -1;
    if (st.mode != AWE_STORE_FULL && st.mode != AWE_STORE_CHECKPOINT) continue;
    d.acc = off;
    off = align256(off + d.npts * 8);
  }
  P->acc_bytes = off - P->acc_off;
  for (int s = 0; s < P->nshot; ++s) {
    ShotDev& d = P->sd[s];
    if (st.mode == AWE_STORE_FULL) {
      d.store = off;
      off = align256(off + (long long)d.nt * d.npts * esz);
      d.scale = off;
      off = align256(off + (long long)d.nt * awe::kScaleSlots * 4);
    } else if (st.mode == AWE_STORE_CHECKPOINT) {
      d.store = off;
      off = align256(off + (long long)st.nslots * 2 * d.npts * esz);
      d.scale = off;
      off = align256(off + (long long)st.nslots * 2 * 4);
    } else if (st.mode == AWE_STORE_PROBED) {
      d.store = off;  // FP64 probe sums B, then A, r per point in blocks of 64 points (probe_sums)
      off = align256(off + (long long)st.nslots * 2 * d.npts * 8);
    }
  }
  P->ws_bytes = (size_t)off;
}

// AUTO storage: FULL when its workspace fits the budget, else CHECKPOINT with the most restart
// slots per shot that fit (at most nslots when nslots > 0, and at most the number of steps).
awe_status choose_storage(awe_plan* P) {
  const awe_storage& req = P->store_req;
  long long budget = (long long)req.budget_mib << 20;
  if (req.budget_mib == 0) {
    size_t free_b = 0, total_b = 0;
    AWE_HIP(hipMemGetInfo(&free_b, &total_b));
    budget = (long long)(0.9 * (double)free_b);
  }
  P->store = {AWE_STORE_FULL, 0, req.prec, 0};
  layout_ws(P);
  if ((long long)P->ws_bytes <= budget) return AWE_OK;
  const long long full = (long long)P->ws_bytes;
  char buf[256];
  if (P->ndim == 3) {
    std::snprintf(buf, sizeof buf, "FULL storage needs %lld bytes of workspace, over the budget of %lld, "
                  "and CHECKPOINT storage is disabled in 3D", full, budget);
    return fail(AWE_ERR_UNSUPPORTED, buf);
  }
  const int kmax = std::max(1, req.nslots > 0 ? std::min(req.nslots, P->nsteps) : P->nsteps);
  auto fits = [&](int k) {
    P->store = {AWE_STORE_CHECKPOINT, k, req.prec, 0};
    layout_ws(P);
    return (long long)P->ws_bytes <= budget;
  };
  if (!fits(1)) {
    std::snprintf(buf, sizeof buf, "FULL storage needs %lld bytes of workspace and CHECKPOINT with one "
                  "restart slot %zu, both over the budget of %lld", full, P->ws_bytes, budget);
    return fail(AWE_ERR_WORKSPACE, buf);
  }
  int lo = 1, hi = kmax;  // fits(lo) holds
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (fits(mid)) lo = mid;
    else hi = mid - 1;
  }
  fits(lo);
  return AWE_OK;
}

// Everything of a plan that needs no device: shots, windows, storage choice and workspace
// layout.  P is filled in place; on error the caller deletes it.
awe_status plan_host(const awe_problem* prob, const awe_storage* store, awe_plan* P) {
  P->ndim = prob->ndim;
  P->nbl = prob->nbl;
  P->h = prob->h;
  P->dt = prob->dt;
  P->vmax = prob->vmax;
  P->vref = prob->damp_vref;
  P->R = prob->damp_R;
  P->store = *store;
  P->store_req = *store;
  P->nshot = prob->nshot;
  P->shots.assign(prob->shots, prob->shots + prob->nshot);
  auto bad = [&](const std::string& m) { return fail(AWE_ERR_INVALID_ARG, m); };
  long long rec_rows = 0;
  for (int s = 0; s < P->nshot; ++s) {
    const awe_shot& sh = P->shots[s];
    const std::string id = "shot " + std::to_string(s) + ": ";
    if (sh.nx < 2 || sh.nz < 2 || sh.ny < 1) return bad(id + "grid too small");
    if (P->ndim == 2 && sh.ny != 1) return bad(id + "ny must be 1 in 2D");
    if (P->ndim == 3 && sh.ny < 2) return bad(id + "ny must be >= 2 in 3D");
    if (sh.nt < 2) return bad(id + "nt must be >= 2");
    if (sh.m_offset < 0 || sh.q_offset < 0 || sh.d_offset < 0 || sh.rec_offset < 0 || sh.nrec < 0)
      return bad(id + "negative offset or count");
    if (sh.nrec > 0 && !prob->rec_pos) return bad("rec_pos is NULL");
    rec_rows = std::max<long long>(rec_rows, (long long)(sh.rec_offset + sh.nrec));
    P->max_nt = std::max(P->max_nt, sh.nt);
  }
  P->nsteps = P->max_nt - 1;
  for (int r = 0; r < 5; ++r) P->c[r] = (float)(kStencil[r] / (P->h * P->h));
  P->amp = P->nbl > 0 ? 3.0 * std::log(1.0 / P->R) / (2.0 * P->nbl * P->h * P->vref) : 0.0;
  P->eta_dt = P->nbl > 0 ? (float)(P->amp / ((double)P->nbl * P->nbl) / P->dt) : 0.f;

  // windows (unique m_offset, consistent dims)
  std::map<long long, int> win_of;
  std::vector<std::vector<int>> wshots;
  for (int s = 0; s < P->nshot; ++s) {
    const awe_shot& sh = P->shots[s];
    auto it = win_of.find(sh.m_offset);
    if (it == win_of.end()) {
      win_of[sh.m_offset] = (int)P->wins.size();
      WinDev w{};
      w.m = sh.m_offset;
      w.nx = sh.nx;
      w.px = awe::pitch_of(sh.nx);
      w.npts = (long long)w.px * sh.ny * sh.nz;
      P->wins.push_back(w);
      P->win_dims.insert(P->win_dims.end(), {sh.nx, sh.ny, sh.nz});
      wshots.emplace_back();
    }
    const int wi = win_of[sh.m_offset];
    if (P->win_dims[3 * wi] != sh.nx || P->win_dims[3 * wi + 1] != sh.ny || P->win_dims[3 * wi + 2] != sh.nz)
      return bad("shots sharing m_offset " + std::to_string(sh.m_offset) + " have different grids");
    wshots[wi].push_back(s);
  }
  for (size_t w = 0; w < P->wins.size(); ++w) {
    P->wins[w].sbegin = (int)P->win_shots.size();
    P->wins[w].scount = (int)wshots[w].size();
    P->win_shots.insert(P->win_shots.end(), wshots[w].begin(), wshots[w].end());
    P->max_win_npts = std::max(P->max_win_npts, P->wins[w].npts);
  }

  P->sd.resize(P->nshot);
  P->shot_win.resize(P->nshot);
  for (int s = 0; s < P->nshot; ++s) {
    const awe_shot& sh = P->shots[s];
    ShotDev& d = P->sd[s];
    d.nx = sh.nx;
    d.px = awe::pitch_of(sh.nx);
    d.ny = sh.ny;
    d.nz = sh.nz;
    d.nt = sh.nt;
    d.off = P->max_nt - sh.nt;
    d.nrec = sh.nrec;
    d.npts = (long long)d.px * sh.ny * sh.nz;
    // the step kernels address a field through a buffer resource with 32-bit byte offsets: the
    // largest per-point field (the FP64 accumulator) must not exceed 1 GiB
    if (d.npts * 8 > (1LL << 30))
      return fail(AWE_ERR_UNSUPPORTED, "shot " + std::to_string(s) + ": " + std::to_string(d.npts) +
                                           " workspace points per field exceed the 2^27 the kernels address");
    P->shot_win[s] = win_of[sh.m_offset];
    d.m = sh.m_offset;
    d.q = sh.q_offset;
    d.d = sh.d_offset;
  }
  P->rec_pos.assign(3 * (size_t)std::max<long long>(rec_rows, 1), 0.0);
  if (prob->rec_pos && rec_rows > 0)
    std::copy(prob->rec_pos, prob->rec_pos + 3 * rec_rows, P->rec_pos.begin());
  if (store->mode == AWE_STORE_AUTO) return choose_storage(P);
  layout_ws(P);
  return AWE_OK;
}

}  // namespace

awe_status awe_plan_create(const awe_problem* prob, const awe_storage* store, awe_plan** out) {
  if (!out) return fail(AWE_ERR_INVALID_ARG, "plan output pointer is NULL");
  *out = nullptr;
  awe_status st = validate(prob, store);
  if (st != AWE_OK) return st;
  awe_plan* P = new awe_plan();
  if ((st = plan_host(prob, store, P)) != AWE_OK) {
    delete P;
    return st;
  }
  // default launch shapes (the fastest measured on MI355X for the 2D and 3D workloads; the
  // autotuner or awe_plan_set_tiles choose others): 2D 32-row forward and 16-row adjoint
  // tiles; 3D 64 x 8 column blocks with 128-plane z-blocks forward, 64 x 16 with 64 adjoint
  P->fw.tz = 32;
  P->rv.tz = 16;
  P->fw.ty = 8;
  P->fw.bz = 128;
  P->rv.ty = 16;
  P->rv.bz = 64;
  if ((st = rebuild(P, 3)) != AWE_OK) {
    awe_plan_destroy(P);
    return st;
  }
  if (P->store.mode == AWE_STORE_CHECKPOINT) {
    awe::build_schedule(P->nsteps, P->store.nslots, P->sched);
    const size_t na = P->sched.size() / 3;
    P->sched_first_reverse = na;
    for (size_t i = 0; i < na; ++i)
      if (P->sched[3 * i] == awe::kReverse) {
        P->sched_first_reverse = i;
        break;
      }
  }
  *out = P;
  return AWE_OK;
}

awe_status awe_storage_select(const awe_problem* prob, const awe_storage* store, awe_storage* chosen,
                              size_t* ws_bytes) {
  awe_status st = validate(prob, store);
  if (st != AWE_OK) return st;
  awe_plan P;
  if ((st = plan_host(prob, store, &P)) != AWE_OK) return st;
  if (chosen) *chosen = P.store;
  if (ws_bytes) *ws_bytes = P.ws_bytes;
  return AWE_OK;
}

awe_status awe_plan_get_storage(const awe_plan* plan, awe_storage* out) {
  if (!plan || !out) return fail(AWE_ERR_INVALID_ARG, "NULL argument");
  *out = plan->store;
  return AWE_OK;
}

awe_status awe_plan_workspace_size(const awe_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(AWE_ERR_INVALID_ARG, "NULL argument");
  *bytes = plan->ws_bytes;
  return AWE_OK;
}

void awe_plan_destroy(awe_plan* plan) {
  if (!plan) return;
  for (hipEvent_t e : plan->prof_ev) (void)hipEventDestroy(e);
  if (plan->fw.dev) (void)hipFree(plan->fw.dev);
  if (plan->rv.dev) (void)hipFree(plan->rv.dev);
  if (plan->chk_dev) (void)hipFree(plan->chk_dev);
  delete plan;
}

awe_status awe_plan_autotune(awe_plan* P, const float* m, const float* q, const float* dd,
                             int32_t probe_steps, void* ws, size_t ws_bytes, void* stream,
                             int32_t chosen[4], double* best_ms) {
  awe_status st = check_ws(P, ws, ws_bytes);
  if (st != AWE_OK) return st;
  if (!m || !q || probe_steps < 1) return fail(AWE_ERR_INVALID_ARG, "autotune needs m, q and probe_steps >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  P->kept_ws = nullptr;
  const int probe = std::min<int>(probe_steps, P->nsteps);
  const char* cache = std::getenv("AWE_TUNE_CACHE");
  std::string key;
  if (cache && *cache) {
    key = tune_key(P, probe);
    const auto entries = read_tune_cache(cache);
    const auto it = entries.find(key);
    if (it != entries.end() && apply_tune_entry(P, it->second, &st)) {
      if (st != AWE_OK) return st;
      if (chosen) {
        chosen[0] = P->fw.tz;
        chosen[1] = P->fw.ty;
        chosen[2] = P->fw.bz;
        chosen[3] = P->fuse2;
      }
      if (best_ms) *best_ms = it->second.ms;
      return AWE_OK;
    }
  }
  // one candidate list per direction; the forward probe times forward levels only, the adjoint
  // probe adjoint levels only, so each direction keeps its own fastest shape
  struct Cand { int tz, ty, bz, fuse; };
  std::vector<Cand> cands;
  const bool fusable = P->store.mode == AWE_STORE_NONE || P->store.mode == AWE_STORE_PROBED ||
                       P->store.mode == AWE_STORE_CHECKPOINT ||
                       (P->store.mode == AWE_STORE_FULL && P->store.prec == AWE_PREC_FP32);
  if (P->ndim == 2) {
    for (int tz : {8, 16, 24, 32, 64}) {
      cands.push_back({tz, 8, 0, 0});
      if (fusable && tz != 64) cands.push_back({tz, 8, 0, 1});
    }
  } else {
    // z-blocks of the full depth, of fixed lengths, and of the depth split evenly into 2 to 8
    // (no short last block)
    int nz = 0;
    for (const ShotDev& d : P->sd) nz = std::max(nz, d.nz);
    std::vector<int> bzs = {0, 128, 64, 32};
    for (int k = 2; k <= 8; ++k) {
      const int b = ((nz + k - 1) / k + 1) & ~1;
      if (b >= 16 && std::find(bzs.begin(), bzs.end(), b) == bzs.end()) bzs.push_back(b);
    }
    for (int ty : {4, 8, 16})
      for (int bz : bzs) cands.push_back({32, ty, bz, 0});
  }
  hipEvent_t e0, e1;
  AWE_HIP(hipEventCreate(&e0));
  AWE_HIP(hipEventCreate(&e1));
  std::vector<hipEvent_t> keep_ev;  // keep the probes out of kernel timing
  keep_ev.swap(P->prof_ev);
  // the probes run the kernels the plan's calls run: with FULL storage the forward stores its
  // levels (FP32 or scaled 16-bit) and the adjoint images from the store; with CHECKPOINT storage
  // the reverse sweep images from the recomputed forward buffers
  const bool full = P->store.mode == AWE_STORE_FULL;
  const int prec = P->store.prec;
  // PROBED storage: the probes accumulate into the probe sums too.  Their coefficients are read
  // from the sums the direction does not write (the forward reads the A sums, the adjoint the B
  // sums; every probe takes the same column, pitch 0), which hold max_nt floats when
  // max_nt <= 2 r npts; timing does not depend on the values.
  const bool probed = P->store.mode == AWE_STORE_PROBED &&
                      (long long)P->max_nt <= 2LL * P->store.nslots * P->sd[0].npts;
  const int fkind = probed ? awe::kStoreProbe
                    : !full ? awe::kStoreNone
                    : prec == AWE_PREC_FP32 ? awe::kStoreF32 : prec == AWE_PREC_BF16 ? awe::kStoreBF16 : awe::kStoreFP16;
  const int img = probed ? awe::kImgProbe
                  : full ? (prec == AWE_PREC_FP32 ? awe::kImgFull32 : prec == AWE_PREC_BF16 ? awe::kImgFullBF16
                                                                                          : awe::kImgFullFP16)
                         : P->sd[0].acc >= 0 ? awe::kImgBuffers : awe::kImgNone;
  double best[2] = {1e300, 1e300};
  Cand win[2] = {cands[0], cands[0]};
  P->cur = 0;  // the probes time the first shot group
  auto fail_out = [&](awe_status e) {
    keep_ev.swap(P->prof_ev);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
  };
  for (int dir = 0; dir < 2; ++dir) {
    Tiling& T = dir == 0 ? P->fw : P->rv;
    const int bit = dir == 0 ? AWE_FUSE_FORWARD : AWE_FUSE_ADJOINT;
    for (const Cand& c : cands) {
      // a checkpointed gradient recomputes one level per launch; its reversals run in pairs
      if (c.fuse && dir == 0 && P->store.mode == AWE_STORE_CHECKPOINT) continue;
      T.tz = c.tz;
      T.ty = c.ty;
      T.bz = c.bz;
      P->fuse2 = (P->fuse2 & ~bit) | (c.fuse ? bit : 0);
      if ((st = rebuild(P, dir == 0 ? 1 : 2)) != AWE_OK) return fail_out(st);
      if ((st = prepare(P, m, ws, true, true, s)) != AWE_OK) return fail_out(st);
      for (int i = 0; i < P->nshot; ++i) {
        if (P->sd[i].acc >= 0)
          if (hipError_t e = awe::launch_fill(static_cast<unsigned char*>(ws), P->sd[i].acc, P->sd[i].npts * 8, s))
            return fail_out(hip_fail(e, "autotune fill"));
        if (full && prec != AWE_PREC_FP32)  // per-level scales the 16-bit stores take their maxima into
          if (hipError_t e = awe::launch_fill(static_cast<unsigned char*>(ws), P->sd[i].scale,
                                              (long long)P->sd[i].nt * awe::kScaleSlots * 4, s))
            return fail_out(hip_fail(e, "autotune fill"));
      }
      awe::StepArgs fa = base_args(P, P->fw, ws);
      fa.q = q;
      awe::StepArgs aa = base_args(P, P->rv, ws);
      aa.dd = dd;
      aa.image_src = img;
      if (probed) {
        const ShotDev& d0 = P->sd[0];
        unsigned char* wsb = static_cast<unsigned char*>(ws);
        fa.probe_c = reinterpret_cast<const float*>(wsb + d0.store + (long long)P->store.nslots * d0.npts * 8);
        aa.probe_c = reinterpret_cast<const float*>(wsb + d0.store);
        fa.probe_r = aa.probe_r = P->store.nslots;
        fa.probe_pitch = aa.probe_pitch = 0;
      }
      if (hipError_t e = hipEventRecord(e0, s)) return fail_out(hip_fail(e, "autotune event"));
      // the last levels of the sweep, where every shot of an end-aligned batch is active (the
      // first levels of uneven batches cover only the longest shots)
      if (dir == 0) {
        const bool f2 = fused_ok(P, AWE_FUSE_FORWARD);
        const int k1 = P->ndim == 2 && fkind == awe::kStoreF32 ? awe::kStoreF32R : fkind;  // as forward_loop
        for (int n = std::max(1, P->nsteps - probe + 1); n + (f2 ? 1 : 0) <= P->nsteps; n += f2 ? 2 : 1)
          if ((st = f2 ? step_fwd2(P, fa, n, fkind, s) : step_fwd(P, fa, n, k1, s)) != AWE_OK)
            return fail_out(st);
      } else {
        const bool a2 = fused_ok(P, AWE_FUSE_ADJOINT);
        for (int n = P->nsteps; n > P->nsteps - probe && n >= 2; n -= a2 ? 2 : 1)
          if ((st = a2 ? step_adj2(P, aa, n, s) : step_adj(P, aa, n, s)) != AWE_OK) return fail_out(st);
      }
      if (hipError_t e = hipEventRecord(e1, s)) return fail_out(hip_fail(e, "autotune event"));
      if (hipError_t e = hipEventSynchronize(e1)) return fail_out(hip_fail(e, "autotune event"));
      float ms = 0.f;
      if (hipError_t e = hipEventElapsedTime(&ms, e0, e1)) return fail_out(hip_fail(e, "autotune event"));
      if (ms < best[dir]) {
        best[dir] = ms;
        win[dir] = c;
      }
    }
  }
  keep_ev.swap(P->prof_ev);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->fw.tz = win[0].tz;
  P->fw.ty = win[0].ty;
  P->fw.bz = win[0].bz;
  P->rv.tz = win[1].tz;
  P->rv.ty = win[1].ty;
  P->rv.bz = win[1].bz;
  P->fuse2 = (win[0].fuse ? AWE_FUSE_FORWARD : 0) | (win[1].fuse ? AWE_FUSE_ADJOINT : 0);
  if ((st = rebuild(P, 3)) != AWE_OK) return st;
  if (chosen) {
    chosen[0] = P->fw.tz;
    chosen[1] = P->fw.ty;
    chosen[2] = P->fw.bz;
    chosen[3] = P->fuse2;
  }
  if (best_ms) *best_ms = best[0] + best[1];
  if (cache && *cache) {
    auto entries = read_tune_cache(cache);
    entries[key] = TuneEntry{{P->fw.tz, P->fw.ty, P->fw.bz}, {P->rv.tz, P->rv.ty, P->rv.bz}, P->fuse2,
                             best[0] + best[1]};
    write_tune_cache(cache, entries);
  }
  return AWE_OK;
}

awe_status awe_plan_set_checks(awe_plan* P, int32_t flags) {
  if (!P) return fail(AWE_ERR_INVALID_ARG, "plan is NULL");
  if (flags < 0 || flags > (AWE_CHECK_INPUTS | AWE_CHECK_OUTPUTS | AWE_CHECK_LAUNCHES))
    return fail(AWE_ERR_INVALID_ARG, "flags must combine AWE_CHECK_INPUTS, AWE_CHECK_OUTPUTS, AWE_CHECK_LAUNCHES");
  if ((flags & (AWE_CHECK_INPUTS | AWE_CHECK_OUTPUTS)) && !P->chk_dev) AWE_HIP(hipMalloc(&P->chk_dev, 2 * kMaxScreened * sizeof(unsigned long long)));
  P->checks = flags;
  return AWE_OK;
}

awe_status awe_plan_get_tiles(const awe_plan* P, int32_t fwd[3], int32_t adj[3], int32_t* fusion) {
  if (!P) return fail(AWE_ERR_INVALID_ARG, "plan is NULL");
  if (fwd) {
    fwd[0] = P->fw.tz;
    fwd[1] = P->fw.ty;
    fwd[2] = P->fw.bz;
  }
  if (adj) {
    adj[0] = P->rv.tz;
    adj[1] = P->rv.ty;
    adj[2] = P->rv.bz;
  }
  if (fusion) *fusion = P->fuse2;
  return AWE_OK;
}

awe_status awe_plan_set_tiles_dir(awe_plan* P, int32_t dirs, int32_t tz, int32_t ty, int32_t bz) {
  if (!P) return fail(AWE_ERR_INVALID_ARG, "plan is NULL");
  if (dirs < 1 || dirs > 3) return fail(AWE_ERR_INVALID_ARG, "dirs must be 1 (forward), 2 (adjoint) or 3");
  if (tz != 8 && tz != 12 && tz != 16 && tz != 20 && tz != 24 && tz != 32 && tz != 64)
    return fail(AWE_ERR_INVALID_ARG, "tz must be 8, 12, 16, 20, 24, 32 or 64");
  if (ty != 4 && ty != 8 && ty != 16) return fail(AWE_ERR_INVALID_ARG, "ty must be 4, 8 or 16");
  if (bz < 0) return fail(AWE_ERR_INVALID_ARG, "bz must be >= 0");
  for (Tiling* T : {&P->fw, &P->rv}) {
    if (!(dirs & (T == &P->fw ? 1 : 2))) continue;
    T->tz = tz;
    T->ty = ty;
    T->bz = bz;
  }
  P->kept_ws = nullptr;
  return rebuild(P, dirs);
}

awe_status awe_plan_set_tiles(awe_plan* P, int32_t tz, int32_t ty, int32_t bz) {
  return awe_plan_set_tiles_dir(P, 3, tz, ty, bz);
}

awe_status awe_plan_set_groups(awe_plan* P, int32_t ngroups, int32_t* actual) {
  if (!P) return fail(AWE_ERR_INVALID_ARG, "plan is NULL");
  if (ngroups < 0) return fail(AWE_ERR_INVALID_ARG, "ngroups must be >= 0");
  P->groups_req = ngroups;
  P->kept_ws = nullptr;
  awe_status st = rebuild(P, 3);
  if (st == AWE_OK && actual) *actual = (int32_t)P->g_nshot.size();
  return st;
}

awe_status awe_plan_set_fusion(awe_plan* P, int32_t mode) {
  if (!P) return fail(AWE_ERR_INVALID_ARG, "plan is NULL");
  if (mode < 0 || mode > AWE_FUSE_BOTH) return fail(AWE_ERR_INVALID_ARG, "fusion mode must be 0..3");
  P->fuse2 = mode;
  // two-level kernels exist for 8, 16, 24 and 32 rows
  awe_status st = AWE_OK;
  for (int bit : {AWE_FUSE_FORWARD, AWE_FUSE_ADJOINT}) {
    Tiling& T = bit == AWE_FUSE_FORWARD ? P->fw : P->rv;
    if ((mode & bit) && !two_level_rows(T.tz))
      if ((st = awe_plan_set_tiles_dir(P, bit, T.tz < 24 ? 16 : 32, T.ty, T.bz)) != AWE_OK) return st;
  }
  return st;
}

awe_status awe_profile_enable(awe_plan* P, int64_t max_launches, int32_t stride) {
  if (!P || max_launches < 1 || stride < 1) return fail(AWE_ERR_INVALID_ARG, "bad profiling arguments");
  P->prof_stride = stride;
  P->prof_seen = 0;
  for (hipEvent_t e : P->prof_ev) (void)hipEventDestroy(e);
  P->prof_ev.clear();
  P->prof_cls.clear();
  P->prof_cnt.clear();
  P->prof_in_run = false;
  P->prof_next = 0;
  P->prof_ev.resize(2 * (size_t)max_launches, nullptr);
  for (auto& e : P->prof_ev) AWE_HIP(hipEventCreate(&e));
  return AWE_OK;
}

awe_status awe_profile_read(awe_plan* P, int64_t counts[3], double ms[3]) {
  if (!P || !counts || !ms) return fail(AWE_ERR_INVALID_ARG, "bad profiling arguments");
  for (int c = 0; c < 3; ++c) {
    counts[c] = 0;
    ms[c] = 0.0;
  }
  if (P->prof_next > 0) AWE_HIP(hipEventSynchronize(P->prof_ev[P->prof_next - 1]));
  for (size_t i = 0; 2 * i + 1 < P->prof_next; ++i) {
    float t = 0.f;
    AWE_HIP(hipEventElapsedTime(&t, P->prof_ev[2 * i], P->prof_ev[2 * i + 1]));
    const int c = P->prof_cls[i];
    counts[c] += P->prof_cnt[i];
    ms[c] += t;
  }
  P->prof_next = 0;
  P->prof_seen = 0;
  P->prof_cls.clear();
  P->prof_cnt.clear();
  return AWE_OK;
}

awe_status awe_profile_disable(awe_plan* P) {
  if (!P) return fail(AWE_ERR_INVALID_ARG, "plan is NULL");
  for (hipEvent_t e : P->prof_ev) (void)hipEventDestroy(e);
  P->prof_ev.clear();
  P->prof_cls.clear();
  P->prof_cnt.clear();
  P->prof_in_run = false;
  P->prof_next = 0;
  return AWE_OK;
}

awe_status awe_forward(awe_plan* P, const float* m, const float* q, float* d, int keep, void* ws,
                       size_t ws_bytes, void* stream) {
  awe_status st = check_ws(P, ws, ws_bytes);
  if (st != AWE_OK) return st;
  if (!m || !q) return fail(AWE_ERR_INVALID_ARG, "m and q must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((P->checks & AWE_CHECK_INPUTS) &&
      (st = screen(P, {{m, false, kPerWindow, "m", true}, {q, false, kPerShotQ, "q", false}}, s)) != AWE_OK)
    return st;
  const bool store = keep && (P->store.mode == AWE_STORE_FULL || P->store.mode == AWE_STORE_CHECKPOINT);
  P->kept_ws = nullptr;
  if ((st = prepare(P, m, ws, true, false, s)) != AWE_OK) return st;
  awe::StepArgs a = base_args(P, P->fw, ws);
  a.q = q;
  a.d = d;
  const int G = (int)P->g_nshot.size();
  if (store && P->store.mode == AWE_STORE_CHECKPOINT) {
    awe::StepArgs aa = base_args(P, P->rv, ws);  // no adjoint step runs before the first reverse
    for (P->cur = 0; P->cur < G; ++P->cur)
      if ((st = run_actions(P, a, aa, 0, P->sched_first_reverse, s)) != AWE_OK) return st;
  } else {
    int kind = awe::kStoreNone;
    if (store) {
      kind = P->store.prec == AWE_PREC_FP32 ? awe::kStoreF32
             : P->store.prec == AWE_PREC_BF16 ? awe::kStoreBF16 : awe::kStoreFP16;
      if (kind != awe::kStoreF32)
        for (int i = 0; i < P->nshot; ++i)
          if ((st = fill(P, a.ws, P->sd[i].scale, (long long)P->sd[i].nt * awe::kScaleSlots * 4, s, "level scales")) != AWE_OK)
            return st;
    }
    for (P->cur = 0; P->cur < G; ++P->cur)
      if ((st = forward_loop(P, a, kind, s)) != AWE_OK) return st;
    if (kind == awe::kStoreBF16 || kind == awe::kStoreFP16)
      AWE_HIP(awe::launch_store_last(a, P->nshot, P->max_win_npts, s));
  }
  if (d) AWE_HIP(awe::launch_gather_last(a, P->nshot, P->total_recs, 0, s));
  if (store) P->kept_ws = ws;
  if ((P->checks & AWE_CHECK_OUTPUTS) && d && (st = screen(P, {{d, false, kPerShotD, "d", false}}, s)) != AWE_OK)
    return st;
  return AWE_OK;
}

awe_status awe_backward(awe_plan* P, const float* m, const float* q, const float* dd, double* g,
                        float* v, void* ws, size_t ws_bytes, void* stream) {
  awe_status st = check_ws(P, ws, ws_bytes);
  if (st != AWE_OK) return st;
  if (!dd || !q) return fail(AWE_ERR_INVALID_ARG, "q and dd must not be NULL");
  if ((P->store.mode != AWE_STORE_FULL && P->store.mode != AWE_STORE_CHECKPOINT) || P->kept_ws != ws)
    return fail(AWE_ERR_STATE, "the workspace holds no kept forward wavefield of this plan");
  (void)m;  // the coefficients of the kept forward are reused
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((P->checks & AWE_CHECK_INPUTS) &&
      (st = screen(P, {{q, false, kPerShotQ, "q", false}, {dd, false, kPerShotD, "dd", false}}, s)) != AWE_OK)
    return st;
  unsigned char* w = static_cast<unsigned char*>(ws);
  for (int i = 0; i < P->nshot; ++i) {
    const ShotDev& d = P->sd[i];
    if ((st = fill(P, w, d.fld + 4 * d.npts * 4, 4 * d.npts * 4, s, "adjoint buffers")) != AWE_OK) return st;
  }
  if (g)
    for (int i = 0; i < P->nshot; ++i)
      if ((st = fill(P, w, P->sd[i].acc, P->sd[i].npts * 8, s, "accumulator")) != AWE_OK) return st;
  awe::StepArgs fa = base_args(P, P->fw, ws);
  fa.q = q;
  awe::StepArgs aa = base_args(P, P->rv, ws);
  aa.dd = dd;
  aa.v = v;
  if (P->store.mode == AWE_STORE_FULL) {
    aa.image_src = !g ? awe::kImgNone
                   : P->store.prec == AWE_PREC_FP32 ? awe::kImgFull32
                   : P->store.prec == AWE_PREC_BF16 ? awe::kImgFullBF16 : awe::kImgFullFP16;
    for (P->cur = 0; P->cur < (int)P->g_nshot.size(); ++P->cur)
      if ((st = adjoint_loop(P, aa, s)) != AWE_OK) return st;
  } else {
    aa.image_src = g ? awe::kImgBuffers : awe::kImgNone;
    for (P->cur = 0; P->cur < (int)P->g_nshot.size(); ++P->cur)
      if ((st = run_actions(P, fa, aa, P->sched_first_reverse, P->sched.size() / 3, s)) != AWE_OK) return st;
    P->kept_ws = nullptr;  // the recomputation overwrote the kept forward state
  }
  if (v) AWE_HIP(awe::launch_src_last(aa, P->nshot, s));
  if (g)
    AWE_HIP(awe::launch_grad_reduce(P->rv.tab, (int)P->wins.size(), P->max_win_npts, w, g,
                                    -1.0 / (P->dt * P->dt), s));
  if ((P->checks & AWE_CHECK_OUTPUTS) && (g || v) &&
      (st = screen(P, {{g, true, kPerWindow, "g", false}, {v, false, kPerShotQ, "v", false}}, s)) != AWE_OK)
    return st;
  return AWE_OK;
}

awe_status awe_gradient(awe_plan* P, const float* m, const float* q, const float* dd, double* g,
                        float* v, float* d, void* ws, size_t ws_bytes, void* stream) {
  if (P && P->store.mode != AWE_STORE_FULL && P->store.mode != AWE_STORE_CHECKPOINT)
    return fail(AWE_ERR_UNSUPPORTED, P->store.mode == AWE_STORE_PROBED
                                         ? "PROBED storage: use awe_gradient_probed"
                                         : "gradient needs FULL or CHECKPOINT storage");
  awe_status st = AWE_OK;
  const int checks = P ? P->checks : 0;
  if (checks & AWE_CHECK_INPUTS) {
    // all three inputs before any compute work; the two sweeps then skip their own input screening
    if ((st = check_ws(P, ws, ws_bytes)) != AWE_OK) return st;
    if (!m || !q || !dd) return fail(AWE_ERR_INVALID_ARG, "m, q and dd must not be NULL");
    if ((st = screen(P, {{m, false, kPerWindow, "m", true}, {q, false, kPerShotQ, "q", false},
                         {dd, false, kPerShotD, "dd", false}}, static_cast<hipStream_t>(stream))) != AWE_OK)
      return st;
    P->checks &= ~AWE_CHECK_INPUTS;
  }
  st = awe_forward(P, m, q, d, 1, ws, ws_bytes, stream);
  if (st == AWE_OK) st = awe_backward(P, m, q, dd, g, v, ws, ws_bytes, stream);
  if (P) P->checks = checks;
  return st;
}

awe_status awe_gradient_probed(awe_plan* P, const float* m, const float* q, const float* dd, const float* C,
                               const double* s_w, double* g, float* v, float* d, void* ws, size_t ws_bytes,
                               void* stream) {
  awe_status st = check_ws(P, ws, ws_bytes);
  if (st != AWE_OK) return st;
  if (P->store.mode != AWE_STORE_PROBED) return fail(AWE_ERR_UNSUPPORTED, "the plan's storage is not PROBED");
  if (!m || !q || !dd || !C || !s_w || !g) return fail(AWE_ERR_INVALID_ARG, "m, q, dd, C, s and g must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((P->checks & AWE_CHECK_INPUTS) &&
      (st = screen(P, {{m, false, kPerWindow, "m", true}, {q, false, kPerShotQ, "q", false},
                       {dd, false, kPerShotD, "dd", false}}, s)) != AWE_OK)
    return st;
  const int r = P->store.nslots;
  awe::ProbeWeights w{};
  for (int j = 0; j < r; ++j) w.s[j] = s_w[j];
  P->kept_ws = nullptr;
  if ((st = prepare(P, m, ws, true, true, s)) != AWE_OK) return st;
  unsigned char* wsb = static_cast<unsigned char*>(ws);
  for (int i = 0; i < P->nshot; ++i)
    if ((st = fill(P, wsb, P->sd[i].store, (long long)r * 2 * P->sd[i].npts * 8, s, "probe sums")) != AWE_OK) return st;
  // forward sweep: B_j += C[j][k] (u^k - 2u^{k-1} + u^{k-2}) in the step kernels
  awe::StepArgs a = base_args(P, P->fw, ws);
  a.q = q;
  a.d = d;
  a.probe_c = C;
  a.probe_r = r;
  a.probe_pitch = P->max_nt;
  for (P->cur = 0; P->cur < (int)P->g_nshot.size(); ++P->cur)
    if ((st = forward_loop(P, a, awe::kStoreProbe, s)) != AWE_OK) return st;
  if (d) AWE_HIP(awe::launch_gather_last(a, P->nshot, P->total_recs, 0, s));
  // reverse sweep: A_j += C[j][k] w^k in the adjoint step kernels
  awe::StepArgs aa = base_args(P, P->rv, ws);
  aa.dd = dd;
  aa.v = v;
  aa.image_src = awe::kImgProbe;
  aa.probe_c = C;
  aa.probe_r = r;
  aa.probe_pitch = P->max_nt;
  for (P->cur = 0; P->cur < (int)P->g_nshot.size(); ++P->cur)
    if ((st = adjoint_loop(P, aa, s)) != AWE_OK) return st;
  if (v) AWE_HIP(awe::launch_src_last(aa, P->nshot, s));
  AWE_HIP(awe::launch_probe_reduce(P->rv.tab, (int)P->wins.size(), P->max_win_npts, wsb, r, w, g,
                                   -1.0 / (P->dt * P->dt), s));
  if ((P->checks & AWE_CHECK_OUTPUTS) &&
      (st = screen(P, {{g, true, kPerWindow, "g", false}, {v, false, kPerShotQ, "v", false},
                       {d, false, kPerShotD, "d", false}}, s)) != AWE_OK)
    return st;
  return AWE_OK;
}

awe_status awe_adjoint(awe_plan* P, const float* m, const float* dd, float* v, void* ws,
                       size_t ws_bytes, void* stream) {
  awe_status st = check_ws(P, ws, ws_bytes);
  if (st != AWE_OK) return st;
  if (!m || !dd || !v) return fail(AWE_ERR_INVALID_ARG, "m, dd and v must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((P->checks & AWE_CHECK_INPUTS) &&
      (st = screen(P, {{m, false, kPerWindow, "m", true}, {dd, false, kPerShotD, "dd", false}}, s)) != AWE_OK)
    return st;
  P->kept_ws = nullptr;
  if ((st = prepare(P, m, ws, false, true, s)) != AWE_OK) return st;
  awe::StepArgs a = base_args(P, P->rv, ws);
  a.dd = dd;
  a.v = v;
  a.image_src = awe::kImgNone;
  for (P->cur = 0; P->cur < (int)P->g_nshot.size(); ++P->cur)
    if ((st = adjoint_loop(P, a, s)) != AWE_OK) return st;
  AWE_HIP(awe::launch_src_last(a, P->nshot, s));
  if ((P->checks & AWE_CHECK_OUTPUTS) && (st = screen(P, {{v, false, kPerShotQ, "v", false}}, s)) != AWE_OK)
    return st;
  return AWE_OK;
}

awe_status awe_born(awe_plan* P, const float* m, const float* q, const float* dm, float* dd,
                    void* ws, size_t ws_bytes, void* stream) {
  awe_status st = check_ws(P, ws, ws_bytes);
  if (st != AWE_OK) return st;
  if (!m || !q || !dm || !dd) return fail(AWE_ERR_INVALID_ARG, "m, q, dm and dd must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((P->checks & AWE_CHECK_INPUTS) &&
      (st = screen(P, {{m, false, kPerWindow, "m", true}, {q, false, kPerShotQ, "q", false},
                       {dm, false, kPerWindow, "dm", false}}, s)) != AWE_OK)
    return st;
  P->kept_ws = nullptr;
  if ((st = prepare(P, m, ws, true, true, s)) != AWE_OK) return st;
  awe::StepArgs a = base_args(P, P->fw, ws);
  a.q = q;
  a.dm = dm;
  a.d = dd;
  // 2D with the forward's two-level mode: levels in pairs (a single first step when the count
  // is odd), as the forward solves
  const bool fuse = fused_ok(P, AWE_FUSE_FORWARD);
  for (P->cur = 0; P->cur < (int)P->g_nshot.size(); ++P->cur) {
    ProfRun run(P, s, 2);
    for (int n = 1; n <= P->nsteps;) {
      const bool two = fuse && (n > 1 || !(P->nsteps & 1));
      set_group(P, P->fw, a, two ? n + 1 : n);
      a.step = n;
      if (a.ntiles > 0) {
        if ((st = check_step(P, P->fw, a, n, two ? n + 1 : n, "Born step")) != AWE_OK) return st;
        ProfScope ps(P, 2, s);
        if (P->ndim == 3) AWE_HIP(awe::launch_born3d(a, P->fw.ty, P->fw.bz, s));
        else if (two) AWE_HIP(awe::launch_born2d2(a, P->fw.tz, s));
        else AWE_HIP(awe::launch_born2d(a, P->fw.tz, s));
      }
      n += two ? 2 : 1;
    }
  }
  AWE_HIP(awe::launch_gather_last(a, P->nshot, P->total_recs, 1, s));
  if ((P->checks & AWE_CHECK_OUTPUTS) && (st = screen(P, {{dd, false, kPerShotD, "dd", false}}, s)) != AWE_OK)
    return st;
  return AWE_OK;
}

size_t awe_reduce_workspace_size(int64_t n) {
  (void)n;
  return (size_t)awe::kReduceBlocks * 8;
}

awe_status awe_residual(const float* d_pred, const float* d_obs, float* r, int64_t n, double* loss,
                        void* ws, size_t ws_bytes, void* stream) {
  if (!d_pred || !d_obs || n < 0) return fail(AWE_ERR_INVALID_ARG, "bad residual arguments");
  if (!ws || ws_bytes < awe_reduce_workspace_size(n)) return fail(AWE_ERR_WORKSPACE, "reduction workspace too small");
  AWE_HIP(awe::launch_residual(d_pred, d_obs, r, n, loss, static_cast<unsigned char*>(ws),
                               static_cast<hipStream_t>(stream)));
  return AWE_OK;
}

awe_status awe_residual_noalloc(const float* d_pred, const float* d_obs, float* r, int64_t n,
                                double* loss, void* stream) {
  if (!d_pred || !d_obs || n < 0) return fail(AWE_ERR_INVALID_ARG, "bad residual arguments");
  double* part = nullptr;
  AWE_HIP(awe::scratch_partials(&part));
  AWE_HIP(awe::launch_residual(d_pred, d_obs, r, n, loss, reinterpret_cast<unsigned char*>(part),
                               static_cast<hipStream_t>(stream)));
  return AWE_OK;
}

awe_status awe_dot_f64(const float* a, const float* b, int64_t n, double* out, void* ws,
                       size_t ws_bytes, void* stream) {
  if (!a || !b || !out || n < 0) return fail(AWE_ERR_INVALID_ARG, "bad dot arguments");
  if (!ws || ws_bytes < awe_reduce_workspace_size(n)) return fail(AWE_ERR_WORKSPACE, "reduction workspace too small");
  AWE_HIP(awe::launch_dot(a, b, n, out, static_cast<unsigned char*>(ws), static_cast<hipStream_t>(stream)));
  return AWE_OK;
}

awe_status awe_dot_f64d(const double* a, const double* b, int64_t n, double* out, void* ws,
                        size_t ws_bytes, void* stream) {
  if (!a || !b || !out || n < 0) return fail(AWE_ERR_INVALID_ARG, "bad dot arguments");
  if (!ws || ws_bytes < awe_reduce_workspace_size(n)) return fail(AWE_ERR_WORKSPACE, "reduction workspace too small");
  AWE_HIP(awe::launch_dotd(a, b, n, out, static_cast<unsigned char*>(ws), static_cast<hipStream_t>(stream)));
  return AWE_OK;
}

awe_status awe_slowness2(const float* v, float* m, int64_t n, void* stream) {
  if (!v || !m || n < 0) return fail(AWE_ERR_INVALID_ARG, "bad slowness arguments");
  AWE_HIP(awe::launch_slowness2(v, m, n, static_cast<hipStream_t>(stream)));
  return AWE_OK;
}

awe_status awe_velocity_gradient(const float* v, const float* gm, float* gv, int64_t n, void* stream) {
  if (!v || !gm || !gv || n < 0) return fail(AWE_ERR_INVALID_ARG, "bad velocity-gradient arguments");
  AWE_HIP(awe::launch_velocity_gradient(v, gm, gv, n, static_cast<hipStream_t>(stream)));
  return AWE_OK;
}

namespace {
awe::PatchyConsts patchy_consts(const awe_patchy_consts* c) {
  if (c) return {c->k_min, c->k_brine, c->k_co2, c->rho_co2, c->rho_brine};
  return {36.6e9, 2.735e9, 0.125e9, 700.0, 1000.0};
}
}  // namespace

awe_status awe_patchy(const float* s, const float* vp, const float* rho, const float* phi, float* vp_new,
                      float* rho_new, int64_t n, const awe_patchy_consts* c, void* stream) {
  if (n < 0 || (n > 0 && (!s || !vp || !rho || !phi || !vp_new)))
    return fail(AWE_ERR_INVALID_ARG, "bad patchy arguments");
  AWE_HIP(awe::launch_patchy(s, vp, rho, phi, vp_new, rho_new, n, patchy_consts(c),
                             static_cast<hipStream_t>(stream)));
  return AWE_OK;
}

awe_status awe_patchy_vjp(const float* s, const float* vp, const float* rho, const float* phi,
                          const float* g_vp, const float* g_rho, float* g_s, int64_t n,
                          const awe_patchy_consts* c, void* stream) {
  if (n < 0 || (n > 0 && (!s || !vp || !rho || !phi || !g_vp || !g_s)))
    return fail(AWE_ERR_INVALID_ARG, "bad patchy vjp arguments");
  AWE_HIP(awe::launch_patchy_vjp(s, vp, rho, phi, g_vp, g_rho, g_s, n, patchy_consts(c),
                                 static_cast<hipStream_t>(stream)));
  return AWE_OK;
}

awe_status awe_checkpoint_schedule(int32_t nsteps, int32_t nslots, int32_t* actions, int64_t cap,
                                   int64_t* count) {
  if (nsteps < 0 || nslots < 0 || !count || (cap > 0 && !actions))
    return fail(AWE_ERR_INVALID_ARG, "bad schedule arguments");
  std::vector<int32_t> v;
  awe::build_schedule(nsteps, nslots, v);
  *count = (int64_t)(v.size() / 3);
  if (*count > cap) return fail(AWE_ERR_INVALID_ARG, "action buffer too small");
  if (!v.empty()) std::memcpy(actions, v.data(), v.size() * sizeof(int32_t));
  return AWE_OK;
}

}  // extern "C"
