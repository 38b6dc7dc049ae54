// Host runtime and C ABI of lbnlm: parameter resolution, workspace layout,
// strip work lists, captured step graphs, convergence checks, observation
// and state transfer. See include/lb.h for the contract of every entry point.
#include "lb.h"
#include "lb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace lbnlm;

// Scratch of the allocation-free observation (lb_observe_noalloc): the
// per-strip partials, per-row profiles and per-channel scalars of one
// observation and the gathered result live in this file-scope device array
// instead of the handle's workspace. Each GPU the library runs on holds its
// own copy until the process ends; every call on that GPU shares it.
constexpr size_t kNoallocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) double scratch[kNoallocScratchBytes / sizeof(double)];

namespace {

constexpr int kDefaultK = 1000;
constexpr size_t kAlign = 256;
#ifndef LB_WG_WAVES
#define LB_WG_WAVES 4
#endif
constexpr int kWaves = LB_WG_WAVES;  // wavefronts (strips) per workgroup


size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// D2Q9 velocities and rest weights, host side (layout conversion only).
constexpr int HCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int HCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int HOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
inline double hweight(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }

struct Layout {
  long long plane = 0;       // nodes per state buffer (multiple of the tile)
  int esize = 8;             // bytes per element
  int total_rows = 0;
  int total_part = 0;
  int max_strips = 0;
  int n_tiles = 0;  // tiles of the tiled step (stress force, or FP64 strip-class channels)
  size_t off_state[2] = {0, 0}, off_ch = 0, off_strips = 0, off_astrips = 0, off_rstrips = 0, off_part = 0,
         off_prof = 0, off_prev = 0, off_scal = 0, off_uref = 0, bytes = 0;
  size_t off_stress[2] = {0, 0};  // viscoelastic model only
  size_t off_saf_u = 0, off_saf_t = 0;  // stress-as-force scratch (u~, Sigma^nN)
  size_t off_tiles = 0;                 // tiles of the tiled step
  // two steps per launch: strips of the other channels for captured blocks
  // (and their reverse), and the two-step strips
  size_t off_bstrips = 0, off_brstrips = 0, off_tstrips = 0;
  size_t off_btiles = 0;  // tiles of the tiled channels without two-step strips
  int strip_cap = 0;      // entries of each one-step strip list
  int max_two = 0;
  std::vector<ChanDev> ch;
};

std::string validate(const lb_channel *c, int n, const lb_options *o) {
  if (!c || n <= 0) return "no channels";
  if (!o) return "options are NULL";
  if (o->precision != LB_FP64 && o->precision != LB_FP32_SHIFTED) return "unknown precision";
  if (o->obs_every < 0 || (o->obs_every > 0 && (o->obs_every < 2 || (o->obs_every & 1))))
    return "obs_every must be 0 or an even number >= 2";
  if (o->strip_rows < 0 || o->strip_rows > 4096) return "strip_rows out of range";
  if (!(o->steady_tol >= 0) || !std::isfinite(o->steady_tol)) return "steady_tol must be >= 0";
  if (o->viscoelastic != 0 && o->viscoelastic != 1) return "viscoelastic must be 0 or 1";
  if (o->stress_force != 0 && o->stress_force != 1) return "stress_force must be 0 or 1";
  if (o->steps_per_sweep < 0 || o->steps_per_sweep > 2) return "steps_per_sweep must be 0, 1 or 2";
  if (o->stress_force && (o->precision != LB_FP64 || o->viscoelastic))
    return "stress_force needs FP64 and the instantaneous model";
  for (int i = 0; i < n; ++i) {
    const lb_channel &q = c[i];
    char buf[160];
    auto bad = [&](const char *what) {
      snprintf(buf, sizeof buf, "channel %d: %s", i, what);
      return std::string(buf);
    };
    if (q.nx < 1 || q.ny < 1) return bad("nx and ny must be >= 1");
    if ((long long)q.nx * q.ny > (1LL << 31)) return bad("too many nodes");
    if (!(q.tau_lb > 0.5) || !std::isfinite(q.tau_lb)) return bad("tau_lb must be > 1/2");
    if (!(q.G >= 0) || !std::isfinite(q.G)) return bad("G must be >= 0");
    if (!(q.tau0 > 0)) return bad("tau0 must be > 0");
    if (!(q.gamma_c > 0)) return bad("gamma_c must be > 0");
    if (!std::isfinite(q.force)) return bad("force must be finite");
    if (!std::isfinite(q.eps)) return bad("eps must be finite");
    if (!(q.visc_split >= 0 && q.visc_split <= 1)) return bad("visc_split must be in [0,1]");
    if (q.visc_split > 0 && std::isinf(q.tau0)) return bad("visc_split > 0 needs a finite tau0");
    if (!(std::fabs(q.wall_velocity) < 0.3)) return bad("wall_velocity must be finite with |u_w| < 0.3");
    if (!std::isfinite(q.pressure_gradient)) return bad("pressure_gradient must be finite");
    if (q.nn_pressure != 0 && q.nn_pressure != 1) return bad("nn_pressure must be 0 or 1");
    if (q.top_wall != LB_WALL_HALFWAY && q.top_wall != LB_WALL_ZOU_HE) return bad("unknown top_wall");
    if (q.top_wall == LB_WALL_ZOU_HE && (q.ny < 2 || q.pressure_gradient != 0 || o->stress_force))
      return bad("a Zou-He top wall needs ny >= 2, no pressure_gradient and no stress_force");
    if (q.pressure_gradient != 0 && (q.force != 0 || q.wall_velocity != 0 || q.nx < 2 || q.nn_pressure))
      return bad("pressure_gradient needs force = 0, wall_velocity = 0, nx >= 2 and nn_pressure = 0");
    if (q.pressure_gradient != 0 && o->stress_force) return bad("pressure_gradient is not combined with stress_force");
    if (o->stress_force && q.nn_pressure) return bad("stress_force needs nn_pressure = 0");
    if (o->stress_force && align_up((size_t)q.nx * q.ny, kTile) * kPlanes > 0xffffffffull)
      return bad("stress_force needs nx * ny <= 429,496,704 per channel");
  }
  return "";
}

// Separation closure and viscosity split of the channel parameters.
void resolve(const lb_channel &q, ChanDev &d) {
  const double eta_s = (q.tau_lb - 0.5) / 3.0;
  const double tau = q.tau0 * std::pow(10.0, std::min(q.eps, 0.0) / 0.05);
  const double Ginf = q.G * (1.0 + std::sqrt(std::max(q.eps, 0.0)));
  const double lgt = q.visc_split > 0 ? q.visc_split * Ginf * tau : 0.0;
  const double tau_eff = 0.5 + 3.0 * (eta_s + lgt);
  d.t = 0;
  d.t_startup = q.t_startup;
  d.nx = q.nx;
  d.ny = q.ny;
  d.active = 1;
  d.g = q.force;
  d.omega = 1.0 / tau_eff;
  d.kf = 1.0 - 0.5 / tau_eff;
  d.sp = -4.5 / tau_eff;
  d.G = Ginf;
  d.inv_tau = std::isinf(tau) ? 0.0 : 1.0 / tau;
  d.inv_gc = 1.0 / q.gamma_c;
  d.lgt = lgt;
  d.uw = q.wall_velocity;
  d.gpbc = q.pressure_gradient != 0;
  d.pd = (q.nx + 1) * q.pressure_gradient;
  d.nnp = q.nn_pressure;
  d.zh = q.top_wall == LB_WALL_ZOU_HE;
}

// Term the pull adds to population i of a top-row node at step t: the link
// reflected at the moving half-way wall during step t - 1 gained
// -2 a c_x u_w / cs2 (a and c of the outgoing population opp(i)); only i = 7,
// 8 are affected (none at a Zou-He wall, which completes them instead).
double wall_pull_term(const lb_channel &q, int i, long long t) {
  const double uw = (q.top_wall == LB_WALL_HALFWAY && t >= 1 && t - 1 < q.t_startup) ? q.wall_velocity : 0.0;
  const int o = HOPP[i];
  return -6.0 * hweight(o) * HCX[o] * uw;
}

// Zou-He completion (the kernels' zou_he_top) of the top row's populations
// entering from above, on a host copy of a channel's state at step t:
// no flow through the wall, n4 = n2, and the diagonals such that
// (m + f/2)/s is the wall velocity of step t.
void host_zou_he_top(const lb_channel &q, long long t, double *pops) {
  const size_t N = (size_t)q.nx * q.ny;
  const double uw = t < q.t_startup ? q.wall_velocity : 0.0, fx = t < q.t_startup ? q.force : 0.0;
  for (int x = 0; x < q.nx; ++x) {
    const size_t id = (size_t)(q.ny - 1) * q.nx + x;
    double f[9];
    for (int i = 0; i < 9; ++i) f[i] = pops[(size_t)i * N + id];
    const double s = (f[0] + f[1] + f[3]) + 2.0 * (f[2] + f[5] + f[6]);
    const double d87 = (s * uw - 0.5 * fx) - ((f[1] - f[3]) + (f[5] - f[6]));
    pops[4 * N + id] = f[2];
    pops[8 * N + id] = 0.5 * ((f[5] + f[6]) + d87);
    pops[7 * N + id] = 0.5 * ((f[5] + f[6]) - d87);
  }
}

int strip_rows_for(int cls, int nx, int ny, int requested) {
  if (is_strip_class(cls)) {
    int s = requested > 0 ? requested : 16;
    return std::max(1, std::min(s, ny));
  }
  const int tyw = 64 / nx;
  int s = requested > 0 ? requested : std::max(64, tyw);
  s = (s + tyw - 1) / tyw * tyw;
  return s;
}

// Strips of one channel in row-band order: the strips of one band of rows
// are consecutive (x neighbours, which share cache lines at their edges,
// land on the same XCD), and bands follow each other upwards.
// With stack set, vector-sweep strips come in stacks of kWaves bands at one
// x, so that one workgroup (one CU) holds vertically adjacent strips, and odd
// bands march against the step's direction: two neighbouring strips then
// reach the rows they share (each one's halo and prefetch overrun) at the
// same time, and the second read hits in cache. That pays while a state
// buffer fits the last-level cache (measured: +1.4 points of HBM peak on
// 4096 x 1024 FP32); on larger states the row-band order of x neighbours is
// faster (-1.3 points with stacks on 16 x 8192 x 2048).
void add_strips(int ci, const ChanDev &d, int esize, int srows, bool stack, std::vector<Strip> &out) {
  const int cls = width_class(d.nx, esize);
  const int w = strip_cols(cls, esize);
  const int nxs = is_strip_class(cls) ? (d.nx + w - 1) / w : 1;
  const int nb = (d.ny + srows - 1) / srows;
  if (cls == kVecClass && stack) {
    for (int b0 = 0; b0 < nb; b0 += kWaves)
      for (int xs = 0; xs < nxs; ++xs)
        for (int b = b0; b < std::min(b0 + kWaves, nb); ++b)
          out.push_back(Strip{ci, xs * w, b * srows, std::min((b + 1) * srows, d.ny), b & 1});
    return;
  }
  for (int b = 0; b < nb; ++b)
    for (int xs = 0; xs < nxs; ++xs)
      out.push_back(Strip{ci, xs * w, b * srows, std::min((b + 1) * srows, d.ny), 0});
}

// Two steps per launch (sweep_vec2_kernel) for the blocks of captured steps:
// vector-class channels without the pressure drive (whose column pass runs
// between steps), with either stress model and any top wall, with blocks a multiple of four steps (a
// block is then an even number of two-step launches and returns the state
// to its buffer, as one-step launches do).
bool two_step_handle(const lb_options *o, int K) {
  return o->steps_per_sweep != 1 && !o->stress_force && K % 4 == 0;
}
bool two_step_channel(const lb_channel &c, int esize) {
  return width_class(c.nx, esize) == kVecClass && c.pressure_gradient == 0;
}
// The narrow widths (nx = 1, 2, ..., 64) of the instantaneous model take
// two steps per launch too (sweep_narrow2_kernel), without the pressure drive.
bool narrow_two_step_channel(const lb_options *o, const lb_channel &c, int esize) {
  return !o->viscoelastic && !is_strip_class(width_class(c.nx, esize)) && c.pressure_gradient == 0;
}
bool two_step_wall(const lb_channel &c) { return c.top_wall == LB_WALL_ZOU_HE || c.wall_velocity != 0; }
// Stored columns of the two-step strips of a width at npl nodes per lane:
// at most two_step_cols(npl) (248 at four, 124 at two), in multiples of
// npl, as even as possible.
std::vector<int> two_step_cuts(int nx, int npl) {
  const int cols = two_step_cols(npl);
  const int units = nx / npl, m = (nx + cols - 1) / cols;
  std::vector<int> x(1, 0);
  for (int i = 0; i < m; ++i) x.push_back(x.back() + npl * (units / m + (i < units % m)));
  return x;
}
// Rows per two-step strip: whole rounds of resident strips cost each
// strip's rows plus its four extra rows of step t and about two rows of
// start-up, so the height minimises rounds x (rows + 6) over 16..56 rows.
// From four rounds on, workgroups that finish early let the next ones
// start, so the cost is the strips' rows (each plus 6) over the slots (the
// tallest strips then win: 16 x 8192 x 2048 at 56 rows 108.7-108.9k MLUPS,
// at 50 rows, the whole-round choice, 107.3k).
int two_step_rows(const std::vector<lb_channel> &chans, int npl, int slots) {
  int best = 16;
  double best_cost = 1e300;
  for (int H = 16; H <= kTwoStepMaxRows; ++H) {
    long long S = 0, work = 0;
    for (const lb_channel &c : chans) {
      const long long cuts = (long long)(two_step_cuts(c.nx, npl).size() - 1), full = c.ny / H, rem = c.ny % H;
      S += cuts * (full + (rem > 0));
      work += cuts * (full * (H + 6) + (rem > 0 ? rem + 6 : 0));
    }
    const double r = (double)S / std::max(slots, 1);
    const double cost = r < 4.0 ? std::ceil(r) * (H + 6) : (double)work / std::max(slots, 1);
    if (S > 0 && cost < best_cost) {
      best_cost = cost;
      best = H;
    }
  }
  return best;
}
// Rows per narrow two-step strip: one height R for every narrow channel
// (1, 2, 4, a multiple of 8 up to 64, or a power of two; a channel's
// strips take it rounded up to its row group), the smallest whose strips
// all fit the GPU's resident workgroups at once (slots), so that the strips
// are as short as one round allows; not above the requested height when
// one is given; within the room left in the strip list. (Measured on
// 8-wide channels of 32..512 rows, 16 to 256 of them: among powers of two
// this height was the fastest in every case, a second round or strips
// twice as tall costing 10-55% per step; the multiples of 8 gained a
// further 14% with all 256 channels active, at 48 rows against 64, and
// lost 2% with 64 active, at 24 rows against 32.)
// a channel's rows per strip for height R: R rounded up to its row group
int narrow_rows(int R, int nx) {
  const int g = 64 / nx;
  return (std::max(R, g) + g - 1) / g * g;
}
int narrow_two_step_rows(const std::vector<lb_channel> &chans, long long slots, int requested, long long room) {
  // candidate heights: 1, 2, 4, every multiple of 8 up to 64, then powers
  // of two
  std::vector<int> cand = {1, 2, 4};
  for (int m = 8; m <= 64; m += 8) cand.push_back(m);
  for (int R = 128; R <= (1 << 30); R *= 2) {
    cand.push_back(R);
    if (R == (1 << 30)) break;
  }
  int last_fit = 0;  // the tallest height so far within the room
  for (const int R : cand) {
    if (requested > 0 && R > requested && last_fit > 0) return last_fit;
    long long S = 0;
    for (const lb_channel &c : chans) {
      const int rows = narrow_rows(R, c.nx);
      S += (c.ny + rows - 1) / rows;
    }
    if (S > room) continue;
    if (S <= slots) return R;
    last_fit = R;
  }
  return last_fit > 0 ? last_fit : 1 << 30;
}
void add_two_step_strips(int ci, const lb_channel &c, int npl, int H, std::vector<Strip> &out) {
  const std::vector<int> x = two_step_cuts(c.nx, npl);
  for (int y0 = 0; y0 < c.ny; y0 += H)
    for (size_t s = 0; s + 1 < x.size(); ++s)
      out.push_back(Strip{ci, x[s], y0, std::min(y0 + H, c.ny), 0, x[s + 1]});
}

// The tiled step: the fused stress-force kernel for every channel of a
// stress-force handle; the FP64 tile sweep for FP64 channels of the strip
// classes whose slots fit 32-bit offsets (the others keep the strip sweeps).
#ifndef LB_TILE_SWEEP
#define LB_TILE_SWEEP 1
#endif
struct TileShape {
  int tx, ty;
};
TileShape tile_shape(const lb_options *o) {
  return o->stress_force ? TileShape{kSafTileX, kSafTileY} : TileShape{kMainTileX, kMainTileY};
}
bool tiled(const lb_options *o, const lb_channel &c) {
  if (o->stress_force) return true;
  return LB_TILE_SWEEP && o->precision == LB_FP64 && is_strip_class(width_class(c.nx, 8)) &&
         align_up((size_t)c.nx * c.ny, kTile) * kPlanes <= 0xffffffffull;
}
// Tiles of channel i. The kernels hand each of the 8 XCDs a contiguous run
// of the list: the tile columns of a channel are split into 8 groups, each
// group listed band by band, so that an XCD's tiles have their horizontal
// and vertical neighbours (which share halo populations) on the same L2.
void add_tiles(int i, const lb_channel &c, TileShape ts, std::vector<Strip> &out) {
  const int cols = (c.nx + ts.tx - 1) / ts.tx;
  for (int g = 0; g < 8; ++g)
    for (int y0 = 0; y0 < c.ny; y0 += ts.ty)
      for (int cx = g * cols / 8; cx < (g + 1) * cols / 8; ++cx)
        out.push_back(Strip{i, cx * ts.tx, y0, std::min(y0 + ts.ty, c.ny), 0});
}

// A state buffer larger than the last-level cache: the sweeps stream it
// (nontemporal stores)
bool streamed(const Layout &L) { return (long long)kPlanes * L.plane * L.esize > kNontemporalBytes; }

Layout make_layout(const lb_channel *c, int n, const lb_options *o) {
  Layout L;
  L.esize = (o->precision == LB_FP32_SHIFTED) ? 4 : 8;
  L.ch.resize(n);
  long long node = 0;
  int rows = 0, part = 0, strips = 0;
  for (int i = 0; i < n; ++i) {
    ChanDev &d = L.ch[i];
    resolve(c[i], d);
    d.off = node;
    node += (long long)align_up((size_t)c[i].nx * c[i].ny, 64);
    d.row_off = rows;
    rows += c[i].ny;
    const int cls = width_class(c[i].nx, L.esize);
    const int w = strip_cols(cls, L.esize);
    d.nxs = is_strip_class(cls) ? (c[i].nx + w - 1) / w : 1;
    d.poff = part;
    part += d.nxs * c[i].ny;
    const int srows = strip_rows_for(cls, c[i].nx, c[i].ny, o->strip_rows);
    strips += d.nxs * ((c[i].ny + srows - 1) / srows);
  }
  // room for the active set's smaller strips when few channels are left
  // (fewer than twice the SIMDs of any GPU this runs on, see upload_strips)
  strips = std::max(strips, 4096 + 2 * n);
  L.strip_cap = strips;
  L.plane = (long long)align_up((size_t)std::max<long long>(node, kTile), kTile);
  L.total_rows = rows;
  L.total_part = part;
  L.max_strips = strips;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t p = at;
    at = align_up(at + bytes, kAlign);
    return p;
  };
  const size_t state = (size_t)kPlanes * L.plane * L.esize;
  L.off_state[0] = take(state);
  L.off_state[1] = take(state);
  L.off_ch = take(sizeof(ChanDev) * n);
  L.off_strips = take(sizeof(Strip) * strips);
  L.off_astrips = take(sizeof(Strip) * strips);
  L.off_rstrips = take(sizeof(Strip) * strips);
  L.off_part = take(sizeof(double) * OF_COUNT * part);
  L.off_prof = take(sizeof(double) * OF_COUNT * rows);
  L.off_prev = take(sizeof(double) * rows);
  L.off_scal = take(sizeof(double) * CS_COUNT * n);
  L.off_uref = take(sizeof(float) * rows);
  if (o->viscoelastic) {
    const size_t stress = (size_t)kStressPlanes * L.plane * L.esize;
    L.off_stress[0] = take(stress);
    L.off_stress[1] = take(stress);
  }
  if (o->stress_force) {
    L.off_saf_u = take(sizeof(double) * 2 * L.plane);
    L.off_saf_t = take(sizeof(double) * 3 * L.plane);
  }
  const TileShape ts = tile_shape(o);
  for (int i = 0; i < n; ++i)
    if (tiled(o, c[i])) L.n_tiles += ((c[i].nx + ts.tx - 1) / ts.tx) * ((c[i].ny + ts.ty - 1) / ts.ty);
  L.off_tiles = take(sizeof(Strip) * L.n_tiles);
  L.off_bstrips = take(sizeof(Strip) * strips);
  L.off_brstrips = take(sizeof(Strip) * strips);
  const int min_rows = o->strip_rows > 0 ? std::min(o->strip_rows, 16) : 16;
  const int npl = two_step_npl(L.esize == 4, streamed(L), o->viscoelastic);
  for (int i = 0; i < n && two_step_handle(o, o->obs_every > 0 ? o->obs_every : kDefaultK); ++i)
    if (two_step_channel(c[i], L.esize))
      L.max_two += (int)(two_step_cuts(c[i].nx, npl).size() - 1) * ((c[i].ny + min_rows - 1) / min_rows);
  L.off_btiles = take(sizeof(Strip) * std::max(L.n_tiles, 1));
  L.off_tstrips = take(sizeof(Strip) * std::max(L.max_two, 1));
  L.bytes = at;
  return L;
}

}  // namespace

struct lb_handle {
  Layout L;
  lb_options opt{};
  int n_ch = 0;
  int K = kDefaultK;
  std::vector<lb_channel> in;
  char *ws = nullptr;
  void *buf[2] = {nullptr, nullptr};
  ChanDev *dch = nullptr;
  Strip *dall = nullptr;     // every channel, for observation
  Strip *dact = nullptr;     // active channels, for stepping
  Strip *dact_rev = nullptr; // the same, each class group in reverse order
  double *dpart = nullptr, *dprof = nullptr, *dprev = nullptr, *dscal = nullptr;
  float *duref = nullptr;    // FP32: reference velocity of every row
  void *sbuf[2] = {nullptr, nullptr};  // viscoelastic model: stress buffers (same parity as buf)
  double *saf_u = nullptr, *saf_t = nullptr;  // stress-as-force scratch
  Strip *tiles = nullptr;                     // tiles of the tiled step (every tiled channel)
  // strips grouped by width class: [begin, begin + count) in the arrays
  int all_begin[kClasses] = {0}, all_count[kClasses] = {0};
  int act_begin[kClasses] = {0}, act_count[kClasses] = {0};
  Strip *dbact = nullptr, *dbact_rev = nullptr;  // captured blocks: active channels without two-step strips
  Strip *dtwo = nullptr;                        // two-step strips of the active channels
  int bact_begin[kClasses] = {0}, bact_count[kClasses] = {0};
  // captured blocks: the narrow two-step strips of each width, after the
  // others in dbact
  int n2_begin[kClasses] = {0}, n2_count[kClasses] = {0};
  int two_count = 0;
  bool two_wall = false;  // some two-step strip's channel has a moving or Zou-He top wall
  Strip *btiles = nullptr;  // captured blocks: tiles of the tiled channels without two-step strips
  int n_btiles = 0;
  bool two_step = false;     // captured blocks pair their steps where eligible
  int slots = 1024;          // two-step strips resident at once on the GPU
  int simds = 1024;          // SIMDs of the GPU (four per CU)
  long long n2slots = 1536;  // narrow two-step strips resident at once
  int cur = 0;               // buffer holding the current state
  hipStream_t stream = nullptr, cap = nullptr;
  bool own_stream = false;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  bool obs_valid = false;
  std::vector<double> hprof, hscal;
  std::vector<long long> t;  // host mirror of every channel's step
  std::vector<int> active;
  int n_checks = 0;
  int since_block = 0;       // steps since the last block boundary (handle clock)
  bool any_gpbc = false;     // some channel has the pressure drive
  bool any_zh = false;       // some channel has a Zou-He top wall
  int device = -1;           // the GPU current at lb_create
  double *noalloc = nullptr; // that GPU's copy of `scratch` (device address)
  hipError_t noalloc_err = hipSuccess;
  std::string err;
};

namespace {

lb_status fail(lb_handle *h, lb_status s, const std::string &msg) {
  if (h) h->err = msg;
  return s;
}

lb_status hipfail(lb_handle *h, hipError_t e, const char *where) {
  return fail(h, LB_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHECK(h, call)                                  \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hipfail((h), e_, #call);  \
  } while (0)

void group_strips(const std::vector<Strip> &s, const std::vector<ChanDev> &ch, int esize,
                  std::vector<Strip> &out, int begin[kClasses], int count[kClasses]) {
  out.clear();
  for (int c = 0; c < kClasses; ++c) {
    begin[c] = (int)out.size();
    for (const Strip &x : s)
      if (width_class(ch[x.ch].nx, esize) == c) out.push_back(x);
    count[c] = (int)out.size() - begin[c];
  }
}

lb_status upload_strips(lb_handle *h, bool all) {
  std::vector<Strip> raw, grouped;
  // stacks while a state buffer fits the last-level cache (the stores are
  // then cached, see sweep_args)
  const bool stack = !streamed(h->L);
  // Strip heights of the active set: the requested (or default) ones, all
  // divided alike while the active channels make fewer strips than the GPU
  // has SIMDs (down to a kernel's row group for the narrow widths, 4 rows
  // otherwise), so that a few small channels left still spread over the
  // GPU. A node's arithmetic does not depend on the strip it falls in.
  int div = 1;
  auto rows_of = [&](int i) {
    const ChanDev &d = h->L.ch[i];
    const int cls = width_class(d.nx, h->L.esize);
    const int base = strip_rows_for(cls, d.nx, d.ny, h->opt.strip_rows);
    if (is_strip_class(cls)) return std::max(std::min(base, 4), base / div);
    const int tyw = 64 / d.nx;
    const int r = std::max(tyw, base / div);
    return (r + tyw - 1) / tyw * tyw;
  };
  if (!all) {
    auto count = [&]() {
      long long S = 0;
      for (int i = 0; i < h->n_ch; ++i) {
        if (!h->active[i] || tiled(&h->opt, h->in[i])) continue;
        const ChanDev &d = h->L.ch[i];
        const int cls = width_class(d.nx, h->L.esize);
        const int w = strip_cols(cls, h->L.esize);
        S += (long long)(is_strip_class(cls) ? (d.nx + w - 1) / w : 1) * ((d.ny + rows_of(i) - 1) / rows_of(i));
      }
      return S;
    };
    for (long long S = count(); S > 0 && S < h->simds && div < 64;) {
      div *= 2;
      const long long S2 = count();
      if (S2 == S || S2 > h->L.strip_cap) {  // every channel at its smallest height, or no room
        div /= 2;
        break;
      }
      S = S2;
    }
  }
  for (int i = 0; i < h->n_ch; ++i) {
    if (!all && (!h->active[i] || tiled(&h->opt, h->in[i]))) continue;
    const ChanDev &d = h->L.ch[i];
    add_strips(i, d, h->L.esize,
               all ? strip_rows_for(width_class(d.nx, h->L.esize), d.nx, d.ny, h->opt.strip_rows) : rows_of(i),
               stack, raw);
  }
  if (all) {
    group_strips(raw, h->L.ch, h->L.esize, grouped, h->all_begin, h->all_count);
    if (!grouped.empty())
      HIPCHECK(h, hipMemcpyAsync(h->dall, grouped.data(), grouped.size() * sizeof(Strip),
                                 hipMemcpyHostToDevice, h->stream));
  } else {
    group_strips(raw, h->L.ch, h->L.esize, grouped, h->act_begin, h->act_count);
    std::vector<Strip> rev(grouped);
    for (int c = 0; c < kClasses; ++c)
      std::reverse(rev.begin() + h->act_begin[c], rev.begin() + h->act_begin[c] + h->act_count[c]);
    if (!grouped.empty()) {
      HIPCHECK(h, hipMemcpyAsync(h->dact, grouped.data(), grouped.size() * sizeof(Strip),
                                 hipMemcpyHostToDevice, h->stream));
      HIPCHECK(h, hipMemcpyAsync(h->dact_rev, rev.data(), rev.size() * sizeof(Strip), hipMemcpyHostToDevice,
                                 h->stream));
    }
    // captured blocks: two-step strips for the eligible active channels, the
    // one-step strips of the others
    std::vector<Strip> braw, bgrouped, two, n2raw, n2grouped;
    bool wall = false;
    if (h->two_step) {
      const int es = h->L.esize;
      std::vector<lb_channel> elig, nelig;
      for (int i = 0; i < h->n_ch; ++i) {
        if (!h->active[i]) continue;
        if (two_step_channel(h->in[i], es)) elig.push_back(h->in[i]);
        else if (narrow_two_step_channel(&h->opt, h->in[i], es)) nelig.push_back(h->in[i]);
      }
      const int npl = two_step_npl(es == 4, streamed(h->L), h->opt.viscoelastic);
      const int H = h->opt.strip_rows > 0 ? std::min(h->opt.strip_rows, kTwoStepMaxRows)
                                          : two_step_rows(elig, npl, h->slots);
      for (int i = 0; i < h->n_ch; ++i) {
        if (!h->active[i]) continue;
        if (two_step_channel(h->in[i], es)) {
          add_two_step_strips(i, h->in[i], npl, H, two);
          wall = wall || two_step_wall(h->in[i]);
        } else if (!narrow_two_step_channel(&h->opt, h->in[i], es) && !tiled(&h->opt, h->in[i])) {
          add_strips(i, h->L.ch[i], es, rows_of(i), stack, braw);
        }
      }
      // the narrow ones, in what room the list has left
      if (!nelig.empty()) {
        const int R2 = narrow_two_step_rows(nelig, h->n2slots, h->opt.strip_rows,
                                            h->L.strip_cap - (long long)braw.size());
        for (int i = 0; i < h->n_ch; ++i)
          if (h->active[i] && narrow_two_step_channel(&h->opt, h->in[i], es))
            add_strips(i, h->L.ch[i], es, narrow_rows(R2, h->in[i].nx), stack, n2raw);
      }
    }
    group_strips(braw, h->L.ch, h->L.esize, bgrouped, h->bact_begin, h->bact_count);
    std::vector<Strip> brev(bgrouped);
    for (int c = 0; c < kClasses; ++c)
      std::reverse(brev.begin() + h->bact_begin[c], brev.begin() + h->bact_begin[c] + h->bact_count[c]);
    // the narrow two-step strips follow in dbact
    group_strips(n2raw, h->L.ch, h->L.esize, n2grouped, h->n2_begin, h->n2_count);
    for (int c = 0; c < kClasses; ++c) h->n2_begin[c] += (int)bgrouped.size();
    bgrouped.insert(bgrouped.end(), n2grouped.begin(), n2grouped.end());
    if ((long long)bgrouped.size() > h->L.strip_cap) return fail(h, LB_ENOMEM, "block strip list exceeds its workspace");
    if (!bgrouped.empty()) {
      HIPCHECK(h, hipMemcpyAsync(h->dbact, bgrouped.data(), bgrouped.size() * sizeof(Strip), hipMemcpyHostToDevice,
                                 h->stream));
      HIPCHECK(h, hipMemcpyAsync(h->dbact_rev, brev.data(), brev.size() * sizeof(Strip), hipMemcpyHostToDevice,
                                 h->stream));
    }
    if ((int)two.size() > h->L.max_two) return fail(h, LB_ENOMEM, "two-step strip list exceeds its workspace");
    h->two_count = (int)two.size();
    h->two_wall = wall;
    if (!two.empty())
      HIPCHECK(h, hipMemcpyAsync(h->dtwo, two.data(), two.size() * sizeof(Strip), hipMemcpyHostToDevice, h->stream));
    // the host vectors die here: make the copies complete first
    HIPCHECK(h, hipStreamSynchronize(h->stream));
  }
  // the host vector dies here: make the copy complete first
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

SweepArgs sweep_args(lb_handle *h, const Strip *strips, int begin, int count, int src, int k) {
  SweepArgs a{};
  a.A = h->buf[src];
  a.B = h->buf[src ^ 1];
  a.plane = h->L.plane;
  a.strips = strips + begin;
  a.ch = h->dch;
  a.part = h->dpart;
  a.n_strips = count;
  a.n_wg = (count + kWaves - 1) / kWaves;
  a.k = k;
  a.nt = streamed(h->L);
  a.uref = h->duref;
  a.ve = h->opt.viscoelastic;
  a.zh = h->any_zh;
  a.SA = h->sbuf[src];
  a.SB = h->sbuf[src ^ 1];
  return a;
}

// Enqueues the sweeps of one step (source buffer src, step offset k), over
// every active channel or (block) over those without two-step strips.
lb_status enqueue_step(lb_handle *h, int src, int k, hipStream_t s, bool block = false) {
  if (h->opt.stress_force) {
    HIPCHECK(h, launch_saf_fused(static_cast<const double *>(h->buf[src]), static_cast<double *>(h->buf[src ^ 1]),
                                 h->dch, h->tiles, h->L.n_tiles, k,
                                 streamed(h->L), s));
    return LB_OK;
  }
  Strip *tl = block ? h->btiles : h->tiles;
  const int ntl = block ? h->n_btiles : h->L.n_tiles;
  if (ntl) HIPCHECK(h, launch_tiles(sweep_args(h, tl, 0, ntl, src, k), s));
  const int *begin = block ? h->bact_begin : h->act_begin, *count = block ? h->bact_count : h->act_count;
  Strip *fwd = block ? h->dbact : h->dact, *rev = block ? h->dbact_rev : h->dact_rev;
  for (int c = 0; c < kClasses; ++c) {
    if (!count[c]) continue;
    // Serpentine order: steps reading buffer 0 take the strips in order and
    // march them upwards, steps reading buffer 1 take them in reverse and
    // march downwards (flipped strips of a stack the other way in both), so
    // that every step starts on what the previous step wrote last, the
    // likeliest to still sit in the last-level cache (MALL).
    SweepArgs a = sweep_args(h, src == 0 ? fwd : rev, begin[c], count[c], src, k);
    a.down = (src == 1);
    HIPCHECK(h, launch_sweep(h->opt.precision == LB_FP32_SHIFTED, c, false, a, s));
  }
  // generalised periodic boundaries: the inlet/outlet column pass on the
  // state just written
  if (h->any_gpbc)
    HIPCHECK(h, launch_gpbc(h->opt.precision == LB_FP32_SHIFTED, h->buf[src ^ 1], h->dch, h->n_ch, k, h->duref,
                            s));
  return LB_OK;
}

// The observation of the current state: per-row, per-strip partials into
// part, then the per-channel reduction into prof and scal (and, with
// update_residual, the residual history in the workspace).
lb_status enqueue_observe_into(lb_handle *h, double *part, double *prof, double *scal, int update_residual,
                               int steps_since) {
  if (h->opt.stress_force) {
    HIPCHECK(h, launch_saf_observe(static_cast<const double *>(h->buf[h->cur]), h->dch, h->n_ch, h->L.plane,
                                   h->L.total_rows, h->saf_u, h->saf_t, part, h->stream));
  }
  for (int c = 0; c < kClasses && !h->opt.stress_force; ++c) {
    if (!h->all_count[c]) continue;
    SweepArgs a = sweep_args(h, h->dall, h->all_begin[c], h->all_count[c], h->cur, 0);
    a.part = part;
    HIPCHECK(h, launch_sweep(h->opt.precision == LB_FP32_SHIFTED, c, true, a, h->stream));
  }
  HIPCHECK(h, launch_reduce(h->dch, h->n_ch, part, prof, h->dprev, scal, h->duref, update_residual, steps_since,
                            h->stream));
  return LB_OK;
}

lb_status enqueue_observe(lb_handle *h, int update_residual, int steps_since) {
  return enqueue_observe_into(h, h->dpart, h->dprof, h->dscal, update_residual, steps_since);
}

void drop_graphs(lb_handle *h) {
  for (int p = 0; p < 2; ++p)
    if (h->graph[p]) {
      (void)hipGraphExecDestroy(h->graph[p]);
      h->graph[p] = nullptr;
    }
}

// Captures K steps starting from buffer src, followed by the step-counter
// advance, as one graph (K is even, so the state returns to buffer src).
lb_status capture(lb_handle *h, int src) {
  hipGraph_t g = nullptr;
  HIPCHECK(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed));
  lb_status st = LB_OK;
  if (h->two_step) {
    // pairs of steps: one two-step launch for the eligible channels (its
    // j-th launch reads buffer src ^ (j & 1) and writes the other one), and
    // the one-step launches of the others
    for (int k = 0; k < h->K && st == LB_OK; k += 2) {
      if (h->two_count) {
        SweepArgs a = sweep_args(h, h->dtwo, 0, h->two_count, src ^ ((k / 2) & 1), k);
        a.wall = h->two_wall;
        a.n_wg = h->two_count;  // one strip per workgroup (a wavefront per stage)
        hipError_t e = launch_two_step(h->opt.precision == LB_FP32_SHIFTED, a, h->cap);
        if (e != hipSuccess) st = hipfail(h, e, "launch_two_step");
      }
      for (int c = 0; c < kClasses && st == LB_OK; ++c) {
        if (!h->n2_count[c]) continue;
        SweepArgs a = sweep_args(h, h->dbact, h->n2_begin[c], h->n2_count[c], src ^ ((k / 2) & 1), k);
        a.n_wg = h->n2_count[c];  // one strip per workgroup (a wavefront per stage)
        hipError_t e = launch_narrow_two_step(h->opt.precision == LB_FP32_SHIFTED, 1 << c, a, h->cap);
        if (e != hipSuccess) st = hipfail(h, e, "launch_narrow_two_step");
      }
      if (st == LB_OK) st = enqueue_step(h, src, k, h->cap, true);
      if (st == LB_OK) st = enqueue_step(h, src ^ 1, k + 1, h->cap, true);
    }
  } else {
    for (int k = 0; k < h->K && st == LB_OK; ++k) st = enqueue_step(h, src ^ (k & 1), k, h->cap);
  }
  if (st == LB_OK) {
    hipError_t e = launch_advance(h->dch, h->n_ch, h->K, h->cap);
    if (e != hipSuccess) st = hipfail(h, e, "launch_advance");
  }
  hipError_t e = hipStreamEndCapture(h->cap, &g);
  if (st != LB_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hipfail(h, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&h->graph[src], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hipfail(h, e, "hipGraphInstantiate");
  return LB_OK;
}

lb_status read_observation(lb_handle *h) {
  if (h->obs_valid) return LB_OK;
  lb_status st = enqueue_observe(h, 0, 0);
  if (st != LB_OK) return st;
  h->hprof.resize((size_t)h->L.total_rows * OF_COUNT);
  h->hscal.resize((size_t)h->n_ch * CS_COUNT);
  HIPCHECK(h, hipMemcpyAsync(h->hprof.data(), h->dprof, h->hprof.size() * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipMemcpyAsync(h->hscal.data(), h->dscal, h->hscal.size() * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->obs_valid = true;
  return LB_OK;
}

// Copies channel ch's tiles (and stress tiles) from the current buffer to
// the other one. A frozen channel is no longer swept, so both buffers must
// hold its state: later steps of odd length change which buffer is current.
lb_status mirror_channel(lb_handle *h, int ch) {
  const ChanDev &d = h->L.ch[ch];
  const size_t Npad = align_up((size_t)d.nx * d.ny, kTile);
  const int es = h->L.esize;
  const size_t off = (size_t)slot(0, d.off) * es, bytes = (size_t)kPlanes * Npad * es;
  HIPCHECK(h, hipMemcpyAsync(static_cast<char *>(h->buf[h->cur ^ 1]) + off,
                             static_cast<const char *>(h->buf[h->cur]) + off, bytes, hipMemcpyDeviceToDevice,
                             h->stream));
  if (h->sbuf[0]) {
    const size_t soff = (size_t)sslot(0, d.off) * es, sbytes = (size_t)kStressPlanes * Npad * es;
    HIPCHECK(h, hipMemcpyAsync(static_cast<char *>(h->sbuf[h->cur ^ 1]) + soff,
                               static_cast<const char *>(h->sbuf[h->cur]) + soff, sbytes, hipMemcpyDeviceToDevice,
                               h->stream));
  }
  return LB_OK;
}

// Convergence check after a graph: residuals of all channels, freeze the
// converged ones and rebuild the active work list.
lb_status check_steady(lb_handle *h) {
  const int first = (h->n_checks == 0);
  lb_status st = enqueue_observe(h, 1, h->K);
  if (st != LB_OK) return st;
  h->n_checks++;
  h->hscal.resize((size_t)h->n_ch * CS_COUNT);
  h->hprof.resize((size_t)h->L.total_rows * OF_COUNT);
  HIPCHECK(h, hipMemcpyAsync(h->hscal.data(), h->dscal, h->hscal.size() * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipMemcpyAsync(h->hprof.data(), h->dprof, h->hprof.size() * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->obs_valid = true;
  // NaN/Inf first: report it before anything is frozen, so that host and
  // device keep the same active channels and step counters
  for (int i = 0; i < h->n_ch; ++i)
    if (h->active[i] && h->hscal[(size_t)i * CS_COUNT + CS_NAN] != 0.0) {
      char buf[96];
      snprintf(buf, sizeof buf, "NaN/Inf seen in channel %d during a convergence check", i);
      return fail(h, LB_EUNSTABLE, buf);
    }
  bool changed = false;
  for (int i = 0; i < h->n_ch; ++i) {
    if (!h->active[i]) continue;
    const double *s = &h->hscal[(size_t)i * CS_COUNT];
    if (!first && s[CS_RESIDUAL] < h->opt.steady_tol) {
      h->active[i] = 0;
      h->L.ch[i].active = 0;
      changed = true;
      lb_status m = mirror_channel(h, i);
      if (m != LB_OK) return m;
    }
  }
  if (changed) {
    // publish the active flags and the new work list, then recapture
    std::vector<ChanDev> cur(h->n_ch);
    HIPCHECK(h, hipMemcpyAsync(cur.data(), h->dch, sizeof(ChanDev) * h->n_ch, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->n_ch; ++i) cur[i].active = h->active[i];
    HIPCHECK(h, hipMemcpyAsync(h->dch, cur.data(), sizeof(ChanDev) * h->n_ch, hipMemcpyHostToDevice, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    lb_status u = upload_strips(h, false);
    if (u != LB_OK) return u;
    drop_graphs(h);
  }
  return LB_OK;
}

// FP32 storage: moves every active row's reference velocity to its current
// mean u_x. Needs the observation of the current state in dprof (taken here
// unless the convergence check just took it).
lb_status rereference(lb_handle *h, bool observed) {
  if (h->opt.precision != LB_FP32_SHIFTED) return LB_OK;
  if (!observed) {
    lb_status st = enqueue_observe(h, 0, 0);
    if (st != LB_OK) return st;
  }
  HIPCHECK(h, launch_rereference(static_cast<float *>(h->buf[h->cur]), h->dch, h->n_ch, h->L.total_rows, h->dprof,
                                 h->duref, h->stream));
  return LB_OK;
}

// E_i(u) of the FP32 storage: the velocity part of the equilibrium at
// density 1, a_i (3 c_ix u + (9/2 c_ix^2 - 3/2) u^2).
double href_eq(int i, double u) {
  const double cx = HCX[i];
  return hweight(i) * (3.0 * cx * u + (4.5 * cx * cx - 1.5) * u * u);
}

lb_status fill_rest(lb_handle *h, int which);

// Device address of `scratch` on GPU dev, looked up once per device (with
// that device current, as the caller of lb_create leaves it) and kept for
// the life of the process. In host code the array's name is only a stand-in
// for the symbol: kernels and copies take this address.
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc[kMaxDevices] = {};

hipError_t noalloc_scratch(int dev, double **out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_noalloc[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_noalloc[dev] = static_cast<double *>(p);
  }
  *out = g_noalloc[dev];
  return hipSuccess;
}

// Observable `what` of channel c as lb_observe reports it, from the reduced
// profiles (prof, [row][OF_COUNT]) or scalars (scal, [channel][CS_COUNT]),
// into out (ny doubles, or one). One thread per row.
__global__ void gather_observable_kernel(const ChanDev *ch, int c, int what, const double *prof,
                                         const double *scal, double *out) {
  const ChanDev d = ch[c];
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (what >= 32) {
    if (y != 0) return;
    const double *s = scal + (long long)c * CS_COUNT;
    double v = 0.0;
    switch (what) {
      case LB_OBS_MASS: v = (double)((long long)d.nx * d.ny) + s[CS_MASS_DEV]; break;
      case LB_OBS_MOMX: v = s[CS_MOMX]; break;
      case LB_OBS_FLUX: v = s[CS_FLUX]; break;
      case LB_OBS_WALL_DRAG: v = s[CS_DRAG]; break;
      case LB_OBS_UMID: v = s[CS_UMID]; break;
      case LB_OBS_NAN: v = s[CS_NAN]; break;
      default: break;
    }
    out[0] = v;
    return;
  }
  if (y >= d.ny) return;
  const double *r = prof + ((long long)d.row_off + y) * OF_COUNT;
  double v = 0.0;
  switch (what) {
    case LB_OBS_UX: v = r[OF_UX]; break;
    case LB_OBS_UY: v = r[OF_UY]; break;
    case LB_OBS_SXX: v = r[OF_SXX]; break;
    case LB_OBS_SXY: v = r[OF_SXY]; break;
    case LB_OBS_SYY: v = r[OF_SYY]; break;
    case LB_OBS_N1: v = r[OF_SXX] - r[OF_SYY]; break;
    case LB_OBS_PRESSURE: v = (1.0 + r[OF_RHOE_DEV]) / 3.0; break;
    case LB_OBS_KXY: v = r[OF_KXY]; break;
    case LB_OBS_TRT: v = r[OF_TRT]; break;
    case LB_OBS_KXX: v = r[OF_KXX]; break;
    default: break;
  }
  out[y] = v;
}

}  // namespace

extern "C" {

const char *lb_status_string(int32_t s) {
  switch (s) {
    case LB_OK: return "LB_OK";
    case LB_EINVAL: return "LB_EINVAL";
    case LB_ENOMEM: return "LB_ENOMEM";
    case LB_EHIP: return "LB_EHIP";
    case LB_EUNSTABLE: return "LB_EUNSTABLE";
    case LB_ESTATE: return "LB_ESTATE";
    default: return "unknown status";
  }
}

const char *lb_last_error(const lb_handle *h) { return h ? h->err.c_str() : "NULL handle"; }

lb_status lb_workspace_bytes(const lb_channel *c, int32_t n, const lb_options *o, size_t *bytes) {
  if (!bytes) return LB_EINVAL;
  if (!validate(c, n, o).empty()) return LB_EINVAL;
  *bytes = make_layout(c, n, o).bytes;
  return LB_OK;
}

lb_status lb_create(const lb_channel *c, int32_t n, const lb_options *o, void *ws, size_t ws_bytes,
                    void *stream, lb_handle **out) {
  if (!out) return LB_EINVAL;
  *out = nullptr;
  if (!validate(c, n, o).empty()) return LB_EINVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign)) return LB_EINVAL;
  lb_handle *h = new (std::nothrow) lb_handle();
  if (!h) return LB_ENOMEM;
  h->L = make_layout(c, n, o);
  if (ws_bytes < h->L.bytes) {
    delete h;
    return LB_ENOMEM;
  }
  h->opt = *o;
  h->n_ch = n;
  for (int i = 0; i < n; ++i) {
    h->any_gpbc = h->any_gpbc || h->L.ch[i].gpbc;
    h->any_zh = h->any_zh || h->L.ch[i].zh;
  }
  h->K = o->obs_every > 0 ? o->obs_every : kDefaultK;
  h->in.assign(c, c + n);
  h->ws = static_cast<char *>(ws);
  h->buf[0] = h->ws + h->L.off_state[0];
  h->buf[1] = h->ws + h->L.off_state[1];
  h->dch = reinterpret_cast<ChanDev *>(h->ws + h->L.off_ch);
  h->tiles = reinterpret_cast<Strip *>(h->ws + h->L.off_tiles);
  h->dall = reinterpret_cast<Strip *>(h->ws + h->L.off_strips);
  h->dact = reinterpret_cast<Strip *>(h->ws + h->L.off_astrips);
  h->dact_rev = reinterpret_cast<Strip *>(h->ws + h->L.off_rstrips);
  h->dbact = reinterpret_cast<Strip *>(h->ws + h->L.off_bstrips);
  h->dbact_rev = reinterpret_cast<Strip *>(h->ws + h->L.off_brstrips);
  h->dtwo = reinterpret_cast<Strip *>(h->ws + h->L.off_tstrips);
  h->btiles = reinterpret_cast<Strip *>(h->ws + h->L.off_btiles);
  h->two_step = false;
  for (int i = 0; i < n && two_step_handle(o, h->K); ++i)
    h->two_step = h->two_step || two_step_channel(c[i], h->L.esize) || narrow_two_step_channel(o, c[i], h->L.esize);
  h->dpart = reinterpret_cast<double *>(h->ws + h->L.off_part);
  h->dprof = reinterpret_cast<double *>(h->ws + h->L.off_prof);
  h->dprev = reinterpret_cast<double *>(h->ws + h->L.off_prev);
  h->dscal = reinterpret_cast<double *>(h->ws + h->L.off_scal);
  h->duref = reinterpret_cast<float *>(h->ws + h->L.off_uref);
  if (o->viscoelastic) {
    h->sbuf[0] = h->ws + h->L.off_stress[0];
    h->sbuf[1] = h->ws + h->L.off_stress[1];
  }
  if (o->stress_force) {
    h->saf_u = reinterpret_cast<double *>(h->ws + h->L.off_saf_u);
    h->saf_t = reinterpret_cast<double *>(h->ws + h->L.off_saf_t);
  }
  h->t.assign(n, 0);
  h->active.assign(n, 1);
  auto bail = [&](lb_status s) {
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return s;
  };
  if (stream) {
    h->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return bail(LB_EHIP);
    h->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) return bail(LB_EHIP);
  if (hipMemcpyAsync(h->dch, h->L.ch.data(), sizeof(ChanDev) * n, hipMemcpyHostToDevice, h->stream) !=
      hipSuccess)
    return bail(LB_EHIP);
  std::vector<double> nanrows(std::max(1, h->L.total_rows), std::numeric_limits<double>::quiet_NaN());
  if (hipMemcpyAsync(h->dprev, nanrows.data(), sizeof(double) * h->L.total_rows, hipMemcpyHostToDevice,
                     h->stream) != hipSuccess)
    return bail(LB_EHIP);
  std::vector<float> zrows(std::max(1, h->L.total_rows), 0.0f);
  if (hipMemcpyAsync(h->duref, zrows.data(), sizeof(float) * h->L.total_rows, hipMemcpyHostToDevice, h->stream) !=
      hipSuccess)
    return bail(LB_EHIP);
  {
    // strips of the two-step sweep resident at once
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return bail(LB_EHIP);
    h->slots = two_step_blocks_per_cu(o->precision == LB_FP32_SHIFTED, streamed(h->L), o->viscoelastic) *
               std::max(cus, 1);
    h->simds = 4 * std::max(cus, 1);
    h->n2slots = (long long)narrow_two_step_blocks_per_cu(o->precision == LB_FP32_SHIFTED) * std::max(cus, 1);
  }
  if (upload_strips(h, true) != LB_OK || upload_strips(h, false) != LB_OK) return bail(LB_EHIP);
  std::vector<Strip> tiles, btiles;  // kept until the synchronisation below
  for (int i = 0; i < n; ++i)
    if (tiled(o, c[i])) {
      add_tiles(i, c[i], tile_shape(o), tiles);
      if (!h->two_step || !two_step_channel(c[i], h->L.esize)) add_tiles(i, c[i], tile_shape(o), btiles);
    }
  if (!tiles.empty() && hipMemcpyAsync(h->tiles, tiles.data(), sizeof(Strip) * tiles.size(),
                                       hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return bail(LB_EHIP);
  h->n_btiles = (int)btiles.size();
  if (!btiles.empty() && hipMemcpyAsync(h->btiles, btiles.data(), sizeof(Strip) * btiles.size(),
                                        hipMemcpyHostToDevice, h->stream) != hipSuccess)
    return bail(LB_EHIP);
  if (fill_rest(h, 0) != LB_OK || fill_rest(h, 1) != LB_OK) return bail(LB_EHIP);
  // zero stress at rest (outside any graph)
  for (int b = 0; b < 2; ++b)
    if (h->sbuf[b] &&
        hipMemsetAsync(h->sbuf[b], 0, (size_t)kStressPlanes * h->L.plane * h->L.esize, h->stream) != hipSuccess)
      return bail(LB_EHIP);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(LB_EHIP);
  // the allocation-free observation's scratch on this GPU (a failure here
  // is reported by lb_observe_noalloc, not by lb_create)
  h->noalloc_err = hipGetDevice(&h->device);
  if (h->noalloc_err == hipSuccess) h->noalloc_err = noalloc_scratch(h->device, &h->noalloc);
  *out = h;
  return LB_OK;
}

lb_status lb_destroy(lb_handle *h) {
  if (!h) return LB_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  drop_graphs(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return LB_OK;
}

lb_status lb_step(lb_handle *h, int64_t n) {
  if (!h) return LB_EINVAL;
  if (n < 0) return fail(h, LB_EINVAL, "negative step count");
  h->obs_valid = false;
  int64_t left = n;
  // Every K steps of the handle's clock end a block: the convergence check
  // (if enabled) and, for FP32 storage, the move of the row reference
  // velocities. Whole blocks run as one graph; steps that start or end off
  // a block boundary are enqueued one by one. The boundaries do not depend
  // on how the steps are split over calls, so neither does the result.
  while (left > 0) {
    bool any = false;
    for (int a : h->active) any |= (a != 0);
    if (!any) break;
    int m;
    if (h->since_block == 0 && left >= h->K) {
      if (!h->graph[h->cur]) {
        lb_status st = capture(h, h->cur);
        if (st != LB_OK) return st;
      }
      HIPCHECK(h, hipGraphLaunch(h->graph[h->cur], h->stream));
      m = h->K;
    } else {
      m = (int)std::min<int64_t>(left, h->K - h->since_block);
      for (int k = 0; k < m; ++k) {
        lb_status st = enqueue_step(h, h->cur ^ (k & 1), k, h->stream);
        if (st != LB_OK) return st;
      }
      HIPCHECK(h, launch_advance(h->dch, h->n_ch, m, h->stream));
      h->cur ^= (m & 1);
    }
    for (int i = 0; i < h->n_ch; ++i)
      if (h->active[i]) h->t[i] += m;
    left -= m;
    h->since_block += m;
    h->obs_valid = false;
    if (h->since_block == h->K) {
      h->since_block = 0;
      bool observed = false;
      if (h->opt.steady_tol > 0) {
        lb_status st = check_steady(h);
        if (st != LB_OK) return st;
        observed = true;
      }
      lb_status st = rereference(h, observed);
      if (st != LB_OK) return st;
      h->obs_valid = false;
    }
  }
  h->obs_valid = false;
  return LB_OK;
}

lb_status lb_observe(lb_handle *h, int32_t ch, int32_t what, double *out, size_t n) {
  if (!h) return LB_EINVAL;
  if (ch < 0 || ch >= h->n_ch || !out) return fail(h, LB_EINVAL, "bad channel or output");
  const ChanDev &d = h->L.ch[ch];
  if (what == LB_OBS_STEP) {
    if (n < 1) return fail(h, LB_EINVAL, "output too small");
    out[0] = (double)h->t[ch];
    return LB_OK;
  }
  if (what == LB_OBS_ACTIVE) {
    if (n < 1) return fail(h, LB_EINVAL, "output too small");
    out[0] = h->active[ch];
    return LB_OK;
  }
  lb_status st = read_observation(h);
  if (st != LB_OK) return st;
  const double *s = &h->hscal[(size_t)ch * CS_COUNT];
  const double *pr = &h->hprof[(size_t)d.row_off * OF_COUNT];
  const long long N = (long long)d.nx * d.ny;
  if (what >= 32) {
    if (n < 1) return fail(h, LB_EINVAL, "output too small");
    switch (what) {
      case LB_OBS_MASS: out[0] = (double)N + s[CS_MASS_DEV]; return LB_OK;
      case LB_OBS_MOMX: out[0] = s[CS_MOMX]; return LB_OK;
      case LB_OBS_FLUX: out[0] = s[CS_FLUX]; return LB_OK;
      case LB_OBS_WALL_DRAG: out[0] = s[CS_DRAG]; return LB_OK;
      case LB_OBS_UMID: out[0] = s[CS_UMID]; return LB_OK;
      case LB_OBS_RESIDUAL: {
        // residual is only meaningful after two checks
        out[0] = h->n_checks >= 2 ? s[CS_RESIDUAL] : INFINITY;
        return LB_OK;
      }
      case LB_OBS_NAN: out[0] = s[CS_NAN]; return LB_OK;
      default: return fail(h, LB_EINVAL, "unknown observable");
    }
  }
  if (n < (size_t)d.ny) return fail(h, LB_EINVAL, "output shorter than ny");
  for (int y = 0; y < d.ny; ++y) {
    const double *r = pr + (size_t)y * OF_COUNT;
    double v;
    switch (what) {
      case LB_OBS_UX: v = r[OF_UX]; break;
      case LB_OBS_UY: v = r[OF_UY]; break;
      case LB_OBS_SXX: v = r[OF_SXX]; break;
      case LB_OBS_SXY: v = r[OF_SXY]; break;
      case LB_OBS_SYY: v = r[OF_SYY]; break;
      case LB_OBS_N1: v = r[OF_SXX] - r[OF_SYY]; break;
      case LB_OBS_PRESSURE: v = (1.0 + r[OF_RHOE_DEV]) / 3.0; break;
      case LB_OBS_KXY: v = r[OF_KXY]; break;
      case LB_OBS_TRT: v = r[OF_TRT]; break;
      case LB_OBS_KXX: v = r[OF_KXX]; break;
      default: return fail(h, LB_EINVAL, "unknown observable");
    }
    out[y] = v;
  }
  return LB_OK;
}

lb_status lb_observe_noalloc(lb_handle *h, int32_t ch, int32_t what, double *out, size_t n) {
  if (!h) return LB_EINVAL;
  if (ch < 0 || ch >= h->n_ch || !out) return fail(h, LB_EINVAL, "bad channel or output");
  const ChanDev &d = h->L.ch[ch];
  if (what == LB_OBS_STEP || what == LB_OBS_ACTIVE) {
    if (n < 1) return fail(h, LB_EINVAL, "output too small");
    out[0] = what == LB_OBS_STEP ? (double)h->t[ch] : (double)h->active[ch];
    return LB_OK;
  }
  const bool scalar = what >= 32;
  const bool known = scalar ? (what >= LB_OBS_MASS && what <= LB_OBS_NAN) : (what >= LB_OBS_UX && what <= LB_OBS_KXX);
  if (!known) return fail(h, LB_EINVAL, "unknown observable");
  const size_t count = scalar ? 1 : (size_t)d.ny;
  if (n < count) return fail(h, LB_EINVAL, scalar ? "output too small" : "output shorter than ny");
  if (what == LB_OBS_RESIDUAL) {
    // the residual of the last convergence check, kept in the workspace
    if (h->n_checks < 2) {
      out[0] = INFINITY;
      return LB_OK;
    }
    HIPCHECK(h, hipMemcpyAsync(out, h->dscal + (size_t)ch * CS_COUNT + CS_RESIDUAL, sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(h, hipStreamSynchronize(h->stream));
    return LB_OK;
  }
  if (h->opt.stress_force)
    return fail(h, LB_EINVAL, "lb_observe_noalloc: the stress-force observation needs per-node scratch (use lb_observe)");
  if (!h->noalloc) return hipfail(h, h->noalloc_err, "lb_observe_noalloc: scratch address");
  // partials, profiles, scalars and the gathered result, 256-byte aligned
  auto chunk = [](size_t doubles) { return align_up(doubles, kAlign / sizeof(double)); };
  const size_t n_part = chunk((size_t)OF_COUNT * h->L.total_part), n_prof = chunk((size_t)OF_COUNT * h->L.total_rows);
  const size_t n_scal = chunk((size_t)CS_COUNT * h->n_ch), n_out = chunk(count);
  const size_t need = (n_part + n_prof + n_scal + n_out) * sizeof(double);
  if (need > kNoallocScratchBytes) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "lb_observe_noalloc: this handle's observation needs %zu bytes of scratch, more than its %zu "
             "(use lb_observe)", need, kNoallocScratchBytes);
    return fail(h, LB_EINVAL, buf);
  }
  double *part = h->noalloc, *prof = part + n_part, *scal = prof + n_prof, *res = scal + n_scal;
  lb_status st = enqueue_observe_into(h, part, prof, scal, 0, 0);
  if (st != LB_OK) return st;
  hipLaunchKernelGGL(gather_observable_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, h->stream,
                     h->dch, ch, what, prof, scal, res);
  HIPCHECK(h, hipGetLastError());
  HIPCHECK(h, hipMemcpyAsync(out, res, count * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return LB_OK;
}

lb_status lb_get_state(lb_handle *h, int32_t ch, double *pops, double *P) {
  if (!h) return LB_EINVAL;
  if (ch < 0 || ch >= h->n_ch || !pops || !P) return fail(h, LB_EINVAL, "bad channel or output");
  const ChanDev &d = h->L.ch[ch];
  const size_t N = (size_t)d.nx * d.ny;
  const size_t Npad = align_up(N, kTile);
  const int es = h->L.esize;
  // the channel's tiles are one contiguous block of the state buffer
  std::vector<char> raw((size_t)kPlanes * Npad * es);
  const char *src = static_cast<const char *>(h->buf[h->cur]);
  HIPCHECK(h, hipMemcpyAsync(raw.data(), src + (size_t)slot(0, d.off) * es, raw.size(),
                             hipMemcpyDeviceToHost, h->stream));
  std::vector<float> ur(d.ny, 0.0f);
  if (es == 4)
    HIPCHECK(h, hipMemcpyAsync(ur.data(), h->duref + d.row_off, sizeof(float) * d.ny, hipMemcpyDeviceToHost,
                               h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  // FP32 slots hold n - a_i - E_i(u_ref) of the row the slot belongs to
  auto at = [&](int p, size_t id) -> double {
    const size_t k = (size_t)slot(p, (long long)id);
    if (es == 8) return reinterpret_cast<const double *>(raw.data())[k];
    const double v = reinterpret_cast<const float *>(raw.data())[k];
    return p < 9 ? v + hweight(p) + href_eq(p, ur[id / d.nx]) : v;
  };
  // the pull: stored slot (plane i, source node) -> n_i at the destination
  for (int y = 0; y < d.ny; ++y)
    for (int x = 0; x < d.nx; ++x) {
      const size_t id = (size_t)y * d.nx + x;
      for (int i = 0; i < 9; ++i) {
        const int ys = y - HCY[i];
        const int xs = ((x - HCX[i]) % d.nx + d.nx) % d.nx;
        double v;
        if (ys < 0)
          v = at(HOPP[i], id);
        else if (ys >= d.ny)
          v = at(HOPP[i], id) + wall_pull_term(h->in[ch], i, h->t[ch]);
        else
          v = at(i, (size_t)ys * d.nx + xs);
        pops[(size_t)i * N + id] = v;
      }
      P[id] = at(9, id);
    }
  if (d.zh) host_zou_he_top(h->in[ch], h->t[ch], pops);
  return LB_OK;
}

lb_status lb_set_state(lb_handle *h, int32_t ch, const double *pops_in, const double *P, int64_t t) {
  if (!h) return LB_EINVAL;
  if (ch < 0 || ch >= h->n_ch || !pops_in || !P || t < 0) return fail(h, LB_EINVAL, "bad arguments");
  const ChanDev &d = h->L.ch[ch];
  const size_t N = (size_t)d.nx * d.ny;
  // a Zou-He top wall replaces what enters its row from above (the next step
  // completes it; completing it here keeps the FP32 row reference consistent)
  std::vector<double> zcopy;
  const double *pops = pops_in;
  if (d.zh) {
    zcopy.assign(pops_in, pops_in + 9 * N);
    host_zou_he_top(h->in[ch], t, zcopy.data());
    pops = zcopy.data();
  }
  const size_t Npad = align_up(N, kTile);
  const int es = h->L.esize;
  // start from the device copy so the padding slots of the last tile keep
  // their values
  std::vector<char> raw((size_t)kPlanes * Npad * es);
  char *dst = static_cast<char *>(h->buf[h->cur]);
  HIPCHECK(h, hipMemcpyAsync(raw.data(), dst + (size_t)slot(0, d.off) * es, raw.size(),
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  // FP32: every row's reference velocity becomes the row mean of u_x of the
  // new state (0 where that is not a finite velocity)
  std::vector<float> ur(d.ny, 0.0f);
  if (es == 4)
    for (int y = 0; y < d.ny; ++y) {
      double su = 0;
      for (int x = 0; x < d.nx; ++x) {
        const size_t id = (size_t)y * d.nx + x;
        double rho = 0, jx = 0;
        for (int i = 0; i < 9; ++i) {
          const double v = pops[(size_t)i * N + id];
          rho += v;
          jx += HCX[i] * v;
        }
        su += jx / rho;
      }
      const double u = su / d.nx;
      ur[y] = (std::isfinite(u) && std::fabs(u) <= 1.0) ? (float)u : 0.0f;
    }
  auto put = [&](int p, size_t id, double v) {
    const size_t k = (size_t)slot(p, (long long)id);
    if (es == 8)
      reinterpret_cast<double *>(raw.data())[k] = v;
    else
      reinterpret_cast<float *>(raw.data())[k] = (float)(p < 9 ? v - hweight(p) - href_eq(p, ur[id / d.nx]) : v);
  };
  // inverse of the pull: every stored slot feeds exactly one (node, i)
  for (int y = 0; y < d.ny; ++y)
    for (int x = 0; x < d.nx; ++x) {
      const size_t id = (size_t)y * d.nx + x;
      for (int i = 0; i < 9; ++i) {
        const int ys = y - HCY[i];
        const int xs = ((x - HCX[i]) % d.nx + d.nx) % d.nx;
        const double v = pops[(size_t)i * N + id];
        if (ys < 0)
          put(HOPP[i], id, v);
        else if (ys >= d.ny)
          put(HOPP[i], id, v - wall_pull_term(h->in[ch], i, t));
        else
          put(i, (size_t)ys * d.nx + xs, v);
      }
      put(9, id, P[id]);
    }
  HIPCHECK(h, hipMemcpyAsync(dst + (size_t)slot(0, d.off) * es, raw.data(), raw.size(),
                             hipMemcpyHostToDevice, h->stream));
  if (es == 4)
    HIPCHECK(h, hipMemcpyAsync(h->duref + d.row_off, ur.data(), sizeof(float) * d.ny, hipMemcpyHostToDevice,
                               h->stream));
  // both buffers: a frozen channel is read from whichever is current later
  {
    lb_status m = mirror_channel(h, ch);
    if (m != LB_OK) return m;
  }
  // step counter and residual history of this channel
  std::vector<ChanDev> cur(h->n_ch);
  HIPCHECK(h, hipMemcpyAsync(cur.data(), h->dch, sizeof(ChanDev) * h->n_ch, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  cur[ch].t = t;
  HIPCHECK(h, hipMemcpyAsync(h->dch, cur.data(), sizeof(ChanDev) * h->n_ch, hipMemcpyHostToDevice, h->stream));
  std::vector<double> nanrows(d.ny, std::numeric_limits<double>::quiet_NaN());
  HIPCHECK(h, hipMemcpyAsync(h->dprev + d.row_off, nanrows.data(), sizeof(double) * d.ny,
                             hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->t[ch] = t;
  h->obs_valid = false;
  return LB_OK;
}

lb_status lb_get_stress(lb_handle *h, int32_t ch, double *sigma) {
  if (!h) return LB_EINVAL;
  if (ch < 0 || ch >= h->n_ch || !sigma) return fail(h, LB_EINVAL, "bad channel or output");
  if (!h->opt.viscoelastic) return fail(h, LB_EINVAL, "the handle runs the instantaneous model (no stored stress)");
  const ChanDev &d = h->L.ch[ch];
  const size_t N = (size_t)d.nx * d.ny;
  const size_t Npad = align_up(N, kTile);
  const int es = h->L.esize;
  // the channel's stress tiles are one contiguous block of the buffer
  std::vector<char> raw((size_t)kStressPlanes * Npad * es);
  const char *src = static_cast<const char *>(h->sbuf[h->cur]);
  HIPCHECK(h, hipMemcpyAsync(raw.data(), src + (size_t)sslot(0, d.off) * es, raw.size(), hipMemcpyDeviceToHost,
                             h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  for (int p = 0; p < kStressPlanes; ++p)
    for (size_t id = 0; id < N; ++id) {
      const size_t k = (size_t)sslot(p, (long long)id);
      sigma[(size_t)p * N + id] = es == 8 ? reinterpret_cast<const double *>(raw.data())[k]
                                          : (double)reinterpret_cast<const float *>(raw.data())[k];
    }
  return LB_OK;
}

lb_status lb_set_stress(lb_handle *h, int32_t ch, const double *sigma) {
  if (!h) return LB_EINVAL;
  if (ch < 0 || ch >= h->n_ch || !sigma) return fail(h, LB_EINVAL, "bad channel or input");
  if (!h->opt.viscoelastic) return fail(h, LB_EINVAL, "the handle runs the instantaneous model (no stored stress)");
  const ChanDev &d = h->L.ch[ch];
  const size_t N = (size_t)d.nx * d.ny;
  const size_t Npad = align_up(N, kTile);
  const int es = h->L.esize;
  // start from the device copy so the padding slots of the last tile keep
  // their values
  std::vector<char> raw((size_t)kStressPlanes * Npad * es);
  char *dst = static_cast<char *>(h->sbuf[h->cur]);
  HIPCHECK(h, hipMemcpyAsync(raw.data(), dst + (size_t)sslot(0, d.off) * es, raw.size(), hipMemcpyDeviceToHost,
                             h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  for (int p = 0; p < kStressPlanes; ++p)
    for (size_t id = 0; id < N; ++id) {
      const size_t k = (size_t)sslot(p, (long long)id);
      const double v = sigma[(size_t)p * N + id];
      if (es == 8)
        reinterpret_cast<double *>(raw.data())[k] = v;
      else
        reinterpret_cast<float *>(raw.data())[k] = (float)v;
    }
  HIPCHECK(h, hipMemcpyAsync(dst + (size_t)sslot(0, d.off) * es, raw.data(), raw.size(), hipMemcpyHostToDevice,
                             h->stream));
  {
    lb_status m = mirror_channel(h, ch);
    if (m != LB_OK) return m;
  }
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->obs_valid = false;
  return LB_OK;
}

lb_status lb_set_profile(lb_handle *h, int32_t ch, const double *ux, const double *n1, int32_t n_pts,
                         int32_t points) {
  if (!h) return LB_EINVAL;
  if (ch < 0 || ch >= h->n_ch || !ux || !n1 || n_pts < 1) return fail(h, LB_EINVAL, "bad arguments");
  if (points != LB_PROFILE_ROWS && points != LB_PROFILE_CHEBYSHEV) return fail(h, LB_EINVAL, "unknown point set");
  const ChanDev &d = h->L.ch[ch];
  if (points == LB_PROFILE_ROWS && n_pts != d.ny) return fail(h, LB_EINVAL, "row profile needs ny values");
  std::vector<double> u(d.ny), q(d.ny);
  if (points == LB_PROFILE_ROWS) {
    for (int y = 0; y < d.ny; ++y) {
      u[y] = ux[y];
      q[y] = n1[y];
    }
  } else {
    // barycentric interpolation on the Chebyshev-Gauss points
    // d_k = cos(pi (2k+1)/(2n)), weights (-1)^k sin(pi (2k+1)/(2n))
    const double H = 0.5 * d.ny, yc = 0.5 * (d.ny - 1);
    for (int y = 0; y < d.ny; ++y) {
      const double dd = (y - yc) / H;
      double num_u = 0, num_q = 0, den = 0;
      int hit = -1;
      for (int k = 0; k < n_pts; ++k) {
        const double th = M_PI * (2 * k + 1) / (2.0 * n_pts);
        const double dk = std::cos(th);
        if (dd == dk) {
          hit = k;
          break;
        }
        const double wk = ((k & 1) ? -1.0 : 1.0) * std::sin(th) / (dd - dk);
        num_u += wk * ux[k];
        num_q += wk * n1[k];
        den += wk;
      }
      u[y] = hit >= 0 ? ux[hit] : num_u / den;
      q[y] = hit >= 0 ? n1[hit] : num_q / den;
    }
  }
  const size_t N = (size_t)d.nx * d.ny;
  std::vector<double> pops(9 * N), P(N);
  for (int y = 0; y < d.ny; ++y) {
    // with the flow-induced density the conserved mass is sum (s + 3/2 P);
    // without it, sum s
    const double rho = d.nnp ? 1.0 - 1.5 * q[y] : 1.0;
    const double usq = u[y] * u[y];
    for (int x = 0; x < d.nx; ++x) {
      const size_t id = (size_t)y * d.nx + x;
      for (int i = 0; i < 9; ++i) {
        const double cu = HCX[i] * u[y];
        pops[(size_t)i * N + id] = hweight(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
      }
      P[id] = q[y];
    }
  }
  return lb_set_state(h, ch, pops.data(), P.data(), h->t[ch]);
}

}  // extern "C"

namespace {

// Rest state: n_i = a_i (stored as 0 when shifted), previous trace 0.
template <typename T>
__global__ void fill_rest_kernel(T *p, long long n_slots, int shifted) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n_slots;
       i += (long long)gridDim.x * blockDim.x) {
    const int f = (int)((i / kTile) % kPlanes);
    p[i] = (f < 9 && !shifted) ? T(f == 0 ? 4.0 / 9.0 : (f < 5 ? 1.0 / 9.0 : 1.0 / 36.0)) : T(0);
  }
}

lb_status fill_rest(lb_handle *h, int which) {
  const long long n = (long long)kPlanes * h->L.plane;
  if (h->L.esize == 8)
    hipLaunchKernelGGL(fill_rest_kernel<double>, dim3(2048), dim3(256), 0, h->stream,
                       static_cast<double *>(h->buf[which]), n, 0);
  else
    hipLaunchKernelGGL(fill_rest_kernel<float>, dim3(2048), dim3(256), 0, h->stream,
                       static_cast<float *>(h->buf[which]), n, 1);
  HIPCHECK(h, hipGetLastError());
  return LB_OK;
}

}  // namespace
