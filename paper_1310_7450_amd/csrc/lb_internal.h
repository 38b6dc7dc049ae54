// Internal types shared by the host runtime and the gfx950 kernels of lbnlm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbnlm {

// Stored fields per node: nine populations and the previous stress trace.
constexpr int kPlanes = 10;
// Nodes per storage tile; field p of node n lives at slot(p, n).
constexpr int kTile = 64;
__host__ __device__ inline long long slot(int p, long long n) {
  return ((n >> 6) * kPlanes + p) * kTile + (n & (kTile - 1));
}
// Time-integrated stress (viscoelastic model): sigma_xx, sigma_xy, sigma_yy
// of the previous step, in buffers of their own tiled like the state.
constexpr int kStressPlanes = 3;
__host__ __device__ inline long long sslot(int p, long long n) {
  return ((n >> 6) * kStressPlanes + p) * kTile + (n & (kTile - 1));
}
// Per-row observation fields accumulated in FP64 (x sums per row).
enum ObsField {
  OF_UX = 0, OF_UY, OF_SXX, OF_SXY, OF_SYY, OF_RHOE_DEV, OF_MASS_DEV, OF_MOMX,
  OF_KXY, OF_TRT, OF_DRAG, OF_KXX, OF_COUNT
};
// Per-channel scalars written by the reduction kernel.
enum ChanScalar {
  CS_MASS_DEV = 0, CS_MOMX, CS_FLUX, CS_DRAG, CS_UMID, CS_RESIDUAL, CS_UMAX, CS_NAN, CS_COUNT
};

// Resolved parameters of one channel as the kernels read them.
struct ChanDev {
  long long off;        // element offset of node (0,0) in every plane
  long long t;          // steps completed before the current launch group
  long long t_startup;  // first step without body force
  int nx, ny;
  int row_off;          // first row of this channel in the per-row buffers
  int poff;             // first partial row of this channel
  int nxs;              // partial columns per row (x strips)
  int active;
  double g;             // body-force density
  double omega;         // 1 / tau_eff
  double kf;            // 1 - 1/(2 tau_eff)
  double sp;            // -9 / (2 tau_eff): stress coefficient of the forcing
  double G;             // G_inf
  double inv_tau;       // 1/tau (0 for tau = inf)
  double inv_gc;        // 1/gamma_c
  double lgt;           // lambda G_inf tau
  double uw;            // top wall x velocity while t < t_startup
  double pd;            // pressure drive: p+ - p- = (nx + 1) G_p while t < t_startup
  int gpbc;             // generalised periodic boundaries in x
  int nnp;              // keep the flow-induced density terms
  int zh;               // top wall: Zou-He velocity boundary on row ny - 1
};

// Work unit of one wavefront: rows [y0, y1) of channel ch, starting at
// column x0 (wide mode: first interior column; narrow mode: 0). flip: the
// vector sweep marches this strip against the step's direction (odd bands).
// x1: the two-step sweep stores columns [x0, x1) (at most two_step_cols).
struct Strip {
  int ch, x0, y0, y1, flip, x1;
};

struct SweepArgs {
  const void *A;        // state read (10 planes)
  void *B;              // state written (10 planes)
  long long plane;      // nodes per buffer (a multiple of the tile)
  const Strip *strips;
  const ChanDev *ch;
  double *part;         // observation partials [row][OF_COUNT]
  int n_strips;
  int n_wg;
  int k;                // step offset added to every channel's t
  int nt;               // store the new state with nontemporal hints
  int down;             // the step marches downwards (vector sweep; flipped strips go upwards)
  const float *uref;    // FP32: reference velocity of every row (all channels)
  const void *SA;       // viscoelastic model: stress read (3 planes)
  void *SB;             // viscoelastic model: stress written (3 planes)
  int ve;               // time-integrated stress in place of the instantaneous one
  int zh;               // some channel of the handle has a Zou-He top wall
  int wall;             // two-step sweep: some strip's channel has a moving or Zou-He top wall
};
// A state buffer larger than this is written with nontemporal stores: it
// cannot stay in the 256 MB last-level cache (MALL) until the next step reads
// it, so caching its lines only evicts the reads in flight.
constexpr long long kNontemporalBytes = 256ll << 20;

// Width classes of the sweep: nx in {1,2,4,...,64} runs a whole period per
// lane group ("narrow", classes 0..6); nx a multiple of 64 lanes times the
// nodes one lane holds (vec_nodes) runs aligned strips of that many columns
// with vector accesses (kVecClass); any other multiple of 64 (>= 128) runs
// aligned 64-column strips (kWide64Class); any other width runs generic
// 64-column strips with wrapped lanes (kWideClass).
#ifndef LB_VEC_SWEEP
#define LB_VEC_SWEEP 1
#endif
constexpr int kWideClass = 7;
constexpr int kWide64Class = 8;
constexpr int kVecClass = 9;
constexpr int kClasses = 10;
// nodes per lane of the vector sweep: four FP32 nodes (one 16-byte access)
// or one FP64 node (measured: an 8-byte FP64 access over 64-column strips
// beats a 16-byte one over 128-column strips on the 4096 x 1024 channel)
#ifndef LB_VEC_NPL32
#define LB_VEC_NPL32 4
#endif
#ifndef LB_VEC_NPL64
#define LB_VEC_NPL64 1
#endif
inline int vec_nodes(int esize) { return esize == 4 ? LB_VEC_NPL32 : LB_VEC_NPL64; }
inline int width_class(int nx, int esize) {
  for (int c = 0; c < 7; ++c)
    if (nx == (1 << c)) return c;
  if (LB_VEC_SWEEP && nx % (64 * vec_nodes(esize)) == 0) return kVecClass;
  if (nx % 64 == 0) return kWide64Class;
  return kWideClass;
}
inline bool is_strip_class(int cls) { return cls >= kWideClass; }
// columns of one strip of a strip class
inline int strip_cols(int cls, int esize) { return cls == kVecClass ? 64 * vec_nodes(esize) : 64; }

// Host launchers (defined in lb_kernels.hip).
hipError_t launch_sweep(int fp32, int cls, bool observe, const SweepArgs &a, hipStream_t s);
hipError_t launch_reduce(const ChanDev *ch, int n_ch, const double *part, double *prof,
                         double *prev_ux, double *scal, const float *uref, int update_residual,
                         int steps_since, hipStream_t s);
hipError_t launch_advance(ChanDev *ch, int n_ch, int steps, hipStream_t s);
hipError_t launch_gpbc(int fp32, void *B, const ChanDev *ch, int n_ch, int k, const float *uref, hipStream_t s);
// FP64 step over tiles of kMainTileX x kMainTileY nodes (x0, y0, y1 of a
// Strip; SweepArgs.strips holds the tiles, n_strips their number).
#ifndef LB_MAIN_TX
#define LB_MAIN_TX 64
#endif
#ifndef LB_MAIN_TY
#define LB_MAIN_TY 8
#endif
#ifndef LB_MAIN_THREADS
#define LB_MAIN_THREADS 512
#endif
constexpr int kMainTileX = LB_MAIN_TX, kMainTileY = LB_MAIN_TY, kMainThreads = LB_MAIN_THREADS;
hipError_t launch_tiles(const SweepArgs &a, hipStream_t s);
// Fused stress-force step: tiles of kSafTileX x kSafTileY output nodes
// (x0, y0, y1 of a Strip), one workgroup each; each of the kSafThreads
// threads takes a column of kSafTileX * kSafTileY / kSafThreads nodes.
#ifndef LB_SAF_TX
#define LB_SAF_TX 64
#endif
#ifndef LB_SAF_TY
#define LB_SAF_TY 16
#endif
#ifndef LB_SAF_THREADS
#define LB_SAF_THREADS 512
#endif
constexpr int kSafTileX = LB_SAF_TX, kSafTileY = LB_SAF_TY, kSafThreads = LB_SAF_THREADS;
hipError_t launch_saf_fused(const double *A, double *B, const ChanDev *ch, const Strip *tiles, int n_tiles, int k,
                            int nt, hipStream_t s);
hipError_t launch_saf_observe(const double *A, const ChanDev *ch, int n_ch, long long plane, int total_rows,
                              double *U, double *Tn, double *part, hipStream_t s);
hipError_t launch_rereference(float *A, const ChanDev *ch, int n_ch, int total_rows, const double *prof,
                              float *uref, hipStream_t s);
// Two steps per launch (sweep_vec2_kernel) on strips of vector-class
// channels without the pressure drive: NPL nodes per lane, four for FP32
// states streamed from HBM with the instantaneous model (16-byte loads keep
// more bytes in flight), two otherwise (fewer registers: three wavefronts
// per SIMD in FP32), in windows of 64 NPL columns of which
// two_step_cols(NPL) are stored (the rest is the halo step t+1 needs).
// SweepArgs.strips holds the strips, n_strips their number; the state (with
// the viscoelastic model also the stress) goes from A to B over steps k and
// k+1.
inline int two_step_npl(bool fp32, bool nt, bool ve) { return (fp32 && nt && !ve) ? 4 : 2; }
inline int two_step_cols(int npl) { return 64 * npl - 2 * npl * ((2 + npl - 1) / npl); }
// wavefronts per strip (one per stage) and the most rows a strip may have
constexpr int kTwoStepWaves = 2, kTwoStepMaxRows = 56;
hipError_t launch_two_step(bool fp32, const SweepArgs &a, hipStream_t s);
// Two steps per launch for the narrow widths (nx a power of two up to 64,
// the instantaneous model): one workgroup of two wavefronts per strip of
// rows, the strips of one width in SweepArgs.strips, n_wg = n_strips.
hipError_t launch_narrow_two_step(bool fp32, int nx, const SweepArgs &a, hipStream_t s);
// workgroups of the narrow two-step kernel one CU holds at once (the fewest
// over the widths)
int narrow_two_step_blocks_per_cu(bool fp32);
// workgroups of the two-step kernel one CU holds at once
int two_step_blocks_per_cu(bool fp32, bool nt, bool ve);

}  // namespace lbnlm
