// Internal declarations shared by the HIP kernel files and the host runtime.
// Not part of the public C ABI (include/lddmm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lddmm {

constexpr int kBlock = 256;        // threads per block for every kernel
constexpr int kPartMax = 4096;     // max blocks of a reducing kernel (partials per launch)
constexpr int kMaxStages = 12;     // radix stages of one 1D transform
constexpr int kFFTElems = 2048;    // complex values held in LDS by one FFT block (16 KB)
constexpr int kEMax = 8;           // complex values one thread holds across an LDS stage
constexpr int kXCD = 8;            // accelerator complex dies of an MI355X

// Unsigned division by a runtime constant d via a precomputed multiplier:
// q = (umulhi(n, m) + n) >> s, exact for every n < 2^31 (all indices here are
// below 2^31 because each axis is at most LDDMM_MAX_DIM = 1024).
struct FastDiv {
  uint32_t d, m;
  int s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  int s = 0;
  while ((1ull << s) < d) ++s;
  const unsigned long long m = ((1ull << 32) * ((1ull << s) - d)) / d + 1;
  return FastDiv{d, (uint32_t)m, s};
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (__umulhi(n, f.m) + n) >> f.s;
}

// Kernel-class timing (lddmm_profile_begin / lddmm_profile_end): HIP events
// recorded on the launch stream around each launch of an enabled class whose
// grid has at least the selected number of voxels.
void prof_open(int cls, long long vox, hipStream_t s, hipEvent_t* a);
void prof_close(int cls, long long vox, hipStream_t s, hipEvent_t a);
struct ProfScope {
  int cls;
  long long vox;
  hipStream_t s;
  hipEvent_t a;
  ProfScope(int c, long long n, hipStream_t st) : cls(c), vox(n), s(st) { prof_open(c, n, st, &a); }
  ~ProfScope() { prof_close(cls, vox, s, a); }
};

// Computational grid of one pyramid level.
struct Geom {
  int nx, ny, nz;   // P (each axis 7-smooth)
  int hx;           // nx/2 + 1: length of the half spectrum along x
  int hs;           // row stride of the half spectrum: hx rounded up to 16
  long long n;      // nx*ny*nz (< 2^30)
  long long nspec;  // hs*ny*nz
  float h, inv_h;   // spacing and its inverse
  FastDiv fx, fy, fz, fhx;   // division by nx, ny, nz, hx
};

// Mixed-radix factorisation of one transform length (radices 2,3,4,5,7,8).
struct FFTPlan {
  int n, nst;
  int radix[kMaxStages];
  FastDiv fnb[kMaxStages];   // division by n / radix[s]
  FastDiv fns[kMaxStages];   // division by the product of the previous radices
};

// Device-side control state of the descent (one per problem).
enum : int { MODE_GRAD = 0, MODE_RETRY = 1, MODE_STOPPED = 2, MODE_INIT = 3 };

struct State {
  int mode;        // what the next slot does
  int base;        // v buffer holding the current iterate
  int eval;        // v buffer the forward sweep evaluates
  int halvings;    // consecutive rejections
  int row;         // next trace row
  int stopped_any; // a level stopped on the guard
  int nonfinite;   // non-finite energy seen
  int pad0;
  double eps, step0;
  double E, R, D, img;       // energy terms of the current iterate
  double min_det;            // min det of the last gradient evaluation (trace column)
  double min_det_final;      // min det of the returned v's maps (LDDMM_WFOLD)
};

// --------------------------------------------------------------- sweeps ----

struct FwdArgs {
  Geom g;
  const float* vA;        // v buffers [T][3][n]; st->eval selects one
  const float* vB;
  int j, T;
  float dt, alpha, gamma;
  const float* u_cur;     // u0_j [3][n] (unused when j == 0)
  float* u_next;          // u0_{j+1} [3][n]
  const float* J0;        // template channels [C][n]
  const float* J1;        // target channels [C][n]
  int nch;                // weighted channels (1 or 2)
  int ch[2];              // their channel index in J0/J1
  float w[2];             // their weights
  int img_ch;             // image channel index for the monitor (-1: none)
  int img_weighted;       // 1 if img_ch is among the weighted channels (slot img_slot)
  int img_slot;
  float* J0t_next;        // deformed templates at j+1 [nch][n] (j+1 < T)
  float* r;               // residual [nch][n] (j+1 == T)
  double* partR;          // [kPartMax] for this j
  double* partD;          // [kPartMax]
  double* partI;          // [kPartMax]
  const State* st;
  int rk4;                // departure points by fourth-order Runge-Kutta
  int zmarch;             // plane-marching traversal (forward_tiles blocks), else grid-stride
  int staged;             // LDS-staged traversal (forward_staged; takes precedence)
};

struct BwdArgs {
  Geom g;
  const float* vA;
  const float* vB;        // st->base selects the iterate
  const float* vfix;      // if non-null: use this v instead of vA/vB
  int T;
  float dt;
  int j;                  // u1_j from u1_{j+1} (j >= 0), else no map step
  const float* u_next;    // u1_{j+1} [3][n] (null: zero)
  float* u_cur;           // u1_j [3][n]
  int jb;                 // body force at time jb = j+1 (< T), else none
  const float* J0t;       // deformed templates at jb, channel stride cstride
  long long cstride;
  const float* r;         // residual [nch][n]
  int nch;
  float w[2];
  float coef;             // 2 / sigma^2
  float* b;               // out: body force [3][n]
  double* partDet;        // [kPartMax] min det per block
  const State* st;
  int need_mode;          // run only when st->mode == need_mode (-1: always)
  int staged;             // body-force steps run the LDS-staged kernel (backward_staged)
  int rk4;                // departure points by fourth-order Runge-Kutta
};

// x-inverse pass epilogue
enum : int { UPD_STEP = 0, UPD_WRITE_G = 1, UPD_WRITE_KB = 2 };

struct UpdArgs {
  int kind;
  int j;                  // time step of v
  float* vA;              // v buffers [T][3][n]
  float* vB;
  const float* vfix;      // UPD_WRITE_G with an explicit v
  float* out;             // UPD_WRITE_G: g [T][3][n]; UPD_WRITE_KB: Kb [3][n]
  const State* st;
  int need_mode;
};

// ------------------------------------------------------------- FFT passes --

// One problem's K smoothing: geometry, plans, tables, buffers and tiles.
struct FftPair {
  Geom g;
  FFTPlan px, py, pz;
  const float2* tw[3];     // twiddles per axis
  const double* lam[3];    // Laplacian symbol per axis
  double alpha, gamma;
  const float* b;          // body force [3][n]
  float2* S;               // half spectrum [3][nspec]
  int ppb;                 // x passes: row pairs per block
  int lgTXy, nbx_y;        // y pass: log2 tile width, tiles along kx
  int lgTXz, nbx_z;        // z pass
  int fused;               // x and y in one pass each way (a plane of one component in LDS)
  const State* st;
  int need_mode;
};

// Launch shape of the five passes of one problem.
struct FftLaunch {
  int x_tiles, y_tiles, z_tiles;
  int ex, ey, ez;          // per-thread register budget (8, 16 or 32 values)
  size_t x_lds, y_lds, z_lds;
};

// ---------------------------------------------------------------- batching --

constexpr int kMaxBatch = 32;     // problems per batched launch
constexpr int kMaxT = 64;         // equals LDDMM_MAX_T

// Tile offsets of one batched launch: problem p owns blocks [off[p], off[p+1]).
struct BatchRef {
  int np;
  int off[kMaxBatch + 1];
  const void* tab[kMaxBatch];     // device PairTab of each problem
};

struct DecideArgs {
  State* st;
  const double *partR, *partD, *partI, *partDet;
  int T, nfw, nbw, has_img, guard, init;
  double dt, h3, inv_sigma2;
  double* trace;
};

struct RetryArgs {
  float* vA;
  float* vB;
  long long count;
  const State* st;
};

// Every launch argument of one problem at the current level, kept in device
// memory so one kernel can serve all problems of a batch.
struct PairTab {
  FwdArgs fwd[kMaxT];
  BwdArgs bwd[kMaxT + 1];   // slot j + 1 for backward launch j = -1 .. T-1
  UpdArgs upd[kMaxT];
  FftPair fft;
  DecideArgs dec[2];        // [0]: after a trial, [1]: first evaluation of a level
  RetryArgs rty;
};

// --------------------------------------------------------------- launchers --
// flow.hip
void launch_pad(const float* src, int Nx, int Ny, int Nz, float* dst, const Geom& g,
                hipStream_t s);
void launch_down2(const float* src, const Geom& fine, float* dst, const Geom& coarse,
                  int nfields, hipStream_t s);
void launch_up2(const float* src, const Geom& coarse, float* dst, const Geom& fine, int nfields,
                hipStream_t s);
int reduce_grid(long long n);
void set_sweep_blocks(int blocks);
void set_fft_x_elems(int elems);
void set_fft_cols(int axis, int cols);   // axis 0: y tiles, 1: z tiles
void launch_forward(const FwdArgs& a, hipStream_t s);
// Forward sweep traversal on grid g and its blocks (= the partials it writes),
// single or batched; set_fwd_tiles(0) selects the grid-stride sweep.
void set_fwd_tiles(int tiles);
bool forward_zmarch(const Geom& g);
bool forward_staged(const Geom& g);
void set_fwd_staged_min_blocks(int blocks);
int forward_tiles(const Geom& g);
void launch_backward(const BwdArgs& a, hipStream_t s);
// Blocks of a body-force launch of the backward sweep on this grid = the min-det
// partials it writes (single or batched).
int backward_partials(const Geom& g);
bool backward_staged(const Geom& g);
void set_staged_min_blocks(int blocks);
void launch_forward_batched(const BatchRef& br, int j, int T, int nch, hipStream_t s);
void launch_backward_batched(const BatchRef& br, int j, int T, int nch, hipStream_t s);
void launch_crop3(const float* u, const Geom& g, int Nx, int Ny, int Nz, float* out,
                  hipStream_t s);
void launch_apply(const float* u, int Nx, int Ny, int Nz, float inv_h, const void* src,
                  int interp, int dtype, void* dst, hipStream_t s);
void launch_make_mask(const float* img, long long n, float tau, float* m, float* mi,
                      hipStream_t s);
void launch_fill(float* p, long long n, float val, hipStream_t s);
void launch_copy(const float* src, float* dst, long long n, hipStream_t s);

// fft.hip
bool make_plan(int n, FFTPlan* p);
void launch_twiddles(float2* tw, int n, hipStream_t s);
void launch_lambda(double* lam, int n, double h, hipStream_t s);
void fft_tiles(FftPair& f, FftLaunch* L);
void set_fft_fused_lds(int bytes);
void launch_fft_x_fwd(const FftPair& f, const FftLaunch& L, hipStream_t s);
void launch_fft_y(const FftPair& f, const FftLaunch& L, int inverse, hipStream_t s);
void launch_fft_z_K(const FftPair& f, const FftLaunch& L, hipStream_t s);
void launch_fft_x_inv(const FftPair& f, const FftLaunch& L, const UpdArgs& u, hipStream_t s);
void launch_fft_batched(int pass, const BatchRef& br, int emax, size_t lds, int j, hipStream_t s);
bool launch_fft_fused_batched(int inverse, const BatchRef& br, const Geom& g, size_t lds, int j,
                              hipStream_t s);

// grad.hip
struct GradArgs {
  Geom g;
  int nch;
  const float* J0;       // template channels [C][n]
  int ch[2];
  float wc[2];
  float coef;            // 2 h^3 / sigma^2
  const float* r;        // residual [nch][n]
  const float* u;        // u0 at the step the kernel needs [3][n]
  const float* v;        // v_j [3][n]
  const float* ub_in;    // ubar_{j+1} [3][n]
  float* ub_out;         // ubar_j or ubar_T [3][n]
  float* w;              // L v_j scratch [3][n]
  float* grad;           // dE/dv_j [3][n]
  float dt, alpha, gamma, reg;   // reg = 2 dt h^3
  const int* radius;     // device: splat radius for this step
  int* overflow;         // device flag: radius beyond the supported maximum
};
void launch_ubar_init(const GradArgs& a, hipStream_t s);
void launch_grad_step(const GradArgs& a, hipStream_t s);

// control.hip
void launch_energy_out_checked(const State* st, const int* overflow, double* out4, hipStream_t s);
void launch_level_begin(State* st, double step, int keep_flags, hipStream_t s);
void launch_decide(State* st, const double* partR, int T, const double* partD,
                   const double* partI, const double* partDet, int nblk_fwd, int nblk_bwd,
                   int has_img, double dt, double h3, double inv_sigma2, int guard,
                   double* trace, int init, hipStream_t s);
void launch_retry(float* vA, float* vB, long long count, const State* st, hipStream_t s);
void launch_decide_batched(const BatchRef& br, int init, hipStream_t s);
void launch_retry_batched(const BatchRef& br, hipStream_t s);
void launch_energy_out(const State* st, double* out4, hipStream_t s);
void launch_final_det(State* st, const double* partDet, int T, int nbw, hipStream_t s);

}  // namespace lddmm
