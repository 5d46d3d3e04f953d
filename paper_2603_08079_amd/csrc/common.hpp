// Host/device shared descriptors of libmabd.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mabd {

// Status bits raised by kernels into a device word (integer atomics only).
enum : uint32_t {
  FLAG_NONFINITE = 1u,  // det A <= 0, polar did not converge, or a non-finite value
  FLAG_SINGULAR = 2u,   // a pivot block of an elimination was not positive definite
  FLAG_NOTCONV = 4u,    // an iterative dual solve stopped above its tolerance
  FLAG_GUARD = 8u,      // a kernel was handed work beyond its static sizes (internal error)
};

// Chain of ball joints in "row space".  Rows r = 0..K-1 are the joints in
// chain order; the body between rows r and r+1 is position beta(r) = r + 1 - hl
// (hl = 1 if row 0 is a one-sided joint to the world / a pinned body), valid
// for 0 <= beta < nb.  Row r's left body is beta(r-1), its right body beta(r).
struct ChainDesc {
  int32_t body0;  // first body (solver order) of the chain
  int32_t nb;     // dynamic bodies
  int32_t row0;   // first global chain row
  int32_t K;      // rows (joints), >= 2
  int32_t hl, hr; // one-sided joint at the start / end
  int32_t tile0;  // first tile
  int32_t ntile;  // tiles; interface rows = ntile + 1
  int32_t grow0;  // first interface row (global index)
  int32_t ngroup; // groups of interface rows; top rows = ngroup + 1
  int32_t group0; // first group (global index; also its record index)
  int32_t gtop0;  // first top row (global index)
  int32_t top_global;  // 1: the top system is reduced by chain_global_kernel
                       // (more than CHAIN_THREADS rows), 0: by the last group
};

// A group covers chain-local interface rows [g0, g0 + T] (T >= 1), reduced in
// one workgroup like a tile.
struct GroupDesc {
  int32_t chain;
  int32_t g0;
  int32_t T;
  int32_t gidx;   // group index inside its chain
};

// A tile covers chain-local rows [r0, r0 + T] (T >= 1).  Its rows r0 and r0+T
// are interface rows shared with the neighbouring tiles.
struct TileDesc {
  int32_t chain;
  int32_t r0;
  int32_t T;
  int32_t tidx;   // tile index inside its chain
};

// a tile of a chain has T + 1 rows with T = tile threads - 2 (64, 128 or 256
// threads), or T = PACK_T for packed tiles (64 threads); groups of interface
// rows use CHAIN_THREADS threads
constexpr int CHAIN_THREADS = 256;
constexpr int TILE_REC = 27;         // doubles per tile record
constexpr int GROW_REC = 56;         // doubles per top-level row (scratch)
constexpr int GROUP_T = 255;         // interface rows per group - 1
// packed tiles: 64-thread tiles of PACK_T rows; after two levels of cyclic
// reduction at most 16 rows of a tile survive, and four tiles' survivors are
// reduced together in one wave (rows of tile ti: lanes 16 (ti mod 4) + j)
constexpr int PACK_T = 60;
constexpr int PACK_SV = 18;          // doubles per surviving row: D 6, b 3, U 9
constexpr int PACK_CF = 21;          // doubles per packed eliminated row: PL 9, PU 9, Pb 3

// per-shape raw constants used by the force: Mbar0..2, m, V, mu, lambda
constexpr int SHAPE_STRIDE = 8;
// per-shape structured inverse of Hbar (layout in dmath.hpp)
constexpr int HINV_STRIDE = 20;

constexpr int NO_FAIL = 0x7fffffff;

// precision form 1: a correction sweep that does not halve the KKT residual
// has reached the FP64 rounding floor; the step is accepted there only if the
// residual is within this factor of kkt_tol
constexpr double IR_STALL_FACTOR = 10.0;
// ... or if rho_p is and |G dq + C| is within this many units of rounding of
// the size of the summands it is formed from (per row: the translation
// difference, both anchor offsets A p, both ends' increments J(p) dq)
constexpr double IR_ROUND_FACTOR = 64.0;
// form-1 partials per tile: the four sums behind rho_p and rho_d, then the
// squared size of the summands of G dq + C
constexpr int IR_PART = 5;

struct ChainArgs {
  const ChainDesc *chains;
  const TileDesc *tiles;
  int ntiles;
  const double *q, *qd;       // input state, SoA with stride ns
  double *q_out, *qd_out;     // output state (distinct buffers)
  int64_t ns;
  const int32_t *shp;         // shape index per body
  const double *hinv;         // HINV_STRIDE per shape
  const double *shape;        // SHAPE_STRIDE per shape
  const double *pl, *pr;      // anchors of the left / right end of each chain row, [3][nrs]
  const uint8_t *flag;        // bit0: left end is side a of the joint, bit1: right end is
  int64_t nrs;
  double g[3];
  double h;
  double *tilerec;            // TILE_REC per tile
  const double *xg;           // 3 per global reduced row
  double *lam;                // 3 per chain row
  uint32_t *status;
  int step;                   // step index inside the current call
  // precision form 1 (FP32 body/assembly, FP64 factor, FP64 residual refinement)
  double *dq;                 // 12 x ns accumulated increment of the current step (SoA)
  double *rp;                 // 12 x ns FP64 primal residual, world frame (SoA)
  double *rd;                 // 3 x nrs FP64 dual residual per chain row (SoA)
  double *part;               // IR_PART partial sums per tile (DIAG_PART with diag)
  double *ir;                 // [0] 0 running / 1 converged / 2 stalled near tol /
                              // 3 stalled above it, [1] sweeps,
                              // [2] rho_p, [3] rho_d, [4] kkt, [5] previous kkt
  const double *wr;           // 6 x ns external wrench [tau; f] per body (SoA), or null
  // packed tiles (per group of four tiles, 64 lanes each): surviving rows
  // [PACK_SV][64] and factors of the rows eliminated in the packed levels
  // [PACK_CF][64]
  double *psv;
  double *pcf;
  // 1: chain_resid_kernel checks a finished step (dq = h qd_out, constraint
  // values at q_out) and writes DIAG_PART partials per tile into part
  int diag;
};

// partials per block of the step diagnostics: sum |H^-1 r_p|^2, sum
// |H^-1 f_A|^2, sum |G H^-1 f_A + C|^2, sum |G dq + C|^2, max |C| of ball
// joints and of hinges at the new state
constexpr int DIAG_PART = 6;

// status words: [0] FLAG_* bits, [1] first failing step of the current call,
// [2] index of the running step (set on the device by a one-thread kernel at
// the start of every step, so that a captured step graph is step-independent)
#ifdef __HIPCC__
// record a failure of the running step (integer atomics only)
__device__ __forceinline__ void raise_flag(uint32_t *st, uint32_t bits, int /*unused*/) {
  atomicOr(st, bits);
  atomicMin(reinterpret_cast<int *>(st + 1), *reinterpret_cast<const volatile int *>(st + 2));
}
// a step after a failed one does nothing, so the last good state survives
// (two relaxed device-scope reads, issued together)
struct StepGate {
  int fail, cur;
  __device__ __forceinline__ bool skip() const { return fail < cur; }
};
__device__ __forceinline__ StepGate step_gate(const uint32_t *st) {
  int *s = const_cast<int *>(reinterpret_cast<const int *>(st));
  return StepGate{__hip_atomic_load(s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                  __hip_atomic_load(s + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
}
__device__ __forceinline__ bool skip_step(const uint32_t *st, int /*unused*/) {
  return step_gate(st).skip();
}
#endif

}  // namespace mabd
