// tlb_internal.h -- declarations shared by the translation units of libtlb.so (the step
// library tlb.hip and the learned-correction library learn.hip).  Not installed, not part of
// the C interface.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>

#include "tlb.h"

// Longest run of time steps replayed as one graph; longer runs replay it repeatedly and a
// shorter remainder replays a graph of its own length.
constexpr int TLBI_GRAPH_CHUNK = 32;

// A torus grid: the caller's state buffers, the stream, and the library's per-row tables.
struct tlb_grid {
  tlb_params p;
  void* f[3];
  void* phi[3];
  hipStream_t stream;
  void* rows;       // RowCoef<T>[nt]
  double* area;     // [nt]: r J dtheta dphi, the area of a node of row q
  double* partial;  // [3 * red_blocks + 3]
  double* half_len; // [nt]: (R + r cos theta_{q+1/2}) dphi, the length of a theta-face
  int red_blocks, rows_per_block;
  size_t elem;
  int ty;                     // tile height of the stage kernel (4, 8 or 16)
  // graphs[c][s]: s = 1, 2, 4, .., TLBI_GRAPH_CHUNK time steps as one graph of kernel nodes,
  // closed by the rebase of the order parameter when c = 1 (FP32), all built on the first call
  // that needs one; graph_version: the grid's version when they were built
  hipGraphExec_t graphs[2][TLBI_GRAPH_CHUNK + 1];
  unsigned graph_version;
  void* dft_work;  // structure-factor workspace (built on first use): row transforms and twiddles
  double n_ref;      // reference density of FP32 storage (see stores_deviation), a float value
  unsigned version;  // changes whenever n_ref does: stage arguments kept in graphs are stale
  unsigned long long uid;  // unique over the process: graphs kept elsewhere key on it
  int* check_flag;   // [1]: set by the non-finite check of tlb_step_n (check_every > 0)
  double* proj;      // [3 nt]: per-row sums of the learned correction (tlb_apply_correction)
  void* ch4;         // TLB_CH4: mu, J u^theta phi, u^phi phi of a stage input (3 planes of T)
  // FP32 grids: the order parameter is phi_base + phi[c] (c = 0, 1, 2 hold deviations from the
  // base); the deviation of copy 0 moves into the base after every TLBI_GRAPH_CHUNK-th time step
  // counted from the last set_state, so the bits of a state do not depend on how the steps that
  // made it were split into calls
  float* phi_base;
  int phase;  // FP32: time steps since the last rebase (0 .. TLBI_GRAPH_CHUNK - 1); FP64: 0
};


// Records `msg` as the thread's last error and returns `code`.
int32_t tlbi_fail(int32_t code, const std::string& msg);

// One kernel launch with a single by-value argument block, replayable as a graph node.
struct tlbi_launch {
  const void* fn;
  dim3 grid, block;
  alignas(16) unsigned char args[512];
};

// FP32 grids: move the deviation of state copy 0 into the order parameter's base (exactly),
// enqueued on `stream`; no-op for FP64 grids.
int32_t tlbi_phi_rebase(const tlb_grid* g, hipStream_t stream);
// the rebase as a launch record (FP32 grids); returns 0 for FP64 grids, else 1
int tlbi_phi_rebase_launch(const tlb_grid* g, tlbi_launch* out);

// The launches of Runge-Kutta stage `stage` (1..3) of one time step of grid g (the stage
// kernel, preceded by a prepass for TLB_CH4); returns their number (1 or 2).
int tlbi_stage_launches(const tlb_grid* g, int stage, tlbi_launch out[2]);

namespace {

// Q = 4 Gauss-Hermite velocity set (eq. vmatrix) and weights w = (3 -/+ sqrt 6)/12, with the
// irrational roots written out as literals so that every constant below folds at compile time.
constexpr double SQRT6 = 2.449489742783178098197284074705891391966;
constexpr double VOUT = 2.334414218338977239317512267210362194489;  // sqrt(3 + sqrt 6)
constexpr double VIN = 0.7419637843027258576485135967263602248295;  // sqrt(3 - sqrt 6)

__host__ __device__ constexpr double vel(int i) {
  return i == 0 ? -VOUT : i == 1 ? -VIN : i == 2 ? VIN : VOUT;
}
__host__ __device__ constexpr double wgt(int i) {
  return (i == 0 || i == 3) ? (3.0 - SQRT6) / 12.0 : (3.0 + SQRT6) / 12.0;
}

// Storage of the populations.  FP32 grids store each population as its deviation from the
// rest equilibrium of the grid's reference density n_ref, f_k - n_ref w_i w_j (k = 4 i + j;
// n_ref is the mean density of the state loaded last, to two significant digits): the stored
// values are a few per cent of f, so their rounding is correspondingly finer, and the small
// per-step increments (relaxation, forcing) are not lost against O(0.1 n) values.  FP64 grids
// store f_k itself.
template <typename T>
__host__ __device__ constexpr bool stores_deviation() {
  return std::is_same<T, float>::value;
}
// the value subtracted before storage, per unit of n_ref: w_i w_j for deviation storage, else 0
template <typename T>
__host__ __device__ constexpr double rest_offset(int k) {
  return stores_deviation<T>() ? wgt(k >> 2) * wgt(k & 3) : 0.0;
}

template <int I>
using ic = std::integral_constant<int, I>;
// compile-time loop: fn(ic<B>{}), fn(ic<B+1>{}), ..., fn(ic<E-1>{})
template <int B, int E, class F>
__host__ __device__ __forceinline__ void static_for(F&& fn) {
  if constexpr (B < E) {
    fn(ic<B>{});
    static_for<B + 1, E>(static_cast<F&&>(fn));
  }
}

}  // namespace
