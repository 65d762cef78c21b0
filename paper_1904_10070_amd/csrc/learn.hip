// learn.hip -- learned correction of a coarsened torus step on MI355X (gfx950): the periodic
// five-layer 3x3 network of include/tlb_learn.h, its training (loss, back-propagation, Adam)
// and the glue between torus grids and the network (restriction, moments and targets, the
// equilibrium-based correction).
//
// Convolutions are implicit GEMMs on the matrix cores, v_mfma_f32_16x16x32_bf16: 16 output
// channels x 16 nodes per instruction, 32-long products (one tap of 32 channels, or four taps
// of 8 channels), bfloat16 operands, FP32 accumulation.
//   forward / input gradient  one wavefront = 16 consecutive nodes of a row x all output
//                             channels; weights are staged once per workgroup in LDS in
//                             fragment order (each lane reads its 16 bytes); the node
//                             operand is one 16-byte load per lane and tap straight from the
//                             channel-last activation tensor, the next tile's in flight
//                             during a tile's products.  The input gradient is the same
//                             kernel with the weights transposed and the taps mirrored.
//   weight gradient           one workgroup = strips of 64 nodes of a row; the error signal
//                             and the nine shifted input tiles are transposed into LDS so that
//                             the contraction over nodes reads 8 consecutive nodes per lane;
//                             the next strip's loads are in flight during a strip's products;
//                             per-workgroup partial sums are added in a fixed order (FP64).
// Grids are sized at network creation from the occupancy of each kernel: one wave of resident
// workgroups where the per-workgroup set-up is large (weight gradient, 32-channel inputs).
// Activations are bfloat16, channel-last [sample][theta][phi][channel].

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "tlb.h"
#include "tlb_internal.h"
#include "tlb_learn.h"

#define LRN_HIP_CHECK(call)                                                             \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return tlbi_fail(TLB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

// ------------------------------------------------------------------------------------------
// the architecture

constexpr int NL = TLB_CNN_LAYERS;
constexpr int WIDTH = TLB_CNN_WIDTH;
constexpr int L_CIN[NL] = {6, 32, 32, 32, 32};   // real input channels
constexpr int L_COUT[NL] = {32, 32, 32, 32, 4};  // real output channels
// storage channels of the tensor each layer reads and of its error signal
constexpr int L_CIS[NL] = {8, 32, 32, 32, 32};
constexpr int L_COS[NL] = {32, 32, 32, 32, 8};

constexpr int layer_params(int l) { return L_COUT[l] * 9 * L_CIN[l] + L_COUT[l]; }
constexpr int layer_offset(int l) { return l == 0 ? 0 : layer_offset(l - 1) + layer_params(l - 1); }
static_assert(layer_offset(NL) == TLB_CNN_PARAMS, "parameter count");

// ------------------------------------------------------------------------------------------
// bfloat16

__device__ __forceinline__ u16 to_bf16(float x) { return __builtin_bit_cast(u16, (__bf16)x); }
__device__ __forceinline__ float from_bf16(u16 b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ bf16x8 zero_frag() {
  bf16x8 z;
#pragma unroll
  for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
  return z;
}

__device__ __forceinline__ int wrap(int i, int n) {
  i = i % n;
  return i < 0 ? i + n : i;
}

// periodic index for i in [-n, 2n): one conditional add or subtract, no division
__device__ __forceinline__ int wrap1(int i, int n) {
  i = i < 0 ? i + n : i;
  return i >= n ? i - n : i;
}

// The eight input features of a node from its raw moments (phi, n, u_theta, u_phi).
struct Features {
  float shift[4], scale[4];
  float r;
  const float* Jrow;  // [n_theta]: R + r cos theta_q
};

__device__ __forceinline__ void features_f(const Features& F, float4 m, int row, float x[8]) {
  x[0] = (m.x - F.shift[0]) * F.scale[0];
  x[1] = (m.y - F.shift[1]) * F.scale[1];
  x[2] = (m.z - F.shift[2]) * F.scale[2];
  x[3] = (m.w - F.shift[3]) * F.scale[3];
  x[4] = F.r;
  x[5] = F.Jrow[row];
  x[6] = 0.0f;
  x[7] = 0.0f;
}

__device__ __forceinline__ bf16x8 features(const Features& F, float4 m, int row) {
  float x[8];
  features_f(F, m, row, x);
  bf16x8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = (__bf16)x[i];
  return v;
}

// the eight bf16 input features of every node of a batch: out[i][p] from the moments of
// sample idx[i] (NULL: i) at node p
struct FeatArgs {
  const float* m;  // float4 moments [*][H][W]
  const int32_t* idx;
  u16* out;        // [n][H][W][8]
  Features F;
  int n, H, W;
};

// one workgroup per row and batch slot: blockIdx.x = slot H + row
__global__ __launch_bounds__(128) void features_kernel(FeatArgs a) {
  const int y = blockIdx.x % a.H, slot = blockIdx.x / a.H;
  const int smp = a.idx ? a.idx[slot] : slot;
  // n H W < 2^28, checked when the network is created
  const float4* src = reinterpret_cast<const float4*>(a.m) + ((size_t)smp * a.H + y) * a.W;
  bf16x8* dst = reinterpret_cast<bf16x8*>(a.out) + ((size_t)slot * a.H + y) * a.W;
  for (int x = threadIdx.x; x < a.W; x += 128) dst[x] = features(a.F, src[x], y);
}

// ------------------------------------------------------------------------------------------
// convolution (forward and input gradient)

enum { IN_BF32 = 0, IN_BF8 = 1 };                  // 32-channel / 8-channel bf16 input
enum { EPI_RELU = 0, EPI_OUT = 1, EPI_MASK = 2 };   // bias+ReLU, bias (FP32 out), ReLU mask

struct ConvArgs {
  const void* in;        // bf16 [n][H][W][32 or 8]
  const bf16x8* w;       // weight fragments [kc][cob][64 lanes]
  const float* bias;     // [c_out] (EPI_RELU, EPI_OUT)
  const u16* mask;       // EPI_MASK: activation whose positive entries pass, [n][H][W][32]
  void* out;             // bf16 [n][H][W][32], or float [n][H][W][4] (EPI_OUT)
  int n, H, W, xt, tiles;  // xt = ceil(W / 16) node groups per row; tiles = n H xt
};

constexpr int CONV_THREADS = 256;
constexpr int CONV_WAVES = CONV_THREADS / 64;

// A tile index t = (n xt + xb) H + y (16 nodes of one row; rows vary fastest) as its
// coordinates; a wavefront walks consecutive tiles, mostly down one column.
struct TileCursor {
  int xb, y, n;
  __device__ __forceinline__ void set(int t, int xt, int H) {
    y = t % H;
    const int rest = t / H;
    xb = rest % xt;
    n = rest / xt;
  }
  __device__ __forceinline__ void next(int xt, int H) {
    if (++y == H) {
      y = 0;
      if (++xb == xt) {
        xb = 0;
        ++n;
      }
    }
  }
};

// The node operand of one tile: for each 32-long chunk c, this lane's 8 products -- tap c
// with channels 8g..8g+7 (32-channel input), or tap 4c+g with all 8 channels (8-channel
// input; taps 9..11 are zero padding).
template <int IN, int KC, int C0 = 0>
__device__ __forceinline__ void load_node_operand(const ConvArgs& a, const TileCursor& tc,
                                                  int px, int g, bf16x8 (&bf)[KC]) {
  const int y = tc.y, n = tc.n;
  const int x = tc.xb * 16 + px;
  // the rows and columns of the three offsets (y and x < W are in range, so one wrap is
  // exact); nodes past the row's end, whose outputs are not stored, read its last node
  int rows[3], cols[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    rows[d] = wrap1(y + d - 1, a.H);
    cols[d] = min(wrap1(x + d - 1, a.W), a.W - 1);
  }
#pragma unroll
  for (int c = C0; c < KC; ++c) {
    const int tap = IN == IN_BF32 ? c : 4 * c + g;
    bf[c] = zero_frag();
    if (tap < 9) {
      const int dy = tap / 3, dx = tap % 3;
      const int yy = dy == 0 ? rows[0] : dy == 1 ? rows[1] : rows[2];
      const int xx = dx == 0 ? cols[0] : dx == 1 ? cols[1] : cols[2];
      // bf16 activations: n H W < 2^28 nodes, checked when the network is created
      const int pix = (n * a.H + yy) * a.W + xx;
      if constexpr (IN == IN_BF32)
        bf[c] = static_cast<const bf16x8*>(a.in)[(size_t)pix * 4 + g];
      else
        bf[c] = static_cast<const bf16x8*>(a.in)[pix];
    }
  }
}

// The ReLU mask of a tile's outputs in this lane: node xb 16 + px (the row's last node for
// lanes past its end, which store nothing), channels 16 b + 4 g .. + 3.
template <int COB>
__device__ __forceinline__ void load_tile_mask(const ConvArgs& a, const TileCursor& tc, int px,
                                               int g, uint2 (&mk)[COB]) {
  const size_t opix = ((size_t)tc.n * a.H + tc.y) * a.W + min(tc.xb * 16 + px, a.W - 1);
#pragma unroll
  for (int b = 0; b < COB; ++b)
    mk[b] = *reinterpret_cast<const uint2*>(a.mask + opix * 32 + 16 * b + 4 * g);
}

template <int IN, int COB, int EPI>
__global__ __launch_bounds__(CONV_THREADS) __attribute__((amdgpu_waves_per_eu(3)))
void conv_kernel(ConvArgs a) {
  constexpr int KC = IN == IN_BF32 ? 9 : 3;  // 32-long product chunks
  __shared__ bf16x8 sw[KC * COB * 64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // tiles are per wave
  const int px = lane & 15, g = lane >> 4;
  // each wavefront takes a contiguous range of tiles
  const int nw = gridDim.x * CONV_WAVES, w = blockIdx.x * CONV_WAVES + wave;
  int t = (int)((long long)w * a.tiles / nw);
  const int t_end = (int)((long long)(w + 1) * a.tiles / nw);
  TileCursor cur;
  cur.set(t, a.xt, a.H);
  // the first tile's node operand is in flight while the weights are staged
  bf16x8 bf[KC];
  uint2 mk[COB], mk2[COB];  // EPI_MASK: the ReLU masks of alternate tiles, loaded with their operands
  if (t < t_end) {
    load_node_operand<IN, KC>(a, cur, px, g, bf);
    if constexpr (EPI == EPI_MASK) load_tile_mask<COB>(a, cur, px, g, mk);
  }
  for (int i = threadIdx.x; i < KC * COB * 64; i += CONV_THREADS) sw[i] = a.w[i];
  // this lane's biases (output channels 16 b + 4 g + i; the output layer's four in lanes
  // g = 0), held in registers: read per tile they would come after the tile's stores, and
  // waiting for them would wait for the next tile's operand loads too
  float bias[COB][4];
#pragma unroll
  for (int b = 0; b < COB; ++b)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      bias[b][i] = EPI == EPI_RELU ? a.bias[16 * b + 4 * g + i] : EPI == EPI_OUT ? a.bias[i] : 0.f;
  __syncthreads();
  // one tile: its products, the next tile's operand and mask (into mnext), its epilogue (with
  // mnow).  The loop alternates the two mask registers, so no copy makes the epilogue wait for
  // the loads just issued.
  auto tile_step = [&](const uint2 (&mnow)[COB], uint2 (&mnext)[COB]) {
    const int y = cur.y, n = cur.n;
    const int x = cur.xb * 16 + px;
    const bool live = x < a.W;
    // lane holds node x, output channels 16 b + 4 g + i
    const size_t opix = ((size_t)n * a.H + y) * a.W + x;
    f32x4 acc[COB];
#pragma unroll
    for (int b = 0; b < COB; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < KC; ++c)
#pragma unroll
      for (int b = 0; b < COB; ++b)
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sw[(c * COB + b) * 64 + lane], bf[c],
                                                         acc[b], 0, 0, 0);
    // the next tile's operand and mask (this tile's again after the last: unused, but
    // loading them unconditionally keeps the epilogue's wait from covering these loads).
    // With 32-channel inputs (chunk c = tap c = 3 dy + dx) the next row's tile of the same
    // column shares taps: its dy = 0, 1 are this tile's dy = 1, 2, and only the new row's
    // three taps are loaded.
    TileCursor next = cur;
    const bool more = t + 1 < t_end;
    if (more) next.next(a.xt, a.H);
    if (IN == IN_BF32 && more && next.y != 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) bf[c] = bf[c + 3];
      load_node_operand<IN, KC, IN == IN_BF32 ? 6 : 0>(a, next, px, g, bf);
    } else {
      load_node_operand<IN, KC>(a, next, px, g, bf);
    }
    if constexpr (EPI == EPI_MASK) load_tile_mask<COB>(a, next, px, g, mnext);
    cur = next;
    if (!live) return;
    if constexpr (EPI == EPI_OUT) {
      if (g == 0) {
        float4 o;
        o.x = acc[0][0] + bias[0][0];
        o.y = acc[0][1] + bias[0][1];
        o.z = acc[0][2] + bias[0][2];
        o.w = acc[0][3] + bias[0][3];
        static_cast<float4*>(a.out)[opix] = o;
      }
    } else {
#pragma unroll
      for (int b = 0; b < COB; ++b) {
        const int co = 16 * b + 4 * g;
        float v[4];
        if constexpr (EPI == EPI_RELU) {
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = fmaxf(acc[b][i] + bias[b][i], 0.0f);
        } else {
          const u16 m4[4] = {(u16)(mnow[b].x & 0xFFFF), (u16)(mnow[b].x >> 16),
                             (u16)(mnow[b].y & 0xFFFF), (u16)(mnow[b].y >> 16)};
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = from_bf16(m4[i]) > 0.0f ? acc[b][i] : 0.0f;
        }
        uint2 st;
        st.x = (unsigned)to_bf16(v[0]) | ((unsigned)to_bf16(v[1]) << 16);
        st.y = (unsigned)to_bf16(v[2]) | ((unsigned)to_bf16(v[3]) << 16);
        *reinterpret_cast<uint2*>(static_cast<u16*>(a.out) + opix * 32 + co) = st;
      }
    }
  };
  while (t < t_end) {
    tile_step(mk, mk2);
    if (++t >= t_end) break;
    tile_step(mk2, mk);
    ++t;
  }
}

// ------------------------------------------------------------------------------------------
// weight gradient: dW[o][t][i] = sum over nodes of e[node][o] a[node + offset(t)][i]

constexpr int WG_PITCH = 72;  // LDS row pitch (bf16): 64 nodes + 8 keeps rows 16-byte aligned
// bf16 index of node j of row r
__device__ __forceinline__ int wg_at(int r, int j) { return r * WG_PITCH + j; }
constexpr int WG_THREADS = 256;

struct WgradArgs {
  const u16* e;        // error signal bf16 [n][H][W][COS]
  const u16* a;        // layer input bf16 [n][H][W][CIS]
  float* partial;      // [gridDim.x][COS * 9 * CIS + COS]
  int n, H, W, xs, strips;  // xs = ceil(W / 64) strips per row; strips = n H xs
};

// A strip s = (n xs + xb) H + y (64 nodes of one row; rows vary fastest) as its
// coordinates; the strips of a workgroup are consecutive, so the next one is one carry away,
// and mostly the next row of the same column.
struct StripPos {
  int xb, y, n;
  __device__ __forceinline__ void set(int s, int xs, int H) {
    y = s % H;
    const int rest = s / H;
    xb = rest % xs;
    n = rest / xs;
  }
  __device__ __forceinline__ void next(int xs, int H) {
    if (++y == H) {
      y = 0;
      if (++xb == xs) {
        xb = 0;
        ++n;
      }
    }
  }
};

// The input tiles in LDS form a window of three rows: tap (dy, dx) of the strip in row y
// (input row y + dy - 1, nodes shifted by dx - 1) sits in tile 3 slot + dx with slot =
// (y + dy + 2) mod 3.  The next row's strip of the same column shares two of the rows, so
// it stages only the new one (its three taps dy = 2); a strip that starts a column stages
// all nine taps.
__device__ __forceinline__ int wg_tile(int y, int t) { return ((y + t / 3 + 2) % 3) * 3 + t % 3; }

// The global loads of one strip, all issued before any is used: the error tile (thread u <
// (COS/8) 64 takes node u % 64, channels 8 (u / 64) .. + 7) and the input taps to stage, by
// pairs of neighbouring nodes (unit u: nodes 2 (u % 32) and +1, channels 8 c8 .. + 7 with
// c8 = (u / 32) % (CIS / 8), tap T0 + (u / 32) / (CIS / 8), so that each LDS store of the
// transposed tile writes two consecutive nodes); the error is zero beyond the row's end.
// With CIS / 8 even, the 64 units of a wavefront share their tap: the taps are then found
// once per thread, from the wavefront index, and are scalars.  The partial last round of
// units goes to the highest threads: the products give the lowest wavefronts the extra
// (tap, input block) pair, so the SIMDs even out.
template <int CIS, int NTAP, int T0>
struct WgradUnits {
  static constexpr int NA = NTAP * (CIS / 8) * 32;
  static constexpr int KA = (NA + WG_THREADS - 1) / WG_THREADS;
  static constexpr int REM = NA - (KA - 1) * WG_THREADS;
  static constexpr bool UNIFORM = (CIS / 8) % 2 == 0;
  int tap[KA];  // UNIFORM: tap of unit k, 9 where the thread has no unit k

  // first unit of round k (units base .. base + WG_THREADS - 1 by thread)
  __device__ __forceinline__ static int base_of(int k) {
    return k < KA - 1 ? k * WG_THREADS : k * WG_THREADS - (WG_THREADS - REM);
  }
  __device__ __forceinline__ static int unit_of(int k) {
    return (k < KA - 1 || (int)threadIdx.x >= WG_THREADS - REM) ? base_of(k) + (int)threadIdx.x
                                                                : -1;
  }
  __device__ __forceinline__ void init(int wave) {
    if constexpr (UNIFORM) {
#pragma unroll
      for (int k = 0; k < KA; ++k) {
        // (u / 32) / (CIS / 8) with u / 32 = base / 32 + 2 wave + lane / 32, base / 32 even:
        // the lane's bit drops
        const bool has = k < KA - 1 || 64 * wave >= WG_THREADS - REM;
        tap[k] = has ? T0 + ((base_of(k) >> 6) + wave) / (CIS / 16) : 9;
      }
    }
  }
  __device__ __forceinline__ int tap_of(int k) const {
    if constexpr (UNIFORM) return tap[k];
    const int u = unit_of(k);
    return u >= 0 ? T0 + (u >> 5) / (CIS / 8) : 9;
  }
};

template <int CIS, int COS>
struct WgradStrip {
  static constexpr int NE = (COS / 8) * 64;
  using Full = WgradUnits<CIS, 9, 0>;  // a strip that starts a column: all nine taps
  using Row = WgradUnits<CIS, 3, 6>;   // the next row's strip: the new row's three taps
  static constexpr int KA = Full::KA;
  // every round starts at a multiple of 32 (CIS / 8) units, so a thread's node pair and
  // channel group are the same in both modes; only the taps differ
  static_assert(Full::REM % (32 * (CIS / 8)) == 0 && Row::REM % (32 * (CIS / 8)) == 0,
                "round bases");
  uint4 e;
  uint4 av[KA][2];  // bf16 inputs of the two nodes
  Full full;
  Row row;

  __device__ __forceinline__ void init(int wave) {
    full.init(wave);
    row.init(wave);
  }
  // tap of this thread's unit in round k (9: none) when staging all taps or the new row's
  __device__ __forceinline__ int tap_of(int k, bool all) const {
    const int tr = k < Row::KA ? row.tap_of(k) : 9;
    return all ? full.tap_of(k) : tr;
  }

  __device__ __forceinline__ void load(const WgradArgs& a, const StripPos& p, bool all) {
    const int y = p.y, n = p.n;
    const int x0 = p.xb * 64;
    const int jp = threadIdx.x & 31, c8 = (threadIdx.x >> 5) % (CIS / 8);
    e = make_uint4(0, 0, 0, 0);
    // bf16 tensors: n H W < 2^28 nodes, checked when the network is created; each load takes
    // its row's start (uniform) and a 32-bit byte offset within the row
    if (threadIdx.x < NE) {
      const int j = threadIdx.x & 63, c8e = threadIdx.x >> 6;
      const char* erow =
          reinterpret_cast<const char*>(a.e) + (size_t)((n * a.H + y) * a.W) * COS * 2;
      if (x0 + j < a.W)
        e = *reinterpret_cast<const uint4*>(erow + (unsigned)(((x0 + j) * COS + 8 * c8e) * 2));
    }
#pragma unroll
    for (int k = 0; k < KA; ++k) {
      const int t = tap_of(k, all);
      if (t < 9) {
        const int yy = wrap1(y + t / 3 - 1, a.H);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          // one wrap is exact for the row's nodes (x0 + 2 jp + h < W); those past its end,
          // whose error is zero, read the row's last node
          const int xx = min(wrap1(x0 + 2 * jp + h + t % 3 - 1, a.W), a.W - 1);
          const char* arow =
              reinterpret_cast<const char*>(a.a) + (size_t)((n * a.H + yy) * a.W) * CIS * 2;
          av[k][h] = *reinterpret_cast<const uint4*>(arow + (unsigned)((xx * CIS + 8 * c8) * 2));
        }
      }
    }
  }

  // transposed into LDS: sE[o][j] = e[n][y][x0 + j][o]; tile wg_tile(y, t) of sA [i][j] =
  // a[n][y + dy - 1][x0 + j + dx - 1][i]; bsum[i] accumulates this thread's error values
  // (channel 8 (tid / 64) + i)
  __device__ __forceinline__ void store(const WgradArgs& a, const StripPos& p, bool all, u16* sE,
                                        u16* sA, float (&bsum)[8]) const {
    if (threadIdx.x < NE) {
      const int j = threadIdx.x & 63, c8e = threadIdx.x >> 6;
      const unsigned w4[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const u16 v = (u16)((w4[i >> 1] >> (16 * (i & 1))) & 0xFFFF);
        sE[wg_at(8 * c8e + i, j)] = v;
        bsum[i] += from_bf16(v);
      }
    }
    const int jp = threadIdx.x & 31, c8 = (threadIdx.x >> 5) % (CIS / 8);
#pragma unroll
    for (int k = 0; k < KA; ++k) {
      const int t = tap_of(k, all);
      if (t < 9) {
        // the two nodes' channels 8 c8 .. + 7, two bf16 per word
        const unsigned w[2][4] = {{av[k][0].x, av[k][0].y, av[k][0].z, av[k][0].w},
                                  {av[k][1].x, av[k][1].y, av[k][1].z, av[k][1].w}};
        // channel 2 i: the low halves of the two nodes' word i; channel 2 i + 1: the high
        // halves (byte selectors 0-3 take the second operand's bytes, 4-7 the first's)
        const int tile = wg_tile(p.y, t);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // rows 2 i and 2 i + 1 of the group share their chunk order
          unsigned* r =
              reinterpret_cast<unsigned*>(sA + wg_at(tile * CIS + 8 * c8 + 2 * i, 2 * jp));
          r[0] = __builtin_amdgcn_perm(w[1][i], w[0][i], 0x05040100u);
          r[WG_PITCH / 2] = __builtin_amdgcn_perm(w[1][i], w[0][i], 0x07060302u);
        }
      }
    }
  }
};

template <int CIS, int COS>
__global__ __launch_bounds__(WG_THREADS) void wgrad_kernel(WgradArgs a) {
  constexpr int CIB = (CIS + 15) / 16, COB = (COS + 15) / 16;
  // 16 x 16 output fragments (tap t, output block bc, input block bi); a wavefront takes
  // whole (t, bi) pairs, so that each node operand it reads from LDS serves every bc
  constexpr int NP = 9 * CIB;            // (tap, input block) pairs
  constexpr int PPW = (NP + 3) / 4;      // pairs per wavefront
  using Strip = WgradStrip<CIS, COS>;
  __shared__ __attribute__((aligned(16))) u16 sE[COS * WG_PITCH];
  __shared__ __attribute__((aligned(16))) u16 sA[9 * CIS * WG_PITCH];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) & 3;
  const int px = lane & 15, g = lane >> 4;
  f32x4 acc[PPW][COB];
#pragma unroll
  for (int k = 0; k < PPW; ++k)
#pragma unroll
    for (int bc = 0; bc < COB; ++bc) acc[k][bc] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int s0 = (int)((long long)blockIdx.x * a.strips / gridDim.x);
  const int s1 = (int)((long long)(blockIdx.x + 1) * a.strips / gridDim.x);
  auto products = [&](int y) {
    bf16x8 A[COB][2];  // the error operand of every output block, both halves of the strip
#pragma unroll
    for (int bc = 0; bc < COB; ++bc)
#pragma unroll
      for (int kc = 0; kc < 2; ++kc)
        A[bc][kc] = 16 * bc + px < COS ? *reinterpret_cast<const bf16x8*>(
                                             &sE[wg_at(16 * bc + px, 32 * kc + 8 * g)])
                                       : zero_frag();
#pragma unroll
    for (int k = 0; k < PPW; ++k) {
      const int pr = wave + 4 * k;
      if (pr < NP) {
        const int t = pr / CIB, bi = pr % CIB;
        const int ci = 16 * bi + px;
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
          const bf16x8 B = ci < CIS ? *reinterpret_cast<const bf16x8*>(
                                          &sA[wg_at(wg_tile(y, t) * CIS + ci, 32 * kc + 8 * g)])
                                    : zero_frag();
#pragma unroll
          for (int bc = 0; bc < COB; ++bc)
            acc[k][bc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[bc][kc], B, acc[k][bc], 0, 0, 0);
        }
      }
    }
  };
  Strip st;
  st.init(wave);
  StripPos pos, nxt;
  pos.set(s0, a.xs, a.H);
  bool all = true;  // the strip stages all nine taps (the workgroup's first, or a new column)
  if (s0 < s1) st.load(a, pos, all);
  for (int s = s0; s < s1; ++s) {
    st.store(a, pos, all, sE, sA, bsum);
    // the next strip's loads are in flight during this strip's products
    nxt = pos;
    nxt.next(a.xs, a.H);
    const bool nall = nxt.y == 0;
    if (s + 1 < s1) st.load(a, nxt, nall);
    __syncthreads();
    products(pos.y);
    __syncthreads();
    pos = nxt;
    all = nall;
  }
  float* out = a.partial + (size_t)blockIdx.x * (COS * 9 * CIS + COS);
#pragma unroll
  for (int k = 0; k < PPW; ++k) {
    const int pr = wave + 4 * k;
    if (pr < NP) {
      const int t = pr / CIB, bi = pr % CIB;
      const int ci = 16 * bi + px;
#pragma unroll
      for (int bc = 0; bc < COB; ++bc)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int co = 16 * bc + 4 * g + i;
          if (co < COS && ci < CIS) out[(co * 9 + t) * CIS + ci] = acc[k][bc][i];
        }
    }
  }
  // bias gradient: the error values of channel 8 w + i sit in wave w's lanes (one node each)
  if (threadIdx.x < Strip::NE) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) bsum[i] += __shfl_xor(bsum[i], d, 64);
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < 8; ++i) out[COS * 9 * CIS + 8 * wave + i] = bsum[i];
  }
}

// per-workgroup partial sums -> gradient of one layer's weights, fixed order, FP64 sums
struct GradArgs {
  const float* partial;
  float* grad;  // the layer's slice of the flat gradient
  int blocks, cis, cos_s, cin, cout;
  double scale;
};

// 64 parameters per block; each of the GR_WAVES wavefronts sums every GR_WAVES-th partial
// block of them, and their sums are added in a fixed order
constexpr int GR_PARAMS = 64;
constexpr int GR_WAVES = 16;

__global__ __launch_bounds__(64 * GR_WAVES) void grad_reduce_kernel(GradArgs a) {
  __shared__ double part[GR_WAVES][GR_PARAMS];
  const int lane = threadIdx.x & 63, quarter = threadIdx.x >> 6;
  const int p = blockIdx.x * GR_PARAMS + lane;
  const int nw = a.cout * 9 * a.cin;
  const bool valid = p < nw + a.cout;
  int src = 0;
  if (valid) {
    if (p < nw) {
      const int co = p / (9 * a.cin), rem = p % (9 * a.cin);
      src = (co * 9 + rem / a.cin) * a.cis + rem % a.cin;
    } else {
      src = a.cos_s * 9 * a.cis + (p - nw);
    }
  }
  const size_t stride = (size_t)a.cos_s * 9 * a.cis + a.cos_s;
  double s = 0.0;
  if (valid) {
#pragma unroll 16
    for (int b = quarter; b < a.blocks; b += GR_WAVES) s += (double)a.partial[b * stride + src];
  }
  part[quarter][lane] = s;
  __syncthreads();
  if (quarter == 0 && valid) {
    double t = 0.0;
    for (int q = 0; q < GR_WAVES; ++q) t += part[q][lane];
    a.grad[p] = (float)(t * a.scale);
  }
}

// ------------------------------------------------------------------------------------------
// loss and the last layer's error signal

constexpr int RED = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
  return t;
}

struct LossArgs {
  const float* z;        // [n][HW][4]
  const float* y;        // targets [*][HW][4]
  const int32_t* idx;
  u16* e;                // [n][HW][8]
  double* partial;       // [gridDim.x]
  long long hw, total;   // nodes per sample, n * hw
  float inv_scale[4], w[4];
};

__global__ __launch_bounds__(RED) void loss_kernel(LossArgs a) {
  __shared__ double sh[RED / 64];
  const long long i = (long long)blockIdx.x * RED + threadIdx.x;
  double l = 0.0;
  if (i < a.total) {
    const long long n = i / a.hw, p = i - n * a.hw;
    const long long smp = a.idx ? a.idx[n] : n;
    const float4 z = reinterpret_cast<const float4*>(a.z)[i];
    const float4 y = reinterpret_cast<const float4*>(a.y)[smp * a.hw + p];
    const float d[4] = {z.x - y.x * a.inv_scale[0], z.y - y.y * a.inv_scale[1],
                        z.z - y.z * a.inv_scale[2], z.w - y.w * a.inv_scale[3]};
    u16 e[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      e[c] = to_bf16(a.w[c] * d[c]);
      l += (double)a.w[c] * (double)d[c] * (double)d[c];
    }
    uint4 st;
    st.x = (unsigned)e[0] | ((unsigned)e[1] << 16);
    st.y = (unsigned)e[2] | ((unsigned)e[3] << 16);
    st.z = 0;
    st.w = 0;
    reinterpret_cast<uint4*>(a.e)[i] = st;
  }
  const double t = block_sum(l, sh);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = t;
}

struct SumArgs {
  const double* partial;
  double* out;
  int blocks, width;  // out[c] = sum_b partial[b * width + c] * scale
  double scale;
};

__global__ __launch_bounds__(RED) void sum_partials_kernel(SumArgs a) {
  __shared__ double sh[RED / 64];
  for (int c = 0; c < a.width; ++c) {
    double s = 0.0;
    for (int b = threadIdx.x; b < a.blocks; b += RED) s += a.partial[(size_t)b * a.width + c];
    const double t = block_sum(s, sh);
    if (threadIdx.x == 0) a.out[c] = t * a.scale;
  }
}

// network output times the output scale
struct ScaleArgs {
  const float* z;
  float* out;
  long long count;  // nodes
  float s[4];
};

__global__ __launch_bounds__(256) void scale_kernel(ScaleArgs a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.count) return;
  const float4 z = reinterpret_cast<const float4*>(a.z)[i];
  reinterpret_cast<float4*>(a.out)[i] = make_float4(z.x * a.s[0], z.y * a.s[1], z.z * a.s[2], z.w * a.s[3]);
}

// ------------------------------------------------------------------------------------------
// Adam and the bf16 weight fragments

struct AdamArgs {
  float* p;
  const float* g;
  float* m;
  float* v;
  int count;
  float lr, b1, b2, eps, c1, c2;  // c = 1 - beta^step
};

__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.count) return;
  const float g = a.g[i];
  const float m = a.b1 * a.m[i] + (1.0f - a.b1) * g;
  const float v = a.b2 * a.v[i] + (1.0f - a.b2) * g * g;
  a.m[i] = m;
  a.v[i] = v;
  a.p[i] -= a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
}

// Fragment order of a weight operand: slot ((c * cob + b) * 64 + lane) * 8 + i holds the
// weight of GEMM row 16 b + lane % 16 and product index k = 32 c + 8 (lane / 16) + i, where
// k is (tap c, channel k % 32) for 32-channel operands and (tap 4c + lane/16, channel i) for
// 8-channel ones.  Forward: rows are output channels, W[row][tap][ch].  Input gradient: rows
// are input channels, taps mirrored, W[ch][8 - tap][row].
struct FragArgs {
  const float* W;  // the layer's W[c_out][9][c_in]
  u16* out;
  int slots, cob, wide, transpose, cin, cout;
};
// every layer's forward and input-gradient fragments in one launch: job blockIdx.y
struct FragJobs {
  FragArgs job[2 * NL - 1];
};

__global__ __launch_bounds__(256) void frag_kernel(FragJobs jobs) {
  const FragArgs& a = jobs.job[blockIdx.y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.slots) return;
  const int i = s & 7, lane = (s >> 3) & 63;
  const int b = (s >> 9) % a.cob, c = (s >> 9) / a.cob;
  const int row = 16 * b + (lane & 15), g = lane >> 4;
  const int tap = a.wide ? c : 4 * c + g;
  const int ch = a.wide ? 8 * g + i : i;
  float v = 0.0f;
  if (tap < 9) {
    if (!a.transpose) {
      if (row < a.cout && ch < a.cin) v = a.W[(row * 9 + tap) * a.cin + ch];
    } else {
      if (row < a.cin && ch < a.cout) v = a.W[(ch * 9 + (8 - tap)) * a.cin + row];
    }
  }
  a.out[s] = to_bf16(v);
}

// ------------------------------------------------------------------------------------------
// torus grid <-> network

// A grid's order parameter: FP32 grids store it as base + deviation (phi plane = deviation),
// FP64 grids whole (base NULL).
template <typename T>
__device__ __forceinline__ double order_parameter(const T* phi, const T* base, long long x) {
  return base ? (double)phi[x] + (double)base[x] : (double)phi[x];
}

template <typename T>
struct MomArgs {
  const T* f;
  const T* phi;
  const T* phib;   // base of phi (FP32) or NULL
  const T* f2;     // truth grid (NULL: moments only)
  const T* phi2;
  const T* phib2;
  float* m;        // [HW][4]
  float* y;        // [HW][4]
  long long plane;
  double n_add, n_add2;  // what a node's population sum lacks of its density, per grid
};

template <typename T>
__device__ __forceinline__ void node_moments(const T* f, const T* phi, const T* phib,
                                             long long plane, long long x, double n_add,
                                             double out[4]) {
  double n = 0.0, nut = 0.0, nup = 0.0;
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const double fk = (double)f[k * plane + x];
    n += fk;
    nut += vel(k >> 2) * fk;
    nup += vel(k & 3) * fk;
  });
  n += n_add;  // FP32 grids store f - n_ref w_i w_j
  out[0] = order_parameter(phi, phib, x);
  out[1] = n;
  out[2] = nut / n;
  out[3] = nup / n;
}

// node_moments on values already loaded: f[16], phi and (FP32) its base
template <typename T>
__device__ __forceinline__ void moments_of(const T (&f)[16], T phi, const T* phib, double n_add,
                                           double out[4]) {
  double n = 0.0, nut = 0.0, nup = 0.0;
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const double fk = (double)f[k];
    n += fk;
    nut += vel(k >> 2) * fk;
    nup += vel(k & 3) * fk;
  });
  n += n_add;
  out[0] = phib ? (double)phi + (double)*phib : (double)phi;
  out[1] = n;
  out[2] = nut / n;
  out[3] = nup / n;
}

template <typename T>
__global__ __launch_bounds__(256) void moments_pair_kernel(MomArgs<T> a) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.plane) return;
  double m[4];
  node_moments(a.f, a.phi, a.phib, a.plane, x, a.n_add, m);
  reinterpret_cast<float4*>(a.m)[x] = make_float4((float)m[0], (float)m[1], (float)m[2], (float)m[3]);
  if (a.f2) {
    double t[4];
    node_moments(a.f2, a.phi2, a.phib2, a.plane, x, a.n_add2, t);
    reinterpret_cast<float4*>(a.y)[x] = make_float4((float)(t[0] - m[0]), (float)(t[1] - m[1]),
                                                    (float)(t[2] - m[2]), (float)(t[3] - m[3]));
  }
}

// area-weighted sums of the phi and n corrections, one block per theta row
struct ProjArgs {
  const float* d;       // corrections [HW][4] (times scale)
  const double* area;   // [H]
  double* partial;      // [H][3]: sum a dphi, sum a dn, sum a
  int W;
  float scale0, scale1;
};

__global__ __launch_bounds__(RED) void proj_kernel(ProjArgs a) {
  __shared__ double sh[RED / 64];
  const int q = blockIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int s = threadIdx.x; s < a.W; s += RED) {
    const float4 d = reinterpret_cast<const float4*>(a.d)[(size_t)q * a.W + s];
    s0 += (double)(d.x * a.scale0);
    s1 += (double)(d.y * a.scale1);
  }
  const double ar = a.area[q];
  const double t0 = block_sum(s0, sh);
  const double t1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    a.partial[3 * q + 0] = ar * t0;
    a.partial[3 * q + 1] = ar * t1;
    a.partial[3 * q + 2] = ar * a.W;
  }
}

template <typename T>
struct ApplyArgs {
  T* f;
  T* phi;
  T* phib;                  // FP32 grids in the learned step: fold phi into this base after
                            // the correction (exact two-sum); NULL: phi itself is corrected
  const float* d;           // corrections [HW][4], times scale
  const double* partial;    // [nparts][3]: sum a dphi, sum a dn, sum a
  int nparts;
  long long plane;
  float scale[4];
  T n_ref;  // reference density of the stored deviations (FP32)
};

template <typename T>
__device__ __forceinline__ T feq_k(int i, int j, T n, T ut, T up) {
  const T c0 = T(1) - T(0.5) * (ut * ut + up * up);
  const T xi = T(vel(i)) * ut + T(vel(j)) * up;
  return (n * T(wgt(i) * wgt(j))) * (c0 + xi * (c0 + xi * (T(0.5) + xi * T(1.0 / 6.0))));
}

template <typename T>
__global__ __launch_bounds__(256) void apply_kernel(ApplyArgs<T> a) {
  __shared__ double mean[2];
  // the node's state and correction are loaded first, so that their latency overlaps the sum
  // of the partial sums below
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool node = x < a.plane;
  float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
  T fk[16];
  T ph = T(0), bb = T(0);
  if (node) {
    d = reinterpret_cast<const float4*>(a.d)[x];
    static_for<0, 16>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      fk[k] = a.f[k * a.plane + x];
    });
    ph = a.phi[x];
    if (a.phib) bb = a.phib[x];
  }
  if (threadIdx.x < 64) {
    double s0 = 0.0, s1 = 0.0, ar = 0.0;
    for (int q = threadIdx.x; q < a.nparts; q += 64) {
      s0 += a.partial[3 * q + 0];
      s1 += a.partial[3 * q + 1];
      ar += a.partial[3 * q + 2];
    }
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) {
      s0 += __shfl_xor(s0, dd, 64);
      s1 += __shfl_xor(s1, dd, 64);
      ar += __shfl_xor(ar, dd, 64);
    }
    if (threadIdx.x == 0) {
      mean[0] = s0 / ar;
      mean[1] = s1 / ar;
    }
  }
  __syncthreads();
  if (!node) return;
  const T dphi = T((double)(d.x * a.scale[0]) - mean[0]);
  const T dn = T((double)(d.y * a.scale[1]) - mean[1]);
  const T dut = T(d.z * a.scale[2]), dup = T(d.w * a.scale[3]);
  T n = T(0), nut = T(0), nup = T(0);
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    n += fk[k];
    nut += T(vel(k >> 2)) * fk[k];
    nup += T(vel(k & 3)) * fk[k];
  });
  if constexpr (stores_deviation<T>()) n += a.n_ref;  // the stored values are f - n_ref w_i w_j
  const T ut = nut / n, up = nup / n;
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    a.f[k * a.plane + x] =
        fk[k] + (feq_k<T>(k >> 2, k & 3, n + dn, ut + dut, up + dup) - feq_k<T>(k >> 2, k & 3, n, ut, up));
  });
  const T dev = ph + dphi;
  if (a.phib) {  // base + dev = sum + err exactly (two-sum); the base takes the sum
    const T sum = bb + dev;
    const T bv = sum - dev;
    const T dv = sum - bv;
    a.phib[x] = sum;
    a.phi[x] = (bb - bv) + (dev - dv);
  } else {
    a.phi[x] = dev;
  }
}

// ------------------------------------------------------------------------------------------
// the network of a learned step in one launch
//
// One workgroup per output tile of NT_H x NT_W nodes.  It forms the moments and input features
// of the tile and of a five-node halo around it (the reach of five 3x3 layers) straight from
// the grid's state, then runs the five layers through LDS: layer l produces the tile plus a
// halo of 4 - l nodes, reading only what the layer before it wrote.  Halo nodes are computed by
// every tile that needs them (about twice the matrix work of the layer-by-layer kernels); in
// exchange the step's network is one launch instead of six and its activations never reach
// HBM.  Products, their order and every bfloat16 rounding are those of conv_kernel (and the
// moments those of moments_pair_kernel), so the output is the same bit for bit.

constexpr int NT_H = 8, NT_W = 24;   // output tile
constexpr int NT_G = 2;              // 16-node groups per layer row
constexpr int NT_PW = 16 * NT_G + 2; // row pitch of the LDS planes in nodes: the groups + 2 read
#ifndef TLB_NT_THREADS  // 1024 threads (two units per wave and layer) measured 2 % slower
#define TLB_NT_THREADS 512
#endif
constexpr int NT_THREADS = TLB_NT_THREADS;
constexpr int NT_WAVES = NT_THREADS / 64;
static_assert(NT_W + 8 <= 16 * NT_G, "layer 0 row of the tile and its halo in NT_G groups");
static_assert(NT_W + 10 <= NT_PW, "feature row of the tile and its halo");
// fragment offsets of the layers in the staged weights (bf16x8 units)
constexpr int nt_frags(int l) { return (L_CIS[l] == 32 ? 9 : 3) * ((L_COUT[l] + 15) / 16) * 64; }
constexpr int nt_frag_offset(int l) { return l == 0 ? 0 : nt_frag_offset(l - 1) + nt_frags(l - 1); }
constexpr int NT_FRAGS = nt_frag_offset(NL);

template <typename T>
struct NetArgs {
  const T* f;
  const T* phi;
  const T* phib;   // base of phi (FP32) or NULL
  long long plane;
  double n_add;    // what a node's population sum lacks of its density
  const bf16x8* w[NL];  // forward weight fragments of each layer
  const float* bias[NL];
  Features F;
  int H, W, tiles_x;
  float* out;      // [H][W][4]: network output
  double* proj;    // [block][3]: sum a z0 s0, sum a z1 s1, sum a over the tile
  const double* area;
  float s0, s1;
};

// One layer over the tile: rows `rows` of 16 NT_G-node groups, input plane `in` (features,
// 8 channels, when IN8; else 32-channel activations), output plane `out` (32 channels) or,
// for the last layer, the network output in HBM.
template <bool IN8, int COB, bool LAST, typename T>
__device__ __forceinline__ void nt_layer(const NetArgs<T>& a, const bf16x8* sw, const void* in,
                                         u16* out, int l, int rows, int y0, int x0,
                                         double (&ps)[3]) {
  constexpr int KC = IN8 ? 3 : 9;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = lane & 15, g = lane >> 4;
  bf16x8 wa[KC][COB];
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int b = 0; b < COB; ++b) wa[c][b] = sw[(c * COB + b) * 64 + lane];
  const float* bias = a.bias[l];
  for (int u = wave; u < rows * NT_G; u += NT_WAVES) {
    const int i = u / NT_G, col = (u % NT_G) * 16 + px;
    bf16x8 bf[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const int tap = IN8 ? 4 * c + g : c;
      if (tap < 9) {
        const int node = (i + tap / 3) * NT_PW + col + tap % 3;
        bf[c] = IN8 ? static_cast<const bf16x8*>(in)[node]
                    : static_cast<const bf16x8*>(in)[node * 4 + g];
      } else {
        bf[c] = zero_frag();
      }
    }
    f32x4 acc[COB];
#pragma unroll
    for (int b = 0; b < COB; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < KC; ++c)
#pragma unroll
      for (int b = 0; b < COB; ++b)
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[c][b], bf[c], acc[b], 0, 0, 0);
    // lane holds node col of row i, output channels 16 b + 4 g + k
    if constexpr (LAST) {
      const int y = y0 + i, x = x0 + col;
      if (g == 0 && col < NT_W && y < a.H && x < a.W) {
        float4 o;
        o.x = acc[0][0] + bias[0];
        o.y = acc[0][1] + bias[1];
        o.z = acc[0][2] + bias[2];
        o.w = acc[0][3] + bias[3];
        reinterpret_cast<float4*>(a.out)[(size_t)y * a.W + x] = o;
        if (a.proj) {
          const double ar = a.area[y];
          ps[0] += ar * (double)(o.x * a.s0);
          ps[1] += ar * (double)(o.y * a.s1);
          ps[2] += ar;
        }
      }
    } else {
#pragma unroll
      for (int b = 0; b < COB; ++b) {
        const int co = 16 * b + 4 * g;
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = fmaxf(acc[b][k] + bias[co + k], 0.0f);
        uint2 st;
        st.x = (unsigned)to_bf16(v[0]) | ((unsigned)to_bf16(v[1]) << 16);
        st.y = (unsigned)to_bf16(v[2]) | ((unsigned)to_bf16(v[3]) << 16);
        *reinterpret_cast<uint2*>(out + (size_t)(i * NT_PW + col) * 32 + co) = st;
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT_THREADS) void net_step_kernel(NetArgs<T> a) {
  __shared__ bf16x8 sw[NT_FRAGS];                      // every layer's weight fragments
  __shared__ bf16x8 sf[(NT_H + 10) * NT_PW];           // input features, tile + 5 halo
  __shared__ __attribute__((aligned(16))) u16 sa[(NT_H + 8) * NT_PW * 32];  // layers 0, 2
  __shared__ __attribute__((aligned(16))) u16 sb[(NT_H + 6) * NT_PW * 32];  // layers 1, 3
  const int ty = blockIdx.x / a.tiles_x, tx = blockIdx.x % a.tiles_x;
  const int y0 = ty * NT_H, x0 = tx * NT_W;
  // Every global load of the prologue is issued before any of them is used: the weight
  // fragments (WK per thread) and the populations of the feature nodes (FK nodes per thread).
  constexpr int WK = (NT_FRAGS + NT_THREADS - 1) / NT_THREADS;
  constexpr int NFEAT = (NT_H + 10) * NT_PW;
  constexpr int FK = (NFEAT + NT_THREADS - 1) / NT_THREADS;
  bf16x8 wv[WK];
#pragma unroll
  for (int k = 0; k < WK; ++k) {
    const int gi = threadIdx.x + k * NT_THREADS;
    const bf16x8* src = a.w[0];
    int off = 0;
#pragma unroll
    for (int m = 1; m < NL; ++m)
      if (gi >= nt_frag_offset(m)) {
        src = a.w[m];
        off = nt_frag_offset(m);
      }
    if (gi < NT_FRAGS) wv[k] = src[gi - off];
  }
  // features of rows y0 - 5 .. y0 + NT_H + 4, columns x0 - 5 .. x0 + NT_W + 4 (periodic)
  T fv[FK][16];
  T pv[FK], pb[FK];
#pragma unroll
  for (int k = 0; k < FK; ++k) {
    const int i = threadIdx.x + k * NT_THREADS;
    if (i < NFEAT) {
      const int fr = i / NT_PW, fc = i % NT_PW;
      const long long x = (long long)wrap(y0 - 5 + fr, a.H) * a.W + wrap(x0 - 5 + fc, a.W);
#pragma unroll
      for (int c = 0; c < 16; ++c) fv[k][c] = a.f[c * a.plane + x];
      pv[k] = a.phi[x];
      pb[k] = a.phib ? a.phib[x] : T(0);
    }
  }
#pragma unroll
  for (int k = 0; k < WK; ++k) {
    const int gi = threadIdx.x + k * NT_THREADS;
    if (gi < NT_FRAGS) sw[gi] = wv[k];
  }
#pragma unroll
  for (int k = 0; k < FK; ++k) {
    const int i = threadIdx.x + k * NT_THREADS;
    if (i < NFEAT) {
      const int y = wrap(y0 - 5 + i / NT_PW, a.H);
      double m[4];
      moments_of(fv[k], pv[k], a.phib ? &pb[k] : nullptr, a.n_add, m);
      sf[i] = features(a.F, make_float4((float)m[0], (float)m[1], (float)m[2], (float)m[3]), y);
    }
  }
  __syncthreads();
  double ps[3] = {0.0, 0.0, 0.0};
  nt_layer<true, 2, false>(a, sw + nt_frag_offset(0), sf, sa, 0, NT_H + 8, y0, x0, ps);
  __syncthreads();
  nt_layer<false, 2, false>(a, sw + nt_frag_offset(1), sa, sb, 1, NT_H + 6, y0, x0, ps);
  __syncthreads();
  nt_layer<false, 2, false>(a, sw + nt_frag_offset(2), sb, sa, 2, NT_H + 4, y0, x0, ps);
  __syncthreads();
  nt_layer<false, 2, false>(a, sw + nt_frag_offset(3), sa, sb, 3, NT_H + 2, y0, x0, ps);
  __syncthreads();
  nt_layer<false, 1, true>(a, sw + nt_frag_offset(4), sb, nullptr, 4, NT_H, y0, x0, ps);
  if (a.proj) {  // uniform: every thread takes part in the fixed-order block sums
    __shared__ double sh[NT_WAVES][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
      for (int k = 0; k < 3; ++k) ps[k] += __shfl_xor(ps[k], d, 64);
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < 3; ++k) sh[wave][k] = ps[k];
    __syncthreads();
    if (threadIdx.x < 3) {
      double v = 0.0;
      for (int w = 0; w < NT_WAVES; ++w) v += sh[w][threadIdx.x];
      a.proj[3 * blockIdx.x + threadIdx.x] = v;
    }
  }
}

// full-weighting restriction by an even factor k, J-weighted along theta
template <typename T>
struct RestrictArgs {
  const T* f;
  const T* phi;
  const T* phib;  // fine base of phi (FP32) or NULL
  T* fc;
  T* phic;
  T* phibc;       // coarse base of phi (FP32: the restriction goes there, phic becomes 0)
  const double* area;  // fine rows, proportional to J
  int Hf, Wf, Hc, Wc, k;
  long long plane_f, plane_c;
};

template <typename T>
__global__ __launch_bounds__(256) void restrict_kernel(RestrictArgs<T> a) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.plane_c) return;
  const int Q = (int)(x / a.Wc), S = (int)(x - (long long)Q * a.Wc);
  const int h = a.k / 2;
  double rw[33];   // k <= 32
  int rq[33];
  double den = 0.0;
  for (int d = -h; d <= h; ++d) {
    const int q = wrap(a.k * Q + d, a.Hf);
    const double w = (d == -h || d == h) ? 0.5 : 1.0;
    rq[d + h] = q;
    rw[d + h] = w * a.area[q];
    den += rw[d + h];
  }
  den *= (double)a.k;  // the phi weights sum to k
  for (int fld = 0; fld < 17; ++fld) {
    const T* src = fld < 16 ? a.f + fld * a.plane_f : a.phi;
    const T* base = fld < 16 ? nullptr : a.phib;
    double acc = 0.0;
    for (int d = 0; d <= 2 * h; ++d) {
      const long long row = (long long)rq[d] * a.Wf;
      double racc = 0.0;
      for (int e = -h; e <= h; ++e) {
        const double w = (e == -h || e == h) ? 0.5 : 1.0;
        racc += w * order_parameter(src, base, row + wrap(a.k * S + e, a.Wf));
      }
      acc += rw[d] * racc;
    }
    if (fld == 16 && a.phibc) {
      a.phibc[x] = T(acc / den);
      a.phic[x] = T(0);
    } else {
      T* dst = fld < 16 ? a.fc + fld * a.plane_c : a.phic;
      dst[x] = T(acc / den);
    }
  }
}

// sums of x and x^2 per channel of float[count][4]
struct StatArgs {
  const float* d;
  long long count;
  double* partial;  // [gridDim.x][8]
};

__global__ __launch_bounds__(RED) void stats_kernel(StatArgs a) {
  __shared__ double sh[RED / 64];
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long i = (long long)blockIdx.x * RED + threadIdx.x; i < a.count;
       i += (long long)gridDim.x * RED) {
    const float4 v = reinterpret_cast<const float4*>(a.d)[i];
    const double c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      s[j] += c[j];
      s[4 + j] += c[j] * c[j];
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double t = block_sum(s[j], sh);
    if (threadIdx.x == 0) a.partial[(size_t)blockIdx.x * 8 + j] = t;
  }
}

// ------------------------------------------------------------------------------------------
// host side

// most workgroups of a weight-gradient launch (each writes one partial gradient of the layer)
#ifndef TLB_WG_BLOCKS
#define TLB_WG_BLOCKS 2048
#endif
constexpr int WG_MAX_BLOCKS = TLB_WG_BLOCKS;
constexpr int CONV_MAX_BLOCKS = 4096;
constexpr int LEARN_GRAPH_CHUNK = 32;

template <class Args>
tlbi_launch make_launch(const void* fn, dim3 grid, dim3 block, const Args& args) {
  static_assert(sizeof(Args) <= sizeof(tlbi_launch::args), "argument block");
  tlbi_launch l;
  l.fn = fn;
  l.grid = grid;
  l.block = block;
  std::memcpy(l.args, &args, sizeof(Args));
  return l;
}

int32_t run(const tlbi_launch& l, hipStream_t stream) {
  void* p[] = {const_cast<unsigned char*>(l.args)};
  LRN_HIP_CHECK(hipLaunchKernel(l.fn, l.grid, l.block, p, 0, stream));
  return TLB_OK;
}

int32_t run_all(const std::vector<tlbi_launch>& seq, hipStream_t stream) {
  for (const tlbi_launch& l : seq) {
    int32_t rc = run(l, stream);
    if (rc != TLB_OK) return rc;
  }
  return TLB_OK;
}

int blocks_for(long long n, int threads) { return (int)((n + threads - 1) / threads); }

// Partials of tlb_learn_stats: STATS_BLOCKS x 8 doubles plus the 8 results, one buffer per
// device, made on the first call on that device and kept until the process ends (calls on
// one device are stream-ordered through it; tlb_learn_stats waits for its stream).
constexpr int STATS_BLOCKS = 512;
constexpr int MAX_DEVICES = 64;

int32_t stats_workspace(double** out) {
  static std::mutex mu;
  static double* ws[MAX_DEVICES] = {};
  int dev = 0;
  LRN_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return tlbi_fail(TLB_EHIP, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ws[dev]) {
    const hipError_t e = hipMalloc(&ws[dev], (STATS_BLOCKS * 8 + 8) * sizeof(double));
    if (e != hipSuccess) {
      ws[dev] = nullptr;
      return tlbi_fail(TLB_ENOMEM, std::string("stats workspace: ") + hipGetErrorString(e));
    }
  }
  *out = ws[dev];
  return TLB_OK;
}

}  // namespace

struct tlb_cnn {
  tlb_cnn_desc d;
  hipStream_t stream;
  int H, W, B;
  long long HW;
  float* params;
  float* grad;
  float* mom;
  float* vel;
  u16* wf[NL];  // forward fragments
  u16* wd[NL];  // input-gradient fragments (layers 1..4)
  u16* act[4];
  float* z;
  u16* e4;
  u16* feat;           // the input features of the batch, bf16 [n][HW][8]
  u16* eA;
  u16* eB;
  float* partial;      // weight-gradient partials
  double* red;         // loss partials / statistics partials
  double* scalars;     // [8]: loss, statistics
  float* Jrow;
  double* proj;        // [H][3]
  int red_blocks;
  int conv_grid[5];    // most workgroups of each convolution variant (conv_variant)
  int wgrad_grid[NL];  // workgroups of each layer's weight-gradient launch
  // graph of LEARN_GRAPH_CHUNK learned steps, bound to one grid's buffers and tile shape
  hipGraphExec_t chunk_exec;
  unsigned long long chunk_grid;  // uid of the grid the graph was built for (0: none)
  void* chunk_key[7];
  unsigned chunk_version;  // the grid's version when the graph was built
};

namespace {

int frag_slots(int l, bool transpose) {
  if (!transpose) {
    const int kc = L_CIS[l] == 32 ? 9 : 3;
    const int cob = (L_COUT[l] + 15) / 16;
    return kc * cob * 64 * 8;
  }
  const int kc = L_COS[l] == 32 ? 9 : 3;
  const int cob = (L_CIN[l] + 15) / 16;
  return kc * cob * 64 * 8;
}

Features make_features(const tlb_cnn* net) {
  Features F;
  for (int c = 0; c < 4; ++c) {
    F.shift[c] = net->d.in_shift[c];
    F.scale[c] = net->d.in_scale[c];
  }
  F.r = (float)net->d.r;
  F.Jrow = net->Jrow;
  return F;
}

// index of a convolution variant: 0 8-channel input with the bias + ReLU epilogue (the first
// layer), 1 8-channel input with the ReLU mask, 2-4 32-channel input with the output layer's,
// the ReLU-mask and the bias + ReLU epilogue
int conv_variant(int in, int epi) {
  if (in == IN_BF8) return epi == EPI_RELU ? 0 : 1;
  return epi == EPI_OUT ? 2 : epi == EPI_MASK ? 3 : 4;
}

const void* conv_fn(int in, int cob, int epi) {
  if (in == IN_BF8)
    return epi == EPI_RELU ? reinterpret_cast<const void*>(&conv_kernel<IN_BF8, 2, EPI_RELU>)
                           : reinterpret_cast<const void*>(&conv_kernel<IN_BF8, 2, EPI_MASK>);
  if (epi == EPI_OUT) return reinterpret_cast<const void*>(&conv_kernel<IN_BF32, 1, EPI_OUT>);
  if (epi == EPI_MASK) return reinterpret_cast<const void*>(&conv_kernel<IN_BF32, 2, EPI_MASK>);
  (void)cob;
  return reinterpret_cast<const void*>(&conv_kernel<IN_BF32, 2, EPI_RELU>);
}

tlbi_launch conv_launch(const tlb_cnn* net, int in, int cob, int epi, const void* src,
                        const u16* w, const float* bias, const u16* mask, void* out, int n) {
  ConvArgs a{};
  a.in = src;
  a.w = reinterpret_cast<const bf16x8*>(w);
  a.bias = bias;
  a.mask = mask;
  a.out = out;
  a.n = n;
  a.H = net->H;
  a.W = net->W;
  a.xt = (net->W + 15) / 16;
  a.tiles = n * net->H * a.xt;
  int blocks = blocks_for(a.tiles, CONV_WAVES);
  const int cap = net->conv_grid[conv_variant(in, epi)];
  if (blocks > cap) blocks = cap;
  return make_launch(conv_fn(in, cob, epi), dim3(blocks), dim3(CONV_THREADS), a);
}

const float* bias_of(const tlb_cnn* net, int l) {
  return net->params + layer_offset(l) + L_COUT[l] * 9 * L_CIN[l];
}

// forward of n samples: moments (sample idx[i]) -> act[0..3] -> z
// the input features of every node of the batch, once (the first layer's convolution and
// weight gradient read them as an 8-channel input)
tlbi_launch features_launch(const tlb_cnn* net, const float* moments, const int32_t* idx, int n) {
  FeatArgs fa{};
  fa.m = moments;
  fa.idx = idx;
  fa.out = net->feat;
  fa.F = make_features(net);
  fa.n = n;
  fa.H = net->H;
  fa.W = net->W;
  return make_launch(reinterpret_cast<const void*>(&features_kernel), dim3(n * net->H), dim3(128),
                     fa);
}

void forward_seq(const tlb_cnn* net, const float* moments, const int32_t* idx, int n,
                 std::vector<tlbi_launch>& seq) {
  seq.push_back(features_launch(net, moments, idx, n));
  seq.push_back(conv_launch(net, IN_BF8, 2, EPI_RELU, net->feat, net->wf[0],
                            bias_of(net, 0), nullptr, net->act[0], n));
  for (int l = 1; l < 4; ++l)
    seq.push_back(conv_launch(net, IN_BF32, 2, EPI_RELU, net->act[l - 1], net->wf[l],
                              bias_of(net, l), nullptr, net->act[l], n));
  seq.push_back(conv_launch(net, IN_BF32, 1, EPI_OUT, net->act[3], net->wf[4],
                            bias_of(net, 4), nullptr, net->z, n));
}

const void* wgrad_fn(int l) {
  if (l == 0) return reinterpret_cast<const void*>(&wgrad_kernel<8, 32>);
  if (l == 4) return reinterpret_cast<const void*>(&wgrad_kernel<32, 8>);
  return reinterpret_cast<const void*>(&wgrad_kernel<32, 32>);
}

// loss, back-propagation and the gradient of every layer into net->grad
void backward_seq(const tlb_cnn* net, const float* moments, const float* targets,
                  const int32_t* idx, int n, std::vector<tlbi_launch>& seq) {
  LossArgs la{};
  la.z = net->z;
  la.y = targets;
  la.idx = idx;
  la.e = net->e4;
  la.partial = net->red;
  la.hw = net->HW;
  la.total = (long long)n * net->HW;
  for (int c = 0; c < 4; ++c) {
    la.inv_scale[c] = 1.0f / net->d.out_scale[c];
    la.w[c] = net->d.loss_weight[c];
  }
  const int lblocks = blocks_for(la.total, RED);
  seq.push_back(make_launch(reinterpret_cast<const void*>(&loss_kernel), dim3(lblocks), dim3(RED), la));
  SumArgs sa{net->red, net->scalars, lblocks, 1, 1.0 / (4.0 * (double)la.total)};
  seq.push_back(make_launch(reinterpret_cast<const void*>(&sum_partials_kernel), dim3(1), dim3(RED), sa));

  const double scale = 2.0 / (4.0 * (double)la.total);
  const u16* e = net->e4;
  for (int l = NL - 1; l >= 0; --l) {
    WgradArgs wa{};
    wa.e = e;
    wa.a = l == 0 ? net->feat : net->act[l - 1];
    wa.partial = net->partial;
    wa.n = n;
    wa.H = net->H;
    wa.W = net->W;
    wa.xs = (net->W + 63) / 64;
    wa.strips = n * net->H * wa.xs;
    const int wblocks = std::min(wa.strips, net->wgrad_grid[l]);
    seq.push_back(make_launch(wgrad_fn(l), dim3(wblocks), dim3(WG_THREADS), wa));
    GradArgs ga{net->partial, net->grad + layer_offset(l), wblocks, L_CIS[l], L_COS[l], L_CIN[l],
                L_COUT[l], scale};
    seq.push_back(make_launch(reinterpret_cast<const void*>(&grad_reduce_kernel),
                              dim3(blocks_for(layer_params(l), GR_PARAMS)),
                              dim3(64 * GR_WAVES), ga));
    if (l > 0) {
      // error signals alternate between two buffers: layer 4 -> eA, 3 -> eB, 2 -> eA, ...
      u16* next = (l == 4 || e == net->eB) ? net->eA : net->eB;
      seq.push_back(conv_launch(net, l == 4 ? IN_BF8 : IN_BF32, 2, EPI_MASK, e,
                                net->wd[l], nullptr, net->act[l - 1], next, n));
      e = next;
    }
  }
}

void frags_seq(const tlb_cnn* net, std::vector<tlbi_launch>& seq) {
  FragJobs jobs{};
  int n = 0, blocks = 1;
  for (int l = 0; l < NL; ++l)
    for (int tr = 0; tr < (l > 0 ? 2 : 1); ++tr) {
      FragArgs& fa = jobs.job[n++];
      fa.W = net->params + layer_offset(l);
      fa.out = tr ? net->wd[l] : net->wf[l];
      fa.slots = frag_slots(l, tr);
      fa.transpose = tr;
      fa.cin = L_CIN[l];
      fa.cout = L_COUT[l];
      fa.cob = tr ? (L_CIN[l] + 15) / 16 : (L_COUT[l] + 15) / 16;
      fa.wide = tr ? (L_COS[l] == 32) : (L_CIS[l] == 32);
      blocks = std::max(blocks, blocks_for(fa.slots, 256));
    }
  seq.push_back(make_launch(reinterpret_cast<const void*>(&frag_kernel), dim3(blocks, n),
                            dim3(256), jobs));
}

int32_t check_batch(const tlb_cnn* net, const float* moments, int32_t n) {
  if (!net) return tlbi_fail(TLB_EINVAL, "network is NULL");
  if (!moments) return tlbi_fail(TLB_EINVAL, "moments is NULL");
  if (n < 1 || n > net->B) return tlbi_fail(TLB_EINVAL, "batch size out of range [1, max_batch]");
  return TLB_OK;
}

template <typename T>
void pair_launch(const tlb_grid* g, const tlb_grid* truth, float* m, float* y,
                 std::vector<tlbi_launch>& seq) {
  MomArgs<T> a{};
  a.f = static_cast<const T*>(g->f[0]);
  a.phi = static_cast<const T*>(g->phi[0]);
  a.phib = reinterpret_cast<const T*>(g->phi_base);
  a.f2 = truth ? static_cast<const T*>(truth->f[0]) : nullptr;
  a.phi2 = truth ? static_cast<const T*>(truth->phi[0]) : nullptr;
  a.phib2 = truth ? reinterpret_cast<const T*>(truth->phi_base) : nullptr;
  a.m = m;
  a.y = y;
  a.plane = (long long)g->p.n_theta * g->p.n_phi;
  a.n_add = stores_deviation<T>() ? g->n_ref : 0.0;
  a.n_add2 = truth && stores_deviation<T>() ? truth->n_ref : 0.0;
  seq.push_back(make_launch(reinterpret_cast<const void*>(&moments_pair_kernel<T>),
                            dim3(blocks_for(a.plane, 256)), dim3(256), a));
}

// the correction of grid g by d; with nparts == 0 the area-weighted sums are made here (one
// block per row), otherwise they are already in proj[nparts][3]
template <typename T>
void apply_launches(tlb_grid* g, const float* d, const float scale[4], double* proj,
                    int nparts, bool rebase, std::vector<tlbi_launch>& seq) {
  if (nparts == 0) {
    ProjArgs pa{d, g->area, proj, g->p.n_phi, scale[0], scale[1]};
    seq.push_back(make_launch(reinterpret_cast<const void*>(&proj_kernel), dim3(g->p.n_theta),
                              dim3(RED), pa));
    nparts = g->p.n_theta;
  }
  ApplyArgs<T> aa{};
  aa.f = static_cast<T*>(g->f[0]);
  aa.phi = static_cast<T*>(g->phi[0]);
  aa.phib = rebase ? reinterpret_cast<T*>(g->phi_base) : nullptr;
  aa.d = d;
  aa.partial = proj;
  aa.nparts = nparts;
  aa.plane = (long long)g->p.n_theta * g->p.n_phi;
  for (int c = 0; c < 4; ++c) aa.scale[c] = scale[c];
  aa.n_ref = T(g->n_ref);
  seq.push_back(make_launch(reinterpret_cast<const void*>(&apply_kernel<T>),
                            dim3(blocks_for(aa.plane, 256)), dim3(256), aa));
}

int net_tiles(int H, int W) { return ((H + NT_H - 1) / NT_H) * ((W + NT_W - 1) / NT_W); }

// the network of a learned step of grid g (net_step_kernel): output in net->z, per-tile
// area-weighted sums of the corrections (times scale[0], scale[1]) in net->proj
template <typename T>
tlbi_launch net_step_launch(const tlb_grid* g, const tlb_cnn* net, const float scale[4]) {
  NetArgs<T> a{};
  a.f = static_cast<const T*>(g->f[0]);
  a.phi = static_cast<const T*>(g->phi[0]);
  a.phib = reinterpret_cast<const T*>(g->phi_base);
  a.plane = (long long)g->p.n_theta * g->p.n_phi;
  a.n_add = stores_deviation<T>() ? g->n_ref : 0.0;
  for (int l = 0; l < NL; ++l) {
    a.w[l] = reinterpret_cast<const bf16x8*>(net->wf[l]);
    a.bias[l] = bias_of(net, l);
  }
  a.F = make_features(net);
  a.H = net->H;
  a.W = net->W;
  a.tiles_x = (net->W + NT_W - 1) / NT_W;
  a.out = net->z;
  a.proj = net->proj;
  a.area = g->area;
  a.s0 = scale[0];
  a.s1 = scale[1];
  return make_launch(reinterpret_cast<const void*>(&net_step_kernel<T>),
                     dim3(net_tiles(net->H, net->W)), dim3(NT_THREADS), a);
}

// one learned step of grid g: three stage launches, the network, the correction
void learned_step_seq(tlb_grid* g, tlb_cnn* net, std::vector<tlbi_launch>& seq) {
  for (int st = 1; st <= 3; ++st) {
    tlbi_launch l[2];
    const int n = tlbi_stage_launches(g, st, l);
    for (int i = 0; i < n; ++i) seq.push_back(l[i]);
  }
  float scale[4];
  for (int c = 0; c < 4; ++c)
    scale[c] = (net->d.apply_mask == 0 || ((net->d.apply_mask >> c) & 1u)) ? net->d.out_scale[c] : 0.0f;
  // moments, features and the five layers in one launch, which also forms the area-weighted
  // sums of the corrections per tile
  if (g->p.precision == 64)
    seq.push_back(net_step_launch<double>(g, net, scale));
  else
    seq.push_back(net_step_launch<float>(g, net, scale));
  const int nparts = (int)seq.back().grid.x;
  // FP32: the correction also folds the order parameter into its base, so every learned step
  // ends with a rebase
  if (g->p.precision == 64)
    apply_launches<double>(g, net->z, scale, net->proj, nparts, false, seq);
  else
    apply_launches<float>(g, net->z, scale, net->proj, nparts, true, seq);
}

void drop_learn_graph(tlb_cnn* net) {
  if (net->chunk_exec) (void)hipGraphExecDestroy(net->chunk_exec);
  net->chunk_exec = nullptr;
  net->chunk_grid = 0;
}

int32_t build_learn_graph(tlb_grid* g, tlb_cnn* net) {
  drop_learn_graph(net);
  std::vector<tlbi_launch> one;
  learned_step_seq(g, net, one);
  hipGraph_t graph;
  LRN_HIP_CHECK(hipGraphCreate(&graph, 0));
  // argument pointers stay valid until the graph is instantiated
  std::vector<void*> argp(one.size());
  for (size_t i = 0; i < one.size(); ++i) argp[i] = one[i].args;
  hipError_t e = hipSuccess;
  hipGraphNode_t prev = nullptr;
  for (int t = 0; t < LEARN_GRAPH_CHUNK && e == hipSuccess; ++t)
    for (size_t i = 0; i < one.size() && e == hipSuccess; ++i) {
      hipKernelNodeParams kp{};
      kp.func = const_cast<void*>(one[i].fn);
      kp.gridDim = one[i].grid;
      kp.blockDim = one[i].block;
      kp.sharedMemBytes = 0;
      kp.kernelParams = &argp[i];
      kp.extra = nullptr;
      hipGraphNode_t node;
      e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
      prev = node;
    }
  if (e == hipSuccess) e = hipGraphInstantiate(&net->chunk_exec, graph, nullptr, nullptr, 0);
  if (e == hipSuccess && (e = hipGraphUpload(net->chunk_exec, g->stream)) != hipSuccess)
    (void)hipGraphExecDestroy(net->chunk_exec);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    net->chunk_exec = nullptr;
    return tlbi_fail(TLB_EHIP, std::string("learned-step graph: ") + hipGetErrorString(e));
  }
  net->chunk_grid = g->uid;
  net->chunk_version = g->version;
  void* key[7] = {g->f[0], g->f[1], g->f[2], g->phi[0], g->phi[1], g->phi[2],
                  reinterpret_cast<void*>((intptr_t)g->ty)};
  std::memcpy(net->chunk_key, key, sizeof(key));
  return TLB_OK;
}

// The graph keeps the stage arguments (time step, parameters, per-row tables) of the grid it
// was built for; a grid is identified by its process-unique id, not its address, since a new
// grid may be created at a destroyed one's address with the same state buffers.
bool graph_matches(const tlb_cnn* net, const tlb_grid* g) {
  if (!net->chunk_exec || net->chunk_grid != g->uid || net->chunk_version != g->version)
    return false;
  void* key[7] = {g->f[0], g->f[1], g->f[2], g->phi[0], g->phi[1], g->phi[2],
                  reinterpret_cast<void*>((intptr_t)g->ty)};
  return std::memcmp(net->chunk_key, key, sizeof(key)) == 0;
}

void free_net(tlb_cnn* net) {
  void* bufs[] = {net->params, net->grad, net->mom, net->vel, net->z, net->e4, net->feat,
                  net->eA, net->eB, net->partial, net->red, net->scalars, net->Jrow, net->proj};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (int l = 0; l < NL; ++l) {
    if (net->wf[l]) (void)hipFree(net->wf[l]);
    if (net->wd[l]) (void)hipFree(net->wd[l]);
  }
  for (int l = 0; l < 4; ++l)
    if (net->act[l]) (void)hipFree(net->act[l]);
  drop_learn_graph(net);
  delete net;
}

bool finite_nonzero(float x) { return std::isfinite(x) && x != 0.0f; }

int32_t check_grid(const tlb_grid* g, const char* what) {
  if (!g) return tlbi_fail(TLB_EINVAL, std::string(what) + " is NULL");
  return TLB_OK;
}

}  // namespace

extern "C" {

int32_t tlb_cnn_create(const tlb_cnn_desc* desc, void* hip_stream, tlb_cnn** out) {
  if (!out) return tlbi_fail(TLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc) return tlbi_fail(TLB_EINVAL, "desc is NULL");
  const tlb_cnn_desc& d = *desc;
  if (!(d.r > 0.0) || !(d.R > d.r) || !std::isfinite(d.R))
    return tlbi_fail(TLB_EINVAL, "radii must satisfy 0 < r < R");
  if (d.n_theta < 1 || d.n_phi < 1 || (long long)d.n_theta * d.n_phi > (1LL << 26))
    return tlbi_fail(TLB_EINVAL, "grid size out of range");
  if (d.max_batch < 1 || (long long)d.max_batch * d.n_theta * d.n_phi > (1LL << 28))
    return tlbi_fail(TLB_EINVAL, "max_batch out of range");
  for (int c = 0; c < 4; ++c)
    if (!std::isfinite(d.in_shift[c]) || !finite_nonzero(d.in_scale[c]) ||
        !finite_nonzero(d.out_scale[c]) || !std::isfinite(d.loss_weight[c]) ||
        d.loss_weight[c] < 0.0f)
      return tlbi_fail(TLB_EINVAL, "normalisation, output scale or loss weight invalid");
  if (d.apply_mask > 15u) return tlbi_fail(TLB_EINVAL, "apply_mask has bits above the four outputs");
  tlb_cnn* net = new (std::nothrow) tlb_cnn{};
  if (!net) return tlbi_fail(TLB_ENOMEM, "host allocation failed");
  net->d = d;
  net->stream = static_cast<hipStream_t>(hip_stream);
  net->H = d.n_theta;
  net->W = d.n_phi;
  net->B = d.max_batch;
  net->HW = (long long)d.n_theta * d.n_phi;
  const size_t nb = (size_t)net->B * net->HW;
  const size_t P = TLB_CNN_PARAMS;
  net->red_blocks = blocks_for((long long)nb, RED);
  if (net->red_blocks < 1024) net->red_blocks = 1024;
  // Convolution grids.  A 32-channel-input workgroup stages 18 KB of weight fragments in LDS
  // before its first tile: those kernels run one wave of resident workgroups, each wavefront
  // then taking many tiles with the next tile's loads in flight (measured on 16 x 128 x 320:
  // 0.72-0.78x the time of 4096 workgroups).  The others stage 6 KB and balance better with
  // up to 4096 workgroups.
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  for (int v = 0; v < 5 && e == hipSuccess; ++v) {
    net->conv_grid[v] = CONV_MAX_BLOCKS;
    if (v < 2) continue;
    int resident = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &resident, conv_fn(IN_BF32, v == 2 ? 1 : 2, v == 2 ? EPI_OUT : v == 3 ? EPI_MASK : EPI_RELU),
        CONV_THREADS, 0);
    if (e == hipSuccess)
      net->conv_grid[v] = (int)std::min<long long>(CONV_MAX_BLOCKS,
                                                   (long long)std::max(resident, 1) * cus);
  }
  // Weight-gradient grids: one wave of resident workgroups (LDS or registers limit them to
  // 3 to 5 per compute unit), each taking consecutive strips, the next strip's loads in
  // flight during a strip's products.
  for (int l = 0; l < NL && e == hipSuccess; ++l) {
    int resident = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, wgrad_fn(l), WG_THREADS, 0);
    if (e == hipSuccess)
      net->wgrad_grid[l] =
          (int)std::min<long long>(WG_MAX_BLOCKS, (long long)std::max(resident, 1) * cus);
  }
  if (e != hipSuccess) {
    free_net(net);
    return tlbi_fail(TLB_EHIP, std::string("occupancy query: ") + hipGetErrorString(e));
  }
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  alloc((void**)&net->params, P * 4);
  alloc((void**)&net->grad, P * 4);
  alloc((void**)&net->mom, P * 4);
  alloc((void**)&net->vel, P * 4);
  for (int l = 0; l < NL; ++l) {
    alloc((void**)&net->wf[l], frag_slots(l, false) * 2);
    if (l > 0) alloc((void**)&net->wd[l], frag_slots(l, true) * 2);
  }
  for (int l = 0; l < 4; ++l) alloc((void**)&net->act[l], nb * WIDTH * 2);
  alloc((void**)&net->z, nb * 16);
  alloc((void**)&net->feat, nb * 16);
  alloc((void**)&net->e4, nb * 16);
  alloc((void**)&net->eA, nb * WIDTH * 2);
  alloc((void**)&net->eB, nb * WIDTH * 2);
  size_t partial = 0;
  for (int l = 0; l < NL; ++l)
    partial = std::max(partial, (size_t)net->wgrad_grid[l] * (L_COS[l] * 9 * L_CIS[l] + L_COS[l]));
  alloc((void**)&net->partial, partial * 4);
  alloc((void**)&net->red, (size_t)net->red_blocks * 8 * 8);
  alloc((void**)&net->scalars, 8 * 8);
  alloc((void**)&net->Jrow, net->H * 4);
  // partial sums of the corrections: one per row (tlb_apply_correction) or per tile of the
  // learned step's network
  const size_t nproj = std::max<size_t>(net->H, net_tiles(net->H, net->W));
  alloc((void**)&net->proj, nproj * 3 * 8);
  if (e != hipSuccess) {
    free_net(net);
    return tlbi_fail(TLB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  std::vector<float> J(net->H);
  for (int q = 0; q < net->H; ++q) J[q] = (float)(d.R + d.r * std::cos(2.0 * M_PI * q / net->H));
  std::vector<float> zero(P, 0.0f);
  e = hipMemcpy(net->Jrow, J.data(), net->H * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->params, zero.data(), P * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->mom, zero.data(), P * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(net->vel, zero.data(), P * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_net(net);
    return tlbi_fail(TLB_EHIP, std::string("upload: ") + hipGetErrorString(e));
  }
  std::vector<tlbi_launch> seq;
  frags_seq(net, seq);
  int32_t rc = run_all(seq, net->stream);
  if (rc == TLB_OK && hipStreamSynchronize(net->stream) != hipSuccess)
    rc = tlbi_fail(TLB_EHIP, "stream synchronisation failed");
  if (rc != TLB_OK) {
    free_net(net);
    return rc;
  }
  *out = net;
  return TLB_OK;
}

void tlb_cnn_destroy(tlb_cnn* net) {
  if (!net) return;
  (void)hipStreamSynchronize(net->stream);
  free_net(net);
}

int32_t tlb_cnn_set_params(tlb_cnn* net, const float* host_params) {
  if (!net || !host_params) return tlbi_fail(TLB_EINVAL, "network or params is NULL");
  for (int i = 0; i < TLB_CNN_PARAMS; ++i)
    if (!std::isfinite(host_params[i])) return tlbi_fail(TLB_EINVAL, "non-finite parameter");
  LRN_HIP_CHECK(hipStreamSynchronize(net->stream));
  std::vector<float> zero(TLB_CNN_PARAMS, 0.0f);
  LRN_HIP_CHECK(hipMemcpy(net->params, host_params, TLB_CNN_PARAMS * 4, hipMemcpyHostToDevice));
  LRN_HIP_CHECK(hipMemcpy(net->mom, zero.data(), TLB_CNN_PARAMS * 4, hipMemcpyHostToDevice));
  LRN_HIP_CHECK(hipMemcpy(net->vel, zero.data(), TLB_CNN_PARAMS * 4, hipMemcpyHostToDevice));
  std::vector<tlbi_launch> seq;
  frags_seq(net, seq);
  int32_t rc = run_all(seq, net->stream);
  if (rc != TLB_OK) return rc;
  LRN_HIP_CHECK(hipStreamSynchronize(net->stream));
  return TLB_OK;
}

int32_t tlb_cnn_get_params(tlb_cnn* net, float* host_params) {
  if (!net || !host_params) return tlbi_fail(TLB_EINVAL, "network or params is NULL");
  LRN_HIP_CHECK(hipStreamSynchronize(net->stream));
  LRN_HIP_CHECK(hipMemcpy(host_params, net->params, TLB_CNN_PARAMS * 4, hipMemcpyDeviceToHost));
  return TLB_OK;
}

int32_t tlb_cnn_forward(tlb_cnn* net, const float* moments, const int32_t* idx, int32_t n,
                        float* out) {
  int32_t rc = check_batch(net, moments, n);
  if (rc != TLB_OK) return rc;
  if (!out) return tlbi_fail(TLB_EINVAL, "out is NULL");
  std::vector<tlbi_launch> seq;
  forward_seq(net, moments, idx, n, seq);
  ScaleArgs sa{net->z, out, (long long)n * net->HW, {0, 0, 0, 0}};
  for (int c = 0; c < 4; ++c) sa.s[c] = net->d.out_scale[c];
  seq.push_back(make_launch(reinterpret_cast<const void*>(&scale_kernel),
                            dim3(blocks_for(sa.count, 256)), dim3(256), sa));
  return run_all(seq, net->stream);
}

int32_t tlb_cnn_gradient(tlb_cnn* net, const float* moments, const float* targets,
                         const int32_t* idx, int32_t n, double* loss, float* host_grad) {
  int32_t rc = check_batch(net, moments, n);
  if (rc != TLB_OK) return rc;
  if (!targets) return tlbi_fail(TLB_EINVAL, "targets is NULL");
  std::vector<tlbi_launch> seq;
  forward_seq(net, moments, idx, n, seq);
  backward_seq(net, moments, targets, idx, n, seq);
  rc = run_all(seq, net->stream);
  if (rc != TLB_OK) return rc;
  LRN_HIP_CHECK(hipStreamSynchronize(net->stream));
  if (loss) LRN_HIP_CHECK(hipMemcpy(loss, net->scalars, 8, hipMemcpyDeviceToHost));
  if (host_grad)
    LRN_HIP_CHECK(hipMemcpy(host_grad, net->grad, TLB_CNN_PARAMS * 4, hipMemcpyDeviceToHost));
  return TLB_OK;
}

int32_t tlb_cnn_train_step(tlb_cnn* net, const float* moments, const float* targets,
                           const int32_t* idx, int32_t n, const tlb_adam* adam, double* loss) {
  int32_t rc = check_batch(net, moments, n);
  if (rc != TLB_OK) return rc;
  if (!targets || !adam) return tlbi_fail(TLB_EINVAL, "targets or adam is NULL");
  if (adam->step < 1 || !(adam->lr >= 0.0f) || !(adam->beta1 >= 0.0f && adam->beta1 < 1.0f) ||
      !(adam->beta2 >= 0.0f && adam->beta2 < 1.0f) || !(adam->eps > 0.0f))
    return tlbi_fail(TLB_EINVAL, "Adam hyper-parameters out of range");
  std::vector<tlbi_launch> seq;
  forward_seq(net, moments, idx, n, seq);
  backward_seq(net, moments, targets, idx, n, seq);
  AdamArgs aa{};
  aa.p = net->params;
  aa.g = net->grad;
  aa.m = net->mom;
  aa.v = net->vel;
  aa.count = TLB_CNN_PARAMS;
  aa.lr = adam->lr;
  aa.b1 = adam->beta1;
  aa.b2 = adam->beta2;
  aa.eps = adam->eps;
  aa.c1 = (float)(1.0 - std::pow((double)adam->beta1, adam->step));
  aa.c2 = (float)(1.0 - std::pow((double)adam->beta2, adam->step));
  seq.push_back(make_launch(reinterpret_cast<const void*>(&adam_kernel),
                            dim3(blocks_for(TLB_CNN_PARAMS, 256)), dim3(256), aa));
  frags_seq(net, seq);
  rc = run_all(seq, net->stream);
  if (rc != TLB_OK) return rc;
  if (loss) {
    LRN_HIP_CHECK(hipStreamSynchronize(net->stream));
    LRN_HIP_CHECK(hipMemcpy(loss, net->scalars, 8, hipMemcpyDeviceToHost));
  }
  return TLB_OK;
}

int32_t tlb_learn_stats(const float* data, int64_t count, void* hip_stream, double out[8]) {
  if (!data || !out || count < 1) return tlbi_fail(TLB_EINVAL, "data, out or count invalid");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const int blocks = STATS_BLOCKS;
  double* part = nullptr;
  int32_t wrc = stats_workspace(&part);
  if (wrc != TLB_OK) return wrc;
  StatArgs a{data, count, part};
  std::vector<tlbi_launch> seq;
  seq.push_back(make_launch(reinterpret_cast<const void*>(&stats_kernel), dim3(blocks), dim3(RED), a));
  SumArgs s{part, part + blocks * 8, blocks, 8, 1.0};
  seq.push_back(make_launch(reinterpret_cast<const void*>(&sum_partials_kernel), dim3(1), dim3(RED), s));
  int32_t rc = run_all(seq, stream);
  hipError_t e = hipSuccess;
  if (rc == TLB_OK)
    e = hipMemcpyAsync(out, part + blocks * 8, 8 * sizeof(double), hipMemcpyDeviceToHost, stream);
  if (rc == TLB_OK && e == hipSuccess) e = hipStreamSynchronize(stream);
  if (rc != TLB_OK) return rc;
  if (e != hipSuccess) return tlbi_fail(TLB_EHIP, std::string("stats: ") + hipGetErrorString(e));
  return TLB_OK;
}

int32_t tlb_restrict(const tlb_grid* fine, tlb_grid* coarse) {
  int32_t rc = check_grid(fine, "fine grid");
  if (rc == TLB_OK) rc = check_grid(coarse, "coarse grid");
  if (rc != TLB_OK) return rc;
  const tlb_params& pf = fine->p;
  const tlb_params& pc = coarse->p;
  if (pf.n_theta % pc.n_theta || pf.n_phi % pc.n_phi)
    return tlbi_fail(TLB_EINVAL, "fine sizes are not multiples of the coarse ones");
  const int k = pf.n_theta / pc.n_theta;
  if (k != pf.n_phi / pc.n_phi || k < 2 || k % 2 || k > 32)
    return tlbi_fail(TLB_EINVAL, "refinement factor must be the same even k in both angles, 2..32");
  if (pf.r != pc.r || pf.R != pc.R || pf.precision != pc.precision ||
      (pf.flags & TLB_FLAT) != (pc.flags & TLB_FLAT))
    return tlbi_fail(TLB_EINVAL, "grids differ in radii, flat flag or precision");
  std::vector<tlbi_launch> seq;
  auto go = [&](auto tag) {
    using T = decltype(tag);
    RestrictArgs<T> a{};
    a.f = static_cast<const T*>(fine->f[0]);
    a.phi = static_cast<const T*>(fine->phi[0]);
    a.phib = reinterpret_cast<const T*>(fine->phi_base);
    a.fc = static_cast<T*>(coarse->f[0]);
    a.phic = static_cast<T*>(coarse->phi[0]);
    a.phibc = reinterpret_cast<T*>(coarse->phi_base);
    a.area = fine->area;
    a.Hf = pf.n_theta;
    a.Wf = pf.n_phi;
    a.Hc = pc.n_theta;
    a.Wc = pc.n_phi;
    a.k = k;
    a.plane_f = (long long)pf.n_theta * pf.n_phi;
    a.plane_c = (long long)pc.n_theta * pc.n_phi;
    seq.push_back(make_launch(reinterpret_cast<const void*>(&restrict_kernel<T>),
                              dim3(blocks_for(a.plane_c, 256)), dim3(256), a));
  };
  if (pf.precision == 64) go(double{}); else go(float{});
  // the restricted deviations are relative to the fine grid's reference density (restriction
  // keeps it: it preserves constants and the area-weighted totals)
  if (pf.precision == 32 && coarse->n_ref != fine->n_ref) {
    coarse->n_ref = fine->n_ref;
    ++coarse->version;
  }
  coarse->phase = 0;  // the coarse order parameter is all base now, as after set_state
  return run_all(seq, coarse->stream);
}

int32_t tlb_learn_pair(const tlb_grid* grid, const tlb_grid* truth, float* moments,
                       float* targets) {
  int32_t rc = check_grid(grid, "grid");
  if (rc != TLB_OK) return rc;
  if (!moments) return tlbi_fail(TLB_EINVAL, "moments is NULL");
  if (truth) {
    if (!targets) return tlbi_fail(TLB_EINVAL, "targets is NULL");
    if (truth->p.n_theta != grid->p.n_theta || truth->p.n_phi != grid->p.n_phi ||
        truth->p.precision != grid->p.precision)
      return tlbi_fail(TLB_EINVAL, "truth grid differs in size or precision");
  }
  std::vector<tlbi_launch> seq;
  if (grid->p.precision == 64)
    pair_launch<double>(grid, truth, moments, targets, seq);
  else
    pair_launch<float>(grid, truth, moments, targets, seq);
  return run_all(seq, grid->stream);
}

int32_t tlb_apply_correction(tlb_grid* grid, const float* corrections) {
  int32_t rc = check_grid(grid, "grid");
  if (rc != TLB_OK) return rc;
  if (!corrections) return tlbi_fail(TLB_EINVAL, "corrections is NULL");
  // the per-row sums go to the grid's own workspace (made with the grid): stream-ordered, so
  // successive corrections on one grid reuse it in order
  const float one[4] = {1.0f, 1.0f, 1.0f, 1.0f};
  std::vector<tlbi_launch> seq;
  if (grid->p.precision == 64)
    apply_launches<double>(grid, corrections, one, grid->proj, 0, false, seq);
  else
    apply_launches<float>(grid, corrections, one, grid->proj, 0, false, seq);
  return run_all(seq, grid->stream);
}

int32_t tlb_learned_step_n(tlb_grid* grid, tlb_cnn* net, int64_t n_steps) {
  int32_t rc = check_grid(grid, "grid");
  if (rc != TLB_OK) return rc;
  if (!net) return tlbi_fail(TLB_EINVAL, "network is NULL");
  if (n_steps < 0) return tlbi_fail(TLB_EINVAL, "n_steps < 0");
  if (grid->p.n_theta != net->H || grid->p.n_phi != net->W)
    return tlbi_fail(TLB_EINVAL, "grid size differs from the network's");
  const bool use_graph = !(grid->p.flags & TLB_NO_GRAPH) && n_steps >= LEARN_GRAPH_CHUNK;
  int64_t done = 0;
  if (use_graph) {
    if (!graph_matches(net, grid)) {
      rc = build_learn_graph(grid, net);
      if (rc != TLB_OK) return rc;
    }
    for (; done + LEARN_GRAPH_CHUNK <= n_steps; done += LEARN_GRAPH_CHUNK)
      LRN_HIP_CHECK(hipGraphLaunch(net->chunk_exec, grid->stream));
  }
  if (done < n_steps) {
    std::vector<tlbi_launch> seq;
    learned_step_seq(grid, net, seq);
    for (; done < n_steps; ++done) {
      rc = run_all(seq, grid->stream);
      if (rc != TLB_OK) return rc;
    }
  }
  if (n_steps > 0) grid->phase = 0;  // every learned step rebases the order parameter
  return TLB_OK;
}

}  // extern "C"
