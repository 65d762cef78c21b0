// tlb.hip -- MI355X (gfx950, CDNA4) implementation of the vielbein lattice Boltzmann
// binary-fluid step on a periodic torus (Ambrus, Busuioc, Wagner, Paillusson, Kusumaatmaja,
// arXiv:1904.10070) behind the C interface of include/tlb.h.
//
// One time step = three launches of one fused stage kernel (three-stage SSP Runge-Kutta).
// Each launch evaluates the whole right-hand side of the semi-discrete system for a tile of
// 64 (phi) x TY (theta, 4, 8 or 16) nodes and writes the Runge-Kutta combination:
//   * the 16 populations stream, two at a time, through a ring of LDS tiles with a 3-node
//     halo filled by asynchronous copies: each thread keeps its node's f_k and accumulates the
//     upwind (UW5) flux difference along phi and theta (eq. boltz_tor advection, metric factors
//     r and J); threads owning a ring node accumulate that node's moments for the CH flux;
//   * order parameter tile with a 2-node halo -> LDS (copied ahead of the populations);
//     chemical potential mu (eq. mu, with the surface Laplace-Beltrami operator) on the tile
//     and its cross-shaped 1-node ring -> LDS;
//   * per node: moments, f_eq (eq. feq), BGK, the velocity-space force and connection terms
//     through the K^H matrix (section II C), the phi grad mu interface force (eq. pbin), the
//     Cahn-Hilliard right-hand side (eq. CH), and the Runge-Kutta combine -> coalesced stores.
// Wavefront = one 64-node row of the tile, so per-row geometry is wavefront-uniform.
// Tiles are numbered so that each of the 8 XCDs owns a contiguous band of theta rows, which
// keeps the theta halos of neighbouring tiles in the same L2.
//
// Discretisation readings (the paper defers its numerical scheme to supplementary material):
// conservative finite differences with fifth-order upwind face values for the advection,
// second-order central flux form for Cahn-Hilliard, SSP-RK3 in time, potential-form force
// n F = -phi grad mu with central differences, u = sum f v / n.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "tlb.h"
#include "tlb_internal.h"

namespace {

// ------------------------------------------------------------------------------------------
// error reporting
thread_local std::string g_last_error;
// a message in static storage, set instead of g_last_error by the entry point that allocates
// nothing (assigning a std::string may allocate)
thread_local const char* g_static_error = nullptr;

int32_t fail(int32_t code, const std::string& msg) {
  g_static_error = nullptr;
  g_last_error = msg;
  return code;
}

int32_t fail_static(int32_t code, const char* msg) {
  g_static_error = msg;
  return code;
}

void clear_error() {
  g_last_error.clear();  // keeps its capacity: no allocation
  g_static_error = nullptr;
}

#define TLB_HIP_CHECK(call)                                                              \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(TLB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

// ------------------------------------------------------------------------------------------
// velocity space (section II C)

// probabilists' Hermite polynomials He_0..He_4, written out
__host__ __device__ constexpr double hermite_e(int l, double x) {
  return l == 0 ? 1.0 : l == 1 ? x : l == 2 ? x * x - 1.0 : l == 3 ? x * x * x - 3.0 * x
       : x * x * x * x - 6.0 * x * x + 3.0;
}
// velocity-derivative kernel K^H_{im} = -w_i sum_{l<Q} He_{l+1}(v_i) He_l(v_m) / l!
__host__ __device__ constexpr double kh(int i, int m) {
  return -wgt(i) * (hermite_e(1, vel(i)) * hermite_e(0, vel(m)) +
                    hermite_e(2, vel(i)) * hermite_e(1, vel(m)) +
                    hermite_e(3, vel(i)) * hermite_e(2, vel(m)) / 2.0 +
                    hermite_e(4, vel(i)) * hermite_e(3, vel(m)) / 6.0);
}
// sum_m K^H_{im} w_m and sum_m K^H_{im} v_m w_m: the velocity derivatives of the rest
// equilibrium (of f = w and of f v^phi = v w)
__host__ __device__ constexpr double kw(int i) {
  return kh(i, 0) * wgt(0) + kh(i, 1) * wgt(1) + kh(i, 2) * wgt(2) + kh(i, 3) * wgt(3);
}
__host__ __device__ constexpr double kvw(int i) {
  return kh(i, 0) * vel(0) * wgt(0) + kh(i, 1) * vel(1) * wgt(1) + kh(i, 2) * vel(2) * wgt(2) +
         kh(i, 3) * vel(3) * wgt(3);
}

// ------------------------------------------------------------------------------------------
// tile geometry of the stage kernel
constexpr int TX = 64;  // nodes along phi per tile = wavefront width
constexpr int HY = 3;   // population halo rows (UW5 needs 3 upwind, 2 downwind)
// LDS tiles hold rows of 72 elements: columns s0-4 .. s0+67, a 16-byte aligned window that
// contains the 3-node phi halo of the populations and the 2-node halo of the order parameter.
constexpr int LXT = TX + 8;
constexpr int CX = 4;   // LDS column of the tile's first node
// A tile is TX x TY nodes, one wavefront per row; the tile height TY (4, 8 or 16) is chosen
// per grid at run time (tlb_set_tile_rows / tlb_autotune).
template <int TY_>
struct Tile {
  static constexpr int TY = TY_;
  static constexpr int NT = TX * TY;            // threads per block
  static constexpr int NWAVE = TY;
  static constexpr int LY = TY + 2 * HY;        // population tile rows q0-3 .. q0+TY+2
  static constexpr int PY = TY + 4;             // order-parameter tile rows q0-2 .. q0+TY+1
  static constexpr int NRING = 2 * TX + 2 * TY; // cross-shaped ring of 1 node
  static_assert(NRING <= NT, "ring nodes must fit one per thread");
};
constexpr int DEFAULT_TY = 8;

// UW5 flux difference (face_{+1/2} - face_{-1/2}) for a positive velocity, offsets -3..+2;
// the negative-velocity stencil is its mirror image with the sign flipped, offsets -2..+3.
__host__ __device__ constexpr double uw5p(int o) {
  return o == -3 ? -2.0 / 60 : o == -2 ? 15.0 / 60 : o == -1 ? -60.0 / 60
       : o == 0 ? 20.0 / 60 : o == 1 ? 30.0 / 60 : o == 2 ? -3.0 / 60 : 0.0;
}
__host__ __device__ constexpr double uw5m(int o) { return -uw5p(-o); }

// WENO-5 face value (Jiang and Shu, J. Comput. Phys. 126, 1996) between h0 and hp1 from the
// upwind side: third-order candidates on {-2,-1,0}, {-1,0,1}, {0,1,2}, combined with weights
// d_k / (eps + beta_k)^2 (d = 1/10, 6/10, 3/10; beta_k the smoothness indicators), normalised.
// On smooth data the weights tend to d and the face value to the UW5 one.
constexpr double WENO_EPS = 1e-6;

template <typename T>
__device__ __forceinline__ T weno5(T hm2, T hm1, T h0, T hp1, T hp2) {
  const T q0 = (T(2) * hm2 - T(7) * hm1 + T(11) * h0) * T(1.0 / 6.0);
  const T q1 = (T(5) * h0 - hm1 + T(2) * hp1) * T(1.0 / 6.0);
  const T q2 = (T(2) * h0 + T(5) * hp1 - hp2) * T(1.0 / 6.0);
  const T d0 = hm2 - T(2) * hm1 + h0, e0 = hm2 - T(4) * hm1 + T(3) * h0;
  const T d1 = hm1 - T(2) * h0 + hp1, e1 = hm1 - hp1;
  const T d2 = h0 - T(2) * hp1 + hp2, e2 = T(3) * h0 - T(4) * hp1 + hp2;
  const T b0 = T(WENO_EPS) + T(13.0 / 12.0) * d0 * d0 + T(0.25) * e0 * e0;
  const T b1 = T(WENO_EPS) + T(13.0 / 12.0) * d1 * d1 + T(0.25) * e1 * e1;
  const T b2 = T(WENO_EPS) + T(13.0 / 12.0) * d2 * d2 + T(0.25) * e2 * e2;
  const T a0 = T(0.1) / (b0 * b0), a1 = T(0.6) / (b1 * b1), a2 = T(0.3) / (b2 * b2);
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// The two WENO-5 flux differences of population k = 4 i + j at a node: b points at the node in
// the LDS population tile (rows LXT apart), Jnb holds J of the rows q-3..q+3.  Along phi the
// stored values are used as they are (the reconstruction is shift-invariant, so deviations
// give the same differences); along theta the flux h = J f of the full population.
template <typename T, int I, int J, int K>
__device__ __forceinline__ void weno_advection(const T* b, const T (&Jnb)[7], T inv_rJdth,
                                               T n_ref, T& dph, T& dth) {
  if constexpr (J >= 2)
    dph = weno5(b[-2], b[-1], b[0], b[1], b[2]) - weno5(b[-3], b[-2], b[-1], b[0], b[1]);
  else
    dph = weno5(b[3], b[2], b[1], b[0], b[-1]) - weno5(b[2], b[1], b[0], b[-1], b[-2]);
  T h[7];
#pragma unroll
  for (int o = 0; o < 7; ++o) h[o] = Jnb[o] * (b[(o - 3) * LXT] + n_ref * T(rest_offset<T>(K)));
  if constexpr (I >= 2)
    dth = weno5(h[1], h[2], h[3], h[4], h[5]) - weno5(h[0], h[1], h[2], h[3], h[4]);
  else
    dth = weno5(h[6], h[5], h[4], h[3], h[2]) - weno5(h[5], h[4], h[3], h[2], h[1]);
  dth *= inv_rJdth;
}

// Per theta-row coefficients (one record per row q), all derived on the host in FP64.
template <typename T>
struct RowCoef {
  T bth_p[6];    // theta advection, v > 0: uw5p(o) J_{q+o} / (r J_q dtheta), o = -3..2
  T bth_m[6];    // theta advection, v < 0: uw5m(o) J_{q+o} / (r J_q dtheta), o = -2..3
  T inv_Jdph;    // 1 / (J_q dphi)
  T J;           // J_q = R + r cos theta_q
  T G;           // sin theta_q / J_q (connection coefficient)
  T lap_n;       // J_{q+1/2} / (r^2 J_q dtheta^2)
  T lap_s;       // J_{q-1/2} / (r^2 J_q dtheta^2)
  T lap_p;       // 1 / (J_q^2 dphi^2)
  T inv_2Jdph;   // 1 / (2 J_q dphi)
  T inv_2rJdth;  // 1 / (2 r J_q dtheta)
  T bsum_p;      // sum of bth_p: the theta advection of a theta-independent value (v > 0)
  T bsum_m;      // sum of bth_m (v < 0)
  // fourth-order Cahn-Hilliard operators (TLB_CH4)
  T l4[4];        // J at theta_{q-3/2}, _{q-1/2}, _{q+1/2}, _{q+3/2}, over 576 r^2 J_q dtheta^2
  T lp4;          // 1 / (12 J_q^2 dphi^2)
  T inv_12Jdph;   // 1 / (12 J_q dphi)
  T inv_12rJdth;  // 1 / (12 r J_q dtheta)
};

template <typename T>
struct Consts {
  T A, kappa, M, inv_tau, inv_2rdth, dt;
  T n_ref;  // reference density of the stored deviations (FP32)
  int ch_adv;
  T inv_12rdth;  // 1 / (12 r dtheta) (TLB_CH4)
};

template <typename T>
struct StageArgs {
  const T* fin;    // stage input populations (read with halos)
  const T* phin;   // stage input order parameter
  const T* f0;     // y^n populations (read at the node only; may alias fout)
  const T* phi0;
  T* fout;
  T* phiout;
  const RowCoef<T>* rows;
  int nt, np, ntx, nty;
  long long plane;  // nt * np
  T a0, b1;         // out = a0 * y^n + b1 * (y_s + dt L(y_s))
  int has_y0;       // a0 != 0
  Consts<T> c;
  const T* phib;    // FP32: the base of the order parameter (phin, phi0, phiout hold deviations)
  const T* mu4;     // TLB_CH4: mu, J u^theta phi, u^phi phi of the stage input (prepass)
  const T* P4;
  const T* Q4;
};

// The fourth-order Cahn-Hilliard prepass (TLB_CH4) of one Runge-Kutta stage: per node of the
// stage input, the chemical potential with the fourth-order surface Laplacian (eq. mu) and the
// two Cahn-Hilliard advection fluxes J u^theta phi and u^phi phi; the stage kernel then reads
// them as halo tiles like the populations.
template <typename T>
struct Ch4Args {
  const T* f;
  const T* phi;
  const T* phib;  // base of the order parameter (FP32) or NULL
  T* mu;
  T* P;
  T* Q;
  const RowCoef<T>* rows;
  int nt, np;
  long long plane;
  T A, kappa, n_ref;
};

__device__ __forceinline__ int wrapi(int x, int n) {
  // the indices wrapped here are almost always in range or one period off; only grids smaller
  // than a halo need the division
  if (x >= 0 && x < n) return x;
  if (x < 0 && x >= -n) return x + n;
  if (x >= n && x < 2 * n) return x - n;
  int m = x % n;
  return m < 0 ? m + n : m;
}

// The order parameter at index i: FP32 grids store it as base + deviation (the deviation plane
// d, the base plane b); FP64 grids store it whole (b = NULL).
template <typename T>
__device__ __forceinline__ T phi_val(const T* d, const T* b, long long i) {
  return b ? d[i] + b[i] : d[i];
}
template <typename T>
__device__ __forceinline__ double phi_val64(const T* d, const T* b, long long i) {
  return b ? (double)d[i] + (double)b[i] : (double)d[i];
}

// Block -> tile mapping: consecutive hardware blocks go round-robin over the 8 XCDs; give
// XCD x the contiguous tile range [start_x, start_x + count_x) of a banded tile order (see
// band_tile), so that the blocks resident on one XCD at a time form a compact patch whose
// halo rows and halo cache lines are shared through that XCD's L2.
__host__ __device__ __forceinline__ int xcd_tile(int b, int nblk) {
  const int xcd = b & 7, local = b >> 3;
  const int full = nblk >> 3, rem = nblk & 7;
  return xcd < rem ? xcd * (full + 1) + local : rem * (full + 1) + (xcd - rem) * full + local;
}

// Banded tile order: the tile columns are cut into bands of BAND columns (the last band may be
// narrower); bands follow each other, and inside a band the tiles go row by row.
#ifndef TLB_BAND
#define TLB_BAND 8
#endif
constexpr int BAND = TLB_BAND;
__host__ __device__ __forceinline__ void band_tile(int t, int ntx, int nty, int& tx, int& ty) {
  const int band = t / (BAND * nty);
  const int width = min(BAND, ntx - band * BAND);
  const int local = t - band * BAND * nty;
  ty = local / width;
  tx = band * BAND + (local - ty * width);
}

// Empty register-to-register asm: the value must exist at this point of the program, so its
// computation cannot be moved past it (used to stop arithmetic from sinking across barriers).
__device__ __forceinline__ void pin_reg(float& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin_reg(double& x) { asm volatile("" : "+v"(x)); }

// s_waitcnt immediate (gfx9 encoding): wait until at most `vm` vector-memory operations of this
// wave are outstanding and all LDS operations are done; exp count not waited on.
template <int VM>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(VM >= 0 && VM < 64, "vmcnt out of range");
  __builtin_amdgcn_s_waitcnt((VM & 0xF) | (0x7 << 4) | (0x0 << 8) | (((VM >> 4) & 0x3) << 14));
}

typedef __attribute__((address_space(3))) void lds_void_t;
// word 3 of a raw buffer resource descriptor on the gfx9 family (32-bit dword format)
constexpr int BUF_DWORD3 = 0x00020000;

// Asynchronous copy (LDS DMA) of one halo tile: ROWS rows of LXT elements of T, starting at
// row q0 + R0 and column s0 - CX of a plane, stored row-major in LDS.  The copy unit is a
// 16-byte chunk (VEC, possible when the row length n_phi keeps every chunk aligned and inside
// one period) or a 4-byte word.  Copy instruction i of wave w moves the contiguous units
// [i NT + w c_i, i NT + (w+1) c_i) with c_i = ceil(units of instruction i / waves), lanes past
// the tile masked off; every wave thus issues every instruction, so all waves count the same
// number of outstanding copies per tile (the waits below rely on it).
template <typename T, bool VEC, int ROWS, int R0, int NT>
struct TileCopy {
  static constexpr int NWAVE = NT / 64;
  static constexpr int UNIT = VEC ? 16 : 4;
  static constexpr int ROW_UNITS = LXT * (int)sizeof(T) / UNIT;
  static constexpr int UNITS = ROWS * ROW_UNITS;
  static constexpr int INSTR = (UNITS + NT - 1) / NT;  // copy instructions per wave per tile
  __host__ __device__ static constexpr int chunk(int i) {
    const int v = UNITS - i * NT < NT ? UNITS - i * NT : NT;
    return (v + NWAVE - 1) / NWAVE;
  }
  __host__ __device__ static constexpr bool every_wave_copies() {
    for (int i = 0; i < INSTR; ++i) {
      const int v = UNITS - i * NT < NT ? UNITS - i * NT : NT;
      if (chunk(i) > 64 || (NWAVE - 1) * chunk(i) >= v) return false;
    }
    return true;
  }
  static_assert(every_wave_copies(), "a wave would issue no copy for some instruction");
  static_assert((LXT * (int)sizeof(T)) % UNIT == 0, "row is not a whole number of units");

  unsigned voff[INSTR];
  bool valid[INSTR];

  __device__ __forceinline__ void init(int lane, int wave, int q0, int s0, int nt, int np,
                                       bool interior) {
#pragma unroll
    for (int i = 0; i < INSTR; ++i) {
      const int u = i * NT + wave * chunk(i) + lane;
      valid[i] = lane < chunk(i) && u < UNITS;
      unsigned off = 0;
      if (valid[i]) {
        const int row = u / ROW_UNITS, uc = u - row * ROW_UNITS;
        int col, byte_in_elem = 0;
        if constexpr (VEC) {
          col = uc * (UNIT / (int)sizeof(T));
        } else {
          col = uc / ((int)sizeof(T) / 4);
          byte_in_elem = 4 * (uc - col * ((int)sizeof(T) / 4));
        }
        int gq = q0 + R0 + row, gs = s0 - CX + col;
        if (!interior) {
          gq = wrapi(gq, nt);
          gs = wrapi(gs, np);
        }
        off = (unsigned)(gq * np + gs) * (unsigned)sizeof(T) + (unsigned)byte_in_elem;
      }
      voff[i] = off;
    }
  }
  // copy from the plane at `base` (plane_bytes long) into the LDS tile `lds`: buffer loads
  // with the plane in a resource descriptor (range-checked by the hardware), written by the
  // load unit straight into LDS
  __device__ __forceinline__ void issue(const T* base, unsigned plane_bytes, T* lds,
                                        int wave) const {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, plane_bytes, BUF_DWORD3);
#pragma unroll
    for (int i = 0; i < INSTR; ++i) {
      char* l = reinterpret_cast<char*>(lds) + UNIT * (i * NT + wave * chunk(i));
      if (valid[i])
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)l, UNIT, voff[i], 0, 0, 0);
    }
  }
};

// chemical potential (eq. mu) at local node (y, x) in [-1, TY] x [-1, TX] of the phi tile
template <typename T>
__device__ __forceinline__ T mu_at(const T* sPhi, int y, int x, const RowCoef<T>& rc, T A,
                                   T kappa) {
  const int c = (y + 2) * LXT + (x + CX);
  const T ph = sPhi[c];
  const T lap = rc.lap_n * (sPhi[c + LXT] - ph) - rc.lap_s * (ph - sPhi[c - LXT]) +
                rc.lap_p * (sPhi[c + 1] - T(2) * ph + sPhi[c - 1]);
  return A * ph * (ph * ph - T(1)) - kappa * lap;
}

// population ring depth D: while a group of PB populations is used, the copies of the next
// D - PB are in flight.  y^n of the node (stages 2 and 3) is loaded during the population loop
// instead of in the epilogue, which hides its latency; costs 16 (FP32) or 32 (FP64) VGPRs
#ifndef TLB_PREFETCH_Y0_32
#define TLB_PREFETCH_Y0_32 1
#endif
#ifndef TLB_PREFETCH_Y0_64
#define TLB_PREFETCH_Y0_64 0
#endif
#ifndef TLB_RING32
#define TLB_RING32 6
#endif
#ifndef TLB_RING64
#define TLB_RING64 6
#endif
// 1 / x: the hardware reciprocal (1 ulp) in FP32, where the correctly rounded division would
// cost about ten instructions of an issue-bound kernel; a correctly rounded division in FP64.
template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (std::is_same<T, float>::value)
    return __builtin_amdgcn_rcpf(x);
  else
    return T(1) / x;
}

// Address of a node's value in plane k: a wavefront-uniform base (row and plane, scalar
// registers) plus the lane's 32-bit byte offset, so that the access takes the scalar-base form
// instead of a 64-bit vector address per plane.
template <typename P>
__device__ __forceinline__ P* at_node(P* base, long long uniform_elems, unsigned lane_bytes) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(base + uniform_elems) + lane_bytes);
}

// Streaming (nontemporal) accesses for the stage outputs and the y^n loads, used on grids whose
// state copies are far larger than the 256 MB last-level cache: there the output streams gain
// nothing from being cached, while on grids that fit it the next stage reads them from there.
template <bool NT, typename T>
__device__ __forceinline__ void put(T* p, T v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
template <bool NT, typename T>
__device__ __forceinline__ T get_y0(const T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// Populations are consumed in groups of PB: one wait and one block barrier per group, after
// which the ring slots of the previous group are refilled with populations k+D-PB .. k+D-1.
// ops_after_copy: the vector-memory instructions a wave issues after the copy of population m
// and before the wait of the group starting at population k, which may still be outstanding
// when population m has landed (vmcnt counts in issue order).  Issue order: the
// order-parameter copy, populations 0..D-1 (DW instructions each), the phi^n load (Y0), then
// in group k the refill copies followed by the y^n loads of the group's populations (Y0).
template <int D, int DW, bool Y0, int PB>
__host__ __device__ constexpr int ops_after_copy(int m, int k) {
  int count = 0;
  bool seen = false;
  for (int p = 0; p < D; ++p) {
    if (seen) count += DW;
    if (p == m) seen = true;
  }
  if (Y0 && seen) count += 1;
  for (int g = 0; g < k; g += PB) {
    if (g >= PB)
      for (int p = g + D - PB; p < g + D && p < 16; ++p) {
        if (seen) count += DW;
        if (p == m) seen = true;
      }
    if (Y0 && seen) count += PB;
  }
  return count;
}

// populations consumed per block barrier (a sweep of 1, 2 and 4 with ring depths 4-8 on both
// precisions: 2 with depth 6 is fastest, by 0.4-2 %)
#ifndef TLB_GROUP32
#define TLB_GROUP32 2
#endif
#ifndef TLB_GROUP64
#define TLB_GROUP64 2
#endif
template <typename T>
struct Ring {
  static constexpr int D = sizeof(T) == 4 ? TLB_RING32 : TLB_RING64;
  static constexpr int PB = sizeof(T) == 4 ? TLB_GROUP32 : TLB_GROUP64;  // populations per barrier
  static constexpr bool PREFETCH = sizeof(T) == 4 ? TLB_PREFETCH_Y0_32 : TLB_PREFETCH_Y0_64;
  static_assert(D % PB == 0 && 16 % PB == 0 && D > PB, "ring depth and group size");
};

// One right-hand-side evaluation + Runge-Kutta combine for the tile (tx, ty) of the grid
// described by `a`, by a block of Tile<TY>::NT threads.  GENREF: the FP32 storage reference
// density is read from the arguments; otherwise it is the constant 1 (every grid near unit
// density), whose products the compiler folds away.
template <typename T, bool VEC, int TY, bool WENO = false, bool STREAM = false,
          bool GENREF = false, bool CH4 = false>
__device__ __forceinline__ void stage_tile(const StageArgs<T>& a, const int tx, const int ty) {
// (the body is device code: the host pass of the single-source compiler skips it; with both
// advection variants instantiated, that pass otherwise rejects the call from the batch kernel)
#if defined(__HIP_DEVICE_COMPILE__)
  using TL = Tile<TY>;
  constexpr int NT = TL::NT, LY = TL::LY, PY = TL::PY, NRING = TL::NRING;
  constexpr int D = Ring<T>::D;
  using CopyF = TileCopy<T, VEC, LY, -HY, NT>;
  using CopyPhi = TileCopy<T, VEC, PY, -2, NT>;
  constexpr int DW = CopyF::INSTR;
  constexpr int TILE_SLOTS = LY * LXT;
  static_assert(D >= 2 && D <= 8, "ring depth");
  // the ring slots are separate LDS objects, so that the compiler can see that reading one
  // slot does not depend on the copies still in flight into the others
  __shared__ T sF0[TILE_SLOTS], sF1[TILE_SLOTS], sF2[D > 2 ? TILE_SLOTS : 1],
      sF3[D > 3 ? TILE_SLOTS : 1], sF4[D > 4 ? TILE_SLOTS : 1], sF5[D > 5 ? TILE_SLOTS : 1],
      sF6[D > 6 ? TILE_SLOTS : 1], sF7[D > 7 ? TILE_SLOTS : 1];
  auto slot = [&](auto sc) -> T* {
    constexpr int S = decltype(sc)::value % D;
    if constexpr (S == 0) return sF0;
    else if constexpr (S == 1) return sF1;
    else if constexpr (S == 2) return sF2;
    else if constexpr (S == 3) return sF3;
    else if constexpr (S == 4) return sF4;
    else if constexpr (S == 5) return sF5;
    else if constexpr (S == 6) return sF6;
    else return sF7;
  };
  __shared__ T sPhi[PY * LXT];
  __shared__ T sPhiB[stores_deviation<T>() ? PY * LXT : 1];  // FP32: base tile, then phi itself
  // TLB_CH4: mu, J u^theta phi and u^phi phi of the prepass, halo tiles like the populations
  __shared__ T sMu4[CH4 ? TILE_SLOTS : 1], sP4[CH4 ? TILE_SLOTS : 1], sQ4[CH4 ? TILE_SLOTS : 1];
  __shared__ T sMu[(TY + 2) * (TX + 2)];
  __shared__ T sPt[(TY + 2) * TX];  // J u^theta phi on the tile and the rows above/below
  __shared__ T sPp[TY * (TX + 2)];  // u^phi phi on the tile and the columns left/right

  const int tid = threadIdx.x;
  const int lx = tid & (TX - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ly = wave;  // wavefront-uniform row of the tile
  const int nt = a.nt, np = a.np;
  const int q0 = ty * TY, s0 = tx * TX;
  const int q = q0 + ly, s = s0 + lx;
  const bool active = (q < nt) && (s < np);
  const int qw = __builtin_amdgcn_readfirstlane(q < nt ? q : wrapi(q, nt));
  // this row's coefficients, read once (scalar loads: the row is wavefront-uniform) and kept
  // in registers -- a reference would be re-read from memory after every barrier
  const RowCoef<T> rc = a.rows[qw];
  // no periodic wrap needed for any halo of this tile
  const bool interior = q0 >= HY && q0 + TY + HY <= nt && s0 >= CX && s0 + LXT - CX <= np;

  // ---- asynchronous halo copies: the order parameter, then populations 0..D-1 (one per slot);
  //      from iteration k = 1 on, iteration k refills slot (k-1) mod D with population k+D-1
  CopyPhi cp_phi;
  CopyF cp_f;
  cp_phi.init(lx, wave, q0, s0, nt, np, interior);
  cp_f.init(lx, wave, q0, s0, nt, np, interior);
  const unsigned plane_bytes = (unsigned)(a.plane * (long long)sizeof(T));
  cp_phi.issue(a.phin, plane_bytes, sPhi, wave);
  if constexpr (stores_deviation<T>()) cp_phi.issue(a.phib, plane_bytes, sPhiB, wave);
  if constexpr (CH4) {  // issued before the populations: the loop's first wait covers them
    cp_f.issue(a.mu4, plane_bytes, sMu4, wave);
    cp_f.issue(a.P4, plane_bytes, sP4, wave);
    cp_f.issue(a.Q4, plane_bytes, sQ4, wave);
  }
  static_for<0, D>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    cp_f.issue(a.fin + k * a.plane, plane_bytes, slot(ic<k>{}), wave);
  });

  // ---- ring role: one cross-ring node per thread for tid < NRING
  int ry, rx;
  if (tid < TX) { ry = -1; rx = tid; }
  else if (tid < 2 * TX) { ry = TY; rx = tid - TX; }
  else if (tid < 2 * TX + TY) { ry = tid - 2 * TX; rx = -1; }
  else { ry = tid - 2 * TX - TY; rx = TX; }
  const bool ring = !CH4 && tid < NRING;  // CH4 takes the ring's fluxes from the prepass
  if (!ring) { ry = 0; rx = 0; }
  const RowCoef<T>& rrc = a.rows[wrapi(q0 + ry, nt)];

  // The order-parameter tile is read only after the population loop (chemical potential,
  // force, Cahn-Hilliard): the loop's first wait covers its copy, which was issued first, and
  // reading it here would make the compiler drain every copy in flight before the loop.
  static_assert(CopyPhi::INSTR + DW * D < 64, "outstanding copies exceed the vmcnt range");

  // ---- stream the 16 populations through the LDS ring
  T f[16], adv[16];
  // y^n at this node for the Runge-Kutta combine, loaded during the population loop
  constexpr bool PF = Ring<T>::PREFETCH;
  T yn[PF ? 16 : 1];
  const long long row0 = (long long)qw * np;  // wavefront-uniform
  const unsigned lane_bytes = (unsigned)(s < np ? s : 0) * (unsigned)sizeof(T);
  T phin = T(0);
  if constexpr (PF)
    if (a.has_y0) phin = get_y0<STREAM>(at_node(a.phi0, row0, lane_bytes));
  // moments of this node and of the ring node, both summed population by population in the
  // same order, so that a node's moments (and all that follows) do not depend on whether it
  // is inside a tile or in a neighbour's ring -- results are independent of the tile shape
  T n = T(0), nut = T(0), nup = T(0);
  T rn = T(0), rut = T(0), rup = T(0);
  const int cN = (ly + HY) * LXT + lx + CX;  // this node in the population tile
  const int cR = (ry + HY) * LXT + rx + CX;  // the ring node
  const T inv_Jdph = rc.inv_Jdph;
  T n_ref = T(1);
  if constexpr (GENREF) n_ref = a.c.n_ref;
  // WENO: J of rows q-3..q+3 (wavefront-uniform scalar loads) and 1 / (r J dtheta)
  T Jnb[7];
  T inv_rJdth = T(0);
  if constexpr (WENO) {
#pragma unroll
    for (int o = 0; o < 7; ++o) Jnb[o] = a.rows[wrapi(qw + o - 3, nt)].J;
    inv_rJdth = T(2) * rc.inv_2rJdth;
  }

  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int i = k >> 2, j = k & 3;
    constexpr int PB = Ring<T>::PB;
    if constexpr (k % PB == 0) {
      // wait until populations k .. k+PB-1 have landed: at most the vector-memory instructions
      // issued after the last one's copy may be outstanding (in FP32 stages with y^n these
      // include the y^n loads)
      constexpr int m = k + PB - 1;
      if constexpr (PF) {
        if (a.has_y0) wait_vm_lgkm0<ops_after_copy<D, DW, true, PB>(m, k)>();
        else wait_vm_lgkm0<ops_after_copy<D, DW, false, PB>(m, k)>();
      } else {
        wait_vm_lgkm0<ops_after_copy<D, DW, false, PB>(m, k)>();
      }
      __builtin_amdgcn_s_barrier();
      // every wave is past populations k-PB .. k-1: their ring slots can be refilled
      if constexpr (k >= PB)
        static_for<k + D - PB, (k + D < 16 ? k + D : 16)>([&](auto pc) {
          constexpr int p = decltype(pc)::value;
          cp_f.issue(a.fin + p * a.plane, plane_bytes, slot(ic<p>{}), wave);
        });
      if constexpr (PF)
        if (a.has_y0)
          static_for<k, k + PB>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            yn[p] = get_y0<STREAM>(at_node(a.f0, p * a.plane + row0, lane_bytes));
          });
    }
    const T* buf = slot(ic<k>{});
    f[k] = buf[cN];
    n += f[k];
    nut += T(vel(i)) * f[k];
    nup += T(vel(j)) * f[k];
    // phi direction: sum_o uw5(o) f_{s+o}, upwind side by the sign of v_j
    T dph, dth;
    if constexpr (WENO) {
      weno_advection<T, i, j, k>(buf + cN, Jnb, inv_rJdth, n_ref, dph, dth);
    } else {
    if constexpr (j >= 2) {
      dph = T(uw5p(-3)) * buf[cN - 3];
      static_for<-2, 3>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        dph += T(uw5p(o)) * buf[cN + o];
      });
    } else {
      dph = T(uw5m(-2)) * buf[cN - 2];
      static_for<-1, 4>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        dph += T(uw5m(o)) * buf[cN + o];
      });
    }
    // theta direction: sum_o uw5(o) J_{q+o} / (r J_q dtheta) f_{q+o}
    if constexpr (i >= 2) {
      dth = rc.bth_p[0] * buf[cN - 3 * LXT];
      static_for<-2, 3>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        dth += rc.bth_p[o + 3] * buf[cN + o * LXT];
      });
    } else {
      dth = rc.bth_m[0] * buf[cN - 2 * LXT];
      static_for<-1, 4>([&](auto oc) {
        constexpr int o = decltype(oc)::value;
        dth += rc.bth_m[o + 2] * buf[cN + o * LXT];
      });
    }
    // deviation storage: the constant n_ref w_i w_j drops out of the phi differences (their
    // weights sum to zero) but not out of the J-weighted theta differences
    if constexpr (stores_deviation<T>())
      dth += (n_ref * T(rest_offset<T>(k))) * (i >= 2 ? rc.bsum_p : rc.bsum_m);
    }
    adv[k] = T(-vel(i)) * dth + (T(-vel(j)) * inv_Jdph) * dph;
    if (ring) {
      const T fr = buf[cR];
      rn += fr;
      rut += T(vel(i)) * fr;
      rup += T(vel(j)) * fr;
    }
    // keep the arithmetic of this population here: without the pin the compiler sinks it to
    // the end of the kernel and holds every stencil value of all 16 populations live
    pin_reg(adv[k]);
    pin_reg(f[k]);
    pin_reg(n);
    pin_reg(nut);
    pin_reg(nup);
    pin_reg(rn);
    pin_reg(rut);
    pin_reg(rup);
  });

  // ---- FP32: the order-parameter tiles hold the stage input's deviation (sPhi) and the base
  //      (sPhiB); their sum, the order parameter itself, replaces the base tile.  dsn is the
  //      node's own deviation, which the Runge-Kutta combine updates.
  const T* sPhiF = sPhi;
  T dsn = T(0);
  if constexpr (stores_deviation<T>()) {
    dsn = sPhi[(ly + 2) * LXT + lx + CX];
    for (int i = tid; i < PY * LXT; i += NT) sPhiB[i] += sPhi[i];
    __syncthreads();
    sPhiF = sPhiB;
  }

  // ---- chemical potential on the tile and the ring (the order-parameter tile has landed:
  //      its copy was issued before population 0's)
  if constexpr (!CH4) sMu[(ly + 1) * (TX + 2) + lx + 1] = mu_at(sPhiF, ly, lx, rc, a.c.A, a.c.kappa);
  if (ring) sMu[(ry + 1) * (TX + 2) + rx + 1] = mu_at(sPhiF, ry, rx, rrc, a.c.A, a.c.kappa);

  // ---- CH fluxes of the tile and the ring
  // with deviation storage the sums above are n - n_ref; dn keeps that small difference
  const T dn = n;
  if constexpr (stores_deviation<T>()) {
    n += n_ref;
    rn += n_ref;
  }
  const T inv_n = recip(n);
  const T ut = nut * inv_n, up = nup * inv_n;
  const T phc = sPhiF[(ly + 2) * LXT + lx + CX];
  if constexpr (!CH4) {
    sPt[(ly + 1) * TX + lx] = rc.J * ut * phc;
    sPp[ly * (TX + 2) + lx + 1] = up * phc;
  }
  if (ring) {
    const T phr = sPhiF[(ry + 2) * LXT + rx + CX];
    const T inv_rn = recip(rn);
    if (ry < 0 || ry >= TY) sPt[(ry + 1) * TX + rx] = rrc.J * (rut * inv_rn) * phr;
    else sPp[ry * (TX + 2) + rx + 1] = (rup * inv_rn) * phr;
  }
  __syncthreads();

  // ---- interface force n F = -phi grad mu and the Cahn-Hilliard right-hand side
  T Fth, Fph, Lphi;
  if constexpr (CH4) {
    // fourth-order central grad mu, the fourth-order surface Laplacian of mu (staggered along
    // theta: face gradients (m_{a-1} - 27 m_a + 27 m_{a+1} - m_{a+2}) at the faces a+1/2,
    // a = q-2 .. q+1, weighted by J_face / (576 r^2 J dtheta^2) with (1, -27, 27, -1); the
    // five-point fourth-order difference along phi) and fourth-order central flux differences
    const T* m = sMu4 + cN;
    auto G = [&](int o) {  // face gradient numerator at the face (q + o) + 1/2
      return m[(o - 1) * LXT] - T(27) * m[o * LXT] + T(27) * m[(o + 1) * LXT] - m[(o + 2) * LXT];
    };
    const T dmu_th = (m[-2 * LXT] - T(8) * m[-LXT]) + (T(8) * m[LXT] - m[2 * LXT]);
    const T dmu_ph = (m[-2] - T(8) * m[-1]) + (T(8) * m[1] - m[2]);
    Fth = -phc * dmu_th * a.c.inv_12rdth * inv_n;
    Fph = -phc * dmu_ph * rc.inv_12Jdph * inv_n;
    const T lap_th = rc.l4[0] * G(-2) - T(27) * (rc.l4[1] * G(-1)) + T(27) * (rc.l4[2] * G(0)) -
                     rc.l4[3] * G(1);
    const T lap_ph = rc.lp4 * ((-m[-2] + T(16) * m[-1]) - T(30) * m[0] + (T(16) * m[1] - m[2]));
    Lphi = a.c.M * (lap_th + lap_ph);
    if (a.c.ch_adv) {
      const T* P = sP4 + cN;
      const T* Q = sQ4 + cN;
      Lphi -= ((P[-2 * LXT] - T(8) * P[-LXT]) + (T(8) * P[LXT] - P[2 * LXT])) * rc.inv_12rJdth +
              ((Q[-2] - T(8) * Q[-1]) + (T(8) * Q[1] - Q[2])) * rc.inv_12Jdph;
    }
  } else {
    const int cm = (ly + 1) * (TX + 2) + lx + 1;
    const T mu_c = sMu[cm], mu_n = sMu[cm + TX + 2], mu_s = sMu[cm - (TX + 2)];
    const T mu_e = sMu[cm + 1], mu_w = sMu[cm - 1];
    Fth = -phc * (mu_n - mu_s) * a.c.inv_2rdth * inv_n;
    Fph = -phc * (mu_e - mu_w) * rc.inv_2Jdph * inv_n;
    const T lapmu = rc.lap_n * (mu_n - mu_c) - rc.lap_s * (mu_c - mu_s) +
                    rc.lap_p * (mu_e - T(2) * mu_c + mu_w);
    Lphi = a.c.M * lapmu;
    if (a.c.ch_adv) {
      const int ct = (ly + 1) * TX + lx, cp = ly * (TX + 2) + lx + 1;
      Lphi -= (sPt[ct + TX] - sPt[ct - TX]) * rc.inv_2rJdth +
              (sPp[cp + 1] - sPp[cp - 1]) * rc.inv_2Jdph;
    }
  }


  const T dt = a.c.dt, a0 = a.a0, b1 = a.b1;
  const bool y0 = a.has_y0;
  if (active) {
    // the stored value at the node: FP32 the deviation from the base, FP64 phi itself
    const T own = stores_deviation<T>() ? dsn : phc;
    const T ys = own + dt * Lphi;
    T yn0 = phin;
    if constexpr (!PF)
      if (y0) yn0 = *at_node(a.phi0, row0, lane_bytes);
    T out = ys;
    if constexpr (stores_deviation<T>()) {
      // FP32: a0 d^n + b1 (d_s + dt L) as d^n + b1 ((d_s - d^n) + dt L) (a0 + b1 = 1), on the
      // deviations from the base, which are small where phi sits near +-1 in the bulk: there
      // the increments are far below half an ulp of 1 and would be lost on phi itself
      if (y0) out = yn0 + b1 * ((own - yn0) + dt * Lphi);
    } else {
      if (y0) out = a0 * yn0 + b1 * ys;
    }
    put<STREAM>(at_node(a.phiout, row0, lane_bytes), out);
  }

  // ---- equilibrium (eq. feq) as a cubic in xi = v.u:
  //      f_eq = n w_i w_j [c0 (1 + xi) + xi^2/2 + xi^3/6],  c0 = 1 - u^2/2
  // ---- velocity derivatives (section II C): (df/dv^theta)_ij = sum_m K_im f_mj,
  //      (df/dv^phi)_ij = sum_m K_jm f_im, (d(f v^phi)/dv^phi)_ij = sum_m K_jm v_m f_im, so the
  //      force and connection terms combine into
  //      S_ij = (G v_j^2 - F^theta) sum_m K_im f_mj - sum_m K_jm (F^phi + G v_i v_m) f_im.
  const T c0 = T(1) - T(0.5) * (ut * ut + up * up);
  const T G = rc.G;
  T g[16];
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int i = k >> 2, m = k & 3;
    g[k] = (Fph + G * T(vel(i) * vel(m))) * f[k];
  });
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int i = k >> 2, j = k & 3;
    T dvt = T(0), dvp = T(0);
    static_for<0, 4>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      dvt += T(kh(i, m)) * f[4 * m + j];
      dvp += T(kh(j, m)) * g[4 * i + m];
    });
    if constexpr (stores_deviation<T>()) {
      // the velocity derivatives of the stored constant n_ref w_i w_j, in closed form
      dvt += n_ref * T(wgt(j) * kw(i));
      dvp += n_ref * (T(wgt(i)) * (Fph * T(kw(j)) + G * T(vel(i) * kvw(j))));
    }
    const T xi = T(vel(i)) * ut + T(vel(j)) * up;
    T relax;  // f_eq - f, in the stored representation
    if constexpr (stores_deviation<T>()) {
      // f_eq - n_ref w_i w_j = w_i w_j (n_ref p1 + dn (1 + p1)), p1 = poly - 1, all small
      const T p1 = T(-0.5) * (ut * ut + up * up) + xi * (c0 + xi * (T(0.5) + xi * T(1.0 / 6.0)));
      relax = T(wgt(i) * wgt(j)) * (n_ref * p1 + dn * (T(1) + p1)) - f[k];
    } else {
      const T poly = c0 + xi * (c0 + xi * (T(0.5) + xi * T(1.0 / 6.0)));
      relax = (n * T(wgt(i) * wgt(j))) * poly - f[k];
    }
    const T L = adv[k] + (G * T(vel(j) * vel(j)) - Fth) * dvt - dvp + relax * a.c.inv_tau;
    const T ys = f[k] + dt * L;
    if (active) {
      T* dst = at_node(a.fout, k * a.plane + row0, lane_bytes);
      if constexpr (PF)
        put<STREAM>(dst, y0 ? a0 * yn[k] + b1 * ys : ys);
      else
        put<STREAM>(dst, y0 ? a0 * *at_node(a.f0, k * a.plane + row0, lane_bytes) + b1 * ys : ys);
    }
  });
#endif
}

// Minimum waves per SIMD the compiler is asked to keep room for (register budget 512 / waves
// VGPRs); 1 leaves the allocation free.
#ifndef TLB_WPE32
#define TLB_WPE32 1
#endif
#ifndef TLB_WPE64
#define TLB_WPE64 1
#endif
template <typename T>
struct StageWaves {
  static constexpr int value = sizeof(T) == 4 ? TLB_WPE32 : TLB_WPE64;
};

template <typename T, bool VEC, int TY, bool WENO = false, bool STREAM = false,
          bool GENREF = false, bool CH4 = false>
__global__ __launch_bounds__(Tile<TY>::NT) __attribute__((amdgpu_waves_per_eu(
    StageWaves<T>::value))) void tlb_stage_kernel(StageArgs<T> a) {
  const int tile = xcd_tile(blockIdx.x, a.ntx * a.nty);
  int tx, ty;
  band_tile(tile, a.ntx, a.nty, tx, ty);
  stage_tile<T, VEC, TY, WENO, STREAM, GENREF, CH4>(a, tx, ty);
}

// The fourth-order surface Laplacian (TLB_CH4) of a plane h at node (q, s), read from global
// memory: staggered along theta (face gradient numerators h_{a-1} - 27 h_a + 27 h_{a+1} -
// h_{a+2} at the faces a+1/2, a = q-2 .. q+1, weighted by rc.l4 with (1, -27, 27, -1)), the
// five-point fourth-order difference along phi.
template <typename T>
__device__ __forceinline__ T lap4_at(const T* h, const T* hb, const RowCoef<T>& rc, int q,
                                     int s, int nt, int np) {
  T c[7];  // rows q-3 .. q+3 of column s
#pragma unroll
  for (int o = -3; o <= 3; ++o) c[o + 3] = phi_val(h, hb, (long long)wrapi(q + o, nt) * np + s);
  auto G = [&](int o) { return c[o + 2] - T(27) * c[o + 3] + T(27) * c[o + 4] - c[o + 5]; };
  const long long row = (long long)q * np;
  const T e1 = phi_val(h, hb, row + wrapi(s + 1, np)), e2 = phi_val(h, hb, row + wrapi(s + 2, np));
  const T w1 = phi_val(h, hb, row + wrapi(s - 1, np)), w2 = phi_val(h, hb, row + wrapi(s - 2, np));
  const T lap_th = rc.l4[0] * G(-2) - T(27) * (rc.l4[1] * G(-1)) + T(27) * (rc.l4[2] * G(0)) -
                   rc.l4[3] * G(1);
  const T lap_ph = rc.lp4 * ((-w2 + T(16) * w1) - T(30) * c[3] + (T(16) * e1 - e2));
  return lap_th + lap_ph;
}

// TLB_CH4 prepass, one thread per node (see Ch4Args)
template <typename T>
__global__ __launch_bounds__(256) void tlb_ch4_prep_kernel(Ch4Args<T> a) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.plane) return;
  const int q = (int)(x / a.np), s = (int)(x - (long long)q * a.np);
  T n = T(0), nut = T(0), nup = T(0);
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const T fk = a.f[k * a.plane + x];
    n += fk;
    nut += T(vel(k >> 2)) * fk;
    nup += T(vel(k & 3)) * fk;
  });
  if constexpr (stores_deviation<T>()) n += a.n_ref;
  const T inv_n = recip(n);
  const RowCoef<T> rc = a.rows[q];
  const T ph = phi_val(a.phi, a.phib, x);
  a.mu[x] = a.A * ph * (ph * ph - T(1)) - a.kappa * lap4_at(a.phi, a.phib, rc, q, s, a.nt, a.np);
  a.P[x] = rc.J * (nut * inv_n) * ph;
  a.Q[x] = (nup * inv_n) * ph;
}

// One stage for an ensemble of grids in one launch, one block per tile.  table[3 g + stage - 1]
// holds the stage arguments of grid g; tile_begin[g] is the first tile of grid g in the
// concatenated tile order (tile_begin[n] = total).  Blocks go round-robin to the 8 XCDs, and
// XCD x takes a contiguous range of that order, so that each XCD's L2 serves whole grids, or
// compact parts of them, as for a single grid.  (A persistent form, the resident blocks walking
// the tiles, was 10-14 % slower: each tile's copies then queued behind the previous tile's
// stores.)
// A pointer read from device memory (the batch's argument table) is generic to the compiler,
// which then accesses it with flat instructions; those also count against the LDS wait
// counter, so every wait for an LDS read would wait for the global loads in flight too.  Cast
// through the global address space, the pointer gets global (and scalar) instructions, as a
// kernel argument does.
template <typename P>
__device__ __forceinline__ P* global_ptr(P* p) {
  return (P*)((__attribute__((address_space(1))) P*)reinterpret_cast<uintptr_t>(p));
}

template <typename T, bool VEC, int TY, bool GENREF = false, bool STREAM = false>
__global__ __launch_bounds__(Tile<TY>::NT) __attribute__((amdgpu_waves_per_eu(
    StageWaves<T>::value))) void tlb_stage_batch_kernel(
    const StageArgs<T>* __restrict__ table, const int* __restrict__ tile_begin, int n, int stage) {
  const int total = tile_begin[n];
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
  const int full = total >> 3, rem = total & 7;
  if (local >= full + (xcd < rem ? 1 : 0)) return;
  const int t = xcd * full + min(xcd, rem) + local;
  int lo = 0, hi = n - 1;  // the grid owning tile t: the last g with tile_begin[g] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_begin[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  StageArgs<T> a = table[3 * lo + stage - 1];
  a.fin = global_ptr(a.fin);
  a.phin = global_ptr(a.phin);
  a.f0 = global_ptr(a.f0);
  a.phi0 = global_ptr(a.phi0);
  a.fout = global_ptr(a.fout);
  a.phiout = global_ptr(a.phiout);
  a.rows = global_ptr(a.rows);
  if (a.phib) a.phib = global_ptr(a.phib);
  int tx, ty;
  band_tile(t - tile_begin[lo], a.ntx, a.nty, tx, ty);
  stage_tile<T, VEC, TY, false, STREAM, GENREF>(a, tx, ty);
}

// ------------------------------------------------------------------------------------------
// f = f_eq(n, u) (eq. feq), one thread per node
template <typename T>
__global__ __launch_bounds__(256) void tlb_init_feq_kernel(T* f, const T* n, const T* ut,
                                                          const T* up, long long plane,
                                                          T n_ref) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= plane) return;
  const T nn = n[x], a = ut[x], b = up[x];
  const T c0 = T(1) - T(0.5) * (a * a + b * b);
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int i = k >> 2, j = k & 3;
    const T xi = T(vel(i)) * a + T(vel(j)) * b;
    if constexpr (stores_deviation<T>()) {
      const T p1 = T(-0.5) * (a * a + b * b) + xi * (c0 + xi * (T(0.5) + xi * T(1.0 / 6.0)));
      f[k * plane + x] = T(wgt(i) * wgt(j)) * (n_ref * p1 + (nn - n_ref) * (T(1) + p1));
    } else {
      f[k * plane + x] = (nn * T(wgt(i) * wgt(j))) * (c0 + xi * (c0 + xi * (T(0.5) + xi * T(1.0 / 6.0))));
    }
  });
}

// between full populations and the stored representation: f += scale * rest_offset
// (scale = -n_ref stores, +n_ref restores, the difference of two n_ref changes the reference)
template <typename T>
__global__ __launch_bounds__(256) void tlb_offset_kernel(T* f, long long plane, T scale) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= plane) return;
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    f[k * plane + x] += scale * T(rest_offset<T>(k));
  });
}

// Non-finite check of a state (tlb_step_n with check_every > 0): sets *flag to 1 if any
// population or phi value is NaN or Inf.  Grid-stride loop, one vector store per wave that saw
// one (several waves may store the same value).
template <typename T>
__global__ __launch_bounds__(256) void tlb_nonfinite_kernel(const T* f, const T* phi,
                                                           const T* phib, long long plane,
                                                           int* flag) {
  bool bad = false;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < plane;
       x += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 16; ++k) bad = bad || !isfinite(f[k * plane + x]);
    bad = bad || !isfinite(phi[x]) || (phib && !isfinite(phib[x]));
  }
  if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) *flag = 1;
}

// *flag = value (a kernel, not a memset: the step loop may be captured into a graph)
__global__ void tlb_set_flag_kernel(int* flag, int value) { *flag = value; }

// FP32 order parameter, stored as base b + deviation d: move the deviation into the base,
// exactly -- b' = fl(b + d) and d' = (b + d) - b', the rounding error of that sum, by the
// error-free two-sum (Knuth) -- so that d stays small (a few ulps of b) and the small
// increments it accumulates keep their precision.  b' + d' = b + d.
// (one by-value argument block, so that it can be a graph node like the stage kernels)
struct RebaseArgs {
  float* b;
  float* d;
  long long plane;
};

__global__ __launch_bounds__(256) void tlb_phi_rebase_kernel(RebaseArgs a) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.plane) return;
  const float bb = a.b[x], dd = a.d[x];
  const float sum = bb + dd;
  const float bv = sum - dd;  // the part of sum that came from bb
  const float dv = sum - bv;  // ... and from dd
  a.b[x] = sum;
  a.d[x] = (bb - bv) + (dd - dv);
}

// out = b + d (FP32 order parameter as one plane; out may alias neither)
__global__ __launch_bounds__(256) void tlb_phi_sum_kernel(float* out, const float* b,
                                                         const float* d, long long plane) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < plane) out[x] = b[x] + d[x];
}

// moments and chemical potential of a state, one thread per node
template <typename T>
__global__ __launch_bounds__(256) void tlb_moments_kernel(const T* f, const T* phi,
                                                         const T* phib, T* n_out,
                                                         T* ut_out, T* up_out, T* phi_out,
                                                         T* mu_out, const RowCoef<T>* rows,
                                                         int nt, int np, T A, T kappa,
                                                         T n_ref, int ch4) {
  const long long plane = (long long)nt * np;
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= plane) return;
  const int q = (int)(x / np), s = (int)(x - (long long)q * np);
  T n = T(0), nut = T(0), nup = T(0);
  static_for<0, 16>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const T fk = f[k * plane + x];
    n += fk;
    nut += T(vel(k >> 2)) * fk;
    nup += T(vel(k & 3)) * fk;
  });
  if constexpr (stores_deviation<T>()) n += n_ref;
  if (n_out) n_out[x] = n;
  if (ut_out) ut_out[x] = nut / n;
  if (up_out) up_out[x] = nup / n;
  const T ph = phi_val(phi, phib, x);
  if (phi_out) phi_out[x] = ph;
  if (mu_out && ch4) {
    mu_out[x] = A * ph * (ph * ph - T(1)) - kappa * lap4_at(phi, phib, rows[q], q, s, nt, np);
  } else if (mu_out) {
    const RowCoef<T>& rc = rows[q];
    const int qn = q + 1 == nt ? 0 : q + 1, qs = q == 0 ? nt - 1 : q - 1;
    const int se = s + 1 == np ? 0 : s + 1, sw = s == 0 ? np - 1 : s - 1;
    const T lap = rc.lap_n * (phi_val(phi, phib, (long long)qn * np + s) - ph) -
                  rc.lap_s * (ph - phi_val(phi, phib, (long long)qs * np + s)) +
                  rc.lap_p * (phi_val(phi, phib, (long long)q * np + se) - T(2) * ph +
                              phi_val(phi, phib, (long long)q * np + sw));
    mu_out[x] = A * ph * (ph * ph - T(1)) - kappa * lap;
  }
}

// ------------------------------------------------------------------------------------------
// conservation diagnostics in FP64: per-block partials in a fixed order, then one block
constexpr int RED_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void tlb_reduce_kernel(const T* f, const T* phi,
                                                                const T* phib,
                                                                const double* area, int nt,
                                                                int np, int rows_per_block,
                                                                double n_add, double* partial) {
  __shared__ double s[3][RED_THREADS / 64];
  const int q_begin = blockIdx.x * rows_per_block;
  const int q_end = min(nt, q_begin + rows_per_block);
  const long long plane = (long long)nt * np;
  double m = 0.0, p = 0.0, bad = 0.0;
  for (int q = q_begin; q < q_end; ++q) {
    double rm = 0.0, rp = 0.0;
    for (int s0 = threadIdx.x; s0 < np; s0 += RED_THREADS) {
      const long long x = (long long)q * np + s0;
      double n = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double fk = (double)f[k * plane + x];
        bad += isfinite(fk) ? 0.0 : 1.0;
        n += fk;
      }
      n += n_add;  // the reference density of deviation storage (else 0)
      const double ph = phi_val64(phi, phib, x);
      bad += isfinite(ph) ? 0.0 : 1.0;
      rm += n;
      rp += ph;
    }
    m += area[q] * rm;
    p += area[q] * rp;
  }
  m = wave_sum(m);
  p = wave_sum(p);
  bad = wave_sum(bad);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s[0][w] = m;
    s[1][w] = p;
    s[2][w] = bad;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int i = 0; i < RED_THREADS / 64; ++i) t += s[threadIdx.x][i];
    partial[3 * blockIdx.x + threadIdx.x] = t;
  }
}

// Diagnostics of sections III B and IV in FP64: per row q, the azimuthal averages of phi and of
// p = n + A(-phi^2/2 + 3 phi^4/4); per block, the interface length (sign changes of phi towards
// the phi neighbour count r dtheta, towards the theta neighbour (R + r cos theta_{q+1/2}) dphi)
// and the area, as partials for tlb_reduce_final_kernel.
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void tlb_diag_kernel(const T* f, const T* phi,
                                                              const T* phib,
                                                              const double* area,
                                                              const double* half_len, double r_dth,
                                                              double A, int nt, int np,
                                                              int rows_per_block, double n_add,
                                                              double* phi_avg, double* p_avg,
                                                              double* partial) {
  __shared__ double s[3][RED_THREADS / 64];
  const int q_begin = blockIdx.x * rows_per_block;
  const int q_end = min(nt, q_begin + rows_per_block);
  const long long plane = (long long)nt * np;
  double len = 0.0, ar = 0.0;
  for (int q = q_begin; q < q_end; ++q) {
    const int qn = q + 1 == nt ? 0 : q + 1;
    double rphi = 0.0, rp = 0.0;
    for (int s0 = threadIdx.x; s0 < np; s0 += RED_THREADS) {
      const long long x = (long long)q * np + s0;
      const int se = s0 + 1 == np ? 0 : s0 + 1;
      const double ph = phi_val64(phi, phib, x);
      if (ph * phi_val64(phi, phib, (long long)q * np + se) < 0.0) len += r_dth;
      if (ph * phi_val64(phi, phib, (long long)qn * np + s0) < 0.0) len += half_len[q];
      double n = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) n += (double)f[k * plane + x];
      n += n_add;
      rphi += ph;
      rp += n + A * (-0.5 * ph * ph + 0.75 * ph * ph * ph * ph);
    }
    rphi = wave_sum(rphi);
    rp = wave_sum(rp);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      s[0][w] = rphi;
      s[1][w] = rp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0;
      for (int i = 0; i < RED_THREADS / 64; ++i) {
        a += s[0][i];
        b += s[1][i];
      }
      if (phi_avg) phi_avg[q] = a / np;
      if (p_avg) p_avg[q] = b / np;
    }
    __syncthreads();
    ar += area[q] * np;
  }
  len = wave_sum(len);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s[2][w] = len;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < RED_THREADS / 64; ++i) t += s[2][i];
    partial[3 * blockIdx.x + 0] = t;
    partial[3 * blockIdx.x + 1] = ar;
    partial[3 * blockIdx.x + 2] = 0.0;
  }
}

// Structure-factor length: a direct DFT of phi in FP64, rows then columns.  The zero mode is
// left out, so the mean of phi need not be removed.  tw holds exp(-2 pi i j / n) for the row
// length n_phi followed by the column length n_theta.
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void tlb_dft_rows_kernel(const T* phi, const T* phib,
                                                                  const double2* tw, double2* X,
                                                                  int np) {
  extern __shared__ double srow[];  // the row, n_phi values
  const int q = blockIdx.x;
  for (int s0 = threadIdx.x; s0 < np; s0 += RED_THREADS)
    srow[s0] = phi_val64(phi, phib, (long long)q * np + s0);
  __syncthreads();
  for (int m = threadIdx.x; m < np; m += RED_THREADS) {
    double re = 0.0, im = 0.0;
    int idx = 0;  // (m s) mod n_phi
    for (int s0 = 0; s0 < np; ++s0) {
      const double2 w = tw[idx];
      re += srow[s0] * w.x;
      im += srow[s0] * w.y;
      idx += m;
      if (idx >= np) idx -= np;
    }
    X[(long long)q * np + m] = make_double2(re, im);
  }
}

// one block per phi mode m': the column transform, |Y|^2, and the sums of S and |k| S
__global__ __launch_bounds__(RED_THREADS) void tlb_dft_cols_kernel(const double2* X,
                                                                  const double2* tw, int nt,
                                                                  int np, double r, double R,
                                                                  double* partial) {
  extern __shared__ double2 scol[];  // the column, n_theta complex values
  __shared__ double sh[2][RED_THREADS / 64];
  const int mp = blockIdx.x;
  for (int q = threadIdx.x; q < nt; q += RED_THREADS) scol[q] = X[(long long)q * np + mp];
  __syncthreads();
  const double kp = (mp <= (np - 1) / 2 ? mp : mp - np) / R;
  double s0 = 0.0, s1 = 0.0;
  for (int m = threadIdx.x; m < nt; m += RED_THREADS) {
    double re = 0.0, im = 0.0;
    int idx = 0;  // (m q) mod n_theta
    for (int q = 0; q < nt; ++q) {
      const double2 w = tw[idx];
      const double2 x = scol[q];
      re += x.x * w.x - x.y * w.y;
      im += x.x * w.y + x.y * w.x;
      idx += m;
      if (idx >= nt) idx -= nt;
    }
    const double S = (m == 0 && mp == 0) ? 0.0 : re * re + im * im;
    const double kt = (m <= (nt - 1) / 2 ? m : m - nt) / r;
    s0 += S;
    s1 += sqrt(kt * kt + kp * kp) * S;
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = s0;
    sh[1][w] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int i = 0; i < RED_THREADS / 64; ++i) t += sh[threadIdx.x][i];
    partial[2 * mp + threadIdx.x] = t;
  }
}

__global__ __launch_bounds__(RED_THREADS) void tlb_reduce_final_kernel(const double* partial,
                                                                      int nblocks,
                                                                      double* out) {
  __shared__ double s[3][RED_THREADS / 64];
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS)
    for (int c = 0; c < 3; ++c) v[c] += partial[3 * b + c];
  for (int c = 0; c < 3; ++c) v[c] = wave_sum(v[c]);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 3; ++c) s[c][w] = v[c];
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int i = 0; i < RED_THREADS / 64; ++i) t += s[threadIdx.x][i];
    out[threadIdx.x] = t;
  }
}

// ------------------------------------------------------------------------------------------
// host side: per-launch constants and the per-row geometry (appendix A), derived in FP64
template <typename T>
Consts<T> make_consts(const tlb_params& p, double n_ref) {
  Consts<T> c{};
  c.n_ref = T(n_ref);
  const double dth = 2.0 * M_PI / p.n_theta;
  c.A = T(p.A);
  c.kappa = T(p.kappa);
  c.M = T(p.M);
  c.inv_tau = T(1.0 / p.tau);
  c.inv_2rdth = T(1.0 / (2.0 * p.r * dth));
  c.inv_12rdth = T(1.0 / (12.0 * p.r * dth));
  c.dt = T(p.dt);
  c.ch_adv = (p.flags & TLB_CH_NO_ADVECTION) ? 0 : 1;
  return c;
}

template <typename T>
void make_rows(const tlb_params& p, RowCoef<T>* rows, double* area) {
  const int nt = p.n_theta;
  const double dth = 2.0 * M_PI / nt, dph = 2.0 * M_PI / p.n_phi;
  const bool flat = p.flags & TLB_FLAT;
  auto Jat = [&](double th) { return flat ? p.R : p.R + p.r * std::cos(th); };
  for (int q = 0; q < nt; ++q) {
    const double th = q * dth;
    const double J = Jat(th);
    RowCoef<T>& rc = rows[q];
    double sp = 0.0, sm = 0.0;
    for (int o = -3; o <= 2; ++o) {
      const int qq = ((q + o) % nt + nt) % nt;
      const double b = uw5p(o) * Jat(qq * dth) / (p.r * J * dth);
      rc.bth_p[o + 3] = T(b);
      sp += b;
    }
    for (int o = -2; o <= 3; ++o) {
      const int qq = ((q + o) % nt + nt) % nt;
      const double b = uw5m(o) * Jat(qq * dth) / (p.r * J * dth);
      rc.bth_m[o + 2] = T(b);
      sm += b;
    }
    rc.bsum_p = T(sp);
    rc.bsum_m = T(sm);
    rc.inv_Jdph = T(1.0 / (J * dph));
    rc.J = T(J);
    rc.G = T(flat ? 0.0 : std::sin(th) / J);
    rc.lap_n = T(Jat(th + 0.5 * dth) / (p.r * p.r * J * dth * dth));
    rc.lap_s = T(Jat(th - 0.5 * dth) / (p.r * p.r * J * dth * dth));
    rc.lap_p = T(1.0 / (J * J * dph * dph));
    rc.inv_2Jdph = T(1.0 / (2.0 * J * dph));
    rc.inv_2rJdth = T(1.0 / (2.0 * p.r * J * dth));
    for (int m = 0; m < 4; ++m)
      rc.l4[m] = T(Jat(th + (m - 1.5) * dth) / (576.0 * p.r * p.r * J * dth * dth));
    rc.lp4 = T(1.0 / (12.0 * J * J * dph * dph));
    rc.inv_12Jdph = T(1.0 / (12.0 * J * dph));
    rc.inv_12rJdth = T(1.0 / (12.0 * p.r * J * dth));
    area[q] = p.r * J * dth * dph;
    area[nt + q] = Jat(th + 0.5 * dth) * dph;
  }
}

}  // namespace

// ------------------------------------------------------------------------------------------
constexpr int GRAPH_CHUNK_B = TLBI_GRAPH_CHUNK;

struct tlb_batch {
  tlb_grid** grids;
  int n;
  int precision, ty, blocks;
  bool vec;
  hipStream_t stream;
  void* table;      // StageArgs<T>[3 n] (device)
  int* tile_begin;  // [n + 1] (device)
  int total_tiles;
  hipGraphExec_t graphs[GRAPH_CHUNK_B + 1];  // as tlb_grid::graphs, for the whole batch
  bool streaming;      // the ensemble's state copies exceed STREAMING_BYTES
  unsigned* versions;  // [n]: the grids' versions when the table was built
};

namespace {

template <typename T>
StageArgs<T> stage_args(const tlb_grid* g, int stage) {
  StageArgs<T> a{};
  const int src = stage == 1 ? 0 : stage - 1;  // stage 1 reads y^n, 2 reads y1, 3 reads y2
  const int dst = stage == 3 ? 0 : stage;      // stage 3 writes y^{n+1} over y^n
  a.fin = static_cast<const T*>(g->f[src]);
  a.phin = static_cast<const T*>(g->phi[src]);
  a.f0 = static_cast<const T*>(g->f[0]);
  a.phi0 = static_cast<const T*>(g->phi[0]);
  a.fout = static_cast<T*>(g->f[dst]);
  a.phiout = static_cast<T*>(g->phi[dst]);
  a.rows = static_cast<const RowCoef<T>*>(g->rows);
  a.nt = g->p.n_theta;
  a.np = g->p.n_phi;
  a.ntx = (a.np + TX - 1) / TX;
  a.nty = (a.nt + g->ty - 1) / g->ty;
  a.plane = (long long)a.nt * a.np;
  a.has_y0 = stage != 1;
  a.a0 = stage == 2 ? T(0.75) : stage == 3 ? T(1.0 / 3.0) : T(0);
  a.b1 = stage == 2 ? T(0.25) : stage == 3 ? T(2.0 / 3.0) : T(1);
  a.c = make_consts<T>(g->p, g->n_ref);
  if constexpr (stores_deviation<T>()) a.phib = reinterpret_cast<const T*>(g->phi_base);
  if (g->ch4) {
    const T* w = static_cast<const T*>(g->ch4);
    a.mu4 = w;
    a.P4 = w + a.plane;
    a.Q4 = w + 2 * a.plane;
  }
  return a;
}

// 16-byte copies need every 16-byte chunk of a row inside one period of phi
template <typename T>
bool vec_ok(int n_phi) {
  return n_phi % (16 / (int)sizeof(T)) == 0;
}

template <typename T, bool VEC, bool GENREF>
const void* stage_fn_ty(int ty, bool streaming) {
  if (streaming) {  // the 16-byte-copy form only (every large grid here has n_phi % 4 == 0)
    if constexpr (VEC) {
      switch (ty) {
        case 4: return reinterpret_cast<const void*>(&tlb_stage_kernel<T, true, 4, false, true, GENREF>);
        case 16: return reinterpret_cast<const void*>(&tlb_stage_kernel<T, true, 16, false, true, GENREF>);
        default: return reinterpret_cast<const void*>(&tlb_stage_kernel<T, true, 8, false, true, GENREF>);
      }
    }
  }
  switch (ty) {
    case 4: return reinterpret_cast<const void*>(&tlb_stage_kernel<T, VEC, 4, false, false, GENREF>);
    case 16: return reinterpret_cast<const void*>(&tlb_stage_kernel<T, VEC, 16, false, false, GENREF>);
    default: return reinterpret_cast<const void*>(&tlb_stage_kernel<T, VEC, 8, false, false, GENREF>);
  }
}

// FP32 grids whose reference density is not 1 need the kernels that read it
template <typename T>
bool general_reference(const tlb_grid* g) {
  return stores_deviation<T>() && g->n_ref != 1.0;
}

// Grids whose three state copies (51 values per node) exceed this use streaming accesses
constexpr double STREAMING_BYTES = 1024.0 * 1024.0 * 1024.0;

bool streaming(const tlb_grid* g) {
  return 51.0 * g->p.n_theta * (double)g->p.n_phi * (double)g->elem > STREAMING_BYTES;
}

template <typename T>
const void* stage_fn(const tlb_grid* g) {
  const bool vec = vec_ok<T>(g->p.n_phi), gen = general_reference<T>(g);
  if (g->p.flags & TLB_CH4) {  // the fourth-order Cahn-Hilliard variant: 8-row tiles only
    if (gen)
      return vec ? reinterpret_cast<const void*>(&tlb_stage_kernel<T, true, DEFAULT_TY, false, false, true, true>)
                 : reinterpret_cast<const void*>(&tlb_stage_kernel<T, false, DEFAULT_TY, false, false, true, true>);
    return vec ? reinterpret_cast<const void*>(&tlb_stage_kernel<T, true, DEFAULT_TY, false, false, false, true>)
               : reinterpret_cast<const void*>(&tlb_stage_kernel<T, false, DEFAULT_TY, false, false, false, true>);
  }
  if (g->p.flags & TLB_WENO5) {  // the WENO variant exists for the default tile height only
    if (gen)
      return vec ? reinterpret_cast<const void*>(&tlb_stage_kernel<T, true, DEFAULT_TY, true, false, true>)
                 : reinterpret_cast<const void*>(&tlb_stage_kernel<T, false, DEFAULT_TY, true, false, true>);
    return vec ? reinterpret_cast<const void*>(&tlb_stage_kernel<T, true, DEFAULT_TY, true>)
               : reinterpret_cast<const void*>(&tlb_stage_kernel<T, false, DEFAULT_TY, true>);
  }
  if (gen)
    return vec ? stage_fn_ty<T, true, true>(g->ty, streaming(g))
               : stage_fn_ty<T, false, true>(g->ty, streaming(g));
  return vec ? stage_fn_ty<T, true, false>(g->ty, streaming(g))
             : stage_fn_ty<T, false, false>(g->ty, streaming(g));
}

template <typename T, bool VEC, bool GENREF>
const void* batch_fn_ty(int ty, bool streaming) {
  if (streaming) {  // as for single grids, the 16-byte-copy form only
    if constexpr (VEC) {
      switch (ty) {
        case 4: return reinterpret_cast<const void*>(&tlb_stage_batch_kernel<T, true, 4, GENREF, true>);
        case 16: return reinterpret_cast<const void*>(&tlb_stage_batch_kernel<T, true, 16, GENREF, true>);
        default: return reinterpret_cast<const void*>(&tlb_stage_batch_kernel<T, true, 8, GENREF, true>);
      }
    }
  }
  switch (ty) {
    case 4: return reinterpret_cast<const void*>(&tlb_stage_batch_kernel<T, VEC, 4, GENREF>);
    case 16: return reinterpret_cast<const void*>(&tlb_stage_batch_kernel<T, VEC, 16, GENREF>);
    default: return reinterpret_cast<const void*>(&tlb_stage_batch_kernel<T, VEC, 8, GENREF>);
  }
}

// the batch kernel for the batch's current grids (the general-reference form if any needs it;
// streaming accesses when the ensemble's state copies together exceed STREAMING_BYTES)
template <typename T>
const void* batch_fn(const tlb_batch* b) {
  bool gen = false;
  for (int i = 0; i < b->n; ++i) gen = gen || general_reference<T>(b->grids[i]);
  if (gen)
    return b->vec ? batch_fn_ty<T, true, true>(b->ty, b->streaming)
                  : batch_fn_ty<T, false, true>(b->ty, b->streaming);
  return b->vec ? batch_fn_ty<T, true, false>(b->ty, b->streaming)
                : batch_fn_ty<T, false, false>(b->ty, b->streaming);
}

int stage_blocks(const tlb_grid* g) {
  return ((g->p.n_phi + TX - 1) / TX) * ((g->p.n_theta + g->ty - 1) / g->ty);
}

// The launches of Runge-Kutta stage `stage` of grid g, each with one by-value argument block:
// the stage kernel, preceded for TLB_CH4 by the fourth-order Cahn-Hilliard prepass on the
// stage input.  Returns their number (1 or 2).
template <typename T>
int stage_launches(const tlb_grid* g, int stage, tlbi_launch out[2]) {
  static_assert(sizeof(StageArgs<T>) <= sizeof(out->args), "argument block");
  static_assert(sizeof(Ch4Args<T>) <= sizeof(out->args), "argument block");
  const StageArgs<T> a = stage_args<T>(g, stage);
  int n = 0;
  if (g->ch4) {
    Ch4Args<T> c{};
    c.f = a.fin;
    c.phi = a.phin;
    c.phib = a.phib;
    c.mu = const_cast<T*>(a.mu4);
    c.P = const_cast<T*>(a.P4);
    c.Q = const_cast<T*>(a.Q4);
    c.rows = a.rows;
    c.nt = a.nt;
    c.np = a.np;
    c.plane = a.plane;
    c.A = T(g->p.A);
    c.kappa = T(g->p.kappa);
    c.n_ref = T(g->n_ref);
    out[n].fn = reinterpret_cast<const void*>(&tlb_ch4_prep_kernel<T>);
    out[n].grid = dim3((unsigned)((a.plane + 255) / 256));
    out[n].block = dim3(256);
    std::memcpy(out[n].args, &c, sizeof(c));
    ++n;
  }
  out[n].fn = stage_fn<T>(g);
  out[n].grid = dim3(stage_blocks(g));
  out[n].block = dim3(TX * g->ty);
  std::memcpy(out[n].args, &a, sizeof(a));
  return n + 1;
}

template <typename T>
int32_t launch_stage(tlb_grid* g, int stage) {
  tlbi_launch l[2];
  const int n = stage_launches<T>(g, stage, l);
  for (int i = 0; i < n; ++i) {
    void* params[] = {l[i].args};
    TLB_HIP_CHECK(hipLaunchKernel(l[i].fn, l[i].grid, l[i].block, params, 0, g->stream));
  }
  return TLB_OK;
}

// A chain of `steps` time steps (3 `steps` kernel nodes, each depending on the one before)
// built explicitly -- no stream capture, so the caller's stream may be the legacy default
// stream -- and replayed with one launch.  Kernel nodes only.  Runs of GRAPH_CHUNK steps
// replay the longest chain; a shorter run, or the remainder of a longer one, replays a chain of
// its own length (built on first use and kept), so every step of the loop is a graph replay.
constexpr int GRAPH_CHUNK = TLBI_GRAPH_CHUNK;

// `make_params(st)` returns the kernel-argument array of stage st (1..3); the arrays must stay
// valid until the graph is instantiated
template <class MakeParams>
hipError_t build_chain(const void* fn, dim3 grid, dim3 block, MakeParams make_params,
                       int steps, hipStream_t stream, hipGraphExec_t* out) {
  hipGraph_t graph;
  hipError_t e = hipGraphCreate(&graph, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t prev = nullptr;
  for (int t = 0; t < steps && e == hipSuccess; ++t)
    for (int st = 1; st <= 3 && e == hipSuccess; ++st) {
      hipKernelNodeParams kp{};
      kp.func = const_cast<void*>(fn);
      kp.gridDim = grid;
      kp.blockDim = block;
      kp.sharedMemBytes = 0;
      kp.kernelParams = make_params(st);
      kp.extra = nullptr;
      hipGraphNode_t node;
      e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
      prev = node;
    }
  if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  if (e == hipSuccess && (e = hipGraphUpload(*out, stream)) != hipSuccess)
    (void)hipGraphExecDestroy(*out);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) *out = nullptr;
  return e;
}

// A chain of `steps` time steps of the grid's stage launches (kernel nodes only), each node
// depending on the one before, closed by the rebase of the order parameter if `close`.
template <typename T>
int32_t build_step_graph(tlb_grid* g, int steps, bool close) {
  tlbi_launch l[3][2];
  int n[3];
  void* argp[3][2];
  for (int st = 1; st <= 3; ++st) {
    n[st - 1] = stage_launches<T>(g, st, l[st - 1]);
    for (int i = 0; i < n[st - 1]; ++i) argp[st - 1][i] = l[st - 1][i].args;
  }
  hipGraph_t graph;
  hipError_t e = hipGraphCreate(&graph, 0);
  if (e != hipSuccess) return fail(TLB_EHIP, std::string("graph build: ") + hipGetErrorString(e));
  hipGraphNode_t prev = nullptr;
  auto add = [&](const tlbi_launch& l, void** params) {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(l.fn);
    kp.gridDim = l.grid;
    kp.blockDim = l.block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = params;
    kp.extra = nullptr;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    prev = node;
  };
  for (int t = 0; t < steps && e == hipSuccess; ++t)
    for (int st = 0; st < 3 && e == hipSuccess; ++st)
      for (int i = 0; i < n[st] && e == hipSuccess; ++i) add(l[st][i], &argp[st][i]);
  tlbi_launch rb;
  void* rbp = rb.args;
  if (e == hipSuccess && close && tlbi_phi_rebase_launch(g, &rb)) add(rb, &rbp);
  hipGraphExec_t& slot = g->graphs[close ? 1 : 0][steps];
  if (e == hipSuccess) e = hipGraphInstantiate(&slot, graph, nullptr, nullptr, 0);
  // uploaded now, so that the first launch of the graph costs what every other launch costs
  if (e == hipSuccess && (e = hipGraphUpload(slot, g->stream)) != hipSuccess)
    (void)hipGraphExecDestroy(slot);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    slot = nullptr;
    return fail(TLB_EHIP, std::string("graph build: ") + hipGetErrorString(e));
  }
  return TLB_OK;
}

// Every graph the step loop uses: runs of 1, 2, 4, .., GRAPH_CHUNK steps, and for FP32 grids
// each also closed by the fold of the order parameter.
template <typename T>
int32_t build_step_graphs(tlb_grid* g) {
  for (int c = 0; c < (g->phi_base ? 2 : 1); ++c)
    for (int len = 1; len <= GRAPH_CHUNK; len <<= 1)
      if (!g->graphs[c][len]) {
        int32_t rc = build_step_graph<T>(g, len, c == 1);
        if (rc != TLB_OK) return rc;
      }
  return TLB_OK;
}

void drop_graph(tlb_grid* g) {
  for (auto& row : g->graphs)
    for (hipGraphExec_t& x : row) {
      if (x) (void)hipGraphExecDestroy(x);
      x = nullptr;
    }
}

// The next run of at most `n` steps of grid g: its length, and whether it ends on a rebase of
// the order parameter (FP32 grids rebase after every GRAPH_CHUNK-th step since set_state).
struct Run {
  int steps;
  bool close;
};
Run next_run(const tlb_grid* g, int64_t n) {
  const int left = GRAPH_CHUNK - g->phase;
  const int s = (int)std::min<int64_t>(left, n);
  return Run{s, g->phi_base != nullptr && s == left};
}
void advance_phase(tlb_grid* g, int steps) {
  g->phase = g->phi_base ? (g->phase + steps) % GRAPH_CHUNK : 0;
}

template <typename T>
int32_t check_t(tlb_grid* g) {
  const long long plane = (long long)g->p.n_theta * g->p.n_phi;
  const int blocks = (int)std::min<long long>(4096, (plane + 255) / 256);
  hipLaunchKernelGGL(tlb_nonfinite_kernel<T>, dim3(blocks), dim3(256), 0, g->stream,
                     static_cast<const T*>(g->f[0]), static_cast<const T*>(g->phi[0]),
                     reinterpret_cast<const T*>(g->phi_base), plane, g->check_flag);
  TLB_HIP_CHECK(hipGetLastError());
  return TLB_OK;
}

template <typename T>
int32_t step_n_t(tlb_grid* g, int64_t n) {
  if (g->graph_version != g->version) {  // stage arguments changed: the graphs are stale
    drop_graph(g);
    g->graph_version = g->version;
  }
  const bool direct = g->p.flags & TLB_NO_GRAPH;  // the same runs as the graphs, launch by launch
  for (int64_t done = 0; done < n;) {
    const Run r = next_run(g, n - done);
    if (direct) {
      for (int t = 0; t < r.steps; ++t)
        for (int st = 1; st <= 3; ++st) {
          int32_t rc = launch_stage<T>(g, st);
          if (rc != TLB_OK) return rc;
        }
      if (r.close) {
        int32_t rc = tlbi_phi_rebase(g, g->stream);
        if (rc != TLB_OK) return rc;
      }
    } else {
      // the run as graphs of 32, 16, 8, 4, 2 and 1 steps (its binary digits, largest first;
      // the last one carries the fold), all built together on first use: no later call builds
      // a graph, whatever its length and the fold phase it starts at
      for (int left = r.steps; left > 0;) {
        int piece = GRAPH_CHUNK;
        while (piece > left) piece >>= 1;
        left -= piece;
        hipGraphExec_t& x = g->graphs[r.close && left == 0 ? 1 : 0][piece];
        if (!x) {
          int32_t rc = build_step_graphs<T>(g);
          if (rc != TLB_OK) return rc;
        }
        TLB_HIP_CHECK(hipGraphLaunch(x, g->stream));
      }
    }
    advance_phase(g, r.steps);
    done += r.steps;
  }
  return TLB_OK;
}

// Time `reps` launches of `launch()` on `stream` (after one untimed launch), in milliseconds.
template <class Launch>
int32_t time_launches(hipStream_t stream, int reps, Launch launch, float* ms) {
  hipEvent_t e0, e1;
  TLB_HIP_CHECK(hipEventCreate(&e0));
  TLB_HIP_CHECK(hipEventCreate(&e1));
  int32_t rc = launch();
  if (rc == TLB_OK) {
    (void)hipEventRecord(e0, stream);
    for (int i = 0; i < reps && rc == TLB_OK; ++i) rc = launch();
    (void)hipEventRecord(e1, stream);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(ms, e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

constexpr int TILE_CHOICES[3] = {4, 8, 16};
constexpr int TUNE_ROUNDS = 3;

// Repetitions per measurement: about 3 ms of work at 1.5e10 node-stages/s, at least 4 and at
// most 200 (small grids need many launches before the launch noise averages out).
int tune_reps(long long nodes) {
  const long long r = 20000000LL / (nodes > 0 ? nodes : 1);
  return (int)std::max(4LL, std::min(200LL, r));
}

// Index into TILE_CHOICES of the smallest time; the default height wins ties.
int fastest(const float (&ms)[3]) {
  int pick = 1;
  for (int c = 0; c < 3; ++c)
    if (ms[c] < ms[pick]) pick = c;
  return pick;
}

// Autotuner: time pairs of stage-1 and stage-2 launches for every tile height (stage 1 reads
// the state and writes the stage-1 copy, stage 2 reads both and writes the stage-2 copy, so the
// state is unchanged, and stage 2 reads as much as stage 3 does); three interleaved rounds, the
// best time of each height counts.
template <typename T>
int32_t autotune_t(tlb_grid* g, int32_t* chosen) {
  const int old_ty = g->ty;
  const int reps = tune_reps((long long)g->p.n_theta * g->p.n_phi);
  float best[3] = {0.0f, 0.0f, 0.0f};
  for (int round = 0; round < TUNE_ROUNDS; ++round)
    for (int c = 0; c < 3; ++c) {
      g->ty = TILE_CHOICES[c];
      float ms = 0.0f;
      int32_t rc = time_launches(g->stream, reps, [&]() {
        int32_t r = launch_stage<T>(g, 1);
        return r == TLB_OK ? launch_stage<T>(g, 2) : r;
      }, &ms);
      if (rc != TLB_OK) {
        g->ty = old_ty;
        return rc;
      }
      if (round == 0 || ms < best[c]) best[c] = ms;
    }
  g->ty = TILE_CHOICES[fastest(best)];
  drop_graph(g);
  if (chosen) *chosen = g->ty;
  return TLB_OK;
}

// ---- ensembles ------------------------------------------------------------------------------

void drop_batch_graph(tlb_batch* b) {
  for (hipGraphExec_t& x : b->graphs) {
    if (x) (void)hipGraphExecDestroy(x);
    x = nullptr;
  }
}

// (Re)build the argument table and the tile offsets of the batch for its tile height, and the
// launch size (one block per tile, rounded up to a multiple of the 8 XCDs).
template <typename T>
int32_t batch_setup_t(tlb_batch* b) {
  std::string err;
  StageArgs<T>* tab = static_cast<StageArgs<T>*>(std::malloc(sizeof(StageArgs<T>) * 3 * b->n));
  int* tb = static_cast<int*>(std::malloc(sizeof(int) * (b->n + 1)));
  if (!tab || !tb) {
    std::free(tab);
    std::free(tb);
    return fail(TLB_ENOMEM, "host allocation failed");
  }
  long long total = 0;
  for (int i = 0; i < b->n; ++i) {
    b->versions[i] = b->grids[i]->version;
    tlb_grid tmp = *b->grids[i];
    tmp.ty = b->ty;
    for (int st = 1; st <= 3; ++st) tab[3 * i + st - 1] = stage_args<T>(&tmp, st);
    tb[i] = (int)total;
    total += stage_blocks(&tmp);
    if (total > (long long)INT_MAX - 8) {
      std::free(tab);
      std::free(tb);
      return fail(TLB_EINVAL, "ensemble has too many tiles");
    }
  }
  tb[b->n] = (int)total;
  b->total_tiles = (int)total;
  hipError_t e = hipMemcpyAsync(b->table, tab, sizeof(StageArgs<T>) * 3 * b->n,
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->tile_begin, tb, sizeof(int) * (b->n + 1), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  std::free(tab);
  std::free(tb);
  if (e != hipSuccess) return fail(TLB_EHIP, std::string("batch upload: ") + hipGetErrorString(e));
  b->blocks = (int)((total + 7) / 8 * 8);  // one block per tile, a multiple of the 8 XCDs
  drop_batch_graph(b);
  return TLB_OK;
}

template <typename T>
int32_t batch_launch_t(tlb_batch* b, int stage) {
  const void* fn = batch_fn<T>(b);
  const StageArgs<T>* table = static_cast<const StageArgs<T>*>(b->table);
  const int* tile_begin = b->tile_begin;
  int n = b->n;
  void* params[] = {&table, &tile_begin, &n, &stage};
  TLB_HIP_CHECK(hipLaunchKernel(fn, dim3(b->blocks), dim3(TX * b->ty), params, 0, b->stream));
  return TLB_OK;
}

template <typename T>
int32_t batch_step_t(tlb_batch* b, int64_t n) {
  for (int64_t done = 0; done < n;) {
    int s = (int)std::min<int64_t>(GRAPH_CHUNK, n - done);  // up to the next rebase of any grid
    for (int i = 0; i < b->n; ++i) s = std::min(s, next_run(b->grids[i], s).steps);
    bool missing = false;  // graphs of 1, 2, 4, .., GRAPH_CHUNK steps, all built on first use
    for (int len = 1; len <= GRAPH_CHUNK; len <<= 1) missing = missing || !b->graphs[len];
    if (missing) {
      const void* fn = batch_fn<T>(b);
      const StageArgs<T>* table = static_cast<const StageArgs<T>*>(b->table);
      const int* tile_begin = b->tile_begin;
      int nn = b->n;
      int stages[3] = {1, 2, 3};
      void* params[3][4] = {{&table, &tile_begin, &nn, &stages[0]},
                            {&table, &tile_begin, &nn, &stages[1]},
                            {&table, &tile_begin, &nn, &stages[2]}};
      for (int len = 1; len <= GRAPH_CHUNK; len <<= 1) {
        if (b->graphs[len]) continue;
        hipError_t e = build_chain(fn, dim3(b->blocks), dim3(TX * b->ty),
                                   [&](int st) { return params[st - 1]; }, len, b->stream,
                                   &b->graphs[len]);
        if (e != hipSuccess)
          return fail(TLB_EHIP, std::string("batch graph build: ") + hipGetErrorString(e));
      }
    }
    for (int left = s; left > 0;) {  // the run's binary digits, largest first
      int piece = GRAPH_CHUNK;
      while (piece > left) piece >>= 1;
      left -= piece;
      TLB_HIP_CHECK(hipGraphLaunch(b->graphs[piece], b->stream));
    }
    for (int i = 0; i < b->n; ++i) {  // each grid rebases where it would when stepped alone
      tlb_grid* g = b->grids[i];
      const bool close = next_run(g, s).close;
      advance_phase(g, s);
      if (close) {
        int32_t rc = tlbi_phi_rebase(g, b->stream);
        if (rc != TLB_OK) return rc;
      }
    }
    done += s;
  }
  return TLB_OK;
}

template <typename T>
int32_t batch_autotune_t(tlb_batch* b, int32_t* chosen) {
  long long nodes = 0;
  for (int i = 0; i < b->n; ++i) nodes += (long long)b->grids[i]->p.n_theta * b->grids[i]->p.n_phi;
  const int reps = tune_reps(nodes);
  float best[3] = {0.0f, 0.0f, 0.0f};
  for (int round = 0; round < TUNE_ROUNDS; ++round)
    for (int c = 0; c < 3; ++c) {
      b->ty = TILE_CHOICES[c];
      int32_t rc = batch_setup_t<T>(b);
      float ms = 0.0f;
      if (rc == TLB_OK)
        rc = time_launches(b->stream, reps, [&]() {
          int32_t r = batch_launch_t<T>(b, 1);
          return r == TLB_OK ? batch_launch_t<T>(b, 2) : r;
        }, &ms);
      if (rc != TLB_OK) {
        b->ty = DEFAULT_TY;
        (void)batch_setup_t<T>(b);
        return rc;
      }
      if (round == 0 || ms < best[c]) best[c] = ms;
    }
  b->ty = TILE_CHOICES[fastest(best)];
  int32_t rc = batch_setup_t<T>(b);
  if (chosen) *chosen = b->ty;
  return rc;
}

template <typename T>
int32_t init_feq_t(tlb_grid* g, const void* n, const void* ut, const void* up) {
  const long long plane = (long long)g->p.n_theta * g->p.n_phi;
  const int blocks = (int)((plane + 255) / 256);
  hipLaunchKernelGGL(tlb_init_feq_kernel<T>, dim3(blocks), dim3(256), 0, g->stream,
                     static_cast<T*>(g->f[0]), static_cast<const T*>(n),
                     static_cast<const T*>(ut), static_cast<const T*>(up), plane, T(g->n_ref));
  TLB_HIP_CHECK(hipGetLastError());
  return TLB_OK;
}

template <typename T>
int32_t offset_t(tlb_grid* g, void* f, T scale) {
  const long long plane = (long long)g->p.n_theta * g->p.n_phi;
  hipLaunchKernelGGL(tlb_offset_kernel<T>, dim3((int)((plane + 255) / 256)), dim3(256), 0,
                     g->stream, static_cast<T*>(f), plane, scale);
  TLB_HIP_CHECK(hipGetLastError());
  return TLB_OK;
}

template <typename T>
int32_t moments_t(tlb_grid* g, void* n, void* ut, void* up, void* phi, void* mu) {
  const long long plane = (long long)g->p.n_theta * g->p.n_phi;
  const int blocks = (int)((plane + 255) / 256);
  hipLaunchKernelGGL(tlb_moments_kernel<T>, dim3(blocks), dim3(256), 0, g->stream,
                     static_cast<const T*>(g->f[0]), static_cast<const T*>(g->phi[0]),
                     reinterpret_cast<const T*>(g->phi_base),
                     static_cast<T*>(n), static_cast<T*>(ut), static_cast<T*>(up),
                     static_cast<T*>(phi), static_cast<T*>(mu),
                     static_cast<const RowCoef<T>*>(g->rows), g->p.n_theta, g->p.n_phi,
                     T(g->p.A), T(g->p.kappa), T(g->n_ref), (g->p.flags & TLB_CH4) ? 1 : 0);
  TLB_HIP_CHECK(hipGetLastError());
  return TLB_OK;
}

// n_add: what each node's population sum lacks of its density (the reference density of the
// stored deviations; 0 for full populations)
template <typename T>
int32_t reduce_t(tlb_grid* g, double n_add) {
  hipLaunchKernelGGL(tlb_reduce_kernel<T>, dim3(g->red_blocks), dim3(RED_THREADS), 0,
                     g->stream, static_cast<const T*>(g->f[0]),
                     static_cast<const T*>(g->phi[0]), reinterpret_cast<const T*>(g->phi_base),
                     g->area, g->p.n_theta, g->p.n_phi,
                     g->rows_per_block, n_add, g->partial);
  TLB_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(tlb_reduce_final_kernel, dim3(1), dim3(RED_THREADS), 0, g->stream,
                     g->partial, g->red_blocks, g->partial + 3 * g->red_blocks);
  TLB_HIP_CHECK(hipGetLastError());
  return TLB_OK;
}

template <typename T>
int32_t diag_t(tlb_grid* g, double* phi_avg, double* p_avg) {
  const double dth = 2.0 * M_PI / g->p.n_theta;
  hipLaunchKernelGGL(tlb_diag_kernel<T>, dim3(g->red_blocks), dim3(RED_THREADS), 0, g->stream,
                     static_cast<const T*>(g->f[0]), static_cast<const T*>(g->phi[0]),
                     reinterpret_cast<const T*>(g->phi_base), g->area,
                     g->half_len, g->p.r * dth, g->p.A, g->p.n_theta, g->p.n_phi,
                     g->rows_per_block, stores_deviation<T>() ? g->n_ref : 0.0, phi_avg, p_avg,
                     g->partial);
  TLB_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(tlb_reduce_final_kernel, dim3(1), dim3(RED_THREADS), 0, g->stream,
                     g->partial, g->red_blocks, g->partial + 3 * g->red_blocks);
  TLB_HIP_CHECK(hipGetLastError());
  return TLB_OK;
}

// Reference density of FP32 storage for a state of area-weighted mean density `mean`: mean to
// two significant digits (so exactly 1 for every state near unit density), as a float value;
// 1 for a state without a positive finite mean.
double reference_density(double mean) {
  if (!(mean > 0.0) || !std::isfinite(mean)) return 1.0;
  const double e = std::pow(10.0, std::floor(std::log10(mean)) - 1.0);
  return (double)(float)(std::round(mean / e) * e);
}

void set_reference(tlb_grid* g, double n_ref) {
  if (n_ref == g->n_ref) return;
  g->n_ref = n_ref;
  ++g->version;
  drop_graph(g);
}

// area-weighted mean density of state copy 0 of an FP32 grid (waits for the stream)
int32_t mean_density(tlb_grid* g, double n_add, double* mean) {
  int32_t rc = reduce_t<float>(g, n_add);
  if (rc != TLB_OK) return rc;
  double out[3];
  TLB_HIP_CHECK(hipMemcpyAsync(out, g->partial + 3 * g->red_blocks, 3 * sizeof(double),
                               hipMemcpyDeviceToHost, g->stream));
  TLB_HIP_CHECK(hipStreamSynchronize(g->stream));
  *mean = out[0] / (4.0 * M_PI * M_PI * g->p.r * g->p.R);
  return TLB_OK;
}

int32_t check_params(const tlb_params* p) {
  if (!p) return fail(TLB_EINVAL, "params is NULL");
  if (!(p->r > 0.0) || !std::isfinite(p->r)) return fail(TLB_EINVAL, "r must be > 0");
  if (!(p->R > p->r) || !std::isfinite(p->R)) return fail(TLB_EINVAL, "R must exceed r");
  if (p->n_theta < 1 || p->n_phi < 1) return fail(TLB_EINVAL, "grid sides must be >= 1");
  if ((long long)p->n_theta * p->n_phi * (p->precision == 64 ? 8 : 4) > 0xFFFFFFFFLL)
    return fail(TLB_EINVAL, "grid too large: one population plane must stay below 4 GiB");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(TLB_EINVAL, "dt must be > 0");
  if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return fail(TLB_EINVAL, "tau must be > 0");
  if (!(p->kappa >= 0.0) || !std::isfinite(p->kappa))
    return fail(TLB_EINVAL, "kappa must be >= 0");
  if (!(p->M >= 0.0) || !std::isfinite(p->M)) return fail(TLB_EINVAL, "M must be >= 0");
  if (!std::isfinite(p->A)) return fail(TLB_EINVAL, "A must be finite");
  if (p->precision != 32 && p->precision != 64)
    return fail(TLB_EINVAL, "precision must be 32 or 64");
  if (p->flags &
      ~(TLB_FLAT | TLB_CH_NO_ADVECTION | TLB_NO_GRAPH | TLB_WENO5 | TLB_STRICT_DT | TLB_CH4))
    return fail(TLB_EINVAL, "unknown flag");
  if ((p->flags & TLB_CH4) && (p->flags & TLB_WENO5))
    return fail(TLB_EINVAL, "TLB_CH4 and TLB_WENO5 cannot be combined");
  if (p->check_every < 0) return fail(TLB_EINVAL, "check_every must be >= 0");
  return TLB_OK;
}

// The explicit stability bound of tlb_stable_dt (see tlb.h), for validated parameters.
double stable_dt_bound(const tlb_params& p) {
  const double v_max = std::sqrt(3.0 + std::sqrt(6.0));
  const double h_t = p.r * 2.0 * M_PI / p.n_theta;
  const double h_p = ((p.flags & TLB_FLAT) ? p.R : p.R - p.r) * 2.0 * M_PI / p.n_phi;
  const double dt_adv = 1.0 / (v_max * (1.0 / h_t + 1.0 / h_p));
  const double dt_bgk = 2.5 * p.tau;
  const double S = 4.0 / (h_t * h_t) + 4.0 / (h_p * h_p);
  const double ch = p.M * p.kappa * S * S + 2.0 * p.M * std::fabs(p.A) * S;
  const double dt_ch = ch > 0.0 ? 2.51 / ch : INFINITY;
  return std::min(dt_adv, std::min(dt_bgk, dt_ch));
}

std::atomic<unsigned long long> g_next_uid{1};

}  // namespace

// ------------------------------------------------------------------------------------------
int32_t tlbi_fail(int32_t code, const std::string& msg) { return fail(code, msg); }

int tlbi_phi_rebase_launch(const tlb_grid* g, tlbi_launch* out) {
  if (!g->phi_base) return 0;
  const RebaseArgs args{g->phi_base, static_cast<float*>(g->phi[0]),
                        (long long)g->p.n_theta * g->p.n_phi};
  static_assert(sizeof(args) <= sizeof(out->args), "argument block");
  out->fn = reinterpret_cast<const void*>(&tlb_phi_rebase_kernel);
  out->grid = dim3((unsigned)((args.plane + 255) / 256));
  out->block = dim3(256);
  std::memcpy(out->args, &args, sizeof(args));
  return 1;
}

int32_t tlbi_phi_rebase(const tlb_grid* g, hipStream_t stream) {
  if (!g->phi_base) return TLB_OK;
  const RebaseArgs args{g->phi_base, static_cast<float*>(g->phi[0]),
                        (long long)g->p.n_theta * g->p.n_phi};
  hipLaunchKernelGGL(tlb_phi_rebase_kernel, dim3((unsigned)((args.plane + 255) / 256)), dim3(256),
                     0, stream, args);
  TLB_HIP_CHECK(hipGetLastError());
  return TLB_OK;
}

int tlbi_stage_launches(const tlb_grid* g, int stage, tlbi_launch out[2]) {
  return g->p.precision == 64 ? stage_launches<double>(g, stage, out)
                              : stage_launches<float>(g, stage, out);
}

namespace {

// workspace: X [nt][np] complex, twiddles (np + nt) complex, partials 2 np doubles
size_t dft_bytes(const tlb_grid* g) {
  const size_t nt = g->p.n_theta, np = g->p.n_phi;
  return (nt * np + np + nt) * sizeof(double2) + 2 * np * sizeof(double);
}

template <typename T>
int32_t structure_t(tlb_grid* g, double out[3]) {
  const int nt = g->p.n_theta, np = g->p.n_phi;
  if ((size_t)np * sizeof(double) > 64 * 1024 || (size_t)nt * sizeof(double2) > 64 * 1024)
    return fail(TLB_EINVAL, "structure factor: a row or column exceeds the 64 KB of LDS per block");
  double2* X = nullptr;
  double2* tw = nullptr;
  double* part = nullptr;
  if (!g->dft_work) {
    hipError_t e = hipMalloc(&g->dft_work, dft_bytes(g));
    if (e != hipSuccess) {
      g->dft_work = nullptr;
      return fail(TLB_ENOMEM, std::string("structure factor workspace: ") + hipGetErrorString(e));
    }
    std::vector<double2> h(np + nt);
    for (int j = 0; j < np; ++j)
      h[j] = make_double2(std::cos(2.0 * M_PI * j / np), -std::sin(2.0 * M_PI * j / np));
    for (int j = 0; j < nt; ++j)
      h[np + j] = make_double2(std::cos(2.0 * M_PI * j / nt), -std::sin(2.0 * M_PI * j / nt));
    X = static_cast<double2*>(g->dft_work);
    TLB_HIP_CHECK(hipMemcpy(X + (size_t)nt * np, h.data(), h.size() * sizeof(double2),
                            hipMemcpyHostToDevice));
  }
  X = static_cast<double2*>(g->dft_work);
  tw = X + (size_t)nt * np;
  part = reinterpret_cast<double*>(tw + np + nt);
  hipLaunchKernelGGL(tlb_dft_rows_kernel<T>, dim3(nt), dim3(RED_THREADS), np * sizeof(double),
                     g->stream, static_cast<const T*>(g->phi[0]),
                     reinterpret_cast<const T*>(g->phi_base), tw, X, np);
  TLB_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(tlb_dft_cols_kernel, dim3(np), dim3(RED_THREADS), nt * sizeof(double2),
                     g->stream, X, tw + np, nt, np, g->p.r, g->p.R, part);
  TLB_HIP_CHECK(hipGetLastError());
  std::vector<double> h(2 * (size_t)np);
  TLB_HIP_CHECK(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                               g->stream));
  TLB_HIP_CHECK(hipStreamSynchronize(g->stream));
  double s0 = 0.0, s1 = 0.0;
  for (int mp = 0; mp < np; ++mp) {
    s0 += h[2 * mp];
    s1 += h[2 * mp + 1];
  }
  out[0] = s1 > 0.0 ? 2.0 * M_PI * s0 / s1 : INFINITY;
  out[1] = s0;
  out[2] = s1;
  return TLB_OK;
}

// ---- the structure-factor length without allocation (tlb_structure_length_noalloc)
//
// Its workspace is `scratch`, a device array of this file: one copy per GPU, kept until the
// process ends, shared by every call on that GPU (calls that overlap on one GPU race).  Host
// code never passes `scratch` itself (the name stands for a host-side shadow): the device
// address of each GPU's copy is taken once per device with hipGetSymbolAddress and kept.
// Layout: X [nt][np] complex, twiddles (np + nt) complex, partials 2 np doubles, 3 results.
constexpr size_t SCRATCH_BYTES = size_t(24) << 20;
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_DEVICES] = {};

size_t scratch_need(int nt, int np) {
  return ((size_t)nt * np + (size_t)np + nt) * sizeof(double2) + 2 * (size_t)np * sizeof(double) +
         3 * sizeof(double);
}

// the device address of the current device's `scratch` (looked up on its first use)
int32_t scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return fail_static(TLB_EHIP, "structure factor (no allocation): hipGetDevice failed");
  if (dev < 0 || dev >= SCRATCH_DEVICES)
    return fail_static(TLB_EHIP, "structure factor (no allocation): device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return fail_static(TLB_EHIP, "structure factor (no allocation): hipGetSymbolAddress failed");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TLB_OK;
}

// exp(-2 pi i j / n) for j < np (row transform) followed by the same for the column length nt
__global__ __launch_bounds__(RED_THREADS) void tlb_twiddle_kernel(double2* tw, int np, int nt) {
  const int j = blockIdx.x * RED_THREADS + threadIdx.x;
  if (j >= np + nt) return;
  const int n = j < np ? np : nt, m = j < np ? j : j - np;
  double sn, cs;
  sincospi(2.0 * m / n, &sn, &cs);
  tw[j] = make_double2(cs, -sn);
}

// sums of the per-mode partials in a fixed order and L_S = 2 pi sum S / sum |k| S
__global__ __launch_bounds__(RED_THREADS) void tlb_structure_final_kernel(const double* part,
                                                                         int np, double* out) {
  __shared__ double sh[2][RED_THREADS / 64];
  double s0 = 0.0, s1 = 0.0;
  for (int mp = threadIdx.x; mp < np; mp += RED_THREADS) {
    s0 += part[2 * mp];
    s1 += part[2 * mp + 1];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = s0;
    sh[1][w] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < RED_THREADS / 64; ++i) {
      a += sh[0][i];
      b += sh[1][i];
    }
    out[0] = b > 0.0 ? 2.0 * M_PI * a / b : INFINITY;
    out[1] = a;
    out[2] = b;
  }
}

template <typename T>
int32_t structure_noalloc_t(tlb_grid* g, double out[3]) {
  const int nt = g->p.n_theta, np = g->p.n_phi;
  if ((size_t)np * sizeof(double) > 64 * 1024 || (size_t)nt * sizeof(double2) > 64 * 1024)
    return fail_static(TLB_EINVAL,
                       "structure factor: a row or column exceeds the 64 KB of LDS per block");
  if (scratch_need(nt, np) > SCRATCH_BYTES)
    return fail_static(TLB_EINVAL,
                       "structure factor (no allocation): grid too large for the 24 MiB "
                       "workspace ((n_theta n_phi + n_theta + n_phi) 16 + n_phi 16 + 24 bytes)");
  void* base = nullptr;
  int32_t rc = scratch_address(&base);
  if (rc != TLB_OK) return rc;
  double2* X = static_cast<double2*>(base);
  double2* tw = X + (size_t)nt * np;
  double* part = reinterpret_cast<double*>(tw + np + nt);
  double* res = part + 2 * (size_t)np;
  hipLaunchKernelGGL(tlb_twiddle_kernel, dim3((np + nt + RED_THREADS - 1) / RED_THREADS),
                     dim3(RED_THREADS), 0, g->stream, tw, np, nt);
  hipLaunchKernelGGL(tlb_dft_rows_kernel<T>, dim3(nt), dim3(RED_THREADS), np * sizeof(double),
                     g->stream, static_cast<const T*>(g->phi[0]),
                     reinterpret_cast<const T*>(g->phi_base), tw, X, np);
  hipLaunchKernelGGL(tlb_dft_cols_kernel, dim3(np), dim3(RED_THREADS), nt * sizeof(double2),
                     g->stream, X, tw + np, nt, np, g->p.r, g->p.R, part);
  hipLaunchKernelGGL(tlb_structure_final_kernel, dim3(1), dim3(RED_THREADS), 0, g->stream, part,
                     np, res);
  if (hipGetLastError() != hipSuccess)
    return fail_static(TLB_EHIP, "structure factor (no allocation): kernel launch failed");
  if (hipMemcpyAsync(out, res, 3 * sizeof(double), hipMemcpyDeviceToHost, g->stream) !=
          hipSuccess ||
      hipStreamSynchronize(g->stream) != hipSuccess)
    return fail_static(TLB_EHIP, "structure factor (no allocation): copy of the result failed");
  return TLB_OK;
}

}  // namespace

extern "C" {

int32_t tlb_structure_length_noalloc(tlb_grid* g, double out[3]) {
  clear_error();
  if (!g || !out) return fail_static(TLB_EINVAL, "grid or out is NULL");
  return g->p.precision == 64 ? structure_noalloc_t<double>(g, out)
                              : structure_noalloc_t<float>(g, out);
}

const char* tlb_last_error(void) {
  return g_static_error ? g_static_error : g_last_error.c_str();
}

int32_t tlb_structure_length(tlb_grid* g, double out[3]) {
  clear_error();
  if (!g || !out) return fail(TLB_EINVAL, "grid or out is NULL");
  return g->p.precision == 64 ? structure_t<double>(g, out) : structure_t<float>(g, out);
}

int32_t tlb_create_torus_grid(const tlb_params* params, const tlb_buffers* buffers,
                              void* hip_stream, tlb_grid** out) {
  clear_error();
  if (!out) return fail(TLB_EINVAL, "out is NULL");
  *out = nullptr;
  int32_t rc = check_params(params);
  if (rc != TLB_OK) return rc;
  if ((params->flags & TLB_STRICT_DT) && params->dt > stable_dt_bound(*params))
    return fail(TLB_EUNSTABLE, "dt " + std::to_string(params->dt) +
                                   " exceeds the stability bound " +
                                   std::to_string(stable_dt_bound(*params)));
  if (!buffers) return fail(TLB_EINVAL, "buffers is NULL");
  for (int i = 0; i < 3; ++i)
    if (!buffers->f[i] || !buffers->phi[i]) return fail(TLB_EINVAL, "a state buffer is NULL");
  for (int i = 0; i < 6; ++i)
    for (int j = i + 1; j < 6; ++j) {
      const void* x = i < 3 ? buffers->f[i] : buffers->phi[i - 3];
      const void* y = j < 3 ? buffers->f[j] : buffers->phi[j - 3];
      if (x == y) return fail(TLB_EINVAL, "state buffers must be distinct");
    }
  tlb_grid* g = new (std::nothrow) tlb_grid{};
  if (!g) return fail(TLB_ENOMEM, "host allocation failed");
  g->p = *params;
  for (int i = 0; i < 3; ++i) {
    g->f[i] = buffers->f[i];
    g->phi[i] = buffers->phi[i];
  }
  g->stream = static_cast<hipStream_t>(hip_stream);
  g->elem = params->precision == 64 ? sizeof(double) : sizeof(float);
  g->ty = DEFAULT_TY;
  g->n_ref = 1.0;
  g->uid = g_next_uid.fetch_add(1);
  const int nt = params->n_theta;
  g->rows_per_block = nt <= 512 ? 1 : (nt + 511) / 512;
  g->red_blocks = (nt + g->rows_per_block - 1) / g->rows_per_block;

  const size_t row_bytes =
      params->precision == 64 ? sizeof(RowCoef<double>) : sizeof(RowCoef<float>);
  void* host_rows = std::malloc(row_bytes * nt);
  // area[q] in host_area[0..nt), theta-face length in host_area[nt..2nt)
  double* host_area = static_cast<double*>(std::malloc(sizeof(double) * 2 * nt));
  auto cleanup = [&](int32_t code, const std::string& msg) {
    std::free(host_rows);
    std::free(host_area);
    if (g->rows) (void)hipFree(g->rows);
    if (g->area) (void)hipFree(g->area);
    if (g->partial) (void)hipFree(g->partial);
    if (g->half_len) (void)hipFree(g->half_len);
    if (g->check_flag) (void)hipFree(g->check_flag);
    if (g->proj) (void)hipFree(g->proj);
    if (g->ch4) (void)hipFree(g->ch4);
    if (g->phi_base) (void)hipFree(g->phi_base);
    delete g;
    return fail(code, msg);
  };
  if (!host_rows || !host_area) return cleanup(TLB_ENOMEM, "host allocation failed");
  if (params->precision == 64)
    make_rows<double>(*params, static_cast<RowCoef<double>*>(host_rows), host_area);
  else
    make_rows<float>(*params, static_cast<RowCoef<float>*>(host_rows), host_area);

  hipError_t e = hipMalloc(&g->rows, row_bytes * nt);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&g->area), sizeof(double) * nt);
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void**>(&g->partial),
                  sizeof(double) * (3 * g->red_blocks + 3));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&g->half_len), sizeof(double) * nt);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&g->check_flag), sizeof(int));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&g->proj), sizeof(double) * 3 * nt);
  if (e == hipSuccess && (params->flags & TLB_CH4))
    e = hipMalloc(&g->ch4, 3 * (size_t)nt * params->n_phi * g->elem);
  if (e == hipSuccess && params->precision == 32)
    e = hipMalloc(reinterpret_cast<void**>(&g->phi_base), (size_t)nt * params->n_phi * sizeof(float));
  if (e != hipSuccess)
    return cleanup(TLB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = hipMemcpyAsync(g->rows, host_rows, row_bytes * nt, hipMemcpyHostToDevice, g->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->area, host_area, sizeof(double) * nt, hipMemcpyHostToDevice,
                       g->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->half_len, host_area + nt, sizeof(double) * nt, hipMemcpyHostToDevice,
                       g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) return cleanup(TLB_EHIP, std::string("upload: ") + hipGetErrorString(e));
  std::free(host_rows);
  std::free(host_area);
  *out = g;
  return TLB_OK;
}

void tlb_destroy(tlb_grid* g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->stream);
  drop_graph(g);
  if (g->dft_work) (void)hipFree(g->dft_work);
  (void)hipFree(g->rows);
  (void)hipFree(g->area);
  (void)hipFree(g->partial);
  (void)hipFree(g->half_len);
  (void)hipFree(g->check_flag);
  (void)hipFree(g->proj);
  if (g->ch4) (void)hipFree(g->ch4);
  if (g->phi_base) (void)hipFree(g->phi_base);
  delete g;
}

int32_t tlb_set_state(tlb_grid* g, const void* f, const void* phi, const void* n,
                      const void* ut, const void* up) {
  clear_error();
  if (!g || !phi) return fail(TLB_EINVAL, "grid or phi is NULL");
  if (!f && (!n || !ut || !up)) return fail(TLB_EINVAL, "f is NULL and a moment field is NULL");
  const size_t plane_bytes = (size_t)g->p.n_theta * g->p.n_phi * g->elem;
  g->phase = 0;
  if (g->phi_base) {  // FP32: phi becomes the base, its deviation zero
    TLB_HIP_CHECK(
        hipMemcpyAsync(g->phi_base, phi, plane_bytes, hipMemcpyDeviceToDevice, g->stream));
    TLB_HIP_CHECK(hipMemsetAsync(g->phi[0], 0, plane_bytes, g->stream));
  } else {
    TLB_HIP_CHECK(hipMemcpyAsync(g->phi[0], phi, plane_bytes, hipMemcpyDeviceToDevice, g->stream));
  }
  if (f) {
    TLB_HIP_CHECK(
        hipMemcpyAsync(g->f[0], f, 16 * plane_bytes, hipMemcpyDeviceToDevice, g->stream));
    if (g->p.precision == 64) return TLB_OK;
    double mean = 0.0;
    int32_t rc = mean_density(g, 0.0, &mean);  // full populations: nothing to add
    if (rc != TLB_OK) return rc;
    set_reference(g, reference_density(mean));
    return offset_t<float>(g, g->f[0], -float(g->n_ref));
  }
  if (g->p.precision == 64) return init_feq_t<double>(g, n, ut, up);
  // FP32: equilibrium with the current reference density, then again with the one the state's
  // mean density asks for if that differs
  int32_t rc = init_feq_t<float>(g, n, ut, up);
  double mean = 0.0;
  if (rc == TLB_OK) rc = mean_density(g, g->n_ref, &mean);
  if (rc != TLB_OK) return rc;
  const double n_ref = reference_density(mean);
  if (n_ref == g->n_ref) return TLB_OK;
  set_reference(g, n_ref);
  return init_feq_t<float>(g, n, ut, up);
}

int32_t tlb_stable_dt(const tlb_params* params, double* dt_max) {
  clear_error();
  if (!dt_max) return fail(TLB_EINVAL, "dt_max is NULL");
  if (!params) return fail(TLB_EINVAL, "params is NULL");
  tlb_params p = *params;
  p.dt = 1.0;  // the bound does not depend on dt; let validation look at the rest
  int32_t rc = check_params(&p);
  if (rc != TLB_OK) return rc;
  *dt_max = stable_dt_bound(p);
  return TLB_OK;
}

int32_t tlb_step_n(tlb_grid* g, int64_t n_steps) {
  clear_error();
  if (!g) return fail(TLB_EINVAL, "grid is NULL");
  if (n_steps < 0) return fail(TLB_EINVAL, "n_steps < 0");
  const bool dbl = g->p.precision == 64;
  const int64_t every = g->p.check_every;
  if (every <= 0) return dbl ? step_n_t<double>(g, n_steps) : step_n_t<float>(g, n_steps);
  // checked run: clear the flag, step in runs of check_every with a check after each run (and
  // after the last step), then wait and report
  hipLaunchKernelGGL(tlb_set_flag_kernel, dim3(1), dim3(1), 0, g->stream, g->check_flag, 0);
  TLB_HIP_CHECK(hipGetLastError());
  int64_t done = 0;
  do {
    const int64_t m = std::min(every, n_steps - done);
    int32_t rc = dbl ? step_n_t<double>(g, m) : step_n_t<float>(g, m);
    if (rc == TLB_OK) rc = dbl ? check_t<double>(g) : check_t<float>(g);
    if (rc != TLB_OK) return rc;
    done += m;
  } while (done < n_steps);
  int flag = 0;
  TLB_HIP_CHECK(hipMemcpyAsync(&flag, g->check_flag, sizeof(int), hipMemcpyDeviceToHost,
                               g->stream));
  TLB_HIP_CHECK(hipStreamSynchronize(g->stream));
  if (flag) return fail(TLB_ENONFINITE, "non-finite values in the state after a checked run");
  return TLB_OK;
}

int32_t tlb_get_moments(tlb_grid* g, void* n, void* ut, void* up, void* phi, void* mu) {
  clear_error();
  if (!g) return fail(TLB_EINVAL, "grid is NULL");
  return g->p.precision == 64 ? moments_t<double>(g, n, ut, up, phi, mu)
                              : moments_t<float>(g, n, ut, up, phi, mu);
}

int32_t tlb_get_state(tlb_grid* g, void* f, void* phi) {
  clear_error();
  if (!g) return fail(TLB_EINVAL, "grid is NULL");
  const size_t plane_bytes = (size_t)g->p.n_theta * g->p.n_phi * g->elem;
  if (f) {
    TLB_HIP_CHECK(
        hipMemcpyAsync(f, g->f[0], 16 * plane_bytes, hipMemcpyDeviceToDevice, g->stream));
    if (g->p.precision == 32) {
      int32_t rc = offset_t<float>(g, f, float(g->n_ref));
      if (rc != TLB_OK) return rc;
    }
  }
  if (phi && g->phi_base) {  // FP32: base + deviation
    const long long plane = (long long)g->p.n_theta * g->p.n_phi;
    hipLaunchKernelGGL(tlb_phi_sum_kernel, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0,
                       g->stream, static_cast<float*>(phi), g->phi_base,
                       static_cast<const float*>(g->phi[0]), plane);
    TLB_HIP_CHECK(hipGetLastError());
  } else if (phi) {
    TLB_HIP_CHECK(
        hipMemcpyAsync(phi, g->phi[0], plane_bytes, hipMemcpyDeviceToDevice, g->stream));
  }
  return TLB_OK;
}

int32_t tlb_invariants(tlb_grid* g, double out[3]) {
  clear_error();
  if (!g || !out) return fail(TLB_EINVAL, "grid or out is NULL");
  int32_t rc = g->p.precision == 64 ? reduce_t<double>(g, 0.0) : reduce_t<float>(g, g->n_ref);
  if (rc != TLB_OK) return rc;
  TLB_HIP_CHECK(hipMemcpyAsync(out, g->partial + 3 * g->red_blocks, 3 * sizeof(double),
                               hipMemcpyDeviceToHost, g->stream));
  TLB_HIP_CHECK(hipStreamSynchronize(g->stream));
  if (out[2] > 0) return fail(TLB_ENONFINITE, "non-finite values in the state");
  return TLB_OK;
}

int32_t tlb_set_tile_rows(tlb_grid* g, int32_t rows) {
  clear_error();
  if (!g) return fail(TLB_EINVAL, "grid is NULL");
  if (rows != 4 && rows != 8 && rows != 16) return fail(TLB_EINVAL, "tile rows must be 4, 8 or 16");
  if ((g->p.flags & (TLB_WENO5 | TLB_CH4)) && rows != DEFAULT_TY)
    return fail(TLB_EINVAL, "the WENO-5 and fourth-order CH variants run with tiles of 8 rows only");
  if (g->ty != rows) {
    g->ty = rows;
    drop_graph(g);
  }
  return TLB_OK;
}

int32_t tlb_autotune(tlb_grid* g, int32_t* rows) {
  clear_error();
  if (!g) return fail(TLB_EINVAL, "grid is NULL");
  if (g->p.flags & (TLB_WENO5 | TLB_CH4)) {  // one tile height only
    if (rows) *rows = g->ty;
    return TLB_OK;
  }
  return g->p.precision == 64 ? autotune_t<double>(g, rows) : autotune_t<float>(g, rows);
}

int32_t tlb_create_batch(tlb_grid* const* grids, int32_t n, void* hip_stream, tlb_batch** out) {
  clear_error();
  if (!out) return fail(TLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grids || n < 1) return fail(TLB_EINVAL, "a batch needs at least one grid");
  for (int i = 0; i < n; ++i) {
    if (!grids[i]) return fail(TLB_EINVAL, "a grid of the batch is NULL");
    if (grids[i]->p.precision != grids[0]->p.precision)
      return fail(TLB_EINVAL, "all grids of a batch must have the same precision");
    for (int j = 0; j < i; ++j)
      if (grids[j] == grids[i]) return fail(TLB_EINVAL, "a grid appears twice in the batch");
    if (grids[i]->p.flags & (TLB_WENO5 | TLB_CH4))
      return fail(TLB_EINVAL, "the WENO-5 and fourth-order CH variants are not available in batches");
  }
  tlb_batch* b = new (std::nothrow) tlb_batch{};
  if (!b) return fail(TLB_ENOMEM, "host allocation failed");
  b->grids = new (std::nothrow) tlb_grid*[n];
  if (!b->grids) {
    delete b;
    return fail(TLB_ENOMEM, "host allocation failed");
  }
  b->versions = new (std::nothrow) unsigned[n];
  if (!b->versions) {
    delete[] b->grids;
    delete b;
    return fail(TLB_ENOMEM, "host allocation failed");
  }
  b->n = n;
  b->precision = grids[0]->p.precision;
  b->ty = DEFAULT_TY;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->vec = true;
  double state_bytes = 0.0;
  for (int i = 0; i < n; ++i) {
    b->grids[i] = grids[i];
    b->vec = b->vec && (b->precision == 64 ? vec_ok<double>(grids[i]->p.n_phi)
                                           : vec_ok<float>(grids[i]->p.n_phi));
    state_bytes += 51.0 * grids[i]->p.n_theta * (double)grids[i]->p.n_phi * (double)grids[i]->elem;
  }
  b->streaming = state_bytes > STREAMING_BYTES;
  const size_t args_bytes = b->precision == 64 ? sizeof(StageArgs<double>) : sizeof(StageArgs<float>);
  hipError_t e = hipMalloc(&b->table, args_bytes * 3 * n);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&b->tile_begin), sizeof(int) * (n + 1));
  int32_t rc = TLB_OK;
  if (e != hipSuccess) rc = fail(TLB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (rc == TLB_OK)
    rc = b->precision == 64 ? batch_setup_t<double>(b) : batch_setup_t<float>(b);
  if (rc != TLB_OK) {
    tlb_destroy_batch(b);
    return rc;
  }
  *out = b;
  return TLB_OK;
}

int32_t tlb_batch_step_n(tlb_batch* b, int64_t n_steps) {
  clear_error();
  if (!b) return fail(TLB_EINVAL, "batch is NULL");
  if (n_steps < 0) return fail(TLB_EINVAL, "n_steps < 0");
  // a grid whose stage arguments changed since the table was built (a new reference density)
  for (int i = 0; i < b->n; ++i)
    if (b->versions[i] != b->grids[i]->version) {
      int32_t rc = b->precision == 64 ? batch_setup_t<double>(b) : batch_setup_t<float>(b);
      if (rc != TLB_OK) return rc;
      break;
    }
  return b->precision == 64 ? batch_step_t<double>(b, n_steps) : batch_step_t<float>(b, n_steps);
}

int32_t tlb_batch_autotune(tlb_batch* b, int32_t* rows) {
  clear_error();
  if (!b) return fail(TLB_EINVAL, "batch is NULL");
  return b->precision == 64 ? batch_autotune_t<double>(b, rows) : batch_autotune_t<float>(b, rows);
}

void tlb_destroy_batch(tlb_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  drop_batch_graph(b);
  if (b->table) (void)hipFree(b->table);
  if (b->tile_begin) (void)hipFree(b->tile_begin);
  delete[] b->grids;
  delete[] b->versions;
  delete b;
}

int32_t tlb_diagnostics(tlb_grid* g, double out[2], double* phi_avg, double* p_avg) {
  clear_error();
  if (!g) return fail(TLB_EINVAL, "grid is NULL");
  int32_t rc = g->p.precision == 64 ? diag_t<double>(g, phi_avg, p_avg)
                                    : diag_t<float>(g, phi_avg, p_avg);
  if (rc != TLB_OK) return rc;
  if (out) {
    double tmp[3];
    TLB_HIP_CHECK(hipMemcpyAsync(tmp, g->partial + 3 * g->red_blocks, 3 * sizeof(double),
                                 hipMemcpyDeviceToHost, g->stream));
    TLB_HIP_CHECK(hipStreamSynchronize(g->stream));
    out[0] = tmp[0];
    out[1] = tmp[1];
  }
  return TLB_OK;
}

}  // extern "C"
