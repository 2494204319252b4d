// libqla: the qubit lattice algorithm (QLA) time step of Vahala et al.,
// arXiv:2301.13601, as hand-written HIP for gfx950 (MI355X), behind the C ABI
// declared in include/qla.h.
//
// One time step is one launch of qla_step_kernel, which applies, for every
// site, the whole operator sequence of Eq. (23) or Eq. (28): U_X (Eq. (18),
// 16 factors), U_Y (Eq. (20), 16 factors) and the potentials V_X, V_Y
// (Eq. (21), (22)), with the collision angles of Eq. (24) and potential
// angles of Eq. (25) computed on the fly from n. State is FP32; the
// diagnostics (Eq. (27), div B, div D) accumulate in FP64.
//
// Work decomposition of the fused step (see the design notes for the why):
//  * a wave owns a strip of 64*C consecutive columns (C per lane) and a
//    segment of rows; it marches down its segment one row per iteration;
//  * the x sweep of the ingested row runs in registers: a streaming shift
//    along x is a register rename for C-1 of the lane's columns and one DPP
//    whole-wave shift for the last; the outermost ceil(4/C) lanes on each
//    side are halo (one step's x support is +-4 cells) and store nothing;
//  * the y sweep is a 16-stage register pipeline: a stage that streams from
//    y-1 reads a one-row delay register, a stage that streams from y+1
//    delays the other two active components by one row instead, so the
//    pipeline emits the fully stepped row R-4 after ingesting row R;
//  * the loop is unrolled four times so that every ring of per-row data
//    (collision coefficients, potential coefficients) is indexed by
//    compile-time slots and stays in registers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>

#include "qla.h"

namespace {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Cross-lane moves (DPP whole-wave shifts by one lane; the lane with no
// source receives 0, which only ever lands in halo lanes).
// ---------------------------------------------------------------------------
// bound_ctrl set: the lane without a source reads 0 (no old value needed)
__device__ __forceinline__ float from_next_lane(float v) {   // wave_shl:1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_prev_lane(float v) {   // wave_shr:1
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}

// Streaming along x in pull form: S^{+x} sets v(x) = v(x + 1).
template <int C>
__device__ __forceinline__ void pull_from_right(float (&v)[C]) {
  const float nb = from_next_lane(v[0]);
#pragma unroll
  for (int k = 0; k < C - 1; ++k) v[k] = v[k + 1];
  v[C - 1] = nb;
}
// S^{-x}: v(x) = v(x - 1).
template <int C>
__device__ __forceinline__ void pull_from_left(float (&v)[C]) {
  const float nb = from_prev_lane(v[C - 1]);
#pragma unroll
  for (int k = C - 1; k > 0; --k) v[k] = v[k - 1];
  v[0] = nb;
}

// ---------------------------------------------------------------------------
// Rotation R(phi) of the pair (a, b): a' = cos a - sin b, b' = sin a + cos b,
// as three shears with t = tan(phi/2), s = sin(phi). SGN = -1 rotates by
// -phi. Both coefficients are small numbers carried at full relative
// precision, which keeps cos^2 + sin^2 = 1 to FP32 rounding (a cos(phi)
// rounded to FP32 does not, and that bias compounds over the 32 rotations
// of every step).
// ---------------------------------------------------------------------------
template <int SGN>
__device__ __forceinline__ void rot(float& a, float& b, float t, float s) {
  if constexpr (SGN > 0) {
    a = fmaf(-t, b, a);
    b = fmaf(s, a, b);
    a = fmaf(-t, b, a);
  } else {
    a = fmaf(t, b, a);
    b = fmaf(-s, a, b);
    a = fmaf(t, b, a);
  }
}

// (t, s) = (tan(theta/2), sin(theta)). The short series is accurate to well
// below an FP32 ulp for |theta| <= kNarrowAngle; wider angles use libm.
constexpr float kNarrowAngle = 0.12f;

template <bool WIDE>
__device__ __forceinline__ void rot_coef(float th, float& t, float& s) {
  if constexpr (WIDE) {
    s = sinf(th);
    t = tanf(0.5f * th);
  } else {
    const float th2 = th * th;
    s = th * fmaf(th2, fmaf(th2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
    t = th * fmaf(th2, fmaf(th2, 1.0f / 240.0f, 1.0f / 24.0f), 0.5f);
  }
}

// Potential coefficients (sin b, 1 - cos b) for an applied angle b.
template <bool WIDE>
__device__ __forceinline__ void pot_coef(float b, float& sb, float& hb) {
  if constexpr (WIDE) {
    sb = sinf(b);
    const float h = sinf(0.5f * b);
    hb = 2.0f * h * h;
  } else {
    const float b2 = b * b;
    sb = b * fmaf(b2, fmaf(b2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
    hb = b2 * fmaf(b2, fmaf(b2, 1.0f / 720.0f, -1.0f / 24.0f), 0.5f);
  }
}

// a' = cos(b) a + sgn * sin(b) p  ==  a - (1 - cos b) a + sgn sin(b) p
__device__ __forceinline__ float pot_row(float a, float p, float sb, float hb) {
  return fmaf(sb, p, fmaf(-hb, a, a));
}

// ---------------------------------------------------------------------------
// Step kernel.
// ---------------------------------------------------------------------------
struct StepArgs {
  const float* __restrict__ qin;   // 6 planes
  float* __restrict__ qout;        // 6 planes
  const float* __restrict__ n;     // 3 planes
  int64_t plane;                   // nx * ny
  int nx, ny;
  int seg_rows;                    // rows per wave segment (multiple of 4)
  int nstrips, nsegs;
  int waves_per_block;
  float a4;                        // delta / 4                    (Eq. (24))
  float kb;                        // kappa * frac / 2             (Eq. (25))
};

template <int C>
struct Cols {
  static constexpr int kHaloLanes = (4 + C - 1) / C;
  static constexpr int kOut = (kWave - 2 * kHaloLanes) * C;   // output columns per strip
};

__device__ __forceinline__ int wrap_index(int64_t i, int n) {
  int64_t r = i % n;
  return static_cast<int>(r < 0 ? r + n : r);
}

// Loads and stores of one row of one plane go through a buffer resource
// whose base is the row (wave-uniform, scalar registers) and whose extent is
// the row's nx floats; the lane supplies a fixed byte offset. A lane that
// must not store uses an offset past the extent, which the hardware drops.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;        // raw 32-bit buffer, gfx9 family
constexpr uint32_t kNoStore = 0x80000000u;    // beyond any row extent

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float* row, int nx) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(row), 0, nx * 4, kRsrcWord3);
}

template <int C, bool VEC>
__device__ __forceinline__ void load_row(const float* row, int nx, const uint32_t (&xb)[C],
                                         float (&out)[C]) {
  const __amdgpu_buffer_rsrc_t r = row_rsrc(row, nx);
  if constexpr (VEC && C == 4) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, xb[0], 0, 0);
    out[0] = __uint_as_float(v.x); out[1] = __uint_as_float(v.y);
    out[2] = __uint_as_float(v.z); out[3] = __uint_as_float(v.w);
  } else if constexpr (VEC && C == 2) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, xb[0], 0, 0);
    out[0] = __uint_as_float(v.x); out[1] = __uint_as_float(v.y);
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) out[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, xb[k], 0, 0));
  }
}

template <int C, bool VEC>
__device__ __forceinline__ void store_row(float* row, int nx, const uint32_t (&sb)[C],
                                          const float (&v)[C]) {
  const __amdgpu_buffer_rsrc_t r = row_rsrc(row, nx);
  if constexpr (VEC && C == 4) {
    u32x4 w;
    w.x = __float_as_uint(v[0]); w.y = __float_as_uint(v[1]);
    w.z = __float_as_uint(v[2]); w.w = __float_as_uint(v[3]);
    __builtin_amdgcn_raw_buffer_store_b128(w, r, sb[0], 0, 0);
  } else if constexpr (VEC && C == 2) {
    u32x2 w;
    w.x = __float_as_uint(v[0]); w.y = __float_as_uint(v[1]);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, sb[0], 0, 0);
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[k]), r, sb[k], 0, 0);
  }
}

// true on every lane if any lane's flag is set (a wave-uniform branch)
__device__ __forceinline__ bool wave_any(bool v) { return __any(v) != 0; }

// Everything a wave carries from one row iteration to the next. The wave
// marches through its segment in direction DIR (+1: increasing y, -1:
// decreasing y); "row R" is the row ingested this iteration and "lag k" the
// row ingested k iterations ago (R - k*DIR).
template <int C>
struct Pipe {
  // y-sweep stream stages (the 8 S^{+-y} of Eq. (20) in the order they act):
  // one-row delay registers for two components each
  float d[8][2][C];
  // collision coefficients (tan(theta_0/2), sin theta_0, tan(theta_2/2),
  // sin theta_2) of rows lag 1..4, slot = iteration mod 4
  float th[4][4][C];
  // V_Y coefficients (sin b1, 1-cos b1, sin b3, 1-cos b3) per row slot, and
  // whether the row has any nonzero y-difference of n_x or n_z (when it
  // has none, beta_1 = beta_3 = 0 and V_Y is exactly the identity)
  float vy[4][4][C];
  bool fy[4];
  // Eq. (23) only: V_X coefficients, their flag and the (q1, q4) pair per row
  // slot, all applied after U_Y
  float vx[4][4][C];
  bool fx[4];
  float q14[4][2][C];
  // the ingested row R and the rows in flight: Q of R and R+DIR, n of R-DIR
  // (x and z components), R, R+DIR and R+2*DIR
  float q[6][C];
  float q1[6][C];
  float nprev[2][C];
  float ncur[3][C];
  float nnext[3][C];
  float nn2[3][C];
};

struct RowBases {
  const float* qld;    // Q row R+2*DIR (plane 0)
  const float* nld;    // n row R+3*DIR (plane 0)
};

// Lag (in rows) of the y-pipeline after each of its 8 stream stages. A stage
// that pulls from the row ahead in marching order (S^{+y} when marching in
// +y, S^{-y} when marching in -y) has to wait one more row.
template <int DIR>
struct YLags {
  // stream stages in acting order: S-03 S+03 S+25 S-25 S+03 S-03 S-25 S+25
  static constexpr int sgn[8] = {-1, +1, +1, -1, +1, -1, -1, +1};
  static constexpr int after(int k) {
    int l = 0;
    for (int j = 0; j <= k; ++j) l += (sgn[j] == DIR) ? 1 : 0;
    return l;
  }
  static constexpr int before(int k) { return k == 0 ? 0 : after(k - 1); }
};

// MODE: 0 = Eq. (23), 1 = Eq. (28). POT: potentials present (kappa != 0).
template <int C, bool VEC, bool WIDE, int MODE, bool POT, int DIR, int SLOT>
__device__ __forceinline__ void row_iteration(Pipe<C>& p, const StepArgs& g, const uint32_t (&xo)[C],
                                              const uint32_t (&so)[C], bool edge_lane, int i,
                                              int seg_h, int y0, const RowBases& rb) {
  // ---- prefetch Q of row R+2*DIR and n of row R+3*DIR ---------------------
  float qld[6][C];
  float nld[3][C];
#pragma unroll
  for (int c = 0; c < 6; ++c) load_row<C, VEC>(rb.qld + c * g.plane, g.nx, xo, qld[c]);
#pragma unroll
  for (int c = 0; c < 3; ++c) load_row<C, VEC>(rb.nld + c * g.plane, g.nx, xo, nld[c]);

  // ---- coefficients of row R (Eq. (24), (25)) -----------------------------
  float u[3][C];
  float tc[3][C], sc[3][C];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      u[c][k] = __builtin_amdgcn_rcpf(p.ncur[c][k]);
      rot_coef<WIDE>(g.a4 * u[c][k], tc[c][k], sc[c][k]);
    }
  }
  // V_X coefficients from the x-differences of n_y (beta_0) and n_z (beta_2).
  // Lanes 0 and 63 see a zero from the DPP shift at the wave edge; their
  // values only reach halo columns, so they do not vote.
  float vxs0[C], vxh0[C], vxs2[C], vxh2[C];
  bool fx = false;
  if constexpr (POT) {
    float dny[C], dnz[C];
    {
      float r1[C], l1[C], r2[C], l2[C];
#pragma unroll
      for (int k = 0; k < C; ++k) {
        r1[k] = l1[k] = p.ncur[1][k];
        r2[k] = l2[k] = p.ncur[2][k];
      }
      pull_from_right<C>(r1); pull_from_left<C>(l1);
      pull_from_right<C>(r2); pull_from_left<C>(l2);
      bool nz = false;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        dny[k] = r1[k] - l1[k];
        dnz[k] = r2[k] - l2[k];
        nz = nz || dny[k] != 0.0f || dnz[k] != 0.0f;
      }
      fx = wave_any(nz && !edge_lane);
    }
    if (fx) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const float b0 = g.kb * dny[k] * (u[1][k] * u[1][k]);
        const float b2 = g.kb * dnz[k] * (u[2][k] * u[2][k]);
        pot_coef<WIDE>(b0, vxs0[k], vxh0[k]);
        pot_coef<WIDE>(b2, vxs2[k], vxh2[k]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < C; ++k) vxs0[k] = vxh0[k] = vxs2[k] = vxh2[k] = 0.0f;
    }
  }

  // ---- U_X (Eq. (18)) with V_X' interleaved (Eq. (28)) on row R ------------
  float (&q)[6][C] = p.q;
  const float (&t1)[C] = tc[1];
  const float (&s1)[C] = sc[1];
  const float (&t2)[C] = tc[2];
  const float (&s2)[C] = sc[2];
  auto cx = [&](auto sgn) {
    constexpr int S = decltype(sgn)::value;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      rot<S>(q[1][k], q[5][k], t1[k], s1[k]);
      rot<S>(q[2][k], q[4][k], t2[k], s2[k]);
    }
  };
  using P_ = std::integral_constant<int, 1>;
  using M_ = std::integral_constant<int, -1>;
  auto vx_apply = [&]() {
    if (fx) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        q[4][k] = pot_row(q[4][k], -q[2][k], vxs2[k], vxh2[k]);
        q[5][k] = pot_row(q[5][k], q[1][k], vxs0[k], vxh0[k]);
      }
    }
  };
  cx(M_{}); pull_from_left<C>(q[1]);  pull_from_left<C>(q[4]);
  cx(P_{}); pull_from_right<C>(q[1]); pull_from_right<C>(q[4]);
  cx(M_{}); pull_from_right<C>(q[2]); pull_from_right<C>(q[5]);
  cx(P_{}); pull_from_left<C>(q[2]);  pull_from_left<C>(q[5]);
  if constexpr (MODE == 1 && POT) vx_apply();
  cx(P_{}); pull_from_right<C>(q[1]); pull_from_right<C>(q[4]);
  cx(M_{}); pull_from_left<C>(q[1]);  pull_from_left<C>(q[4]);
  cx(P_{}); pull_from_left<C>(q[2]);  pull_from_left<C>(q[5]);
  cx(M_{}); pull_from_right<C>(q[2]); pull_from_right<C>(q[5]);
  if constexpr (MODE == 1 && POT) vx_apply();

  // rows of this iteration relative to y0: R, and R - 4*DIR which leaves
  // the pipeline; both lie in the segment for the same range of i
  const int R_rel = DIR > 0 ? i - 4 : seg_h + 3 - i;
  const int O_rel = DIR > 0 ? i - 8 : seg_h + 7 - i;
  const bool R_out = i >= 4 && i < seg_h + 4;
  const bool O_out = i >= 8 && i < seg_h + 8;
  if constexpr (MODE == 1) {
    // q1 and q4 are final once U_X and V_X' are done: U_Y and V_Y leave them
    if (R_out) {
      float* row = g.qout + static_cast<int64_t>(y0 + R_rel) * g.nx;
      store_row<C, VEC>(row + 1 * g.plane, g.nx, so, q[1]);
      store_row<C, VEC>(row + 4 * g.plane, g.nx, so, q[4]);
    }
  }

  // ---- U_Y (Eq. (20)) as a pipeline over rows ------------------------------
  // active components: a0 = q0, a5 = q5 (angle theta_0), b2 = q2, b3 = q3
  // (angle theta_2); C_Y rotates both pairs by -theta (Eq. (19)).
  float (&a0)[C] = q[0];
  float (&a5)[C] = q[5];
  float (&b2)[C] = q[2];
  float (&b3)[C] = q[3];
  using Lg = YLags<DIR>;
  // collision k (0..7) acts on the row at lag Lg::before(k); lag 0 is the
  // row just computed above, older rows come from the ring
  auto cy = [&](auto sgn, auto kk) {
    constexpr int S = decltype(sgn)::value;
    constexpr int lag = Lg::before(decltype(kk)::value);
    if constexpr (lag == 0) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        rot<-S>(a0[k], a5[k], tc[0][k], sc[0][k]);
        rot<-S>(b2[k], b3[k], tc[2][k], sc[2][k]);
      }
    } else {
      constexpr int sl = (SLOT - lag) & 3;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        rot<-S>(a0[k], a5[k], p.th[sl][0][k], p.th[sl][1][k]);
        rot<-S>(b2[k], b3[k], p.th[sl][2][k], p.th[sl][3][k]);
      }
    }
  };
  auto swap_in = [&](float (&cur)[C], float (&dly)[C]) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const float t = cur[k];
      cur[k] = dly[k];
      dly[k] = t;
    }
  };
  // stream stage k shifting (sa, sb) and leaving (ka, kb) of the active four
  auto sy = [&](auto kk, float (&sa)[C], float (&sb)[C], float (&ka)[C], float (&kb)[C]) {
    constexpr int k = decltype(kk)::value;
    if constexpr (Lg::sgn[k] == DIR) {
      // pulls from the row ahead: the other two wait one row
      swap_in(ka, p.d[k][0]);
      swap_in(kb, p.d[k][1]);
    } else {
      // pulls from the row behind: the shifted two come from the delay line
      swap_in(sa, p.d[k][0]);
      swap_in(sb, p.d[k][1]);
    }
  };
  auto vy_apply = [&](auto lag) {
    constexpr int sl = (SLOT - decltype(lag)::value) & 3;
    if (p.fy[sl]) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        b3[k] = pot_row(b3[k], b2[k], p.vy[sl][2][k], p.vy[sl][3][k]);
        a5[k] = pot_row(a5[k], -a0[k], p.vy[sl][0][k], p.vy[sl][1][k]);
      }
    }
  };
  using K0 = std::integral_constant<int, 0>;
  using K1 = std::integral_constant<int, 1>;
  using K2 = std::integral_constant<int, 2>;
  using K3 = std::integral_constant<int, 3>;
  using K4 = std::integral_constant<int, 4>;
  using K5 = std::integral_constant<int, 5>;
  using K6 = std::integral_constant<int, 6>;
  using K7 = std::integral_constant<int, 7>;
  static_assert(Lg::after(3) == 2 && Lg::after(7) == 4, "V_Y' acts at lags 2 and 4");
  // Eq. (20), right to left
  cy(M_{}, K0{});  sy(K0{}, a0, b3, a5, b2);      // C_Y^dagger, S^{-y}_{03}
  cy(P_{}, K1{});  sy(K1{}, a0, b3, a5, b2);      // C_Y,        S^{+y}_{03}
  cy(M_{}, K2{});  sy(K2{}, b2, a5, a0, b3);      // C_Y^dagger, S^{+y}_{25}
  cy(P_{}, K3{});  sy(K3{}, b2, a5, a0, b3);      // C_Y,        S^{-y}_{25}
  if constexpr (MODE == 1 && POT) vy_apply(std::integral_constant<int, 2>{});   // V_Y' (Eq. (28))
  cy(P_{}, K4{});  sy(K4{}, a0, b3, a5, b2);      // C_Y,        S^{+y}_{03}
  cy(M_{}, K5{});  sy(K5{}, a0, b3, a5, b2);      // C_Y^dagger, S^{-y}_{03}
  cy(P_{}, K6{});  sy(K6{}, b2, a5, a0, b3);      // C_Y,        S^{-y}_{25}
  cy(M_{}, K7{});  sy(K7{}, b2, a5, a0, b3);      // C_Y^dagger, S^{+y}_{25}
  // the pipeline now holds the row at lag 4
  float o1[C], o4[C];
  if constexpr (MODE == 1) {
    if constexpr (POT) vy_apply(std::integral_constant<int, 4>{});   // V_Y' (Eq. (28))
  } else {
    // Eq. (23): V_X then V_Y after U_Y, on the row at lag 4
    constexpr int sl = (SLOT - 4) & 3;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      o1[k] = p.q14[sl][0][k];
      o4[k] = p.q14[sl][1][k];
    }
    if constexpr (POT) {
      if (p.fx[sl]) {
#pragma unroll
        for (int k = 0; k < C; ++k) {
          o4[k] = pot_row(o4[k], -b2[k], p.vx[sl][2][k], p.vx[sl][3][k]);
          a5[k] = pot_row(a5[k], o1[k], p.vx[sl][0][k], p.vx[sl][1][k]);
        }
      }
      vy_apply(std::integral_constant<int, 4>{});
    }
  }
  if (O_out) {
    float* row = g.qout + static_cast<int64_t>(y0 + O_rel) * g.nx;
    store_row<C, VEC>(row + 0 * g.plane, g.nx, so, a0);
    store_row<C, VEC>(row + 2 * g.plane, g.nx, so, b2);
    store_row<C, VEC>(row + 3 * g.plane, g.nx, so, b3);
    store_row<C, VEC>(row + 5 * g.plane, g.nx, so, a5);
    if constexpr (MODE == 0) {
      store_row<C, VEC>(row + 1 * g.plane, g.nx, so, o1);
      store_row<C, VEC>(row + 4 * g.plane, g.nx, so, o4);
    }
  }

  // ---- per-row data kept for later rows (slot SLOT held the row at lag 4,
  // consumed above) ------------------------------------------------------------
#pragma unroll
  for (int k = 0; k < C; ++k) {
    p.th[SLOT][0][k] = tc[0][k];
    p.th[SLOT][1][k] = sc[0][k];
    p.th[SLOT][2][k] = tc[2][k];
    p.th[SLOT][3][k] = sc[2][k];
  }
  if constexpr (MODE == 0) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      p.q14[SLOT][0][k] = p.q[1][k];
      p.q14[SLOT][1][k] = p.q[4][k];
    }
    if constexpr (POT) {
      p.fx[SLOT] = fx;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        p.vx[SLOT][0][k] = vxs0[k];
        p.vx[SLOT][1][k] = vxh0[k];
        p.vx[SLOT][2][k] = vxs2[k];
        p.vx[SLOT][3][k] = vxh2[k];
      }
    }
  }
  if constexpr (POT) {
    // V_Y coefficients of row R from the y-differences n(R+1) - n(R-1) of
    // n_x (beta_1) and n_z (beta_3)
    float d1[C], d3[C];
    bool nz = false;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      if constexpr (DIR > 0) {
        d1[k] = p.nnext[0][k] - p.nprev[0][k];
        d3[k] = p.nnext[2][k] - p.nprev[1][k];
      } else {
        d1[k] = p.nprev[0][k] - p.nnext[0][k];
        d3[k] = p.nprev[1][k] - p.nnext[2][k];
      }
      nz = nz || d1[k] != 0.0f || d3[k] != 0.0f;
    }
    const bool fy = wave_any(nz);
    p.fy[SLOT] = fy;
    if (fy) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const float b1 = g.kb * d1[k] * (u[0][k] * u[0][k]);
        const float b3c = g.kb * d3[k] * (u[2][k] * u[2][k]);
        pot_coef<WIDE>(b1, p.vy[SLOT][0][k], p.vy[SLOT][1][k]);
        pot_coef<WIDE>(b3c, p.vy[SLOT][2][k], p.vy[SLOT][3][k]);
      }
    }
  }
  // advance the row window
#pragma unroll
  for (int k = 0; k < C; ++k) {
    p.nprev[0][k] = p.ncur[0][k];
    p.nprev[1][k] = p.ncur[2][k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p.ncur[c][k] = p.nnext[c][k];
      p.nnext[c][k] = p.nn2[c][k];
      p.nn2[c][k] = nld[c][k];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      p.q[c][k] = p.q1[c][k];
      p.q1[c][k] = qld[c][k];
    }
  }
}

// One wave's march over its segment in direction DIR.
template <int C, bool VEC, bool WIDE, int MODE, bool POT, int DIR>
__device__ __forceinline__ void march(const StepArgs& g, const uint32_t (&xo)[C],
                                      const uint32_t (&so)[C], bool edge_lane, int y0, int seg_h) {
  Pipe<C> p;
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int k = 0; k < C; ++k) p.d[s][c][k] = 0.0f;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    p.fy[s] = false;
    p.fx[s] = false;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int k = 0; k < C; ++k) {
        p.th[s][c][k] = 0.0f;
        p.vy[s][c][k] = 0.0f;
        p.vx[s][c][k] = 0.0f;
      }
#pragma unroll
    for (int k = 0; k < C; ++k) p.q14[s][0][k] = p.q14[s][1][k] = 0.0f;
  }

  // first ingested row: 4 rows before the segment in marching order
  const int64_t R0 = DIR > 0 ? static_cast<int64_t>(y0) - 4 : static_cast<int64_t>(y0) + seg_h + 3;
  const int64_t nx64 = g.nx;
  {
    const float* q0r = g.qin + wrap_index(R0, g.ny) * nx64;
    const float* q1r = g.qin + wrap_index(R0 + DIR, g.ny) * nx64;
    const float* nm = g.n + wrap_index(R0 - DIR, g.ny) * nx64;
    const float* n0 = g.n + wrap_index(R0, g.ny) * nx64;
    const float* n1 = g.n + wrap_index(R0 + DIR, g.ny) * nx64;
    const float* n2 = g.n + wrap_index(R0 + 2 * DIR, g.ny) * nx64;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      load_row<C, VEC>(q0r + c * g.plane, g.nx, xo, p.q[c]);
      load_row<C, VEC>(q1r + c * g.plane, g.nx, xo, p.q1[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      load_row<C, VEC>(n0 + c * g.plane, g.nx, xo, p.ncur[c]);
      load_row<C, VEC>(n1 + c * g.plane, g.nx, xo, p.nnext[c]);
      load_row<C, VEC>(n2 + c * g.plane, g.nx, xo, p.nn2[c]);
    }
    load_row<C, VEC>(nm + 0 * g.plane, g.nx, xo, p.nprev[0]);
    load_row<C, VEC>(nm + 2 * g.plane, g.nx, xo, p.nprev[1]);
  }
  // rows in flight: Q of R+2*DIR, n of R+3*DIR (wrapped incrementally)
  int rq = wrap_index(R0 + 2 * DIR, g.ny);
  int rn = wrap_index(R0 + 3 * DIR, g.ny);
  const int iters = ((seg_h + 8) + 3) & ~3;
  for (int i = 0; i < iters; i += 4) {
#define QLA_ITER(S)                                                                            \
  {                                                                                            \
    const RowBases rb{g.qin + rq * nx64, g.n + rn * nx64};                                     \
    row_iteration<C, VEC, WIDE, MODE, POT, DIR, S>(p, g, xo, so, edge_lane, i + S, seg_h, y0,  \
                                                   rb);                                        \
    if constexpr (DIR > 0) {                                                                   \
      rq = (rq + 1 == g.ny) ? 0 : rq + 1;                                                      \
      rn = (rn + 1 == g.ny) ? 0 : rn + 1;                                                      \
    } else {                                                                                   \
      rq = (rq == 0) ? g.ny - 1 : rq - 1;                                                      \
      rn = (rn == 0) ? g.ny - 1 : rn - 1;                                                      \
    }                                                                                          \
  }
    QLA_ITER(0)
    QLA_ITER(1)
    QLA_ITER(2)
    QLA_ITER(3)
#undef QLA_ITER
  }
}

template <int C, bool VEC, bool WIDE, int MODE, bool POT>
__global__ void __launch_bounds__(256) qla_step_kernel(StepArgs g) {
  const int lane = threadIdx.x & (kWave - 1);
  // wave index within the block, as a wave-uniform (scalar) value
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));
  // blocks are dealt round-robin to the 8 XCDs; regroup them so that each
  // XCD gets a contiguous band of the lattice (neighbouring strips and
  // segments share halo data through that XCD's L2)
  const int nblk = gridDim.x;
  const int b = blockIdx.x;
  const int per = nblk / 8;
  const int rem = nblk % 8;
  const int xcd = b % 8;
  const int k8 = b / 8;
  const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
  const int strip = logical % g.nstrips;
  const int seg = (logical / g.nstrips) * g.waves_per_block + wave;
  if (seg >= g.nsegs) return;

  const int y0 = seg * g.seg_rows;
  const int seg_h = min(g.seg_rows, g.ny - y0);
  const int x0 = strip * Cols<C>::kOut;
  const int64_t col0 = static_cast<int64_t>(x0) - Cols<C>::kHaloLanes * C + lane * C;
  // byte offsets of the lane's columns within a row: loads wrap
  // periodically, stores only for output columns of this strip
  uint32_t xo[C], so[C];
  const bool lane_in = lane >= Cols<C>::kHaloLanes && lane < kWave - Cols<C>::kHaloLanes;
  const bool edge_lane = lane == 0 || lane == kWave - 1;
#pragma unroll
  for (int k = 0; k < C; ++k) {
    xo[k] = 4u * static_cast<uint32_t>(wrap_index(col0 + k, g.nx));
    so[k] = (lane_in && col0 + k < g.nx) ? xo[k] : kNoStore;
  }
  if constexpr (VEC) {
    // the lane's C columns are stored together or not at all
#pragma unroll
    for (int k = 1; k < C; ++k) so[k] = so[0];
  }
  // Neighbouring segments march in opposite directions, so that the 8 halo
  // rows two segments share are read by both at about the same time (at
  // the start of both marches or at the end of both) and come from L2 for
  // the second reader.
  if (seg & 1)
    march<C, VEC, WIDE, MODE, POT, +1>(g, xo, so, edge_lane, y0, seg_h);
  else
    march<C, VEC, WIDE, MODE, POT, -1>(g, xo, so, edge_lane, y0, seg_h);
}

// ---------------------------------------------------------------------------
// Validation scan of n at init: smallest n, largest applied potential angle,
// and a flag for any n <= 0 or not finite. One partial per block.
// ---------------------------------------------------------------------------
struct ScanPartial {
  double nmin;
  double bmax;
  double bad;
  double pad;
};

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__global__ void __launch_bounds__(256) qla_scan_kernel(const float* __restrict__ n, int nx, int ny,
                                                       double kb, ScanPartial* __restrict__ out) {
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  double nmin = INFINITY, bmax = 0.0, bad = 0.0;
  for (int64_t s = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; s < plane;
       s += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int y = static_cast<int>(s / nx);
    const int x = static_cast<int>(s - static_cast<int64_t>(y) * nx);
    const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
    const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
    double v[3];
    for (int c = 0; c < 3; ++c) {
      v[c] = n[c * plane + s];
      if (!(v[c] > 0.0) || !isfinite(v[c])) bad = 1.0;
      nmin = fmin(nmin, v[c]);
    }
    if (bad == 0.0) {
      const double d0 = n[1 * plane + static_cast<int64_t>(y) * nx + xp] - n[1 * plane + static_cast<int64_t>(y) * nx + xm];
      const double d1 = n[0 * plane + static_cast<int64_t>(yp) * nx + x] - n[0 * plane + static_cast<int64_t>(ym) * nx + x];
      const double d2 = n[2 * plane + static_cast<int64_t>(y) * nx + xp] - n[2 * plane + static_cast<int64_t>(y) * nx + xm];
      const double d3 = n[2 * plane + static_cast<int64_t>(yp) * nx + x] - n[2 * plane + static_cast<int64_t>(ym) * nx + x];
      bmax = fmax(bmax, fabs(kb * d0 / (v[1] * v[1])));
      bmax = fmax(bmax, fabs(kb * d1 / (v[0] * v[0])));
      bmax = fmax(bmax, fabs(kb * d2 / (v[2] * v[2])));
      bmax = fmax(bmax, fabs(kb * d3 / (v[2] * v[2])));
    }
  }
  __shared__ double sh[3][4];
  nmin = wave_min(nmin);
  bmax = wave_max(bmax);
  bad = wave_max(bad);
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sh[0][w] = nmin;
    sh[1][w] = bmax;
    sh[2][w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    for (int k = 1; k < nw; ++k) {
      nmin = fmin(nmin, sh[0][k]);
      bmax = fmax(bmax, sh[1][k]);
      bad = fmax(bad, sh[2][k]);
    }
    out[blockIdx.x] = ScanPartial{nmin, bmax, bad, 0.0};
  }
}

__global__ void qla_scan_final(ScanPartial* __restrict__ parts, int count) {
  double nmin = INFINITY, bmax = 0.0, bad = 0.0;
  for (int k = threadIdx.x; k < count; k += blockDim.x) {
    nmin = fmin(nmin, parts[k].nmin);
    bmax = fmax(bmax, parts[k].bmax);
    bad = fmax(bad, parts[k].bad);
  }
  nmin = wave_min(nmin);
  bmax = wave_max(bmax);
  bad = wave_max(bad);
  if (threadIdx.x == 0) parts[count] = ScanPartial{nmin, bmax, bad, 0.0};
}

// ---------------------------------------------------------------------------
// Diagnostics (Eq. (27), div B, div D): per-block FP64 partials, then one
// block folds them.
// ---------------------------------------------------------------------------
constexpr int kDiagVals = 8;   // energy, sum divB^2, max|divB|, max|B|^2, sum|B|^2,
                               // sum divD^2, max|divD|, max|D|^2
constexpr int kDiagBlocks = 1024;

__global__ void __launch_bounds__(256) qla_diag_kernel(const float* __restrict__ q,
                                                       const float* __restrict__ n, int nx, int ny,
                                                       double* __restrict__ out) {
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  double e = 0, sdb = 0, mdb = 0, mb = 0, sb = 0, sdd = 0, mdd = 0, md = 0;
  for (int64_t s = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; s < plane;
       s += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int y = static_cast<int>(s / nx);
    const int x = static_cast<int>(s - static_cast<int64_t>(y) * nx);
    const int64_t row = static_cast<int64_t>(y) * nx;
    const int64_t sxp = row + (x + 1 == nx ? 0 : x + 1);
    const int64_t sxm = row + (x == 0 ? nx - 1 : x - 1);
    const int64_t syp = static_cast<int64_t>(y + 1 == ny ? 0 : y + 1) * nx + x;
    const int64_t sym = static_cast<int64_t>(y == 0 ? ny - 1 : y - 1) * nx + x;
    double qq[6];
    for (int c = 0; c < 6; ++c) {
      qq[c] = q[c * plane + s];
      e += qq[c] * qq[c];
    }
    const double divb = 0.5 * (static_cast<double>(q[3 * plane + sxp]) - q[3 * plane + sxm]) +
                        0.5 * (static_cast<double>(q[4 * plane + syp]) - q[4 * plane + sym]);
    const double divd =
        0.5 * (static_cast<double>(n[0 * plane + sxp]) * q[0 * plane + sxp] -
               static_cast<double>(n[0 * plane + sxm]) * q[0 * plane + sxm]) +
        0.5 * (static_cast<double>(n[1 * plane + syp]) * q[1 * plane + syp] -
               static_cast<double>(n[1 * plane + sym]) * q[1 * plane + sym]);
    const double b2 = qq[3] * qq[3] + qq[4] * qq[4] + qq[5] * qq[5];
    const double dx = n[0 * plane + s] * qq[0], dy = n[1 * plane + s] * qq[1],
                 dz = n[2 * plane + s] * qq[2];
    const double d2 = dx * dx + dy * dy + dz * dz;
    sdb += divb * divb;
    mdb = fmax(mdb, fabs(divb));
    mb = fmax(mb, b2);
    sb += b2;
    sdd += divd * divd;
    mdd = fmax(mdd, fabs(divd));
    md = fmax(md, d2);
  }
  e = wave_sum(e); sdb = wave_sum(sdb); sb = wave_sum(sb); sdd = wave_sum(sdd);
  mdb = wave_max(mdb); mb = wave_max(mb); mdd = wave_max(mdd); md = wave_max(md);
  __shared__ double sh[kDiagVals][4];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sh[0][w] = e; sh[1][w] = sdb; sh[2][w] = mdb; sh[3][w] = mb;
    sh[4][w] = sb; sh[5][w] = sdd; sh[6][w] = mdd; sh[7][w] = md;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    for (int k = 1; k < nw; ++k) {
      e += sh[0][k]; sdb += sh[1][k]; mdb = fmax(mdb, sh[2][k]); mb = fmax(mb, sh[3][k]);
      sb += sh[4][k]; sdd += sh[5][k]; mdd = fmax(mdd, sh[6][k]); md = fmax(md, sh[7][k]);
    }
    double* o = out + static_cast<int64_t>(blockIdx.x) * kDiagVals;
    o[0] = e; o[1] = sdb; o[2] = mdb; o[3] = mb; o[4] = sb; o[5] = sdd; o[6] = mdd; o[7] = md;
  }
}

__global__ void qla_diag_final(double* __restrict__ parts, int count) {
  // one wave; parts[count * kDiagVals ..] receives the folded values
  double v[kDiagVals];
  for (int j = 0; j < kDiagVals; ++j) v[j] = 0.0;   // sums and maxima of non-negative values
  for (int k = threadIdx.x; k < count; k += blockDim.x) {
    const double* o = parts + static_cast<int64_t>(k) * kDiagVals;
    v[0] += o[0]; v[1] += o[1]; v[2] = fmax(v[2], o[2]); v[3] = fmax(v[3], o[3]);
    v[4] += o[4]; v[5] += o[5]; v[6] = fmax(v[6], o[6]); v[7] = fmax(v[7], o[7]);
  }
  v[0] = wave_sum(v[0]); v[1] = wave_sum(v[1]); v[4] = wave_sum(v[4]); v[5] = wave_sum(v[5]);
  v[2] = wave_max(v[2]); v[3] = wave_max(v[3]); v[6] = wave_max(v[6]); v[7] = wave_max(v[7]);
  if (threadIdx.x == 0)
    for (int j = 0; j < kDiagVals; ++j) parts[static_cast<int64_t>(count) * kDiagVals + j] = v[j];
}

// E_c = q_c / n_c for c < 3, B copied: (E, B) planes of Eq. (15).
__global__ void __launch_bounds__(256) qla_fields_kernel(const float* __restrict__ q,
                                                         const float* __restrict__ n, int64_t plane,
                                                         float* __restrict__ out) {
  for (int64_t s = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; s < plane;
       s += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    for (int c = 0; c < 3; ++c) out[c * plane + s] = q[c * plane + s] / n[c * plane + s];
    for (int c = 3; c < 6; ++c) out[c * plane + s] = q[c * plane + s];
  }
}

}  // namespace

// ===========================================================================
// Host side: context, launch selection, C ABI.
// ===========================================================================

namespace {

thread_local char g_last_error[512] = "";

qla_status fail(qla_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
qla_status fail(qla_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return st;
}

constexpr uint64_t kMagic = 0x514c41435458ull;   // "QLACTX"

// One compiled instance of the step kernel: how to launch it and how many
// of its blocks fit on a CU.
struct StepImpl {
  void (*launch)(const StepArgs&, dim3, dim3, hipStream_t);
  hipError_t (*blocks_per_cu)(int* nb, int threads);
  int cols;
};

template <int C, bool VEC, bool WIDE, int MODE, bool POT>
void launch_step(const StepArgs& a, dim3 grid, dim3 block, hipStream_t st) {
  hipLaunchKernelGGL((qla_step_kernel<C, VEC, WIDE, MODE, POT>), grid, block, 0, st, a);
}

template <int C, bool VEC, bool WIDE, int MODE, bool POT>
hipError_t step_blocks_per_cu(int* nb, int threads) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, qla_step_kernel<C, VEC, WIDE, MODE, POT>,
                                                      threads, 0);
}

template <int C, bool VEC, bool WIDE, int MODE, bool POT>
StepImpl impl() {
  return StepImpl{launch_step<C, VEC, WIDE, MODE, POT>, step_blocks_per_cu<C, VEC, WIDE, MODE, POT>, C};
}

template <int C, bool VEC>
StepImpl pick_step_c(bool wide, int mode, bool pot) {
  if (wide) {
    if (mode == QLA_POT_EQ28) return pot ? impl<C, VEC, true, 1, true>() : impl<C, VEC, true, 1, false>();
    return pot ? impl<C, VEC, true, 0, true>() : impl<C, VEC, true, 0, false>();
  }
  if (mode == QLA_POT_EQ28) return pot ? impl<C, VEC, false, 1, true>() : impl<C, VEC, false, 1, false>();
  return pot ? impl<C, VEC, false, 0, true>() : impl<C, VEC, false, 0, false>();
}

StepImpl pick_step(int cols, bool vec, bool wide, int mode, bool pot) {
  if (cols == 4)
    return vec ? pick_step_c<4, true>(wide, mode, pot) : pick_step_c<4, false>(wide, mode, pot);
  return vec ? pick_step_c<2, true>(wide, mode, pot) : pick_step_c<2, false>(wide, mode, pot);
}

}  // namespace

struct qla_ctx {
  uint64_t magic;
  qla_params p;
  const float* n;
  float* buf[2];
  int cur;                 // index of the buffer holding the current state
  void* work;
  hipStream_t stream;
  int64_t steps;
  bool wide;
  bool poisoned;
  int cus;                 // compute units of the device
  qla_launch launch;       // requested geometry (0 fields: library default)
  qla_launch planned;      // geometry in use
  StepArgs args;
  dim3 grid, block;
  StepImpl step;
  double nmin, bmax;
};

namespace {

size_t work_bytes() {
  // diagnostics partials (+ one folded row) and scan partials
  return static_cast<size_t>(kDiagBlocks + 1) * kDiagVals * sizeof(double) +
         static_cast<size_t>(kDiagBlocks + 1) * sizeof(ScanPartial);
}

qla_status check_params(const qla_params* p) {
  if (!p) return fail(QLA_EINVAL, "qla: null params");
  if (p->nx < 1 || p->ny < 1) return fail(QLA_EINVAL, "qla: lattice %d x %d must be at least 1 x 1", p->nx, p->ny);
  if (static_cast<int64_t>(p->nx) * p->ny > (int64_t{1} << 40))
    return fail(QLA_EINVAL, "qla: lattice too large");
  if (!(p->delta > 0.0) || !std::isfinite(p->delta)) return fail(QLA_EINVAL, "qla: delta must be finite and > 0");
  if (p->pot_mode != QLA_POT_EQ23 && p->pot_mode != QLA_POT_EQ28)
    return fail(QLA_EINVAL, "qla: pot_mode %d is not QLA_POT_EQ23 or QLA_POT_EQ28", p->pot_mode);
  if (p->beta_scale < QLA_BETA_PHYS || p->beta_scale > QLA_BETA_OFF)
    return fail(QLA_EINVAL, "qla: beta_scale %d unknown", p->beta_scale);
  return QLA_OK;
}

qla_status hip_fail(qla_ctx* ctx, hipError_t e, const char* what) {
  if (ctx) ctx->poisoned = true;
  return fail(QLA_EDEVICE, "qla: %s: %s", what, hipGetErrorString(e));
}

qla_status check_ctx(qla_ctx* ctx) {
  if (!ctx || ctx->magic != kMagic) return fail(QLA_ESTATE, "qla: invalid context");
  if (ctx->poisoned) return fail(QLA_ESTATE, "qla: context unusable after an earlier device error");
  return QLA_OK;
}

double kappa_of(const qla_params& p) {
  if (p.beta_scale == QLA_BETA_PHYS) return p.delta;
  if (p.beta_scale == QLA_BETA_LATTICE) return p.delta * p.delta;
  return 0.0;
}

// Launch geometry of the step kernel. A wave covers 64*C columns (C = 2 by
// default) of which (64 - 2*ceil(4/C))*C are output; the lattice is cut into
// strips (x) and segments (y) so that the whole grid is resident at once
// (one round, no tail), with segments as tall as that allows (each segment
// re-reads 8 halo rows). Requested fields of ctx->launch override the
// defaults.
qla_status plan_step(qla_ctx* c) {
  const int nx = c->p.nx, ny = c->p.ny;
  int C = c->launch.cols > 0 ? c->launch.cols : 2;
  if (C != 2 && C != 4) return fail(QLA_EINVAL, "qla: cols must be 2 or 4");
  const int wpb = c->launch.waves_per_block > 0 ? c->launch.waves_per_block : 1;
  if (wpb > 4) return fail(QLA_EINVAL, "qla: waves_per_block must be 1..4");
  const bool vec = (nx % C) == 0;
  const bool pot = c->p.beta_scale != QLA_BETA_OFF;
  c->step = pick_step(C, vec, c->wide, c->p.pot_mode, pot);
  const int halo = (4 + C - 1) / C;
  const int out_cols = (kWave - 2 * halo) * C;
  const int nstrips = (nx + out_cols - 1) / out_cols;
  int seg_rows = c->launch.seg_rows;
  if (seg_rows <= 0) {
    int bpc = 0;
    hipError_t e = c->step.blocks_per_cu(&bpc, kWave * wpb);
    if (e != hipSuccess || bpc < 1) bpc = 1;
    const int slots = c->cus * bpc;                      // resident blocks
    int block_rows = slots / nstrips;
    if (block_rows < 1) block_rows = 1;
    seg_rows = (ny + block_rows * wpb - 1) / (block_rows * wpb);
    if (seg_rows < 8) seg_rows = 8;
  }
  seg_rows = (seg_rows + 3) & ~3;
  const int nsegs = (ny + seg_rows - 1) / seg_rows;
  const int64_t nblocks64 = static_cast<int64_t>(nstrips) * ((nsegs + wpb - 1) / wpb);
  if (nblocks64 > (int64_t{1} << 30)) return fail(QLA_EINVAL, "qla: launch geometry too large");
  c->args.plane = static_cast<int64_t>(nx) * ny;
  c->args.nx = nx;
  c->args.ny = ny;
  c->args.seg_rows = seg_rows;
  c->args.nstrips = nstrips;
  c->args.nsegs = nsegs;
  c->args.waves_per_block = wpb;
  c->args.a4 = static_cast<float>(c->p.delta / 4.0);
  const double frac = c->p.pot_mode == QLA_POT_EQ28 ? 0.5 : 1.0;
  c->args.kb = static_cast<float>(kappa_of(c->p) * frac * 0.5);
  c->grid = dim3(static_cast<unsigned>(nblocks64));
  c->block = dim3(kWave * wpb);
  c->planned = qla_launch{seg_rows, wpb, C};
  return QLA_OK;
}

}  // namespace

extern "C" {

qla_status qla_workspace_size(const qla_params* p, size_t* bytes) {
  qla_status st = check_params(p);
  if (st != QLA_OK) return st;
  if (!bytes) return fail(QLA_EINVAL, "qla: null bytes pointer");
  *bytes = work_bytes();
  return QLA_OK;
}

qla_status qla_init(const qla_params* p, const float* d_n, float* d_q, float* d_q_pong,
                    void* d_work, void* hip_stream, qla_ctx** out) {
  if (!out) return fail(QLA_EINVAL, "qla: null output pointer");
  *out = nullptr;
  qla_status st = check_params(p);
  if (st != QLA_OK) return st;
  if (!d_n || !d_q || !d_q_pong || !d_work)
    return fail(QLA_EINVAL, "qla: null device buffer");
  if (d_q == d_q_pong) return fail(QLA_EINVAL, "qla: the two state buffers must differ");
  if ((reinterpret_cast<uintptr_t>(d_work) & 255) != 0)
    return fail(QLA_EINVAL, "qla: workspace must be 256-byte aligned");
  qla_ctx* c = new (std::nothrow) qla_ctx();
  if (!c) return fail(QLA_ENOMEM, "qla: host allocation failed");
  c->magic = kMagic;
  c->p = *p;
  c->n = d_n;
  c->buf[0] = d_q;
  c->buf[1] = d_q_pong;
  c->cur = 0;
  c->work = d_work;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->steps = 0;
  c->poisoned = false;

  // validate n and size the coefficient series
  const double frac = p->pot_mode == QLA_POT_EQ28 ? 0.5 : 1.0;
  const double kb = kappa_of(*p) * frac * 0.5;
  const int64_t plane = static_cast<int64_t>(p->nx) * p->ny;
  int blocks = static_cast<int>((plane + 255) / 256);
  if (blocks > kDiagBlocks) blocks = kDiagBlocks;
  ScanPartial* parts = reinterpret_cast<ScanPartial*>(
      static_cast<char*>(d_work) + static_cast<size_t>(kDiagBlocks + 1) * kDiagVals * sizeof(double));
  hipLaunchKernelGGL(qla_scan_kernel, dim3(blocks), dim3(256), 0, c->stream, d_n, p->nx, p->ny, kb, parts);
  hipLaunchKernelGGL(qla_scan_final, dim3(1), dim3(kWave), 0, c->stream, parts, blocks);
  ScanPartial res{};
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&res, parts + blocks, sizeof(res), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    st = hip_fail(nullptr, e, "validating n");
    delete c;
    return st;
  }
  if (res.bad != 0.0) {
    delete c;
    return fail(QLA_EINVAL, "qla: every refractive index must be finite and > 0");
  }
  c->nmin = res.nmin;
  c->bmax = res.bmax;
  const double theta_max = p->delta / (4.0 * res.nmin);
  c->wide = !(theta_max <= kNarrowAngle && res.bmax <= kNarrowAngle);
  int dev = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess || cus < 1) {
    delete c;
    return hip_fail(nullptr, e == hipSuccess ? hipErrorInvalidDevice : e, "querying the device");
  }
  c->cus = cus;
  c->launch = qla_launch{0, 0, 0};
  st = plan_step(c);
  if (st != QLA_OK) {
    delete c;
    return st;
  }
  *out = c;
  return QLA_OK;
}

qla_status qla_step(qla_ctx* ctx, int64_t nsteps) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (nsteps < 0) return fail(QLA_EINVAL, "qla: negative step count");
  for (int64_t s = 0; s < nsteps; ++s) {
    StepArgs a = ctx->args;
    a.qin = ctx->buf[ctx->cur];
    a.qout = ctx->buf[ctx->cur ^ 1];
    a.n = ctx->n;
    ctx->step.launch(a, ctx->grid, ctx->block, ctx->stream);
    ctx->cur ^= 1;
    ++ctx->steps;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "launching the step kernel");
  return QLA_OK;
}

qla_status qla_energy(qla_ctx* ctx, qla_diag* out) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!out) return fail(QLA_EINVAL, "qla: null diag pointer");
  const int64_t plane = static_cast<int64_t>(ctx->p.nx) * ctx->p.ny;
  int blocks = static_cast<int>((plane + 255) / 256);
  if (blocks > kDiagBlocks) blocks = kDiagBlocks;
  double* parts = static_cast<double*>(ctx->work);
  hipLaunchKernelGGL(qla_diag_kernel, dim3(blocks), dim3(256), 0, ctx->stream, ctx->buf[ctx->cur],
                     ctx->n, ctx->p.nx, ctx->p.ny, parts);
  hipLaunchKernelGGL(qla_diag_final, dim3(1), dim3(kWave), 0, ctx->stream, parts, blocks);
  double v[kDiagVals];
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(v, parts + static_cast<int64_t>(blocks) * kDiagVals, sizeof(v),
                       hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "computing diagnostics");
  out->step = ctx->steps;
  out->energy = v[0] / static_cast<double>(plane);
  out->divB_l2 = std::sqrt(v[1]);
  out->divB_max = v[2];
  out->B_max = std::sqrt(v[3]);
  out->B_l2 = std::sqrt(v[4]);
  out->divD_l2 = std::sqrt(v[5]);
  out->divD_max = v[6];
  out->D_max = std::sqrt(v[7]);
  return QLA_OK;
}

qla_status qla_fields(qla_ctx* ctx, float* dst, int32_t what, int32_t dst_is_host) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!dst) return fail(QLA_EINVAL, "qla: null destination");
  if (what != 0 && what != 1) return fail(QLA_EINVAL, "qla: what must be 0 (Q) or 1 (E, B)");
  const int64_t plane = static_cast<int64_t>(ctx->p.nx) * ctx->p.ny;
  const size_t bytes = static_cast<size_t>(plane) * 6 * sizeof(float);
  const float* src = ctx->buf[ctx->cur];
  hipError_t e = hipSuccess;
  if (what == 1) {
    // (E, B) is written into the idle state buffer, then copied out
    float* tmp = ctx->buf[ctx->cur ^ 1];
    int blocks = static_cast<int>((plane + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(qla_fields_kernel, dim3(blocks), dim3(256), 0, ctx->stream, src, ctx->n, plane, tmp);
    e = hipGetLastError();
    src = tmp;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst, src, bytes, dst_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                       ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "exporting fields");
  return QLA_OK;
}

qla_status qla_get_launch(qla_ctx* ctx, qla_launch* out) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!out) return fail(QLA_EINVAL, "qla: null launch pointer");
  *out = ctx->planned;
  return QLA_OK;
}

qla_status qla_set_launch(qla_ctx* ctx, const qla_launch* req) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!req) return fail(QLA_EINVAL, "qla: null launch pointer");
  if (req->seg_rows < 0 || req->waves_per_block < 0 || req->waves_per_block > 4 ||
      (req->cols != 0 && req->cols != 2 && req->cols != 4))
    return fail(QLA_EINVAL, "qla: launch fields out of range");
  const qla_launch keep = ctx->launch;
  ctx->launch = *req;
  st = plan_step(ctx);
  if (st != QLA_OK) {
    ctx->launch = keep;
    plan_step(ctx);
  }
  return st;
}

qla_status qla_state(qla_ctx* ctx, float** d_current) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!d_current) return fail(QLA_EINVAL, "qla: null output pointer");
  *d_current = ctx->buf[ctx->cur];
  return QLA_OK;
}

void qla_free(qla_ctx* ctx) {
  if (!ctx || ctx->magic != kMagic) return;
  ctx->magic = 0;
  delete ctx;
}

const char* qla_last_error(void) { return g_last_error; }

}  // extern "C"
