// Device code of the fused QLA time step (Vahala et al., arXiv:2301.13601),
// shared by the translation units that instantiate it. See qla.hip for the
// host side and the C ABI.
//
// One launch of qla_step_kernel applies one or two whole time steps: for
// every site of every lattice in a batch, the operator sequence of Eq. (23)
// or Eq. (28): U_X (Eq. (18), 16 factors), U_Y (Eq. (20), 16 factors) and the
// potentials V_X, V_Y (Eq. (21), (22)), with the collision angles of
// Eq. (24) and the potential angles of Eq. (25) computed on the fly from n.
//
// Work decomposition:
//  * a wave owns a strip of 64*C consecutive columns (C per lane) and a
//    segment of rows of one lattice, and marches through the segment one row
//    per iteration;
//  * the x sweep of the ingested row runs in registers: a streaming shift
//    along x is a register rename for C-1 of the lane's columns and one DPP
//    whole-wave shift for the last; the outermost lanes on each side are
//    halo (one step's x support is +-4 cells) and store nothing;
//  * the y sweep is a 16-stage register pipeline: a stage that pulls from
//    the row behind in marching order reads a one-row delay register, a
//    stage that pulls from the row ahead delays the other two active
//    components instead, so the pipeline emits the fully stepped row four
//    rows behind the one it ingests;
//  * the loop is unrolled four times so that every ring of per-row data
//    (collision coefficients, potential coefficients) is indexed by
//    compile-time slots and stays in registers;
//  * a two-step launch pairs two waves on one segment: the first runs the
//    step on rows from memory and passes each finished row through LDS to
//    the second, which steps it again and stores it (temporal blocking).
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

namespace qla_dev {

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

// The potentials act once per half step and, unlike the collisions, are
// not undone by a partner operator, so the rounding of their updates adds
// up over a run. Both forms below therefore form the small increment first
// and round the full value only once.
//
// a' = cos(b) a + sin(b) p  ==  a + (sin(b) p - (1 - cos b) a)
__device__ __forceinline__ float pot_row(float a, float p, float sb, float hb) {
  return a + fmaf(sb, p, -(hb * a));
}

// Rotation of the pair (a, b) by SGN * phi (a' = cos a - sin b, b' = sin a +
// cos b for SGN = +1) from s = sin(phi), h = 1 - cos(phi): each component
// moves by its increment (-h a - s b, s a - h b), one rounding each.
template <int SGN>
__device__ __forceinline__ void rot_inc(float& a, float& b, float s, float h) {
  const float sa = SGN > 0 ? s : -s;
  const float da = fmaf(-h, a, -(sa * b));
  const float db = fmaf(-h, b, sa * a);
  a = a + da;
  b = b + db;
}

// ---------------------------------------------------------------------------
// Step kernel.
// ---------------------------------------------------------------------------
// One lattice as a wave sees it during a step.
struct StepArgs {
  const float* __restrict__ qin;   // 6 planes
  float* __restrict__ qout;        // 6 planes
  const float* __restrict__ n;     // 3 planes
  // per row y: the first and last column at which an index plane the step
  // reads differs from 1 (nx and -1 for a row of vacuum)
  const int* __restrict__ span;
  int64_t plane;                   // nx * ny
  int nx, ny;
  float a4;                        // delta / 4                    (Eq. (24))
  float kb;                        // kappa * frac / 2             (Eq. (25))
  // the wave's column window as a vacuum test (vacuum_span): a row is
  // vacuum for the wave if its span ends before wa, starts after wb, or lies
  // within the gap (g0, g1) that a window wrapping around the lattice
  // leaves open
  int wa, wb, g0, g1;
};

// Columns of a strip: a pass of STEPS steps has an x support of 4*STEPS
// cells on each side, held by the outermost halo lanes.
template <int C, int STEPS = 1>
struct Cols {
  static constexpr int kHaloLanes = (4 * STEPS + C - 1) / C;
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
// Cache policy of a buffer access (the instruction's cache-policy bits):
// default, or non-temporal ("nt"): the line is not kept for reuse. The step
// writes every row once and no wave of the launch reads it back, so stores
// are non-temporal (per two-step launch on the 4096^2 cylinder 241.5 ->
// 235.7 us). State rows can be read non-temporally as a launch option
// (KOpt::STREAM, six components): that took the cylinder to 225.7 us while
// every index row was fetched, but once index rows of vacuum are skipped
// the default policy is 1 % faster there, and a batch of narrow lattices in
// 128-row segments, whose neighbouring segments reread their halo rows from
// L2, ran 8 % slower with it. Non-temporal index loads, and TM state loads,
// were slower.
constexpr int kCacheDefault = 0;
constexpr int kCacheStream = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float* row, int nx) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(row), 0, nx * 4, kRsrcWord3);
}

template <int C, bool VEC, int POL = kCacheDefault>
__device__ __forceinline__ void load_row(const float* row, int nx, const uint32_t (&xb)[C],
                                         float (&out)[C]) {
  const __amdgpu_buffer_rsrc_t r = row_rsrc(row, nx);
  if constexpr (VEC && C == 4) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, xb[0], 0, POL);
    out[0] = __uint_as_float(v.x); out[1] = __uint_as_float(v.y);
    out[2] = __uint_as_float(v.z); out[3] = __uint_as_float(v.w);
  } else if constexpr (VEC && C == 2) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, xb[0], 0, POL);
    out[0] = __uint_as_float(v.x); out[1] = __uint_as_float(v.y);
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) out[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, xb[k], 0, POL));
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
    __builtin_amdgcn_raw_buffer_store_b128(w, r, sb[0], 0, kCacheStream);
  } else if constexpr (VEC && C == 2) {
    u32x2 w;
    w.x = __float_as_uint(v[0]); w.y = __float_as_uint(v[1]);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, sb[0], 0, kCacheStream);
  } else {
#pragma unroll
    for (int k = 0; k < C; ++k) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[k]), r, sb[k], 0, kCacheStream);
  }
}

// true on every lane if any lane's flag is set (a wave-uniform branch)
__device__ __forceinline__ bool wave_any(bool v) { return __any(v) != 0; }

// Compile-time options of one kernel instance.
//   MODE    0: potentials after U_Y (Eq. (23)); 1: interleaved (Eq. (28))
//   POT     potentials present (kappa != 0)
//   WIDE    libm coefficients instead of the short series
//   VEC     nx % C == 0: vector row I/O
//   FIELDS  0: all six components; 1: only (q2, q3, q4) = (n_z E_z, B_x, B_y)
//           (TM); 2: only (q0, q1, q5) = (n_x E_x, n_y E_y, B_z) (TE). The two
//           triples never mix under C_X, C_Y, V_X, V_Y, so a state living in
//           one triple stays there, and the other three planes are neither
//           read nor written.
//   SKEW    0: the potentials of Eq. (21)/(22) as printed; 1: their
//           skew-symmetric part, a rotation by half the angle in the same
//           pairs (an orthogonal, energy-conserving variant)
//   STREAM  state rows are loaded non-temporally (six components only; a
//           launch option the autotuner tries)
template <int MODE_, bool POT_, bool WIDE_, bool VEC_, int FIELDS_, int SKEW_, int STREAM_ = 0>
struct KOpt {
  static constexpr int MODE = MODE_;
  static constexpr bool POT = POT_;
  static constexpr bool WIDE = WIDE_;
  static constexpr bool VEC = VEC_;
  static constexpr int FIELDS = FIELDS_;
  static constexpr bool SKEW = SKEW_ != 0;
  static constexpr bool STREAM = STREAM_ != 0;
  static constexpr bool TE = FIELDS_ != 1;     // (q0, q1, q5) live
  static constexpr bool TM = FIELDS_ != 2;     // (q2, q3, q4) live
  static constexpr bool live(int c) { return (c == 0 || c == 1 || c == 5) ? TE : TM; }
  // index planes read: n_x and n_y serve the TE triple, n_z the TM triple
  static constexpr bool nlive(int c) { return c == 2 ? TM : TE; }
};

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
  // V_Y coefficients per row slot ((sin phi, 1 - cos phi) of the applied
  // angles of beta_1 and beta_3: phi = b for the printed potentials, b/2 for
  // the skew rotations), and whether the row has any
  // nonzero y-difference of n_x or n_z (when it has none, beta_1 = beta_3 =
  // 0 and V_Y is exactly the identity)
  float vy[4][4][C];
  bool fy[4];
  // Eq. (23) only: V_X coefficients, their flag and the (q1, q2, q4) values
  // per row slot, all needed after U_Y
  float vx[4][4][C];
  bool fx[4];
  float q14[4][3][C];
  // the ingested row R and the rows in flight: Q of R and R+DIR, n of R-DIR
  // (x and z components), R and R+DIR
  float q[6][C];
  float q1[6][C];
  float nprev[2][C];
  float ncur[3][C];
  float nnext[3][C];
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

// Potential coefficients of an applied angle b: (sin phi, 1 - cos phi) with
// phi = b for the printed form and phi = b/2 for the skew rotation by b/2.
template <class O>
__device__ __forceinline__ void vcoef(float b, float& c0, float& c1) {
  pot_coef<O::WIDE>(O::SKEW ? 0.5f * b : b, c0, c1);
}

// Prefetch of the rows a pipeline needs later: Q of row R+2*DIR (stage fed
// from memory only) and n of row R+2*DIR.
template <int C, class O>
__device__ __forceinline__ void load_q(const StepArgs& g, const float* row, const uint32_t (&xo)[C],
                                       float (&qld)[6][C]) {
#pragma unroll
  for (int c = 0; c < 6; ++c)
    if (O::live(c)) load_row<C, O::VEC, O::STREAM ? kCacheStream : kCacheDefault>(row + c * g.plane, g.nx, xo, qld[c]);
}

// n of a row whose window is vacuum (every index the step uses is 1 on
// the wave's columns) is not fetched: its loads get an empty extent, so the
// hardware returns 0 without touching memory, and fix_n puts the 1 the row
// holds in their place once they have landed. The loads stay in the
// instruction stream either way, so the march keeps one schedule (and one
// set of waits) for both kinds of row; skipping the instructions with a
// branch measured slower. Scattering scenes are mostly vacuum, and the
// index is a fifth of the bytes a site moves per launch. No wave reads an
// index row that is vacuum on its window.
template <int C, class O>
__device__ __forceinline__ void load_n(const StepArgs& g, const float* row, const uint32_t (&xo)[C],
                                       float (&nld)[3][C], bool vacuum) {
  const int extent = vacuum ? 0 : g.nx;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (O::nlive(c)) load_row<C, O::VEC>(row + c * g.plane, extent, xo, nld[c]);
}

template <int C, class O>
__device__ __forceinline__ void fix_n(float (&nld)[3][C], bool vacuum) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (O::nlive(c)) {
#pragma unroll
      for (int k = 0; k < C; ++k) nld[c][k] = vacuum ? 1.0f : nld[c][k];
    }
}

// The columns [lo, hi] of a row at which an index the step uses is not 1
// (lo > hi: none), read for the whole wave when a march primes its index
// window. The span table does not change during a launch, so it is read
// through the constant address space: a scalar load.
struct Span {
  int lo, hi;
};
typedef const __attribute__((address_space(4))) int ConstInt;
__device__ __forceinline__ Span row_span(const StepArgs& g, int r) {
  const ConstInt* s = (const ConstInt*)(g.span);
  const int ru = __builtin_amdgcn_readfirstlane(r);
  return Span{s[2 * ru], s[2 * ru + 1]};
}
// Whether the wave's window of a row with span sp holds only vacuum.
__device__ __forceinline__ bool vacuum_span(const StepArgs& g, Span sp) {
  return sp.hi < g.wa || sp.lo > g.wb || (sp.lo > g.g0 && sp.hi < g.g1);
}
__device__ __forceinline__ bool vacuum_row(const StepArgs& g, int r) { return vacuum_span(g, row_span(g, r)); }

// Whether the wave's window is vacuum on each of the next 64 index rows a
// march loads, from row r on in direction DIR: bit k for row r + k*DIR
// (taken periodically). Each lane tests one row's span and a ballot
// gathers the answers, so a march that refreshes the mask every 64 rows
// tests a row with a shift, with no memory access and no wait per row (a
// scalar load per row waited on the LDS operations in flight too).
template <int DIR>
__device__ __forceinline__ uint64_t vacuum_mask(const StepArgs& g, int r) {
  const int rr = wrap_index(static_cast<int64_t>(r) + DIR * static_cast<int>(__lane_id()), g.ny);
  return __ballot(vacuum_span(g, Span{g.span[2 * rr], g.span[2 * rr + 1]}));
}

// Where a pipeline's row coefficients (Eq. (24), (25)) come from.
enum { kCoefCompute = 0, kCoefExport = 1, kCoefImport = 2 };

// LDS rows through which a two-step pair shares row coefficients: cy holds,
// per column, the collision (tan(theta/2), sin theta) of n_x and n_z and the
// V_Y pairs of beta_1, beta_3 (8 rows); cx the collision pair of n_y and the
// V_X pairs of beta_0, beta_2 (6 rows); fy, fx the wave-uniform flags that say
// whether the row has any index difference.
// Eq. (23) pairs also keep in LDS what the row at lag 4 needs after U_Y:
// cxo, fxo point at that row's V_X pairs and flag in the cx ring, and q14
// at the wave's four row slots of (q1, q4).
template <int C>
struct CoefIO {
  float* cy;   // rows of kWave * C floats, numbered by RingMap::cy
  float* cx;   // rows numbered by RingMap::cx
  int* fy;
  int* fx;
  int lane;
  const float* cxo = nullptr;
  const int* fxo = nullptr;
  float* q14 = nullptr;   // [4 slots][q1, q4][kWave * C]
};

// Rows of the two-step LDS ring that a field triple uses, packed: the
// emitted Q planes, and the cy / cx coefficient rows in the numbering above
// (cy: 0, 1 collision n_x; 2, 3 collision n_z; 4, 5 V_Y beta_1; 6, 7 V_Y
// beta_3. cx: 0, 1 collision n_y; 2, 3 V_X beta_0; 4, 5 V_X beta_2).
template <class O>
struct RingMap {
  static constexpr int NQ = O::FIELDS == 0 ? 6 : 3;
  static constexpr int NCY = O::FIELDS == 0 ? 8 : 4;
  static constexpr int NCX = O::FIELDS == 0 ? 6 : (O::FIELDS == 2 ? 4 : 2);
  static constexpr int q(int c) { return O::FIELDS == 0 ? c : (O::FIELDS == 1 ? c - 2 : (c == 5 ? 2 : c)); }
  static constexpr int cy(int r) {
    return O::FIELDS == 0 ? r : ((r & 3) - (O::FIELDS == 1 ? 2 : 0)) + (r >= 4 ? 2 : 0);
  }
  static constexpr int cx(int r) { return O::FIELDS == 1 ? r - 4 : r; }
};

// One row iteration of a y pipeline: the whole step of Eq. (23)/(28) on
// the ingested row R (p.q) for the x sweep, and on the rows in flight for
// the y sweep; the row at lag 4 leaves the pipeline fully stepped. With
// EMIT it is handed over in `emit` (all six components, for a second
// pipeline stage); otherwise it is stored to g.qout when it lies in the
// segment. LAG0 is the iteration at which this pipeline ingests the first
// row of the segment (4 for a pipeline fed from memory, 12 for the second
// stage of a two-step pass), so that rows map to iterations as
// R = y0 + i - LAG0 (marching in +y). CMODE: kCoefCompute computes the
// coefficients of row R from the n window; kCoefExport also writes the
// collision pair of n_y and the V_X pairs of row R to io.cx / io.fx as soon
// as they are known; kCoefImport reads every coefficient of row R from io
// (the n window is then not used).
template <int C, class O, int DIR, int SLOT, bool EMIT, int LAG0, int CMODE>
__device__ __forceinline__ void process_row(Pipe<C>& p, const StepArgs& g, const uint32_t (&so)[C],
                                            bool edge_lane, int i, int seg_h, int y0,
                                            float (&emit)[6][C], const CoefIO<C>& io) {
  constexpr bool VEC = O::VEC, WIDE = O::WIDE, POT = O::POT, TE = O::TE, TM = O::TM;
  constexpr int MODE = O::MODE;
  constexpr bool IMPORT = CMODE == kCoefImport;
  // Eq. (23) in a two-step pair: the lag-4 row's (q1, q4) and V_X pairs
  // come from LDS (the cx ring and the wave's q14 slots)
  constexpr bool LDSROW = MODE == 0 && CMODE != kCoefCompute;

  // ---- coefficients of row R (Eq. (24), (25)) -----------------------------
  float u[3][C];
  float tc[3][C], sc[3][C];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (!O::nlive(c)) continue;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      if constexpr (IMPORT) {
        const int x = io.lane * C + k;
        if (c == 1) {
          tc[c][k] = io.cx[RingMap<O>::cx(0) * (kWave * C) + x];
          sc[c][k] = io.cx[RingMap<O>::cx(1) * (kWave * C) + x];
        } else {
          tc[c][k] = io.cy[RingMap<O>::cy(c) * (kWave * C) + x];     // rows 0, 1 for n_x; 2, 3 for n_z
          sc[c][k] = io.cy[RingMap<O>::cy(c + 1) * (kWave * C) + x];
        }
      } else {
        u[c][k] = __builtin_amdgcn_rcpf(p.ncur[c][k]);
        rot_coef<WIDE>(g.a4 * u[c][k], tc[c][k], sc[c][k]);
      }
    }
  }
  // V_X coefficients from the x-differences of n_y (beta_0) and n_z (beta_2).
  // Lanes 0 and 63 see a zero from the DPP shift at the wave edge; their
  // values only reach halo columns, so they do not vote.
  float vx00[C], vx01[C], vx20[C], vx21[C];
  bool fx = false;
  if constexpr (POT && IMPORT) {
    fx = *io.fx != 0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const int x = io.lane * C + k;
      vx00[k] = vx01[k] = vx20[k] = vx21[k] = 0.0f;
      if constexpr (TE) {
        vx00[k] = io.cx[RingMap<O>::cx(2) * (kWave * C) + x];
        vx01[k] = io.cx[RingMap<O>::cx(3) * (kWave * C) + x];
      }
      if constexpr (TM) {
        vx20[k] = io.cx[RingMap<O>::cx(4) * (kWave * C) + x];
        vx21[k] = io.cx[RingMap<O>::cx(5) * (kWave * C) + x];
      }
    }
  } else if constexpr (POT) {
    float dny[C], dnz[C];
    bool nz = false;
#pragma unroll
    for (int k = 0; k < C; ++k) dny[k] = dnz[k] = 0.0f;
    if constexpr (TE) {
      float r1[C], l1[C];
#pragma unroll
      for (int k = 0; k < C; ++k) r1[k] = l1[k] = p.ncur[1][k];
      pull_from_right<C>(r1);
      pull_from_left<C>(l1);
#pragma unroll
      for (int k = 0; k < C; ++k) {
        dny[k] = r1[k] - l1[k];
        nz = nz || dny[k] != 0.0f;
      }
    }
    if constexpr (TM) {
      float r2[C], l2[C];
#pragma unroll
      for (int k = 0; k < C; ++k) r2[k] = l2[k] = p.ncur[2][k];
      pull_from_right<C>(r2);
      pull_from_left<C>(l2);
#pragma unroll
      for (int k = 0; k < C; ++k) {
        dnz[k] = r2[k] - l2[k];
        nz = nz || dnz[k] != 0.0f;
      }
    }
    fx = wave_any(nz && !edge_lane);
#pragma unroll
    for (int k = 0; k < C; ++k) vx00[k] = vx01[k] = vx20[k] = vx21[k] = 0.0f;
    if (fx) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        if constexpr (TE) vcoef<O>(g.kb * dny[k] * (u[1][k] * u[1][k]), vx00[k], vx01[k]);
        if constexpr (TM) vcoef<O>(g.kb * dnz[k] * (u[2][k] * u[2][k]), vx20[k], vx21[k]);
      }
    }
  }
  if constexpr (CMODE == kCoefExport) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const int x = io.lane * C + k;
      if constexpr (TE) {
        io.cx[RingMap<O>::cx(0) * (kWave * C) + x] = tc[1][k];
        io.cx[RingMap<O>::cx(1) * (kWave * C) + x] = sc[1][k];
        if constexpr (POT) {
          io.cx[RingMap<O>::cx(2) * (kWave * C) + x] = vx00[k];
          io.cx[RingMap<O>::cx(3) * (kWave * C) + x] = vx01[k];
        }
      }
      if constexpr (TM && POT) {
        io.cx[RingMap<O>::cx(4) * (kWave * C) + x] = vx20[k];
        io.cx[RingMap<O>::cx(5) * (kWave * C) + x] = vx21[k];
      }
    }
    if (io.lane == 0) *io.fx = fx ? 1 : 0;
  }

  // ---- U_X (Eq. (18)) with V_X' interleaved (Eq. (28)) on row R ------------
  float (&q)[6][C] = p.q;
  using P_ = std::integral_constant<int, 1>;
  using M_ = std::integral_constant<int, -1>;
  auto cx = [&](auto sgn) {
    constexpr int S = decltype(sgn)::value;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      if constexpr (TE) rot<S>(q[1][k], q[5][k], tc[1][k], sc[1][k]);
      if constexpr (TM) rot<S>(q[2][k], q[4][k], tc[2][k], sc[2][k]);
    }
  };
  auto sx = [&](auto right, int ca, int cb) {
    // streams components ca, cb along x (pull from x+1 if right, else x-1)
    constexpr bool R = decltype(right)::value;
    if (O::live(ca)) {
      if constexpr (R) pull_from_right<C>(q[ca]); else pull_from_left<C>(q[ca]);
    }
    if (O::live(cb)) {
      if constexpr (R) pull_from_right<C>(q[cb]); else pull_from_left<C>(q[cb]);
    }
  };
  // V_X: q4 <- cos b2 q4 - sin b2 q2,  q5 <- sin b0 q1 + cos b0 q5 (Eq. (21))
  auto vx_apply = [&](const float (&c00)[C], const float (&c01)[C], const float (&c20)[C],
                      const float (&c21)[C], float (&q1v)[C], float (&q2v)[C], float (&q4v)[C],
                      float (&q5v)[C]) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      if constexpr (O::SKEW) {
        if constexpr (TM) rot_inc<+1>(q4v[k], q2v[k], c20[k], c21[k]);
        if constexpr (TE) rot_inc<+1>(q1v[k], q5v[k], c00[k], c01[k]);
      } else {
        if constexpr (TM) q4v[k] = pot_row(q4v[k], -q2v[k], c20[k], c21[k]);
        if constexpr (TE) q5v[k] = pot_row(q5v[k], q1v[k], c00[k], c01[k]);
      }
    }
  };
  using T_ = std::integral_constant<bool, true>;
  using F_ = std::integral_constant<bool, false>;
  cx(M_{}); sx(F_{}, 1, 4);
  cx(P_{}); sx(T_{}, 1, 4);
  cx(M_{}); sx(T_{}, 2, 5);
  cx(P_{}); sx(F_{}, 2, 5);
  if constexpr (MODE == 1 && POT) {
    if (fx) vx_apply(vx00, vx01, vx20, vx21, q[1], q[2], q[4], q[5]);
  }
  cx(P_{}); sx(T_{}, 1, 4);
  cx(M_{}); sx(F_{}, 1, 4);
  cx(P_{}); sx(F_{}, 2, 5);
  cx(M_{}); sx(T_{}, 2, 5);
  if constexpr (MODE == 1 && POT) {
    if (fx) vx_apply(vx00, vx01, vx20, vx21, q[1], q[2], q[4], q[5]);
  }

  // rows of this iteration relative to y0: R, and R - 4*DIR which leaves
  // the pipeline; both lie in the segment for the same range of i
  const int R_rel = DIR > 0 ? i - LAG0 : seg_h + LAG0 - 1 - i;
  const int O_rel = DIR > 0 ? i - LAG0 - 4 : seg_h + LAG0 + 3 - i;
  const bool R_out = i >= LAG0 && i < seg_h + LAG0;
  const bool O_out = i >= LAG0 + 4 && i < seg_h + LAG0 + 4;
  if constexpr (MODE == 1 && !EMIT) {
    // q1 and q4 are final once U_X and V_X' are done: U_Y and V_Y leave them
    if (R_out) {
      float* row = g.qout + static_cast<int64_t>(y0 + R_rel) * g.nx;
      if constexpr (TE) store_row<C, VEC>(row + 1 * g.plane, g.nx, so, q[1]);
      if constexpr (TM) store_row<C, VEC>(row + 4 * g.plane, g.nx, so, q[4]);
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
        if constexpr (TE) rot<-S>(a0[k], a5[k], tc[0][k], sc[0][k]);
        if constexpr (TM) rot<-S>(b2[k], b3[k], tc[2][k], sc[2][k]);
      }
    } else {
      constexpr int sl = (SLOT - lag) & 3;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        if constexpr (TE) rot<-S>(a0[k], a5[k], p.th[sl][0][k], p.th[sl][1][k]);
        if constexpr (TM) rot<-S>(b2[k], b3[k], p.th[sl][2][k], p.th[sl][3][k]);
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
  // stream stage k shifting (sa, sb) and leaving (ka, kb) of the active four;
  // the flags say which of the four belong to a live triple
  auto sy = [&](auto kk, float (&sa)[C], bool la, float (&sb)[C], bool lb, float (&ka)[C], bool lka,
                float (&kb)[C], bool lkb) {
    constexpr int k = decltype(kk)::value;
    if constexpr (Lg::sgn[k] == DIR) {
      // pulls from the row ahead: the other two wait one row
      if (lka) swap_in(ka, p.d[k][0]);
      if (lkb) swap_in(kb, p.d[k][1]);
    } else {
      // pulls from the row behind: the shifted two come from the delay line
      if (la) swap_in(sa, p.d[k][0]);
      if (lb) swap_in(sb, p.d[k][1]);
    }
  };
  // V_Y: q3 <- sin b3 q2 + cos b3 q3,  q5 <- -sin b1 q0 + cos b1 q5 (Eq. (22))
  auto vy_apply = [&](auto lag) {
    constexpr int sl = (SLOT - decltype(lag)::value) & 3;
    if (p.fy[sl]) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        if constexpr (O::SKEW) {
          if constexpr (TM) rot_inc<+1>(b2[k], b3[k], p.vy[sl][2][k], p.vy[sl][3][k]);
          if constexpr (TE) rot_inc<-1>(a0[k], a5[k], p.vy[sl][0][k], p.vy[sl][1][k]);
        } else {
          if constexpr (TM) b3[k] = pot_row(b3[k], b2[k], p.vy[sl][2][k], p.vy[sl][3][k]);
          if constexpr (TE) a5[k] = pot_row(a5[k], -a0[k], p.vy[sl][0][k], p.vy[sl][1][k]);
        }
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
  // Eq. (20), right to left; S_{03} shifts (a0, b3), S_{25} shifts (b2, a5)
  cy(M_{}, K0{});  sy(K0{}, a0, TE, b3, TM, a5, TE, b2, TM);   // C_Y^dagger, S^{-y}_{03}
  cy(P_{}, K1{});  sy(K1{}, a0, TE, b3, TM, a5, TE, b2, TM);   // C_Y,        S^{+y}_{03}
  cy(M_{}, K2{});  sy(K2{}, b2, TM, a5, TE, a0, TE, b3, TM);   // C_Y^dagger, S^{+y}_{25}
  cy(P_{}, K3{});  sy(K3{}, b2, TM, a5, TE, a0, TE, b3, TM);   // C_Y,        S^{-y}_{25}
  if constexpr (MODE == 1 && POT) vy_apply(std::integral_constant<int, 2>{});   // V_Y' (Eq. (28))
  cy(P_{}, K4{});  sy(K4{}, a0, TE, b3, TM, a5, TE, b2, TM);   // C_Y,        S^{+y}_{03}
  cy(M_{}, K5{});  sy(K5{}, a0, TE, b3, TM, a5, TE, b2, TM);   // C_Y^dagger, S^{-y}_{03}
  cy(P_{}, K6{});  sy(K6{}, b2, TM, a5, TE, a0, TE, b3, TM);   // C_Y,        S^{-y}_{25}
  cy(M_{}, K7{});  sy(K7{}, b2, TM, a5, TE, a0, TE, b3, TM);   // C_Y^dagger, S^{+y}_{25}
  // the pipeline now holds the row at lag 4
  float o1[C], o4[C];
  if constexpr (MODE == 1) {
    if constexpr (POT) vy_apply(std::integral_constant<int, 4>{});   // V_Y' (Eq. (28))
  } else {
    // Eq. (23): V_X then V_Y after U_Y, on the row at lag 4. q2 comes out of
    // U_Y; q1, q4 are the x-sweep values kept for this row (the skew V_X
    // also rotates q2, which the y sweep has moved on, so it uses b2).
    constexpr int sl = (SLOT - 4) & 3;
    if constexpr (LDSROW) {
      // the two-step pair keeps these in LDS (registers are spent)
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const int x = io.lane * C + k;
        o1[k] = io.q14[(sl * 2 + 0) * (kWave * C) + x];
        o4[k] = io.q14[(sl * 2 + 1) * (kWave * C) + x];
      }
      if constexpr (POT) {
        if (*io.fxo != 0) {
          float c00[C], c01[C], c20[C], c21[C];
#pragma unroll
          for (int k = 0; k < C; ++k) {
            const int x = io.lane * C + k;
            c00[k] = c01[k] = c20[k] = c21[k] = 0.0f;
            if constexpr (TE) {
              c00[k] = io.cxo[RingMap<O>::cx(2) * (kWave * C) + x];
              c01[k] = io.cxo[RingMap<O>::cx(3) * (kWave * C) + x];
            }
            if constexpr (TM) {
              c20[k] = io.cxo[RingMap<O>::cx(4) * (kWave * C) + x];
              c21[k] = io.cxo[RingMap<O>::cx(5) * (kWave * C) + x];
            }
          }
          vx_apply(c00, c01, c20, c21, o1, b2, o4, a5);
        }
        vy_apply(std::integral_constant<int, 4>{});
      }
    } else {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        o1[k] = p.q14[sl][0][k];
        o4[k] = p.q14[sl][1][k];
      }
      if constexpr (POT) {
        if (p.fx[sl]) vx_apply(p.vx[sl][0], p.vx[sl][1], p.vx[sl][2], p.vx[sl][3], o1, b2, o4, a5);
        vy_apply(std::integral_constant<int, 4>{});
      }
    }
  }
  if constexpr (EMIT) {
    if constexpr (MODE == 1) {
      // q1, q4 of the row at lag 4, kept since its x sweep
      constexpr int sl = (SLOT - 4) & 3;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        o1[k] = p.q14[sl][0][k];
        o4[k] = p.q14[sl][1][k];
      }
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
      emit[0][k] = a0[k];
      emit[1][k] = o1[k];
      emit[2][k] = b2[k];
      emit[3][k] = b3[k];
      emit[4][k] = o4[k];
      emit[5][k] = a5[k];
    }
  } else if (O_out) {
    float* row = g.qout + static_cast<int64_t>(y0 + O_rel) * g.nx;
    if constexpr (TE) store_row<C, VEC>(row + 0 * g.plane, g.nx, so, a0);
    if constexpr (TM) store_row<C, VEC>(row + 2 * g.plane, g.nx, so, b2);
    if constexpr (TM) store_row<C, VEC>(row + 3 * g.plane, g.nx, so, b3);
    if constexpr (TE) store_row<C, VEC>(row + 5 * g.plane, g.nx, so, a5);
    if constexpr (MODE == 0) {
      if constexpr (TE) store_row<C, VEC>(row + 1 * g.plane, g.nx, so, o1);
      if constexpr (TM) store_row<C, VEC>(row + 4 * g.plane, g.nx, so, o4);
    }
  }

  // ---- per-row data kept for later rows (slot SLOT held the row at lag 4,
  // consumed above) ------------------------------------------------------------
#pragma unroll
  for (int k = 0; k < C; ++k) {
    if constexpr (TE) {
      p.th[SLOT][0][k] = tc[0][k];
      p.th[SLOT][1][k] = sc[0][k];
    }
    if constexpr (TM) {
      p.th[SLOT][2][k] = tc[2][k];
      p.th[SLOT][3][k] = sc[2][k];
    }
  }
  if constexpr (LDSROW) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const int x = io.lane * C + k;
      if constexpr (TE) io.q14[(SLOT * 2 + 0) * (kWave * C) + x] = p.q[1][k];
      if constexpr (TM) io.q14[(SLOT * 2 + 1) * (kWave * C) + x] = p.q[4][k];
    }
  } else if constexpr (MODE == 0 || EMIT) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      if constexpr (TE) p.q14[SLOT][0][k] = p.q[1][k];
      if constexpr (TM) p.q14[SLOT][1][k] = p.q[4][k];
    }
  }
  if constexpr (MODE == 0 && !LDSROW) {
    if constexpr (POT) {
      p.fx[SLOT] = fx;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        p.vx[SLOT][0][k] = vx00[k];
        p.vx[SLOT][1][k] = vx01[k];
        p.vx[SLOT][2][k] = vx20[k];
        p.vx[SLOT][3][k] = vx21[k];
      }
    }
  }
  if constexpr (POT && IMPORT) {
    p.fy[SLOT] = *io.fy != 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if ((c < 2 && !TE) || (c >= 2 && !TM)) continue;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const int x = io.lane * C + k;
        p.vy[SLOT][c][k] = io.cy[RingMap<O>::cy(4 + c) * (kWave * C) + x];
      }
    }
  } else if constexpr (POT) {
    // V_Y coefficients of row R from the y-differences n(R+1) - n(R-1) of
    // n_x (beta_1) and n_z (beta_3)
    float d1[C], d3[C];
    bool nz = false;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      d1[k] = d3[k] = 0.0f;
      if constexpr (TE) d1[k] = DIR > 0 ? p.nnext[0][k] - p.nprev[0][k] : p.nprev[0][k] - p.nnext[0][k];
      if constexpr (TM) d3[k] = DIR > 0 ? p.nnext[2][k] - p.nprev[1][k] : p.nprev[1][k] - p.nnext[2][k];
      nz = nz || d1[k] != 0.0f || d3[k] != 0.0f;
    }
    const bool fy = wave_any(nz);
    p.fy[SLOT] = fy;
    if (fy) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        if constexpr (TE) vcoef<O>(g.kb * d1[k] * (u[0][k] * u[0][k]), p.vy[SLOT][0][k], p.vy[SLOT][1][k]);
        if constexpr (TM) vcoef<O>(g.kb * d3[k] * (u[2][k] * u[2][k]), p.vy[SLOT][2][k], p.vy[SLOT][3][k]);
      }
    }
  }
}

// Advance a pipeline's row window by one row: n rows shift by one (nld is
// n of row R+2*DIR, first used at the end of the next row's iteration);
// with FEED, Q rows too (qld is Q of row R+2*DIR), else the caller puts the
// next ingested row into p.q.
template <int C, class O, bool FEED>
__device__ __forceinline__ void advance(Pipe<C>& p, const float (&qld)[6][C], const float (&nld)[3][C]) {
#pragma unroll
  for (int k = 0; k < C; ++k) {
    if constexpr (O::TE) p.nprev[0][k] = p.ncur[0][k];
    if constexpr (O::TM) p.nprev[1][k] = p.ncur[2][k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (!O::nlive(c)) continue;
      p.ncur[c][k] = p.nnext[c][k];
      p.nnext[c][k] = nld[c][k];
    }
    if constexpr (FEED) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        if (!O::live(c)) continue;
        p.q[c][k] = p.q1[c][k];
        p.q1[c][k] = qld[c][k];
      }
    }
  }
}

// A pipeline before its first row: empty delay lines and rings, n = 1.
template <int C>
__device__ __forceinline__ void pipe_clear(Pipe<C>& p) {
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
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < C; ++k) p.q14[s][c][k] = 0.0f;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c)
#pragma unroll
    for (int k = 0; k < C; ++k) p.q[c][k] = p.q1[c][k] = 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < C; ++k) p.ncur[c][k] = p.nnext[c][k] = 1.0f;
#pragma unroll
  for (int k = 0; k < C; ++k) p.nprev[0][k] = p.nprev[1][k] = 1.0f;
}

// The n window of a pipeline whose first ingested row is R0: rows R0-DIR
// (n_x, n_z), R0 and R0+DIR (rows of vacuum keep the 1 pipe_clear put
// there).
template <int C, class O, int DIR>
__device__ __forceinline__ void prime_n(Pipe<C>& p, const StepArgs& g, const uint32_t (&xo)[C], int64_t R0) {
  constexpr bool VEC = O::VEC;
  const int64_t nx64 = g.nx;
  const int rm = wrap_index(R0 - DIR, g.ny);
  const int r0 = wrap_index(R0, g.ny);
  const int r1 = wrap_index(R0 + DIR, g.ny);
  if (!vacuum_row(g, r0)) load_n<C, O>(g, g.n + r0 * nx64, xo, p.ncur, false);
  if (!vacuum_row(g, r1)) load_n<C, O>(g, g.n + r1 * nx64, xo, p.nnext, false);
  if (!vacuum_row(g, rm)) {
    const float* nm = g.n + rm * nx64;
    if (O::nlive(0)) load_row<C, VEC>(nm + 0 * g.plane, g.nx, xo, p.nprev[0]);
    if (O::nlive(2)) load_row<C, VEC>(nm + 2 * g.plane, g.nx, xo, p.nprev[1]);
  }
}

// Row iterations of a march of STEPS steps over a segment of seg_h rows:
// the segment and 4 rows of y support per step on each side, in whole
// groups of four.
template <int STEPS>
__device__ __forceinline__ int march_iters(int seg_h) {
  return ((seg_h + 8 * STEPS) + 3) & ~3;
}

template <int DIR>
__device__ __forceinline__ int next_row(int r, int ny) {
  if constexpr (DIR > 0)
    return (r + 1 == ny) ? 0 : r + 1;
  else
    return (r == 0) ? ny - 1 : r - 1;
}

// One wave's march over its segment in direction DIR: one step.
template <int C, class O, int DIR>
__device__ __forceinline__ void march(const StepArgs& g, const uint32_t (&xo)[C],
                                      const uint32_t (&so)[C], bool edge_lane, int y0, int seg_h) {
  constexpr bool VEC = O::VEC;
  Pipe<C> p;
  pipe_clear(p);
  // first ingested row: 4 rows before the segment in marching order
  const int64_t R0 = DIR > 0 ? static_cast<int64_t>(y0) - 4 : static_cast<int64_t>(y0) + seg_h + 3;
  const int64_t nx64 = g.nx;
  {
    const float* q0r = g.qin + wrap_index(R0, g.ny) * nx64;
    const float* q1r = g.qin + wrap_index(R0 + DIR, g.ny) * nx64;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      if (!O::live(c)) continue;
      load_row<C, VEC>(q0r + c * g.plane, g.nx, xo, p.q[c]);
      load_row<C, VEC>(q1r + c * g.plane, g.nx, xo, p.q1[c]);
    }
    prime_n<C, O, DIR>(p, g, xo, R0);
  }
  // rows in flight: Q and n of R+2*DIR (wrapped incrementally)
  int rq = wrap_index(R0 + 2 * DIR, g.ny);
  int rn = rq;
  uint64_t vmask = 0;   // vacuum flags of the index rows to load (vacuum_mask)
  const int iters = march_iters<1>(seg_h);
  float unused[6][C];
  const CoefIO<C> io{nullptr, nullptr, nullptr, nullptr, 0};
  for (int i = 0; i < iters; i += 4) {
    if ((i & 63) == 0) vmask = vacuum_mask<DIR>(g, rn);
#define QLA_ITER(S)                                                                            \
  {                                                                                            \
    float qld[6][C], nld[3][C];                                                                \
    load_q<C, O>(g, g.qin + rq * nx64, xo, qld);                                               \
    const bool vac = (vmask & 1) != 0;                                                         \
    vmask >>= 1;                                                                               \
    load_n<C, O>(g, g.n + rn * nx64, xo, nld, vac);                                            \
    process_row<C, O, DIR, S, false, 4, kCoefCompute>(p, g, so, edge_lane, i + S, seg_h, y0, unused, io); \
    fix_n<C, O>(nld, vac);                                                                     \
    advance<C, O, true>(p, qld, nld);                                                          \
    rq = next_row<DIR>(rq, g.ny);                                                              \
    rn = next_row<DIR>(rn, g.ny);                                                              \
  }
    QLA_ITER(0)
    QLA_ITER(1)
    QLA_ITER(2)
    QLA_ITER(3)
#undef QLA_ITER
  }
}

// Two steps per launch (temporal blocking) on a pair of waves. The
// producer wave runs the step on rows read from memory and hands each fully
// stepped row, through a two-slot LDS ring, to the consumer wave, which
// runs the second step on it and stores the result: HBM sees one read of Q
// and n and one write of Q per two steps, and each wave holds one pipeline
// (so two pairs fit on a SIMD). The producer starts 8 rows before the
// segment (the y support of two steps); the consumer ingests the rows the
// producer emits, 4 rows behind and one iteration later. Rows the producer
// cannot produce exactly (its first 8 and last 8 iterations, and the outer
// 8 columns of the strip) only ever reach halo rows and columns of the
// consumer, which are not stored.
//
// The consumer's rows are the producer's rows of four iterations earlier,
// with the same index values, so it takes their coefficients from the
// producer instead of recomputing them (and never reads n): the collision
// coefficients of n_x and n_z and the V_Y coefficients come from the
// producer's own four-row rings, sent when they are four rows old; those of
// n_y and the V_X coefficients, which the producer keeps for one row only,
// are sent at once through a six-slot ring and read four iterations later.
template <int C, class O>
struct Ring {
  using M = RingMap<O>;
  // cx rows kept: the consumer reads a row's four iterations after the
  // producer wrote it, and with Eq. (23) once more four iterations later
  static constexpr int NR = O::MODE == 0 ? 10 : 6;
  float q[2][M::NQ][kWave * C];    // the emitted row (live planes)
  float cy[2][M::NCY][kWave * C];  // its collision (n_x, n_z) and V_Y coefficients
  float cx[NR][M::NCX][kWave * C]; // collision (n_y) and V_X coefficients, by row
  // Eq. (23): each wave's four row slots of (q1, q4)
  float q14[O::MODE == 0 ? 2 * 4 * 2 * kWave * C : 1];
  int fy[2];
  int fx[NR];
};

template <int C, class O, int DIR>
__device__ __forceinline__ void march2(const StepArgs& g, const uint32_t (&xo)[C],
                                       const uint32_t (&so)[C], bool edge_lane, int y0, int seg_h,
                                       bool producer, int lane, Ring<C, O>& ring) {
  using M = RingMap<O>;
  constexpr bool VEC = O::VEC, TE = O::TE, TM = O::TM, POT = O::POT;
  Pipe<C> p;
  pipe_clear(p);
  const int64_t RA = DIR > 0 ? static_cast<int64_t>(y0) - 8 : static_cast<int64_t>(y0) + seg_h + 7;
  const int64_t nx64 = g.nx;
  const int iters = march_iters<2>(seg_h);
  float unused[6][C];
  constexpr int NR = Ring<C, O>::NR;
  // Eq. (23): this wave's (q1, q4) row slots start at zero, like the
  // registers of a one-step pipeline
  float* const q14 = O::MODE == 0 ? ring.q14 + (producer ? 0 : 4 * 2 * kWave * C) : nullptr;
  if constexpr (O::MODE == 0) {
    for (int e = lane; e < 4 * 2 * kWave * C; e += kWave) q14[e] = 0.0f;
  }
  if (producer) {
    if constexpr (O::MODE == 0) {
      // the lag-4 rows of its first four iterations (ahead of the halo)
      // read slots nobody has written yet: zero, as the consumer makes them
      for (int sl = NR - 4; sl < NR; ++sl) {
#pragma unroll
        for (int c = 0; c < M::NCX; ++c)
#pragma unroll
          for (int k = 0; k < C; ++k) ring.cx[sl][c][lane * C + k] = 0.0f;
        if (lane == 0) ring.fx[sl] = 0;
      }
    }
    {
      const float* q0r = g.qin + wrap_index(RA, g.ny) * nx64;
      const float* q1r = g.qin + wrap_index(RA + DIR, g.ny) * nx64;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        if (!O::live(c)) continue;
        load_row<C, VEC>(q0r + c * g.plane, g.nx, xo, p.q[c]);
        load_row<C, VEC>(q1r + c * g.plane, g.nx, xo, p.q1[c]);
      }
      prime_n<C, O, DIR>(p, g, xo, RA);
    }
    int rq = wrap_index(RA + 2 * DIR, g.ny);
    int rn = rq;
    uint64_t vmask = 0;   // vacuum flags of the index rows to load (vacuum_mask)
    int r6 = 0;   // iteration mod NR
    for (int i = 0; i < iters; i += 4) {
      if ((i & 63) == 0) vmask = vacuum_mask<DIR>(g, rn);
#define QLA_ITER_A(S)                                                                          \
  {                                                                                            \
    float qld[6][C], nld[3][C], e[6][C];                                                       \
    load_q<C, O>(g, g.qin + rq * nx64, xo, qld);                                               \
    const bool vac = (vmask & 1) != 0;                                                         \
    vmask >>= 1;                                                                               \
    load_n<C, O>(g, g.n + rn * nx64, xo, nld, vac);                                            \
    /* the ring entries of slot S hold the row four iterations old: the row */                \
    /* the consumer takes in this iteration */                                                 \
    _Pragma("unroll") for (int k = 0; k < C; ++k) {                                            \
      const int x = lane * C + k;                                                              \
      if constexpr (TE) {                                                                      \
        ring.cy[(S) & 1][M::cy(0)][x] = p.th[S][0][k];                                                \
        ring.cy[(S) & 1][M::cy(1)][x] = p.th[S][1][k];                                                \
        if constexpr (POT) {                                                                   \
          ring.cy[(S) & 1][M::cy(4)][x] = p.vy[S][0][k];                                              \
          ring.cy[(S) & 1][M::cy(5)][x] = p.vy[S][1][k];                                              \
        }                                                                                      \
      }                                                                                        \
      if constexpr (TM) {                                                                      \
        ring.cy[(S) & 1][M::cy(2)][x] = p.th[S][2][k];                                                \
        ring.cy[(S) & 1][M::cy(3)][x] = p.th[S][3][k];                                                \
        if constexpr (POT) {                                                                   \
          ring.cy[(S) & 1][M::cy(6)][x] = p.vy[S][2][k];                                              \
          ring.cy[(S) & 1][M::cy(7)][x] = p.vy[S][3][k];                                              \
        }                                                                                      \
      }                                                                                        \
    }                                                                                          \
    if (lane == 0) ring.fy[(S) & 1] = p.fy[S] ? 1 : 0;                                         \
    {                                                                                          \
      const int ro = r6 >= 4 ? r6 - 4 : r6 + NR - 4;   /* the row at lag 4 */                 \
      const CoefIO<C> io{&ring.cy[(S) & 1][0][0], &ring.cx[r6][0][0], &ring.fy[(S) & 1], &ring.fx[r6], lane, \
                         &ring.cx[ro][0][0], &ring.fx[ro], q14};                                    \
      process_row<C, O, DIR, S, true, 8, kCoefExport>(p, g, so, edge_lane, i + S, seg_h, y0, e, io); \
    }                                                                                          \
    _Pragma("unroll") for (int c = 0; c < 6; ++c) {                                            \
      if (!O::live(c)) continue;                                                               \
      _Pragma("unroll") for (int k = 0; k < C; ++k) ring.q[(S) & 1][M::q(c)][lane * C + k] = e[c][k]; \
    }                                                                                          \
    fix_n<C, O>(nld, vac);                                                                     \
    advance<C, O, true>(p, qld, nld);                                                          \
    rq = next_row<DIR>(rq, g.ny);                                                              \
    rn = next_row<DIR>(rn, g.ny);                                                              \
    r6 = r6 == NR - 1 ? 0 : r6 + 1;                                                            \
    __syncthreads();                                                                           \
  }
      QLA_ITER_A(0)
      QLA_ITER_A(1)
      QLA_ITER_A(2)
      QLA_ITER_A(3)
#undef QLA_ITER_A
    }
    __syncthreads();     // the consumer's last row
  } else {
    // slots the consumer reads before the producer has written them (its
    // first four rows, and with Eq. (23) the lag-4 rows of its first eight,
    // which only reach halo rows) start at zero
    for (int sl = O::MODE == 0 ? NR - 8 : NR - 4; sl < NR; ++sl) {
#pragma unroll
      for (int c = 0; c < M::NCX; ++c)
#pragma unroll
        for (int k = 0; k < C; ++k) ring.cx[sl][c][lane * C + k] = 0.0f;
      if (lane == 0) ring.fx[sl] = 0;
    }
    __syncthreads();     // the producer's first row
    int r6 = NR - 4;     // (iteration - 4) mod NR
    for (int i = 0; i < iters; i += 4) {
#define QLA_ITER_B(S)                                                                          \
  {                                                                                            \
    _Pragma("unroll") for (int c = 0; c < 6; ++c) {                                            \
      if (!O::live(c)) continue;                                                               \
      _Pragma("unroll") for (int k = 0; k < C; ++k) p.q[c][k] = ring.q[(S) & 1][M::q(c)][lane * C + k]; \
    }                                                                                          \
    {                                                                                          \
      const int ro = r6 >= 4 ? r6 - 4 : r6 + NR - 4;   /* the row at lag 4 */                 \
      const CoefIO<C> io{&ring.cy[(S) & 1][0][0], &ring.cx[r6][0][0], &ring.fy[(S) & 1], &ring.fx[r6], lane, \
                         &ring.cx[ro][0][0], &ring.fx[ro], q14};                                    \
      process_row<C, O, DIR, S, false, 12, kCoefImport>(p, g, so, edge_lane, i + S, seg_h, y0, unused, io); \
    }                                                                                          \
    r6 = r6 == NR - 1 ? 0 : r6 + 1;                                                            \
    __syncthreads();                                                                           \
  }
      QLA_ITER_B(0)
      QLA_ITER_B(1)
      QLA_ITER_B(2)
      QLA_ITER_B(3)
#undef QLA_ITER_B
    }
  }
}

// One lattice of a batch as the step kernel reads it from device memory.
struct InstDesc {
  const float* q[2];     // the two state buffers (6 planes each)
  const float* n;        // 3 planes
  int64_t plane;         // nx * ny
  int nx, ny;
  int seg_rows;          // rows per wave segment (multiple of 4)
  int nstrips, nsegs;
  int first_block;       // blocks of the lattices before this one
  float a4, kb;
  const int* span;       // 2 * ny ints: per row, first and last non-vacuum column
};
static_assert(sizeof(InstDesc) == 72, "descriptor layout");

struct BatchArgs {
  const InstDesc* __restrict__ desc;
  int count;             // lattices in the batch
  int parity;            // state buffer holding the input of this step
  int waves_per_block;
  int read_all_n;        // 1: read every index row (no vacuum rows taken as 1)
};

// Row pos of the order 0, 8, 16, ..., 1, 9, 17, ..., 7, 15, ... of the rows
// 0 .. n-1 (a permutation).
__device__ __forceinline__ int interleave8(int pos, int n) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int cnt = (n - r + 7) / 8;   // rows r, r + 8, ... below n
    if (pos < cnt) return r + 8 * pos;
    pos -= cnt;
  }
  return n;   // pos >= n: no row
}

// STEPS time steps per launch (1, or 2 with temporal blocking).
template <int C, class O, int STEPS>
__global__ void __launch_bounds__(256) qla_step_kernel(BatchArgs ba) {
  using Cl = Cols<C, STEPS>;
  const int lane = threadIdx.x & (kWave - 1);
  // wave index within the block, as a wave-uniform (scalar) value
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x / kWave));
  // blocks are dealt round-robin to the 8 XCDs; regroup them so that each
  // XCD gets a contiguous band of work (neighbouring strips share halo
  // columns through that XCD's L2), the band's rows of blocks taken from
  // the lattice eight rows apart (so that every XCD gets a share of an
  // object's rows, which take longest)
  const int nblk = gridDim.x;
  const int b = blockIdx.x;
  const int per = nblk / 8;
  const int rem = nblk % 8;
  const int xcd = b % 8;
  const int k8 = b / 8;
  const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
  // the lattice this block works on: the last one starting at or before it
  int lo = 0, hi = ba.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ba.desc[mid].first_block <= logical) lo = mid; else hi = mid - 1;
  }
  const InstDesc& d = ba.desc[lo];
  const int local = logical - d.first_block;
  const int strip = local % d.nstrips;
  const int brows = STEPS == 2 ? d.nsegs : (d.nsegs + ba.waves_per_block - 1) / ba.waves_per_block;
  const int brow = interleave8(local / d.nstrips, brows);
  // a two-step block is one producer/consumer pair of waves on one segment
  const int seg = STEPS == 2 ? brow : brow * ba.waves_per_block + wave;
  if (seg >= d.nsegs) return;

  StepArgs g;
  g.qin = d.q[ba.parity];
  g.qout = const_cast<float*>(d.q[ba.parity ^ 1]);
  g.n = d.n;
  g.span = d.span;
  g.plane = d.plane;
  g.nx = d.nx;
  g.ny = d.ny;
  g.a4 = d.a4;
  g.kb = d.kb;

  const int y0 = seg * d.seg_rows;
  const int seg_h = min(d.seg_rows, g.ny - y0);
  const int x0 = strip * Cl::kOut;
  const int64_t col0 = static_cast<int64_t>(x0) - Cl::kHaloLanes * C + lane * C;
  {
    // the columns the wave loads, [wa, wb] taken periodically
    int wa = x0 - Cl::kHaloLanes * C;
    int wb = wa + kWave * C - 1;
    int g0 = INT_MAX, g1 = INT_MIN;
    if (ba.read_all_n != 0) {          // never vacuum
      wa = INT_MIN;
      wb = INT_MAX;
    } else if (wb - wa + 1 >= g.nx) {  // every column: only a row without a span
      wa = 0;
      wb = INT_MAX;
    } else if (wa < 0) {               // [0, wb] and [wa + nx, nx - 1]
      g0 = wb;
      g1 = wa + g.nx;
      wa = 0;
      wb = INT_MAX;
    } else if (wb >= g.nx) {           // [wa, nx - 1] and [0, wb - nx]
      g0 = wb - g.nx;
      g1 = wa;
      wa = 0;
      wb = INT_MAX;
    }
    g.wa = wa;
    g.wb = wb;
    g.g0 = g0;
    g.g1 = g1;
  }
  // byte offsets of the lane's columns within a row: loads wrap
  // periodically, stores only for output columns of this strip
  uint32_t xo[C], so[C];
  const bool lane_in = lane >= Cl::kHaloLanes && lane < kWave - Cl::kHaloLanes;
  const bool edge_lane = lane == 0 || lane == kWave - 1;
#pragma unroll
  for (int k = 0; k < C; ++k) {
    xo[k] = 4u * static_cast<uint32_t>(wrap_index(col0 + k, g.nx));
    so[k] = (lane_in && col0 + k < g.nx) ? xo[k] : kNoStore;
  }
  if constexpr (O::VEC) {
    // the lane's C columns are stored together or not at all
#pragma unroll
    for (int k = 1; k < C; ++k) so[k] = so[0];
  }
  // Neighbouring segments march in opposite directions, so that the 8 halo
  // rows two segments share are read by both at about the same time (at
  // the start of both marches or at the end of both) and come from L2 for
  // the second reader.
  if constexpr (STEPS == 2) {
    __shared__ Ring<C, O> ring;
    const bool producer = wave == 0;
    // the producer is on the pair's critical path (it also computes the
    // row coefficients): let its instructions issue first on a shared SIMD
    if (producer) __builtin_amdgcn_s_setprio(2);
    if (seg & 1)
      march2<C, O, +1>(g, xo, so, edge_lane, y0, seg_h, producer, lane, ring);
    else
      march2<C, O, -1>(g, xo, so, edge_lane, y0, seg_h, producer, lane, ring);
  } else {
    if (seg & 1)
      march<C, O, +1>(g, xo, so, edge_lane, y0, seg_h);
    else
      march<C, O, -1>(g, xo, so, edge_lane, y0, seg_h);
  }
}

// One compiled set of options of the step kernel: its one-step and
// two-step launches.
struct StepImpl {
  const void* func[2];                                   // __global__ function, 1 and 2 steps
  hipError_t (*blocks_per_cu[2])(int* nb, int threads);  // occupancy queries
  int cols;
};

template <int C, class O, int STEPS>
hipError_t step_blocks_per_cu(int* nb, int threads) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, qla_step_kernel<C, O, STEPS>, threads, 0);
}

template <int C, class O>
StepImpl impl() {
  return StepImpl{{reinterpret_cast<const void*>(&qla_step_kernel<C, O, 1>),
                   reinterpret_cast<const void*>(&qla_step_kernel<C, O, 2>)},
                  {step_blocks_per_cu<C, O, 1>, step_blocks_per_cu<C, O, 2>},
                  C};
}

// Options every instance is selected by at run time.
struct StepChoice {
  int mode;        // QLA_POT_EQ23 (0) or QLA_POT_EQ28 (1)
  bool pot;        // kappa != 0
  bool wide;
  bool vec;
  int fields;      // 0 all, 1 TM, 2 TE
  int skew;        // 0 printed potentials, 1 skew-symmetric
  bool stream;     // non-temporal state loads (six components only)
};

// One translation unit per (placement, field triple) instantiates these.
template <int MODE, int FIELDS>
StepImpl pick_step(const StepChoice& ch) {
  constexpr int C = 2;
  auto pick_pot = [&](auto vecc, auto widec) -> StepImpl {
    constexpr bool V = decltype(vecc)::value, Wd = decltype(widec)::value;
    if constexpr (FIELDS == 0) {
      if (ch.stream) {
        if (!ch.pot) return impl<C, KOpt<MODE, false, Wd, V, FIELDS, 0, 1>>();
        if (ch.skew) return impl<C, KOpt<MODE, true, Wd, V, FIELDS, 1, 1>>();
        return impl<C, KOpt<MODE, true, Wd, V, FIELDS, 0, 1>>();
      }
    }
    if (!ch.pot) return impl<C, KOpt<MODE, false, Wd, V, FIELDS, 0>>();
    if (ch.skew) return impl<C, KOpt<MODE, true, Wd, V, FIELDS, 1>>();
    return impl<C, KOpt<MODE, true, Wd, V, FIELDS, 0>>();
  };
  using T = std::integral_constant<bool, true>;
  using F = std::integral_constant<bool, false>;
  if (ch.vec) return ch.wide ? pick_pot(T{}, T{}) : pick_pot(T{}, F{});
  return ch.wide ? pick_pot(F{}, T{}) : pick_pot(F{}, F{});
}

// The units (qla_step_inst.hip built once per placement and field triple)
StepImpl pick_step_m0_f0(const StepChoice& ch);
StepImpl pick_step_m0_f1(const StepChoice& ch);
StepImpl pick_step_m0_f2(const StepChoice& ch);
StepImpl pick_step_m1_f0(const StepChoice& ch);
StepImpl pick_step_m1_f1(const StepChoice& ch);
StepImpl pick_step_m1_f2(const StepChoice& ch);

}  // namespace qla_dev
