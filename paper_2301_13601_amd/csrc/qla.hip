// libqla: the qubit lattice algorithm (QLA) of Vahala et al.,
// arXiv:2301.13601, as hand-written HIP for gfx950 (MI355X), behind the C ABI
// declared in include/qla.h. This file holds the host side (contexts,
// launch planning, graphs, the C entry points) and the auxiliary kernels
// (validation scan, FP64 diagnostics, field export); the fused step kernel is
// in qla_step.hpp and its instances in qla_step_inst.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <vector>

#include "qla.h"
#include "qla_step.hpp"

namespace {

using qla_dev::BatchArgs;
using qla_dev::InstDesc;
using qla_dev::kNarrowAngle;
using qla_dev::kWave;
using qla_dev::StepImpl;

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
// Vacuum spans of n at init: per row, the first and last column at which
// one of the index planes in `planes` (bit c: plane c) differs from 1, or
// (nx, -1) for a row of vacuum. The step kernel takes a row's index window
// as 1 without reading it when the window lies outside the span.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) qla_span_kernel(const float* __restrict__ n, int nx, int ny,
                                                       int planes, int* __restrict__ span) {
  const int64_t plane = static_cast<int64_t>(nx) * ny;
  __shared__ int sh[2][256 / kWave];
  for (int y = blockIdx.x; y < ny; y += gridDim.x) {
    int lo = nx, hi = -1;
    for (int x = threadIdx.x; x < nx; x += blockDim.x) {
      const int64_t s = static_cast<int64_t>(y) * nx + x;
      bool other = false;
      for (int c = 0; c < 3; ++c)
        if ((planes >> c) & 1) other = other || n[c * plane + s] != 1.0f;
      if (other) {
        lo = min(lo, x);
        hi = max(hi, x);
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o));
      hi = max(hi, __shfl_xor(hi, o));
    }
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
      sh[0][w] = lo;
      sh[1][w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 1; k < static_cast<int>(blockDim.x / kWave); ++k) {
        lo = min(lo, sh[0][k]);
        hi = max(hi, sh[1][k]);
      }
      span[2 * y] = lo;
      span[2 * y + 1] = hi;
    }
    __syncthreads();
  }
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

// Sums and maxima of the per-block partials over `count` blocks, by one
// wave; every lane ends with the folded values.
__device__ __forceinline__ void diag_fold(const double* __restrict__ parts, int count, double (&v)[kDiagVals]) {
  for (int j = 0; j < kDiagVals; ++j) v[j] = 0.0;   // sums and maxima of non-negative values
  for (int k = threadIdx.x; k < count; k += blockDim.x) {
    const double* o = parts + static_cast<int64_t>(k) * kDiagVals;
    v[0] += o[0]; v[1] += o[1]; v[2] = fmax(v[2], o[2]); v[3] = fmax(v[3], o[3]);
    v[4] += o[4]; v[5] += o[5]; v[6] = fmax(v[6], o[6]); v[7] = fmax(v[7], o[7]);
  }
  v[0] = wave_sum(v[0]); v[1] = wave_sum(v[1]); v[4] = wave_sum(v[4]); v[5] = wave_sum(v[5]);
  v[2] = wave_max(v[2]); v[3] = wave_max(v[3]); v[6] = wave_max(v[6]); v[7] = wave_max(v[7]);
}

__global__ void qla_diag_final(double* __restrict__ parts, int count) {
  // one wave; parts[count * kDiagVals ..] receives the folded values
  double v[kDiagVals];
  diag_fold(parts, count, v);
  if (threadIdx.x == 0)
    for (int j = 0; j < kDiagVals; ++j) parts[static_cast<int64_t>(count) * kDiagVals + j] = v[j];
}

// One wave: the folded partials as a finished qla_diag in device memory
// (the same conversion qla_energy makes on the host).
__global__ void qla_diag_finish(const double* __restrict__ parts, int count, int64_t plane, int64_t step,
                                qla_diag* __restrict__ out) {
  double v[kDiagVals];
  diag_fold(parts, count, v);
  if (threadIdx.x == 0) {
    qla_diag o;
    o.step = step;
    o.energy = v[0] / static_cast<double>(plane);
    o.divB_l2 = sqrt(v[1]);
    o.divB_max = v[2];
    o.B_max = sqrt(v[3]);
    o.B_l2 = sqrt(v[4]);
    o.divD_l2 = sqrt(v[5]);
    o.divD_max = v[6];
    o.D_max = sqrt(v[7]);
    *out = o;
  }
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

// Zero three planes of a state (the triple a polarised context holds at
// zero): planes c0, c1, c2 of q.
__global__ void __launch_bounds__(256) qla_clear_kernel(float* __restrict__ q, int64_t plane, int c0,
                                                        int c1, int c2) {
  for (int64_t s = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; s < plane;
       s += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    q[c0 * plane + s] = 0.0f;
    q[c1 * plane + s] = 0.0f;
    q[c2 * plane + s] = 0.0f;
  }
}


}  // namespace

// Device buffer of qla_energy_noalloc: the per-block partials of one
// diagnostics call, kDiagBlocks blocks of kDiagVals doubles (64 KiB). Each
// GPU holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that GPU.
constexpr int kNoAllocDoubles = kDiagBlocks * kDiagVals;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

// ===========================================================================
// Host side.
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
constexpr int kDefaultGraphSteps = 32;
constexpr int kDefaultStepsPerPass = 2;
constexpr int kCols = 2;                          // lattice columns per lane
// output columns of a strip for a launch of `steps` steps (x support 4 per step)
constexpr int out_cols(int steps) { return (kWave - 2 * ((4 * steps + kCols - 1) / kCols)) * kCols; }

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// workspace layout: diagnostics partials | scan partials | lattice
// descriptors of the one-step launch | of the two-step launch | the vacuum
// spans of each lattice's rows
size_t diag_bytes() { return align256(static_cast<size_t>(kDiagBlocks + 1) * kDiagVals * sizeof(double)); }
size_t scan_bytes() { return align256(static_cast<size_t>(kDiagBlocks + 1) * sizeof(ScanPartial)); }
size_t desc_bytes(int count) { return align256(sizeof(InstDesc) * count); }
size_t span_bytes(int ny) { return align256(2 * sizeof(int) * static_cast<size_t>(ny)); }
size_t work_bytes(int count, const qla_instance* inst) {
  size_t b = diag_bytes() + scan_bytes() + 2 * desc_bytes(count);
  for (int i = 0; i < count; ++i) b += span_bytes(inst[i].p.ny);
  return b;
}

}  // namespace

// error reporting shared with the surrogate kernels (qnn.hip)
namespace qnn {
void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}
}  // namespace qnn

struct qla_ctx {
  uint64_t magic;
  int count;
  int pot_mode, beta_scale, polarisation, v_form;
  std::vector<qla_params> p;
  std::vector<const float*> n;
  std::vector<float*> buf[2];
  std::vector<int*> span;  // per lattice: its rows' vacuum spans (workspace)
  int cur;                 // which buffer (0 or 1) holds the current state
  void* work;
  hipStream_t stream;
  int64_t steps;
  bool wide;
  bool poisoned;
  int cus;
  qla_launch launch;       // requested geometry (0 fields: default)
  qla_launch planned;      // geometry in use
  StepImpl step;
  // per steps-per-launch (index 0: one step, 1: two steps)
  struct Geometry {
    std::vector<InstDesc> desc;
    InstDesc* d_desc;
    dim3 grid, block;
    int seg_rows;
    hipGraphExec_t graph[2];   // graph_steps steps starting from buffer 0 / 1
  } geo[2];
};

namespace {

qla_status check_params(const qla_params* p) {
  if (!p) return fail(QLA_EINVAL, "qla: null params");
  if (p->nx < 1 || p->ny < 1) return fail(QLA_EINVAL, "qla: lattice %d x %d must be at least 1 x 1", p->nx, p->ny);
  if (static_cast<int64_t>(p->nx) * p->ny > (int64_t{1} << 40))
    return fail(QLA_EINVAL, "qla: lattice too large");
  if (p->nx > (1 << 28)) return fail(QLA_EINVAL, "qla: rows longer than 2^28 sites are not supported");
  if (!(p->delta > 0.0) || !std::isfinite(p->delta)) return fail(QLA_EINVAL, "qla: delta must be finite and > 0");
  if (p->pot_mode != QLA_POT_EQ23 && p->pot_mode != QLA_POT_EQ28)
    return fail(QLA_EINVAL, "qla: pot_mode %d is not QLA_POT_EQ23 or QLA_POT_EQ28", p->pot_mode);
  if (p->beta_scale < QLA_BETA_PHYS || p->beta_scale > QLA_BETA_OFF)
    return fail(QLA_EINVAL, "qla: beta_scale %d unknown", p->beta_scale);
  if (p->polarisation < QLA_POL_BOTH || p->polarisation > QLA_POL_TE)
    return fail(QLA_EINVAL, "qla: polarisation %d unknown", p->polarisation);
  if (p->v_form != QLA_V_PRINTED && p->v_form != QLA_V_SKEW)
    return fail(QLA_EINVAL, "qla: v_form %d unknown", p->v_form);
  return QLA_OK;
}

qla_status check_batch(int32_t count, const qla_instance* inst) {
  if (count < 1) return fail(QLA_EINVAL, "qla: a batch holds at least one lattice");
  if (!inst) return fail(QLA_EINVAL, "qla: null instance array");
  for (int i = 0; i < count; ++i) {
    qla_status st = check_params(&inst[i].p);
    if (st != QLA_OK) return st;
    if (inst[i].p.pot_mode != inst[0].p.pot_mode || inst[i].p.beta_scale != inst[0].p.beta_scale ||
        inst[i].p.polarisation != inst[0].p.polarisation || inst[i].p.v_form != inst[0].p.v_form)
      return fail(QLA_EINVAL,
                  "qla: pot_mode, beta_scale, polarisation and v_form must be the same for every lattice "
                  "of a batch");
  }
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

double kb_of(const qla_params& p) {
  const double frac = p.pot_mode == QLA_POT_EQ28 ? 0.5 : 1.0;
  return kappa_of(p) * frac * 0.5;
}

// In a TM or TE context, zero the planes of the other triple of lattice i in
// state buffer b (a kernel, not a memset, so that a caller may capture it).
hipError_t clear_dead(qla_ctx* c, int i, int b) {
  if (c->polarisation == QLA_POL_BOTH) return hipSuccess;
  const qla_params& p = c->p[i];
  const int64_t plane = static_cast<int64_t>(p.nx) * p.ny;
  const int blocks = static_cast<int>(std::min<int64_t>((plane + 255) / 256, 4096));
  if (c->polarisation == QLA_POL_TM)
    hipLaunchKernelGGL(qla_clear_kernel, dim3(blocks), dim3(256), 0, c->stream, c->buf[b][i], plane, 0, 1, 5);
  else
    hipLaunchKernelGGL(qla_clear_kernel, dim3(blocks), dim3(256), 0, c->stream, c->buf[b][i], plane, 2, 3, 4);
  return hipGetLastError();
}

void drop_graphs(qla_ctx* c) {
  for (auto& geo : c->geo)
    for (auto& g : geo.graph) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Launch geometry. A wave covers 128 columns of which 120 are output (112
// for a two-step launch); each lattice is cut into strips (x) and segments
// (y), and every segment costs its rows plus 8 halo rows per step. A
// requested segment height applies to every lattice. Otherwise the planner
// takes a target height S, gives each lattice the whole number of segments
// closest to its height / S (so segments of all lattices are about equally
// tall), and keeps the S whose blocks, handed in launch order to the
// resident block slots (earliest free slot first), finish soonest; among
// near ties it prefers taller segments (fewer halo rows).
struct SegPlan {
  std::vector<int> seg;     // rows per segment, per lattice
  int64_t blocks = 0;
  int64_t makespan = 0;     // in row iterations
};

SegPlan segment_plan(const qla_ctx* c, const std::vector<int>& nstrips, int wpb, int halo, int S, bool uniform,
                     int64_t slots) {
  SegPlan pl;
  pl.seg.resize(c->count);
  for (int i = 0; i < c->count; ++i) {
    const int ny = c->p[i].ny;
    int h = S;
    if (!uniform) {
      const int nseg = std::max(1, static_cast<int>((static_cast<int64_t>(ny) + S / 2) / S));
      h = (ny + nseg - 1) / nseg;
    }
    h = std::max(4, (h + 3) & ~3);
    pl.seg[i] = h;
    const int nsegs = (ny + h - 1) / h;
    pl.blocks += static_cast<int64_t>(nstrips[i]) * ((nsegs + wpb - 1) / wpb);
  }
  if (slots <= 0) return pl;
  // earliest-free-slot simulation of the launch order; a block of wpb
  // segments lasts as long as its tallest segment
  std::vector<int64_t> heap(static_cast<size_t>(std::min<int64_t>(slots, pl.blocks)), 0);
  auto cmp = std::greater<int64_t>();
  for (int i = 0; i < c->count; ++i) {
    const int ny = c->p[i].ny, h = pl.seg[i];
    const int nsegs = (ny + h - 1) / h;
    for (int j = 0; j < nsegs; j += wpb) {
      const int64_t d = std::min(h, ny - j * h) + halo;
      for (int k = 0; k < nstrips[i]; ++k) {
        std::pop_heap(heap.begin(), heap.end(), cmp);
        heap.back() += d;
        pl.makespan = std::max(pl.makespan, heap.back());
        std::push_heap(heap.begin(), heap.end(), cmp);
      }
    }
  }
  return pl;
}

qla_status plan_geometry(qla_ctx* c, int steps, int wpb) {
  auto& geo = c->geo[steps - 1];
  // a two-step block is one producer/consumer pair of waves
  if (steps == 2) wpb = 1;
  const int threads = steps == 2 ? 2 * kWave : kWave * wpb;
  const int oc = out_cols(steps);
  const int halo = 8 * steps;
  int max_ny = 1;
  for (const auto& p : c->p) max_ny = std::max(max_ny, p.ny);
  std::vector<int> nstrips(c->count);
  for (int i = 0; i < c->count; ++i) nstrips[i] = (c->p[i].nx + oc - 1) / oc;
  SegPlan pl;
  if (c->launch.seg_rows > 0) {
    pl = segment_plan(c, nstrips, wpb, halo, c->launch.seg_rows, true, 0);
  } else {
    int bpc = 0;
    hipError_t e = c->step.blocks_per_cu[steps - 1](&bpc, threads);
    if (e != hipSuccess || bpc < 1) bpc = 1;
    const int64_t slots = static_cast<int64_t>(c->cus) * bpc;
    const int top = (max_ny + 3) & ~3;
    // about 96 candidate targets, denser where segments are short
    std::vector<int> cand;
    for (int s = 8; s <= top; s += std::max(4, (s / 24) & ~3)) cand.push_back(s);
    if (cand.empty() || cand.back() != top) cand.push_back(top);
    std::vector<int64_t> span(cand.size());
    int64_t best = -1;
    for (size_t k = 0; k < cand.size(); ++k) {
      span[k] = segment_plan(c, nstrips, wpb, halo, cand[k], false, slots).makespan;
      if (best < 0 || span[k] < best) best = span[k];
    }
    // the tallest target within 1% of the best makespan
    size_t pick = 0;
    for (size_t k = 0; k < cand.size(); ++k)
      if (span[k] * 100 <= best * 101) pick = k;
    pl = segment_plan(c, nstrips, wpb, halo, cand[pick], false, 0);
  }
  if (pl.blocks > (int64_t{1} << 30)) return fail(QLA_EINVAL, "qla: launch geometry too large");
  geo.desc.assign(c->count, InstDesc{});
  int first = 0;
  int tallest = 4;
  for (int i = 0; i < c->count; ++i) {
    const qla_params& p = c->p[i];
    InstDesc& d = geo.desc[i];
    d.q[0] = c->buf[0][i];
    d.q[1] = c->buf[1][i];
    d.n = c->n[i];
    d.plane = static_cast<int64_t>(p.nx) * p.ny;
    d.nx = p.nx;
    d.ny = p.ny;
    d.seg_rows = pl.seg[i];
    d.nstrips = nstrips[i];
    d.nsegs = (p.ny + d.seg_rows - 1) / d.seg_rows;
    d.first_block = first;
    d.a4 = static_cast<float>(p.delta / 4.0);
    d.kb = static_cast<float>(kb_of(p));
    d.span = c->span[i];
    first += d.nstrips * ((d.nsegs + wpb - 1) / wpb);
    tallest = std::max(tallest, d.seg_rows);
  }
  hipError_t e = hipMemcpyAsync(geo.d_desc, geo.desc.data(), sizeof(InstDesc) * c->count,
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "uploading the lattice descriptors");
  geo.grid = dim3(static_cast<unsigned>(pl.blocks));
  geo.block = dim3(threads);
  geo.seg_rows = tallest;
  return QLA_OK;
}

qla_status plan_step(qla_ctx* c) {
  const int wpb = c->launch.waves_per_block > 0 ? c->launch.waves_per_block : 1;
  if (wpb > 4) return fail(QLA_EINVAL, "qla: waves_per_block must be 1..4");
  const int spp = c->launch.steps_per_pass > 0 ? c->launch.steps_per_pass : kDefaultStepsPerPass;
  if (spp > 2) return fail(QLA_EINVAL, "qla: steps_per_pass must be 1 or 2");
  int gsteps = c->launch.graph_steps > 0 ? c->launch.graph_steps : kDefaultGraphSteps;
  // a replay must return to the buffer it started from: an even number of
  // launches
  const int unit = 2 * spp;
  if (gsteps > 1) gsteps = (gsteps + unit - 1) / unit * unit;
  bool vec = true;
  for (const auto& p : c->p) vec = vec && (p.nx % kCols) == 0;
  qla_dev::StepChoice ch;
  ch.mode = c->pot_mode;
  ch.pot = c->beta_scale != QLA_BETA_OFF;
  ch.wide = c->wide;
  ch.vec = vec;
  ch.fields = c->polarisation;
  ch.skew = c->v_form;
  // non-temporal state loads only when asked for: with the index rows of
  // vacuum skipped they no longer pay off on a single lattice either
  ch.stream = c->polarisation == QLA_POL_BOTH && c->launch.stream_loads == 1;
  using Pick = StepImpl (*)(const qla_dev::StepChoice&);
  static constexpr Pick kPick[2][3] = {
      {qla_dev::pick_step_m0_f0, qla_dev::pick_step_m0_f1, qla_dev::pick_step_m0_f2},
      {qla_dev::pick_step_m1_f0, qla_dev::pick_step_m1_f1, qla_dev::pick_step_m1_f2}};
  c->step = kPick[ch.mode][ch.fields](ch);
  drop_graphs(c);
  for (int steps = 1; steps <= 2; ++steps) {
    qla_status st = plan_geometry(c, steps, wpb);
    if (st != QLA_OK) return st;
  }
  c->planned = qla_launch{c->geo[spp - 1].seg_rows, wpb, gsteps, spp, ch.stream ? 1 : 2,
                          c->launch.vacuum_rows == 2 ? 2 : 1};
  return QLA_OK;
}

BatchArgs batch_args(const qla_ctx* c, int steps, int parity) {
  const auto& geo = c->geo[steps - 1];
  return BatchArgs{geo.d_desc, c->count, parity, steps == 2 ? 1 : static_cast<int>(geo.block.x / kWave),
                   c->planned.vacuum_rows == 2 ? 1 : 0};
}

// One launch advancing `steps` (1 or 2) time steps from buffer `parity`.
hipError_t launch_one(qla_ctx* c, int steps, int parity) {
  BatchArgs a = batch_args(c, steps, parity);
  void* args[] = {&a};
  return hipLaunchKernel(c->step.func[steps - 1], c->geo[steps - 1].grid, c->geo[steps - 1].block, args, 0,
                         c->stream);
}

// A graph of graph_steps consecutive steps (launches of steps_per_pass
// steps, alternating buffers), built node by node so that it can be
// replayed on any stream.
hipError_t build_graph(qla_ctx* c, int parity) {
  const int spp = c->planned.steps_per_pass;
  auto& geo = c->geo[spp - 1];
  hipGraph_t g = nullptr;
  hipError_t e = hipGraphCreate(&g, 0);
  if (e != hipSuccess) return e;
  hipGraphNode_t prev = nullptr;
  const int launches = c->planned.graph_steps / spp;
  std::vector<BatchArgs> args(launches);
  for (int j = 0; j < launches && e == hipSuccess; ++j) {
    args[j] = batch_args(c, spp, parity ^ (j & 1));
    void* kp[] = {&args[j]};
    hipKernelNodeParams np{};
    np.func = const_cast<void*>(c->step.func[spp - 1]);
    np.gridDim = geo.grid;
    np.blockDim = geo.block;
    np.sharedMemBytes = 0;
    np.kernelParams = kp;
    np.extra = nullptr;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &np);
    prev = node;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&geo.graph[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

// Validate the index of lattice i and fold its angle ranges into nmin/bmax.
qla_status scan_instance(qla_ctx* c, int i, double* theta_max, double* bmax) {
  const qla_params& p = c->p[i];
  const int64_t plane = static_cast<int64_t>(p.nx) * p.ny;
  int blocks = static_cast<int>(std::min<int64_t>((plane + 255) / 256, kDiagBlocks));
  ScanPartial* parts = reinterpret_cast<ScanPartial*>(static_cast<char*>(c->work) + diag_bytes());
  hipLaunchKernelGGL(qla_scan_kernel, dim3(blocks), dim3(256), 0, c->stream, c->n[i], p.nx, p.ny,
                     kb_of(p), parts);
  hipLaunchKernelGGL(qla_scan_final, dim3(1), dim3(kWave), 0, c->stream, parts, blocks);
  ScanPartial res{};
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&res, parts + blocks, sizeof(res), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "validating n");
  if (res.bad != 0.0)
    return fail(QLA_EINVAL, "qla: lattice %d: every refractive index must be finite and > 0", i);
  *theta_max = std::max(*theta_max, p.delta / (4.0 * res.nmin));
  *bmax = std::max(*bmax, res.bmax);
  // the index planes the step reads: n_x, n_y for the TE triple, n_z for TM
  const int planes = c->polarisation == QLA_POL_TM ? 4 : (c->polarisation == QLA_POL_TE ? 3 : 7);
  hipLaunchKernelGGL(qla_span_kernel, dim3(std::min(p.ny, 4096)), dim3(256), 0, c->stream, c->n[i], p.nx, p.ny,
                     planes, c->span[i]);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(nullptr, e, "summarising n");
  return QLA_OK;
}

qla_status init_common(int32_t count, const qla_instance* inst, void* d_work, void* hip_stream,
                       qla_ctx** out) {
  if (!out) return fail(QLA_EINVAL, "qla: null output pointer");
  *out = nullptr;
  qla_status st = check_batch(count, inst);
  if (st != QLA_OK) return st;
  if (!d_work) return fail(QLA_EINVAL, "qla: null workspace");
  if ((reinterpret_cast<uintptr_t>(d_work) & 255) != 0)
    return fail(QLA_EINVAL, "qla: workspace must be 256-byte aligned");
  for (int i = 0; i < count; ++i) {
    if (!inst[i].d_n || !inst[i].d_q || !inst[i].d_q_pong)
      return fail(QLA_EINVAL, "qla: lattice %d: null device buffer", i);
    if (inst[i].d_q == inst[i].d_q_pong)
      return fail(QLA_EINVAL, "qla: lattice %d: the two state buffers must differ", i);
  }
  qla_ctx* c = new (std::nothrow) qla_ctx();
  if (!c) return fail(QLA_ENOMEM, "qla: host allocation failed");
  c->magic = kMagic;
  c->count = count;
  c->pot_mode = inst[0].p.pot_mode;
  c->beta_scale = inst[0].p.beta_scale;
  c->polarisation = inst[0].p.polarisation;
  c->v_form = inst[0].p.v_form;
  try {
    for (int i = 0; i < count; ++i) {
      c->p.push_back(inst[i].p);
      c->n.push_back(inst[i].d_n);
      c->buf[0].push_back(inst[i].d_q);
      c->buf[1].push_back(inst[i].d_q_pong);
    }
    char* s = static_cast<char*>(d_work) + diag_bytes() + scan_bytes() + 2 * desc_bytes(count);
    for (int i = 0; i < count; ++i) {
      c->span.push_back(reinterpret_cast<int*>(s));
      s += span_bytes(inst[i].p.ny);
    }
  } catch (...) {
    delete c;
    return fail(QLA_ENOMEM, "qla: host allocation failed");
  }
  c->cur = 0;
  c->work = d_work;
  c->geo[0].d_desc = reinterpret_cast<InstDesc*>(static_cast<char*>(d_work) + diag_bytes() + scan_bytes());
  c->geo[1].d_desc = reinterpret_cast<InstDesc*>(static_cast<char*>(d_work) + diag_bytes() + scan_bytes() +
                                                 desc_bytes(count));
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->steps = 0;
  c->poisoned = false;
  for (auto& geo : c->geo) geo.graph[0] = geo.graph[1] = nullptr;
  double theta_max = 0.0, bmax = 0.0;
  for (int i = 0; i < count; ++i) {
    st = scan_instance(c, i, &theta_max, &bmax);
    if (st != QLA_OK) {
      delete c;
      return st;
    }
  }
  c->wide = !(theta_max <= kNarrowAngle && bmax <= kNarrowAngle);
  hipError_t e = hipSuccess;
  for (int i = 0; i < count && e == hipSuccess; ++i)
    for (int b = 0; b < 2 && e == hipSuccess; ++b) e = clear_dead(c, i, b);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(nullptr, e, "clearing the unused field triple");
  }
  int dev = 0, cus = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess || cus < 1) {
    delete c;
    return hip_fail(nullptr, e == hipSuccess ? hipErrorInvalidDevice : e, "querying the device");
  }
  c->cus = cus;
  c->launch = qla_launch{0, 0, 0, 0, 0, 0};
  st = plan_step(c);
  if (st != QLA_OK) {
    delete c;
    return st;
  }
  *out = c;
  return QLA_OK;
}

// This device's address of `scratch`, looked up on the first call on each
// device with that device current (every GPU holds its own copy).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch[kMaxDevices] = {};

qla_status device_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "querying the current device");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(QLA_EINVAL, "qla: device %d is beyond the %d devices this library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(nullptr, e, "looking up the static diagnostics buffer");
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return QLA_OK;
}

}  // namespace

extern "C" {

qla_status qla_workspace_size(const qla_params* p, size_t* bytes) {
  qla_status st = check_params(p);
  if (st != QLA_OK) return st;
  if (!bytes) return fail(QLA_EINVAL, "qla: null bytes pointer");
  const qla_instance one{*p, nullptr, nullptr, nullptr};
  *bytes = work_bytes(1, &one);
  return QLA_OK;
}

qla_status qla_batch_workspace_size(int32_t count, const qla_instance* inst, size_t* bytes) {
  qla_status st = check_batch(count, inst);
  if (st != QLA_OK) return st;
  if (!bytes) return fail(QLA_EINVAL, "qla: null bytes pointer");
  *bytes = work_bytes(count, inst);
  return QLA_OK;
}

qla_status qla_init(const qla_params* p, const float* d_n, float* d_q, float* d_q_pong,
                    void* d_work, void* hip_stream, qla_ctx** out) {
  if (!out) return fail(QLA_EINVAL, "qla: null output pointer");
  *out = nullptr;
  qla_status st = check_params(p);
  if (st != QLA_OK) return st;
  const qla_instance one{*p, d_n, d_q, d_q_pong};
  return init_common(1, &one, d_work, hip_stream, out);
}

qla_status qla_init_batch(int32_t count, const qla_instance* inst, void* d_work, void* hip_stream,
                          qla_ctx** out) {
  return init_common(count, inst, d_work, hip_stream, out);
}

qla_status qla_count(qla_ctx* ctx, int32_t* count) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!count) return fail(QLA_EINVAL, "qla: null count pointer");
  *count = ctx->count;
  return QLA_OK;
}

qla_status qla_step(qla_ctx* ctx, int64_t nsteps) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (nsteps < 0) return fail(QLA_EINVAL, "qla: negative step count");
  const int gsteps = ctx->planned.graph_steps;
  const int spp = ctx->planned.steps_per_pass;
  auto& graph = ctx->geo[spp - 1].graph;
  hipError_t e = hipSuccess;
  while (e == hipSuccess && nsteps > 0) {
    if (gsteps > 1 && nsteps >= gsteps) {
      if (!graph[ctx->cur]) {
        e = build_graph(ctx, ctx->cur);
        if (e != hipSuccess) return hip_fail(ctx, e, "building the step graph");
      }
      e = hipGraphLaunch(graph[ctx->cur], ctx->stream);
      nsteps -= gsteps;
      ctx->steps += gsteps;      // an even number of launches: the state stays in buffer cur
    } else {
      const int k = (spp == 2 && nsteps >= 2) ? 2 : 1;
      e = launch_one(ctx, k, ctx->cur);
      ctx->cur ^= 1;
      ctx->steps += k;
      nsteps -= k;
    }
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(ctx, e, "launching the step kernel");
  return QLA_OK;
}

qla_status qla_energy(qla_ctx* ctx, qla_diag* out) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!out) return fail(QLA_EINVAL, "qla: null diag pointer");
  double* parts = static_cast<double*>(ctx->work);
  for (int i = 0; i < ctx->count; ++i) {
    const qla_params& p = ctx->p[i];
    const int64_t plane = static_cast<int64_t>(p.nx) * p.ny;
    int blocks = static_cast<int>(std::min<int64_t>((plane + 255) / 256, kDiagBlocks));
    hipLaunchKernelGGL(qla_diag_kernel, dim3(blocks), dim3(256), 0, ctx->stream,
                       ctx->buf[ctx->cur][i], ctx->n[i], p.nx, p.ny, parts);
    hipLaunchKernelGGL(qla_diag_final, dim3(1), dim3(kWave), 0, ctx->stream, parts, blocks);
    double v[kDiagVals];
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(v, parts + static_cast<int64_t>(blocks) * kDiagVals, sizeof(v),
                         hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "computing diagnostics");
    qla_diag& o = out[i];
    o.step = ctx->steps;
    o.energy = v[0] / static_cast<double>(plane);
    o.divB_l2 = std::sqrt(v[1]);
    o.divB_max = v[2];
    o.B_max = std::sqrt(v[3]);
    o.B_l2 = std::sqrt(v[4]);
    o.divD_l2 = std::sqrt(v[5]);
    o.divD_max = v[6];
    o.D_max = std::sqrt(v[7]);
  }
  return QLA_OK;
}

qla_status qla_energy_noalloc(const qla_params* p, const float* d_n, const float* d_q, int64_t step,
                              qla_diag* d_out, void* hip_stream) {
  qla_status st = check_params(p);
  if (st != QLA_OK) return st;
  if (!d_n || !d_q || !d_out) return fail(QLA_EINVAL, "qla: null device pointer");
  if ((reinterpret_cast<uintptr_t>(d_out) & 7) != 0) return fail(QLA_EINVAL, "qla: d_out must be 8-byte aligned");
  const int64_t plane = static_cast<int64_t>(p->nx) * p->ny;
  const int blocks = static_cast<int>(std::min<int64_t>((plane + 255) / 256, kDiagBlocks));
  if (static_cast<int64_t>(blocks) * kDiagVals > kNoAllocDoubles)
    return fail(QLA_EINVAL, "qla: %d diagnostics blocks exceed the static buffer of %d", blocks,
                kNoAllocDoubles / kDiagVals);
  double* parts = nullptr;
  st = device_scratch(&parts);
  if (st != QLA_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(qla_diag_kernel, dim3(blocks), dim3(256), 0, s, d_q, d_n, p->nx, p->ny, parts);
  hipLaunchKernelGGL(qla_diag_finish, dim3(1), dim3(kWave), 0, s, parts, blocks, plane, step, d_out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(nullptr, e, "launching the diagnostics");
  return QLA_OK;
}

namespace {

// export lattice i (or every lattice when i < 0) to dst
qla_status fields_impl(qla_ctx* ctx, int i_only, float* dst, int32_t what, int32_t dst_is_host) {
  if (!dst) return fail(QLA_EINVAL, "qla: null destination");
  if (what != 0 && what != 1) return fail(QLA_EINVAL, "qla: what must be 0 (Q) or 1 (E, B)");
  hipError_t e = hipSuccess;
  float* o = dst;
  for (int i = 0; i < ctx->count && e == hipSuccess; ++i) {
    if (i_only >= 0 && i != i_only) continue;
    const qla_params& p = ctx->p[i];
    const int64_t plane = static_cast<int64_t>(p.nx) * p.ny;
    const size_t bytes = static_cast<size_t>(plane) * 6 * sizeof(float);
    const float* src = ctx->buf[ctx->cur][i];
    if (what == 1) {
      // (E, B) is written into the idle state buffer, then copied out
      float* tmp = ctx->buf[ctx->cur ^ 1][i];
      int blocks = static_cast<int>(std::min<int64_t>((plane + 255) / 256, 8192));
      hipLaunchKernelGGL(qla_fields_kernel, dim3(blocks), dim3(256), 0, ctx->stream, src, ctx->n[i],
                         plane, tmp);
      e = hipGetLastError();
      src = tmp;
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(o, src, bytes, dst_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                         ctx->stream);
    o += plane * 6;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "exporting fields");
  return QLA_OK;
}

}  // namespace

qla_status qla_fields(qla_ctx* ctx, float* dst, int32_t what, int32_t dst_is_host) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  return fields_impl(ctx, -1, dst, what, dst_is_host);
}

qla_status qla_fields_at(qla_ctx* ctx, int32_t index, float* dst, int32_t what, int32_t dst_is_host) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (index < 0 || index >= ctx->count) return fail(QLA_EINVAL, "qla: lattice index %d out of range", index);
  return fields_impl(ctx, index, dst, what, dst_is_host);
}

qla_status qla_load_at(qla_ctx* ctx, int32_t index, const float* src, int32_t src_is_host) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!src) return fail(QLA_EINVAL, "qla: null source");
  if (index < 0 || index >= ctx->count) return fail(QLA_EINVAL, "qla: lattice index %d out of range", index);
  const qla_params& p = ctx->p[index];
  const size_t bytes = static_cast<size_t>(p.nx) * p.ny * 6 * sizeof(float);
  hipError_t e = hipMemcpyAsync(ctx->buf[ctx->cur][index], src, bytes,
                                src_is_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = clear_dead(ctx, index, ctx->cur);
  if (e == hipSuccess && src_is_host) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "loading a state");
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
  if (req->seg_rows < 0 || req->seg_rows > (1 << 28) || req->waves_per_block < 0 ||
      req->waves_per_block > 4 || req->graph_steps < 0 || req->graph_steps > 4096 ||
      req->steps_per_pass < 0 || req->steps_per_pass > 2 || req->stream_loads < 0 || req->stream_loads > 2 ||
      req->vacuum_rows < 0 || req->vacuum_rows > 2)
    return fail(QLA_EINVAL, "qla: launch fields out of range");
  const qla_launch keep = ctx->launch;
  ctx->launch = *req;
  st = plan_step(ctx);
  if (st != QLA_OK && !ctx->poisoned) {
    ctx->launch = keep;
    plan_step(ctx);
  }
  return st;
}

qla_status qla_state(qla_ctx* ctx, float** d_current) { return qla_state_at(ctx, 0, d_current); }

qla_status qla_state_at(qla_ctx* ctx, int32_t index, float** d_current) {
  qla_status st = check_ctx(ctx);
  if (st != QLA_OK) return st;
  if (!d_current) return fail(QLA_EINVAL, "qla: null output pointer");
  if (index < 0 || index >= ctx->count) return fail(QLA_EINVAL, "qla: lattice index %d out of range", index);
  *d_current = ctx->buf[ctx->cur][index];
  return QLA_OK;
}

void qla_free(qla_ctx* ctx) {
  if (!ctx || ctx->magic != kMagic) return;
  ctx->magic = 0;
  drop_graphs(ctx);
  delete ctx;
}

const char* qla_last_error(void) { return g_last_error; }

}  // extern "C"
