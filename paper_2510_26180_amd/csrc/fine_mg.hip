// Multigrid-preconditioned fine propagator for grids too large to stay on one CU
// (Algorithm 2 step 1: J backward-Euler steps per (sample, slice), each solved for its
// increment in float32 and refined in float64 as in the CU-resident kernel).
//
// Each pass of the method over the unknowns is its own launch over a chunk of systems:
// grid (row bands of the level, systems), 256-thread work-groups, every wave walking its
// rows and every lane its columns, so the passes stream at full occupancy with few live
// registers.  Per-system sums and maxima are written as one partial per band and reduced
// by a per-system wave in a fixed order (deterministic), which also takes the CG and
// refinement decisions; the host reads one counter after the decisions that end a loop.
//
// Preconditioner: one V-cycle of the aggregation multigrid of mg.h (2x2 aggregates,
// Galerkin coarse operators, red-black Gauss-Seidel smoothing, coarse correction scaled by
// kMgScale), with the same sweep order.  The coarse operators depend only on the sample and
// are built once per call and shared by the sample's slices; level 0 reads the sample's
// scaled float32 couplings directly (its diagonal is 1).  Levels of at most 64 x 64 nodes
// run in one 1024-thread work-group per system with the level data in LDS.  Two fusions
// keep the level-0 passes to four per V-cycle at one sweep: the first sweep's red half
// (x = b / d from x = 0) is folded into its black half, and the prolongation x += s P e into
// the first post-smoothing half sweeps, each half adding s P e to the values it reads.
// On levels of even side the first sweep, the restriction and the level-0 product take
// node pairs per lane (float2 accesses), the direction update four nodes (float4).
#include <algorithm>
#include <string>

#include "common.h"
#include "fine_common.h"
#include "mg.h"
#include "reduce.h"

namespace kc {

namespace {

constexpr int kT = 256;            // threads of a streamed pass (4 waves)
constexpr int kOnChipMax = 64;     // levels of at most this many nodes per side run in LDS
constexpr int kOnChipT = 1024;     // threads of the on-chip work-group (one per CU, LDS-bound)
constexpr int kRing = 1024;        // counters of the host-visible decisions

// --------------------------------------------------------------- host-side level table
struct Layout {
  int n, L, lc;                    // level count; first level run in LDS (L if none)
  int sweeps;
  int m[kMgMaxLevels];
  int rb[kMgMaxLevels];            // rows per band
  int nb[kMgMaxLevels];            // bands
  int64_t coef_off[kMgMaxLevels];  // per-sample offset of level l >= 1: cw, cs, dg
  int64_t coef_per_sample;
  int64_t x_off[kMgMaxLevels];     // per-system offsets of x_l (l <= lc) and b_l (1 <= l <= lc)
  int64_t b_off[kMgMaxLevels];
  int64_t f32_per_sys;             // floats per system: X, R, P, Q, then the level vectors
  size_t lds_bytes;                // the on-chip levels
};

int rows_per_band(int m) {
  int rb = (2048 + m - 1) / m;
  rb = (rb + 3) / 4 * 4;
  return std::min(rb, (m + 3) / 4 * 4);
}

Layout make_layout(int n, int sweeps) {
  Layout y{};
  y.n = n;
  y.sweeps = sweeps >= 1 ? sweeps : kMgSweeps;
  int m = n, L = 1;
  y.m[0] = n;
  while (m > 2 && L < kMgMaxLevels) {
    m = (m + 1) / 2;
    y.m[L++] = m;
  }
  y.L = L;
  y.lc = L;
  for (int l = 1; l < L; ++l)
    if (y.m[l] <= kOnChipMax) {
      y.lc = l;
      break;
    }
  int64_t c = 0;
  for (int l = 1; l < L; ++l) {
    y.coef_off[l] = c;
    c += 3LL * y.m[l] * y.m[l];
  }
  y.coef_per_sample = std::max<int64_t>(c, 1);
  const int64_t Nx = (int64_t)n * n;
  int64_t v = 4 * Nx;
  for (int l = 0; l <= std::min(y.lc, L - 1); ++l) {
    y.x_off[l] = v;
    v += (int64_t)y.m[l] * y.m[l];
    if (l >= 1) {
      y.b_off[l] = v;
      v += (int64_t)y.m[l] * y.m[l];
    }
  }
  y.f32_per_sys = v;
  for (int l = 0; l < L; ++l) {
    y.rb[l] = rows_per_band(y.m[l]);
    y.nb[l] = (y.m[l] + y.rb[l] - 1) / y.rb[l];
  }
  size_t lds = 0;
  for (int l = y.lc; l < L; ++l) lds += 5 * sizeof(float) * (size_t)y.m[l] * y.m[l];
  y.lds_bytes = lds;
  return y;
}

// --------------------------------------------------------------- device-side pieces
// per-system state: float64 refinement and float32 CG scalars, decisions, counters
struct Sys {
  double rmax, sig, wref, target;
  float r0, stop, rr, rz, al, be;
  int alive, refine, incg;         // a system of the chunk; needs a float32 pass; inside CG
  int it, pass, tot_it, tot_pass, max_it, missed, fail;
};

// One level of the V-cycle as the streamed kernels see it.  Level 0: cw = sf (row stride
// n + 1), cs = sf + n (n + 1) (row stride n), dg = 1; levels >= 1: per-sample arrays.
struct Lv {
  int m, rb, l0;
  const float* cw;   // + sample * cstride
  const float* cs;
  const float* dg;
  int64_t cstride;
  float* x;          // + local system * vstride
  const float* b;
  int64_t vstride;
};

struct LvS {   // one system's view of a level
  int m, cwr, l0;
  const float *cw, *cs, *dg;
  float* x;
  const float* b;
  __device__ __forceinline__ float d(int p) const { return l0 ? 1.f : dg[p]; }
  __device__ __forceinline__ float cW(int i, int j) const { return cw[j * cwr + i]; }
  __device__ __forceinline__ float cS(int i, int j) const { return cs[j * m + i]; }
};

__device__ __forceinline__ LvS view(const Lv& v, int64_t sample, int64_t ls) {
  LvS s;
  s.m = v.m;
  s.l0 = v.l0;
  s.cwr = v.l0 ? v.m + 1 : v.m;
  s.cw = v.cw + sample * v.cstride;
  s.cs = v.cs + sample * v.cstride;
  s.dg = v.l0 ? nullptr : v.dg + sample * v.cstride;
  s.x = v.x + ls * v.vstride;
  s.b = v.b + ls * v.vstride;
  return s;
}

// the rows of band blockIdx.x: wave w takes rows j0 + w, j0 + w + 4, ...; lanes columns
template <class F>
__device__ __forceinline__ void band_nodes(int m, int rb, F&& f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j0 = blockIdx.x * rb, j1 = min(m, j0 + rb);
  for (int j = j0 + w; j < j1; j += 4) {
    const int row = j * m;
    for (int i = lane; i < m; i += 64) f(row + i, i, j);
  }
}
template <class F>
__device__ __forceinline__ void band_colour(int m, int rb, int col, F&& f) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j0 = blockIdx.x * rb, j1 = min(m, j0 + rb);
  for (int j = j0 + w; j < j1; j += 4) {
    const int row = j * m;
    for (int i = 2 * lane + ((col + j) & 1); i < m; i += 128) f(row + i, i, j);
  }
}

// work-group sums / maxima of K values; thread 0 stores them as the band's partials
template <int K>
__device__ __forceinline__ void band_partials(double (&v)[K], const bool (&is_max)[K], double* part) {
  __shared__ double sl[K][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = is_max[k] ? wave_nanmax(v[k]) : wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sl[k][w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double a = sl[k][0];
      for (int q = 1; q < 4; ++q) a = is_max[k] ? nanmax(a, sl[k][q]) : a + sl[k][q];
      part[k] = a;
    }
}

// (L x)_p of a level with x read through X(q, i, j)
template <class XF>
__device__ __forceinline__ float apply_at(const LvS& v, int p, int i, int j, XF X) {
  float acc = v.d(p) * X(p, i, j);
  if (i > 0) acc = fmaf(-v.cW(i, j), X(p - 1, i - 1, j), acc);
  if (i < v.m - 1) acc = fmaf(-v.cW(i + 1, j), X(p + 1, i + 1, j), acc);
  if (j > 0) acc = fmaf(-v.cS(i, j), X(p - v.m, i, j - 1), acc);
  if (j < v.m - 1) acc = fmaf(-v.cS(i, j + 1), X(p + v.m, i, j + 1), acc);
  return acc;
}

struct Chunk {   // what every streamed kernel of a chunk needs to find its system
  int64_t sys0;  // first global system of the chunk
  int N;         // slices per sample
  Sys* st;
};

// the system of a streamed kernel is blockIdx.y (the grid is (bands, systems of the chunk))
__device__ __forceinline__ bool pick(const Chunk& c, int which, int64_t& sample, int64_t& ls) {
  ls = blockIdx.y;
  const Sys& s = c.st[ls];
  const int on = which == 0 ? s.alive : which == 1 ? s.refine : s.incg;
  sample = (c.sys0 + ls) / c.N;
  return on != 0;
}
constexpr int kAlive = 0, kRefine = 1, kInCg = 2;

// ---- V-cycle passes (systems inside CG)
// first sweep from x = 0: red x = b / d; black x = (b + sum c_q b_q / d_q) / d
__global__ __launch_bounds__(kT) void k_first_sweep(Lv lv, Chunk c) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const LvS v = view(lv, sample, ls);
  band_nodes(v.m, lv.rb, [&](int p, int i, int j) {
    float xv;
    if (((i + j) & 1) == 0) {
      xv = v.b[p] / v.d(p);
    } else {
      float acc = v.b[p];
      if (i > 0) acc = fmaf(v.cW(i, j), v.b[p - 1] / v.d(p - 1), acc);
      if (i < v.m - 1) acc = fmaf(v.cW(i + 1, j), v.b[p + 1] / v.d(p + 1), acc);
      if (j > 0) acc = fmaf(v.cS(i, j), v.b[p - v.m] / v.d(p - v.m), acc);
      if (j < v.m - 1) acc = fmaf(v.cS(i, j + 1), v.b[p + v.m] / v.d(p + v.m), acc);
      xv = acc / v.d(p);
    }
    v.x[p] = xv;
  });
}

// The same first sweep on a level of even side with 8-byte aligned vectors: each lane takes
// a red and a black node of its row (columns 2k, 2k + 1), reads the pair's b and d as one
// float2 and writes both x as one; the black node's value is formed in the order above, so
// both kernels give the same bits.
__global__ __launch_bounds__(kT) void k_first_sweep_pairs(Lv lv, Chunk c) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const LvS v = view(lv, sample, ls);
  const int m = v.m;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j0 = blockIdx.x * lv.rb, j1 = min(m, j0 + lv.rb);
  for (int j = j0 + w; j < j1; j += 4) {
    const int row = j * m, odd = j & 1;   // red at column 2k + odd, black at 2k + 1 - odd
    for (int i = 2 * lane; i < m; i += 128) {
      const int p = row + i;
      const float2 b2 = *reinterpret_cast<const float2*>(v.b + p);
      const float2 d2 = v.l0 ? make_float2(1.f, 1.f) : *reinterpret_cast<const float2*>(v.dg + p);
      const int ib = i + 1 - odd, pb = row + ib;
      const float bb = odd ? b2.x : b2.y, db = odd ? d2.x : d2.y;
      const float br = odd ? b2.y : b2.x, dr = odd ? d2.y : d2.x;
      float acc = bb;
      if (odd) {   // west neighbour outside the pair, east one the pair's red node
        if (ib > 0) acc = fmaf(v.cW(ib, j), v.b[pb - 1] / v.d(pb - 1), acc);
        acc = fmaf(v.cW(ib + 1, j), br / dr, acc);
      } else {
        acc = fmaf(v.cW(ib, j), br / dr, acc);
        if (ib < m - 1) acc = fmaf(v.cW(ib + 1, j), v.b[pb + 1] / v.d(pb + 1), acc);
      }
      if (j > 0) acc = fmaf(v.cS(ib, j), v.b[pb - m] / v.d(pb - m), acc);
      if (j < m - 1) acc = fmaf(v.cS(ib, j + 1), v.b[pb + m] / v.d(pb + m), acc);
      const float xr = br / dr, xb = acc / db;
      *reinterpret_cast<float2*>(v.x + p) = odd ? make_float2(xb, xr) : make_float2(xr, xb);
    }
  }
}

// half sweep of colour col: x_p += (b_p - (L x)_p) / d_p.  The prolongation x += s P e (e the
// coarse level's x) is folded into the first post-smoothing sweep: its black half (emode 1)
// reads every value as x + s e(parent), the other colour unchanged in memory; its red half
// (emode 2) adds s e to the node's own old value only, its black neighbours being final.
// With part, the band's sum of b_p x_p over the updated nodes goes to part[slot] (the r.z
// of the last sweep at level 0).
__global__ __launch_bounds__(kT) void k_half(Lv lv, Chunk c, int col, const float* __restrict__ ec, int mc,
                                             int64_t evstride, int emode, double* __restrict__ part, int nb,
                                             int slot) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const LvS v = view(lv, sample, ls);
  const float* e = ec ? ec + ls * evstride : nullptr;
  double dot = 0.0;
  band_colour(v.m, lv.rb, col, [&](int p, int i, int j) {
    // neighbours: prolonged on the fly only in the black half (emode 1)
    auto nbr = [&](int q, int qi, int qj) {
      const float xq = v.x[q];
      return emode == 1 ? fmaf(kMgScale, e[(qj >> 1) * mc + (qi >> 1)], xq) : xq;
    };
    const float own = emode ? fmaf(kMgScale, e[(j >> 1) * mc + (i >> 1)], v.x[p]) : v.x[p];
    const float dp = v.d(p);
    float acc = dp * own;
    if (i > 0) acc = fmaf(-v.cW(i, j), nbr(p - 1, i - 1, j), acc);
    if (i < v.m - 1) acc = fmaf(-v.cW(i + 1, j), nbr(p + 1, i + 1, j), acc);
    if (j > 0) acc = fmaf(-v.cS(i, j), nbr(p - v.m, i, j - 1), acc);
    if (j < v.m - 1) acc = fmaf(-v.cS(i, j + 1), nbr(p + v.m, i, j + 1), acc);
    const float bp = v.b[p];
    const float xn = own + (bp - acc) / dp;
    v.x[p] = xn;
    dot += (double)(bp * xn);
  });
  if (part) {
    double d1[1] = {dot};
    const bool mx[1] = {false};
    band_partials<1>(d1, mx, part + ((ls * nb + blockIdx.x) * 4 + slot));
  }
}

// restriction of the residual: b_{l+1}[I, J] = sum over the 2x2 block of (b - L x)
__global__ __launch_bounds__(kT) void k_restrict(Lv lv, Lv cv, Chunk c) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const LvS v = view(lv, sample, ls);
  float* bc = const_cast<float*>(cv.b) + ls * cv.vstride;
  const int m = v.m;
  band_nodes(cv.m, cv.rb, [&](int P, int I, int J) {
    float sum = 0.f;
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) {
        const int i = 2 * I + di, j = 2 * J + dj;
        if (i < m && j < m) {
          const int p = j * m + i;
          sum += v.b[p] - apply_at(v, p, i, j, [&](int q, int, int) { return v.x[q]; });
        }
      }
    bc[P] = sum;
  });
}

// The same restriction from a level of even side with 8-byte aligned vectors: the 2x2 block
// and the rows above and below it are read as float2 (the columns beside it as single
// floats), and the block is summed in the order above, so both kernels give the same bits.
__global__ __launch_bounds__(kT) void k_restrict_pairs(Lv lv, Lv cv, Chunk c) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const LvS v = view(lv, sample, ls);
  float* bc = const_cast<float*>(cv.b) + ls * cv.vstride;
  const int m = v.m;
  auto ld2 = [](const float* q) { return *reinterpret_cast<const float2*>(q); };
  band_nodes(cv.m, cv.rb, [&](int P, int I, int J) {
    const int i0 = 2 * I, j0 = 2 * J;
    const int p0 = j0 * m + i0, p1 = p0 + m;
    const bool hw = i0 > 0, he = i0 + 2 < m, hs = j0 > 0, hn = j0 + 2 < m;
    const float2 zero = make_float2(0.f, 0.f);
    const float2 x0 = ld2(v.x + p0), x1 = ld2(v.x + p1);
    const float2 xs = hs ? ld2(v.x + p0 - m) : zero, xn = hn ? ld2(v.x + p1 + m) : zero;
    const float xw0 = hw ? v.x[p0 - 1] : 0.f, xw1 = hw ? v.x[p1 - 1] : 0.f;
    const float xe0 = he ? v.x[p0 + 2] : 0.f, xe1 = he ? v.x[p1 + 2] : 0.f;
    const float2 b0 = ld2(v.b + p0), b1 = ld2(v.b + p1);
    const float2 d0 = v.l0 ? make_float2(1.f, 1.f) : ld2(v.dg + p0);
    const float2 d1 = v.l0 ? make_float2(1.f, 1.f) : ld2(v.dg + p1);
    // couplings: west / middle / east of each block row, south / middle / north of each column
    const float ww0 = hw ? v.cW(i0, j0) : 0.f, wm0 = v.cW(i0 + 1, j0), we0 = he ? v.cW(i0 + 2, j0) : 0.f;
    const float ww1 = hw ? v.cW(i0, j0 + 1) : 0.f, wm1 = v.cW(i0 + 1, j0 + 1),
                we1 = he ? v.cW(i0 + 2, j0 + 1) : 0.f;
    const float2 ss = hs ? ld2(v.cs + j0 * m + i0) : zero, sm = ld2(v.cs + (j0 + 1) * m + i0),
                 sn = hn ? ld2(v.cs + (j0 + 2) * m + i0) : zero;
    float sum = 0.f, acc;
    acc = d0.x * x0.x;   // (i0, j0)
    if (hw) acc = fmaf(-ww0, xw0, acc);
    acc = fmaf(-wm0, x0.y, acc);
    if (hs) acc = fmaf(-ss.x, xs.x, acc);
    acc = fmaf(-sm.x, x1.x, acc);
    sum += b0.x - acc;
    acc = d0.y * x0.y;   // (i0 + 1, j0)
    acc = fmaf(-wm0, x0.x, acc);
    if (he) acc = fmaf(-we0, xe0, acc);
    if (hs) acc = fmaf(-ss.y, xs.y, acc);
    acc = fmaf(-sm.y, x1.y, acc);
    sum += b0.y - acc;
    acc = d1.x * x1.x;   // (i0, j0 + 1)
    if (hw) acc = fmaf(-ww1, xw1, acc);
    acc = fmaf(-wm1, x1.y, acc);
    acc = fmaf(-sm.x, x0.x, acc);
    if (hn) acc = fmaf(-sn.x, xn.x, acc);
    sum += b1.x - acc;
    acc = d1.y * x1.y;   // (i0 + 1, j0 + 1)
    acc = fmaf(-wm1, x1.x, acc);
    if (he) acc = fmaf(-we1, xe1, acc);
    acc = fmaf(-sm.y, x0.y, acc);
    if (hn) acc = fmaf(-sn.y, xn.y, acc);
    sum += b1.y - acc;
    bc[P] = sum;
  });
}

// the paired kernels' condition: even side, every vector and coupling array 8-byte aligned
// with even strides
bool pairs_ok(const Lv& v) {
  const auto al = [](const void* q) { return (reinterpret_cast<uintptr_t>(q) & 7) == 0; };
  return v.m % 2 == 0 && v.vstride % 2 == 0 && v.cstride % 2 == 0 && al(v.x) && al(v.b) && al(v.cs) &&
         (v.l0 || al(v.dg));
}

// The levels lc..L-1 of one system in LDS: b of level lc in, x of level lc out, with the
// V-cycle's sweep order (down: first sweep, restriction; coarsest: the transposed sweeps;
// up: prolongation and sweeps).
struct OnChip {
  int lc, L, sweeps;
  int m[kMgMaxLevels];
  int64_t coef_off[kMgMaxLevels];
  int lds_off[kMgMaxLevels];   // floats: cw, cs, d, x, b of level l, m^2 each, from here
};

__device__ __forceinline__ void lds_half(int m, const float* cw, const float* cs, const float* dg, const float* b,
                                         float* x, int col) {
  for (int q = threadIdx.x; q < m * ((m + 1) / 2); q += blockDim.x) {
    const int hw = (m + 1) / 2;
    const int j = q / hw;
    const int i = 2 * (q - j * hw) + ((col + j) & 1);
    if (i < m) {
      const int p = j * m + i;
      float acc = dg[p] * x[p];
      if (i > 0) acc = fmaf(-cw[p], x[p - 1], acc);
      if (i < m - 1) acc = fmaf(-cw[p + 1], x[p + 1], acc);
      if (j > 0) acc = fmaf(-cs[p], x[p - m], acc);
      if (j < m - 1) acc = fmaf(-cs[p + m], x[p + m], acc);
      x[p] += (b[p] - acc) / dg[p];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kOnChipT) void k_onchip(OnChip oc, const float* __restrict__ coef, int64_t cps,
                                               const float* __restrict__ bin, float* __restrict__ xout,
                                               int64_t vstride, Chunk c) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  extern __shared__ float lds[];
  // the level arrays, found from the per-level offsets (wave-uniform, no per-thread table)
  auto arr = [&](int l, int k) { return lds + oc.lds_off[l] + k * oc.m[l] * oc.m[l]; };
  auto CW = [&](int l) { return arr(l, 0); };
  auto CS = [&](int l) { return arr(l, 1); };
  auto DG = [&](int l) { return arr(l, 2); };
  auto XL = [&](int l) { return arr(l, 3); };
  auto BL = [&](int l) { return arr(l, 4); };
  {
    for (int l = oc.lc; l < oc.L; ++l) {
      const int mm = oc.m[l] * oc.m[l];
      const float* src = coef + sample * cps + oc.coef_off[l];
      for (int p = threadIdx.x; p < mm; p += blockDim.x) {
        CW(l)[p] = src[p];
        CS(l)[p] = src[mm + p];
        DG(l)[p] = src[2 * mm + p];
      }
    }
    const int m0 = oc.m[oc.lc];
    for (int p = threadIdx.x; p < m0 * m0; p += blockDim.x) BL(oc.lc)[p] = bin[ls * vstride + p];
  }
  __syncthreads();
  for (int l = oc.lc; l < oc.L; ++l) {
    const int m = oc.m[l];
    for (int p = threadIdx.x; p < m * m; p += blockDim.x) {
      const int j = p / m, i = p - j * m;
      XL(l)[p] = ((i + j) & 1) == 0 ? BL(l)[p] / DG(l)[p] : 0.f;
    }
    __syncthreads();
    lds_half(m, CW(l), CS(l), DG(l), BL(l), XL(l), 1);
    for (int s = 1; s < oc.sweeps; ++s) {
      lds_half(m, CW(l), CS(l), DG(l), BL(l), XL(l), 0);
      lds_half(m, CW(l), CS(l), DG(l), BL(l), XL(l), 1);
    }
    if (l + 1 < oc.L) {
      const int mc = oc.m[l + 1];
      for (int P = threadIdx.x; P < mc * mc; P += blockDim.x) {
        const int J = P / mc, I = P - J * mc;
        float sum = 0.f;
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) {
            const int i = 2 * I + di, j = 2 * J + dj;
            if (i < m && j < m) {
              const int p = j * m + i;
              float acc = DG(l)[p] * XL(l)[p];
              if (i > 0) acc = fmaf(-CW(l)[p], XL(l)[p - 1], acc);
              if (i < m - 1) acc = fmaf(-CW(l)[p + 1], XL(l)[p + 1], acc);
              if (j > 0) acc = fmaf(-CS(l)[p], XL(l)[p - m], acc);
              if (j < m - 1) acc = fmaf(-CS(l)[p + m], XL(l)[p + m], acc);
              sum += BL(l)[p] - acc;
            }
          }
        BL(l + 1)[P] = sum;
      }
      __syncthreads();
    } else {
      for (int s = 0; s < oc.sweeps; ++s) {
        lds_half(m, CW(l), CS(l), DG(l), BL(l), XL(l), 1);
        lds_half(m, CW(l), CS(l), DG(l), BL(l), XL(l), 0);
      }
    }
  }
  for (int l = oc.L - 2; l >= oc.lc; --l) {
    const int m = oc.m[l], mc = oc.m[l + 1];
    for (int p = threadIdx.x; p < m * m; p += blockDim.x) {
      const int j = p / m, i = p - j * m;
      XL(l)[p] = fmaf(kMgScale, XL(l + 1)[(j >> 1) * mc + (i >> 1)], XL(l)[p]);
    }
    __syncthreads();
    for (int s = 0; s < oc.sweeps; ++s) {
      lds_half(m, CW(l), CS(l), DG(l), BL(l), XL(l), 1);
      lds_half(m, CW(l), CS(l), DG(l), BL(l), XL(l), 0);
    }
  }
  const int m0 = oc.m[oc.lc];
  for (int p = threadIdx.x; p < m0 * m0; p += blockDim.x) xout[ls * vstride + p] = XL(oc.lc)[p];
}

// Galerkin coarse operator of level l from level l - 1 (level 0 from the scaled couplings
// sf, diagonal 1), per sample
__global__ __launch_bounds__(kT) void k_coarsen(Lv fv, float* __restrict__ coef, int64_t cps, int64_t off, int mc,
                                                int rbc, const uint8_t* __restrict__ need) {
  const int64_t sample = blockIdx.y;
  if (!need[sample]) return;
  const LvS f = view(fv, sample, 0);
  float* cw = coef + sample * cps + off;
  float* cs = cw + (int64_t)mc * mc;
  float* dg = cs + (int64_t)mc * mc;
  const int mf = f.m;
  band_nodes(mc, rbc, [&](int Pn, int I, int J) {
    const int i0 = 2 * I, j0 = 2 * J;
    const bool two_i = i0 + 1 < mf, two_j = j0 + 1 < mf;
    float d = 0.f, cwc = 0.f, csc = 0.f, inner = 0.f;
    for (int dj = 0; dj < (two_j ? 2 : 1); ++dj)
      for (int di = 0; di < (two_i ? 2 : 1); ++di) {
        const int i = i0 + di, j = j0 + dj, p = j * mf + i;
        d += f.d(p);
        if (di == 1) inner += f.cW(i, j);
        if (dj == 1) inner += f.cS(i, j);
        if (di == 0 && I > 0) cwc += f.cW(i, j);
        if (dj == 0 && J > 0) csc += f.cS(i, j);
      }
    dg[Pn] = d - 2.f * inner;
    cw[Pn] = cwc;
    cs[Pn] = csc;
  });
}

// ---- CG passes at level 0 (systems inside CG); part slot 0
__global__ __launch_bounds__(kT) void k_matvec(Lv l0, const float* __restrict__ P, float* __restrict__ Q,
                                               int64_t vs, Chunk c, double* __restrict__ part, int nb) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const LvS v = view(l0, sample, ls);
  const float* p_ = P + ls * vs;
  float* q_ = Q + ls * vs;
  double acc = 0.0;
  band_nodes(v.m, l0.rb, [&](int p, int i, int j) {
    const float qv = apply_at(v, p, i, j, [&](int q, int, int) { return p_[q]; });
    q_[p] = qv;
    acc += (double)(p_[p] * qv);
  });
  double d1[1] = {acc};
  const bool mx[1] = {false};
  band_partials<1>(d1, mx, part + (ls * nb + blockIdx.x) * 4);
}

// The same product on a level of even side with 8-byte aligned vectors: each lane takes two
// neighbouring nodes of its row (columns 2k, 2k + 1), reading P's rows as float2 and writing
// both Q values as one; each node is formed in the order of apply_at.
__global__ __launch_bounds__(kT) void k_matvec_pairs(Lv l0, const float* __restrict__ P, float* __restrict__ Q,
                                                     int64_t vs, Chunk c, double* __restrict__ part, int nb) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const LvS v = view(l0, sample, ls);
  const float* p_ = P + ls * vs;
  float* q_ = Q + ls * vs;
  const int m = v.m;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j0 = blockIdx.x * l0.rb, j1 = min(m, j0 + l0.rb);
  auto ld2 = [](const float* q) { return *reinterpret_cast<const float2*>(q); };
  const float2 zero = make_float2(0.f, 0.f);
  double acc = 0.0;
  for (int j = j0 + w; j < j1; j += 4) {
    const int row = j * m;
    const bool hs = j > 0, hn = j < m - 1;
    for (int i = 2 * lane; i < m; i += 128) {
      const int p = row + i;
      const bool hw = i > 0, he = i + 2 < m;
      const float2 x = ld2(p_ + p);
      const float2 xs = hs ? ld2(p_ + p - m) : zero, xn = hn ? ld2(p_ + p + m) : zero;
      const float xw = hw ? p_[p - 1] : 0.f, xe = he ? p_[p + 2] : 0.f;
      const float2 d2 = v.l0 ? make_float2(1.f, 1.f) : ld2(v.dg + p);
      const float cw0 = hw ? v.cW(i, j) : 0.f, cw1 = v.cW(i + 1, j), cw2 = he ? v.cW(i + 2, j) : 0.f;
      const float2 cs0 = hs ? ld2(v.cs + row + i) : zero, cs1 = hn ? ld2(v.cs + row + m + i) : zero;
      float a0 = d2.x * x.x;
      if (hw) a0 = fmaf(-cw0, xw, a0);
      a0 = fmaf(-cw1, x.y, a0);
      if (hs) a0 = fmaf(-cs0.x, xs.x, a0);
      if (hn) a0 = fmaf(-cs1.x, xn.x, a0);
      float a1 = d2.y * x.y;
      a1 = fmaf(-cw1, x.x, a1);
      if (he) a1 = fmaf(-cw2, xe, a1);
      if (hs) a1 = fmaf(-cs0.y, xs.y, a1);
      if (hn) a1 = fmaf(-cs1.y, xn.y, a1);
      *reinterpret_cast<float2*>(q_ + p) = make_float2(a0, a1);
      acc += (double)(x.x * a0);
      acc += (double)(x.y * a1);
    }
  }
  double d1[1] = {acc};
  const bool mx[1] = {false};
  band_partials<1>(d1, mx, part + (ls * nb + blockIdx.x) * 4);
}
__global__ __launch_bounds__(kT) void k_xr(int m, int rb, float* __restrict__ X, float* __restrict__ R,
                                           const float* __restrict__ P, const float* __restrict__ Q, int64_t vs,
                                           Chunk c, double* __restrict__ part, int nb) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const float al = c.st[ls].al;
  float* x = X + ls * vs;
  float* r = R + ls * vs;
  const float* p_ = P + ls * vs;
  const float* q_ = Q + ls * vs;
  double acc = 0.0;
  band_nodes(m, rb, [&](int p, int, int) {
    x[p] = fmaf(al, p_[p], x[p]);
    const float rv = fmaf(-al, q_[p], r[p]);
    r[p] = rv;
    acc += (double)(rv * rv);
  });
  double d1[1] = {acc};
  const bool mx[1] = {false};
  band_partials<1>(d1, mx, part + (ls * nb + blockIdx.x) * 4);
}

// P = Z + beta P (beta = 0 on the first iteration of a pass)
__global__ __launch_bounds__(kT) void k_pupd(int m, int rb, float* __restrict__ P, const float* __restrict__ Z,
                                             int64_t vs, Chunk c, int first) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const float be = first ? 0.f : c.st[ls].be;
  float* p_ = P + ls * vs;
  const float* z = Z + ls * vs;
  band_nodes(m, rb, [&](int p, int, int) { p_[p] = first ? z[p] : fmaf(be, p_[p], z[p]); });
}

// The same update as float4 over the band's rows taken as one range (side a multiple of 4,
// 16-byte aligned vectors and stride): elementwise, so both kernels give the same bits.
__global__ __launch_bounds__(kT) void k_pupd4(int m, int rb, float* __restrict__ P, const float* __restrict__ Z,
                                              int64_t vs, Chunk c, int first) {
  int64_t sample, ls;
  if (!pick(c, kInCg, sample, ls)) return;
  const float be = first ? 0.f : c.st[ls].be;
  float4* p4 = reinterpret_cast<float4*>(P + ls * vs);
  const float4* z4 = reinterpret_cast<const float4*>(Z + ls * vs);
  const int a = blockIdx.x * rb * (m / 4), b = min(m, (int)(blockIdx.x + 1) * rb) * (m / 4);
  for (int q = a + threadIdx.x; q < b; q += kT) {
    const float4 z = z4[q];
    if (first) {
      p4[q] = z;
    } else {
      const float4 pv = p4[q];
      p4[q] = make_float4(fmaf(be, pv.x, z.x), fmaf(be, pv.y, z.y), fmaf(be, pv.z, z.z), fmaf(be, pv.w, z.w));
    }
  }
}

// ---- float64 refinement passes
struct F64 {
  const double* a;     // faces [M][Fc]
  const double* dinv;  // [M][Nx]
  double c, tauf;
  double* out;         // states (the system's row is w)
  double* res;         // [S][Nx]
  double* inc;         // [S][2][Nx]: increment, previous increment
  int n;
  int rb;
};

__global__ __launch_bounds__(kT) void k_setup(F64 f, StartRef sr, Chunk c) {
  int64_t sample, ls;
  if (!pick(c, kAlive, sample, ls)) return;
  const int64_t Nx = (int64_t)f.n * f.n;
  const int s = (int)((c.sys0 + ls) % c.N);
  const double* src = sr.row(sample, s, c.N, Nx);
  double* w = f.out + (c.sys0 + ls) * Nx;
  double* inc = f.inc + ls * 2 * Nx;
  band_nodes(f.n, f.rb, [&](int p, int, int) {
    w[p] = src ? src[p] : 0.0;
    inc[p] = 0.0;
  });
}

// start of step j >= 1: w_j = w_{j-1} + inc, the new increment g = 2 inc - inc_prev (inc at
// the second step of a slice), inc_prev = inc
__global__ __launch_bounds__(kT) void k_step_start(F64 f, Chunk c, int step) {
  int64_t sample, ls;
  if (!pick(c, kAlive, sample, ls)) return;
  const int64_t Nx = (int64_t)f.n * f.n;
  double* w = f.out + (c.sys0 + ls) * Nx;
  double* inc = f.inc + ls * 2 * Nx;
  double* incp = inc + Nx;
  band_nodes(f.n, f.rb, [&](int p, int, int) {
    const double i1 = inc[p];
    const double g = step > 1 ? 2.0 * i1 - incp[p] : i1;
    w[p] += g;
    incp[p] = i1;
    inc[p] = g;
  });
}

// float64 residual tau f - tau A (w + inc) - inc ... with w already holding w_j + inc:
// res = tau f - c h^2 A w - inc; partials max |res|, max |w|, max d^{-1/2} |res|
__global__ __launch_bounds__(kT) void k_residual(F64 f, Chunk c, double* __restrict__ part, int nb) {
  int64_t sample, ls;
  if (!pick(c, kAlive, sample, ls)) return;
  const int n = f.n;
  const int64_t Nx = (int64_t)n * n;
  const Grid2 g{n, (int64_t)n * (n + 1)};
  const double* af = f.a + sample * 2 * g.nx;
  const double* dv = f.dinv + sample * Nx;
  const double* w = f.out + (c.sys0 + ls) * Nx;
  const double* inc = f.inc + ls * 2 * Nx;
  double* res = f.res + ls * Nx;
  double acc[3] = {0.0, 0.0, 0.0};
  band_nodes(n, f.rb, [&](int p, int i, int j) {
    const double rv = f.tauf - f.c * stencil64(af, w, g, i, j) - inc[p];
    res[p] = rv;
    acc[0] = nanmax(acc[0], fabs(rv));
    acc[1] = nanmax(acc[1], fabs(w[p]));
    acc[2] = nanmax(acc[2], dv[p] * fabs(rv));
  });
  const bool mx[3] = {true, true, true};
  band_partials<3>(acc, mx, part + (ls * nb + blockIdx.x) * 4);
}

// float32 right-hand side of a pass: R = d^{-1/2} res / sig, X = 0; partial sum R.R
__global__ __launch_bounds__(kT) void k_rhs(F64 f, float* __restrict__ X, float* __restrict__ R, int64_t vs, Chunk c,
                                            double* __restrict__ part, int nb) {
  int64_t sample, ls;
  if (!pick(c, kRefine, sample, ls)) return;
  const int64_t Nx = (int64_t)f.n * f.n;
  const double* dv = f.dinv + sample * Nx;
  const double* res = f.res + ls * Nx;
  const double isig = 1.0 / c.st[ls].sig;
  float* x = X + ls * vs;
  float* r = R + ls * vs;
  double acc = 0.0;
  band_nodes(f.n, f.rb, [&](int p, int, int) {
    const float v = (float)(isig * dv[p] * res[p]);
    r[p] = v;
    x[p] = 0.f;
    acc += (double)(v * v);
  });
  double d1[1] = {acc};
  const bool mx[1] = {false};
  band_partials<1>(d1, mx, part + (ls * nb + blockIdx.x) * 4);
}

// float64 update with the correction e = sig d^{-1/2} X: res -= (I + tau A) e, w += e,
// inc += e; partials max |res|, max d^{-1/2} |res|, max |w|
__global__ __launch_bounds__(kT) void k_update64(F64 f, const float* __restrict__ X, int64_t vs, Chunk c,
                                                 double* __restrict__ part, int nb) {
  int64_t sample, ls;
  if (!pick(c, kRefine, sample, ls)) return;
  const int n = f.n;
  const int64_t Nx = (int64_t)n * n;
  const Grid2 g{n, (int64_t)n * (n + 1)};
  const double* af = f.a + sample * 2 * g.nx;
  const double* dv = f.dinv + sample * Nx;
  double* w = f.out + (c.sys0 + ls) * Nx;
  double* inc = f.inc + ls * 2 * Nx;
  double* res = f.res + ls * Nx;
  const float* x = X + ls * vs;
  const double sig = c.st[ls].sig;
  double acc[3] = {0.0, 0.0, 0.0};
  band_nodes(n, f.rb, [&](int p, int i, int j) {
    const double ep = sig * dv[p] * (double)x[p];
    const double ew = i > 0 ? sig * dv[p - 1] * (double)x[p - 1] : 0.0;
    const double ee = i < n - 1 ? sig * dv[p + 1] * (double)x[p + 1] : 0.0;
    const double es = j > 0 ? sig * dv[p - n] * (double)x[p - n] : 0.0;
    const double en = j < n - 1 ? sig * dv[p + n] * (double)x[p + n] : 0.0;
    const double Me = ep + f.c * (af[g.fW(i, j)] * (ep - ew) + af[g.fE(i, j)] * (ep - ee) +
                                  af[g.fS(i, j)] * (ep - es) + af[g.fN(i, j)] * (ep - en));
    const double rv = res[p] - Me;
    res[p] = rv;
    const double wv = w[p] + ep;
    w[p] = wv;
    inc[p] += ep;
    acc[0] = nanmax(acc[0], fabs(rv));
    acc[1] = nanmax(acc[1], dv[p] * fabs(rv));
    acc[2] = nanmax(acc[2], fabs(wv));
  });
  const bool mx[3] = {true, true, true};
  band_partials<3>(acc, mx, part + (ls * nb + blockIdx.x) * 4);
}

// ---- per-system decisions: one wave per system reduces its band partials in a fixed order
enum Phase { PH_RESID, PH_R0, PH_RZ, PH_ALPHA, PH_RR, PH_BETA, PH_UPD, PH_END };

struct Ctl {
  double tol, tauf;
  const double* dmax;   // [M] max diagonal of I + tau A per sample
  float pcg_rtol;
  int cap;
  int* ring;            // host-visible counters
  int slot;
};

__global__ __launch_bounds__(64) void k_decide(Chunk c, const double* __restrict__ part, int nb, int phase, Ctl k) {
  const int64_t ls = blockIdx.x;
  Sys& s = c.st[ls];
  const int lane = threadIdx.x;
  const int64_t sample = (c.sys0 + ls) / c.N;
  const bool want = phase == PH_RESID || phase == PH_END ? s.alive
                    : phase == PH_R0 || phase == PH_UPD   ? s.refine
                                                          : s.incg;
  if (!want) return;
  double v[3] = {0.0, 0.0, 0.0};
  const bool sum = phase == PH_R0 || phase == PH_RZ || phase == PH_ALPHA || phase == PH_RR || phase == PH_BETA;
  for (int b = lane; b < nb; b += 64) {
    const double* q = part + (ls * nb + b) * 4;
    if (sum) {
      v[0] += (phase == PH_RZ || phase == PH_BETA) ? q[1] + q[2] : q[0];
    } else {
      v[0] = nanmax(v[0], q[0]);
      v[1] = nanmax(v[1], q[1]);
      v[2] = nanmax(v[2], q[2]);
    }
  }
  for (int k2 = 0; k2 < 3; ++k2) v[k2] = sum ? wave_sum(v[k2]) : wave_nanmax(v[k2]);
  if (lane != 0) return;
  int count = 0;
  switch (phase) {
    case PH_RESID:   // start of a step
      s.rmax = v[0];
      s.wref = v[1];
      s.sig = v[2];
      s.target = residual_target(k.tol, s.wref, k.tauf, k.dmax[sample]);
      s.pass = 0;
      s.refine = s.rmax > s.target && s.sig > 0.0;
      count = s.refine;
      break;
    case PH_R0: {
      // a pass reduces its residual only as far as the float64 target needs (with a margin:
      // CG measures the 2-norm, the target bounds the max-norm), never beyond pcg_rtol
      s.r0 = (float)v[0];
      const float red = (float)fmin(0.5, fmax((double)k.pcg_rtol, kPassMargin * s.target / s.rmax));
      s.stop = red * red * s.r0;
      s.rr = s.r0;
      s.it = 0;
      s.incg = s.rr > s.stop;
      count = s.incg;
      break;
    }
    case PH_RZ:
      s.rz = (float)v[0];
      break;
    case PH_ALPHA:
      s.al = s.rz / (float)v[0];
      break;
    case PH_RR: {
      const float rr = (float)v[0];
      s.rr = rr;
      s.it += 1;
      if (!(rr < 3.0e38f)) {   // a non-finite float32 pass is discarded; the step reports failure
        s.incg = 0;
        s.refine = 0;
        s.fail = 1;
        s.tot_it += s.it;
        s.max_it = max(s.max_it, s.it);
      } else if (rr <= s.stop || s.it >= k.cap) {
        s.incg = 0;
      }
      count = s.incg;
      break;
    }
    case PH_BETA: {
      const float rzn = (float)v[0];
      s.be = rzn / s.rz;
      s.rz = rzn;
      break;
    }
    case PH_UPD:
      s.tot_it += s.it;
      s.max_it = max(s.max_it, s.it);
      s.rmax = v[0];
      s.sig = v[1];
      s.wref = fmax(s.wref, v[2]);
      s.target = residual_target(k.tol, s.wref, k.tauf, k.dmax[sample]);
      s.pass += 1;
      s.refine = s.rmax > s.target && s.sig > 0.0 && s.pass < kMaxRefinePasses;
      count = s.refine;
      break;
    case PH_END:
      s.tot_pass += s.pass;
      if (s.rmax > s.target) {
        s.fail = 1;
        s.missed += 1;
      }
      break;
  }
  if (count) atomicAdd(&k.ring[k.slot], 1);
}

__global__ void k_init_sys(Sys* st, int64_t S, int64_t sys0, int N, int skip_first, const uint8_t* __restrict__ active,
                           int64_t M) {
  for (int64_t ls = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ls < S; ls += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sys = sys0 + ls;
    const int64_t m = sys / N;
    const int s = (int)(sys % N);
    Sys z{};
    z.alive = m < M && !(active && !active[m]) && !(skip_first && s == 0);
    st[ls] = z;
  }
}

__global__ void k_stats(const Sys* __restrict__ st, int64_t S, int J, int* __restrict__ flag,
                        unsigned long long* __restrict__ cnt) {
  for (int64_t ls = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ls < S; ls += (int64_t)gridDim.x * blockDim.x) {
    const Sys& s = st[ls];
    if (!s.alive) continue;
    if (s.fail) atomicOr(flag, 1);
    atomicAdd(&cnt[0], (unsigned long long)s.tot_it);
    atomicAdd(&cnt[1], (unsigned long long)s.tot_pass);
    atomicAdd(&cnt[2], (unsigned long long)J);
    atomicMax(&cnt[3], (unsigned long long)s.max_it);
    atomicAdd(&cnt[5], (unsigned long long)s.missed);
  }
}

// the largest diagonal of I + tau A over each sample (the rounding floor of the residual)
__global__ __launch_bounds__(kT) void k_dmax(const double* __restrict__ dinv, int64_t Nx, double* __restrict__ dmax,
                                             const uint8_t* __restrict__ need) {
  const int64_t m = blockIdx.x;
  if (!need[m]) return;
  double v = 0.0;
  for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) v = nanmax(v, 1.0 / (dinv[m * Nx + p] * dinv[m * Nx + p]));
  double d1[1] = {v};
  const bool mx[1] = {true};
  double out[1];
  band_partials<1>(d1, mx, out);
  if (threadIdx.x == 0) dmax[m] = out[0];
}

__global__ void k_samples_needed(int64_t M, int N, int skip_first, const uint8_t* __restrict__ active,
                                 uint8_t* __restrict__ need) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x)
    need[m] = !(active && !active[m]) && !(skip_first && N == 1);
}

unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024)); }

}  // namespace

// Fine propagation of nsys = M N systems with the streamed multigrid-preconditioned CG.
// dinv [M][Nx] float64 and sf [M][Fc] float32 (scaled couplings) are built by the caller.
int fine_mg_streamed(klecgc_ctx* ctx, const klecgc_problem& p, const FineArgs& fa, double tau, int J, int N,
                     const double* dinv, const float* sf, int* flag, unsigned long long* cnt) {
  hipStream_t st = ctx->stream;
  const int n = p.n;
  const int64_t M = fa.M, nsys = M * N;
  const int64_t Nx = (int64_t)n * n;
  const int64_t Fc = 2LL * n * (n + 1);
  const double h = 1.0 / (n + 1);
  const double c = tau / (h * h);
  const KcTuning tu = tuning_for(ctx, n);
  const Layout y = make_layout(n, tu.mg_sweeps);
  const int nb0 = y.nb[0];
  // per-sample buffers: coarse operators, largest diagonal, which samples run
  float* coef = (float*)ctx->ws.get(WS_MG_COEF, sizeof(float) * y.coef_per_sample * M + sizeof(double) * M + M);
  double* dmax = (double*)(coef + y.coef_per_sample * M);
  uint8_t* need = (uint8_t*)(dmax + M);
  // per-system buffers for a chunk of systems: float32 Krylov and level vectors, float64
  // residual and increments, band partials, state; a chunk is as large as 16 GiB (or the
  // fixed workspace of an allocation-free call) holds
  const int64_t per_sys = (int64_t)sizeof(float) * y.f32_per_sys + 3 * (int64_t)sizeof(double) * Nx +
                          (int64_t)sizeof(double) * 4 * nb0 + (int64_t)sizeof(Sys) + 64;
  const bool fixed = ctx->ws.arena != nullptr;
  const int64_t budget = fixed ? (int64_t)ctx->ws.arena_left() - 6 * 256 - (int64_t)sizeof(int) * kRing
                               : (int64_t)16 << 30;
  const int64_t chunk = std::min<int64_t>(nsys, budget / per_sys);
  KC_REQUIRE(chunk >= 1, KC_EINVAL, "allocation-free call: one multigrid system needs " + std::to_string(per_sys) +
                                        " bytes, more than the device scratch array has left");
  float* f32 = (float*)ctx->ws.get(WS_FINE_AUX, sizeof(float) * y.f32_per_sys * chunk);
  double* res = (double*)ctx->ws.get(WS_KRYLOV, sizeof(double) * Nx * chunk);
  double* incb = (double*)ctx->ws.get(WS_FINE_INC, 2 * sizeof(double) * Nx * chunk);
  char* small = (char*)ctx->ws.get(WS_MG_SMALL, sizeof(double) * 4 * nb0 * chunk + sizeof(Sys) * chunk +
                                                    sizeof(int) * kRing + 256);
  double* part = (double*)small;
  Sys* sysst = (Sys*)(small + sizeof(double) * 4 * nb0 * chunk);
  int* ring = (int*)(((uintptr_t)(sysst + chunk) + 255) & ~(uintptr_t)255);
  launch_zero_bytes(st, ring, sizeof(int) * kRing);
  int slot = 0;
  auto counted = [&](auto&& launch) -> int {   // a decision whose count the host needs
    if (slot == kRing) {
      launch_zero_bytes(st, ring, sizeof(int) * kRing);
      slot = 0;
    }
    Ctl k{p.inner_rtol > 0 ? p.inner_rtol : 1e-13, tau * p.forcing, dmax, tu.fine_pcg_rtol,
          std::min(p.inner_max_iter > 0 ? p.inner_max_iter : 4000, 400), ring, slot};
    launch(k);
    int hv = 0;
    KC_TRY_HIP(hipMemcpyAsync(&hv, ring + slot, sizeof(int), hipMemcpyDeviceToHost, st));
    KC_TRY_HIP(hipStreamSynchronize(st));
    ++slot;
    return hv;
  };
  const Ctl k0{p.inner_rtol > 0 ? p.inner_rtol : 1e-13, tau * p.forcing, dmax, tu.fine_pcg_rtol,
               std::min(p.inner_max_iter > 0 ? p.inner_max_iter : 4000, 400), ring, kRing - 1};

  // per-sample set-up: which samples run, their largest diagonal, their coarse operators
  k_samples_needed<<<grid1(M), 256, 0, st>>>(M, N, fa.skip_first, fa.active, need);
  KC_LAUNCH_CHECK();
  k_dmax<<<(unsigned)M, kT, 0, st>>>(dinv, Nx, dmax, need);
  KC_LAUNCH_CHECK();
  const int64_t nxf = (int64_t)n * (n + 1);
  auto level = [&](int l, int64_t vs_base_off) {
    Lv v{};
    v.m = y.m[l];
    v.rb = y.rb[l];
    v.l0 = l == 0;
    if (l == 0) {
      v.cw = sf;
      v.cs = sf + nxf;
      v.dg = nullptr;
      v.cstride = Fc;
    } else {
      v.cw = coef + y.coef_off[l];
      v.cs = v.cw + (int64_t)y.m[l] * y.m[l];
      v.dg = v.cs + (int64_t)y.m[l] * y.m[l];
      v.cstride = y.coef_per_sample;
    }
    v.vstride = y.f32_per_sys;
    (void)vs_base_off;
    return v;
  };
  for (int l = 1; l < y.L; ++l) {
    Lv f = level(l - 1, 0);
    k_coarsen<<<dim3((unsigned)y.nb[l], (unsigned)M), kT, 0, st>>>(f, coef, y.coef_per_sample, y.coef_off[l], y.m[l],
                                                                  y.rb[l], need);
    KC_LAUNCH_CHECK();
  }
  OnChip oc{};
  oc.lc = y.lc;
  oc.L = y.L;
  oc.sweeps = y.sweeps;
  for (int l = 0, off = 0; l < y.L; ++l) {
    oc.m[l] = y.m[l];
    oc.coef_off[l] = y.coef_off[l];
    oc.lds_off[l] = off;
    if (l >= y.lc) off += 5 * y.m[l] * y.m[l];
  }

  double last_line = 0.0;
  progress_line("multigrid fine propagation: %lld systems of %dx%d, %d steps, chunks of %lld", (long long)nsys, n, n,
                J, (long long)chunk);
  F64 f{fa.a, dinv, c, tau * p.forcing, fa.out, res, incb, n, y.rb[0]};
  StartRef sr{fa.start, fa.u0, fa.start_shift};
  const int sw = y.sweeps;
  for (int64_t s0 = 0; s0 < nsys; s0 += chunk) {
    const int64_t S = std::min<int64_t>(chunk, nsys - s0);
    Chunk ch{s0, N, sysst};
    // level views of this chunk's per-system vectors
    float* X = f32;
    float* R = f32 + Nx;
    float* P = f32 + 2 * Nx;
    float* Q = f32 + 3 * Nx;
    const int64_t vs = y.f32_per_sys;
    Lv lv[kMgMaxLevels];
    for (int l = 0; l < y.L; ++l) {
      lv[l] = level(l, 0);
      if (l <= y.lc && l < y.L) {
        lv[l].x = f32 + y.x_off[l];
        lv[l].b = l == 0 ? R : f32 + y.b_off[l];
      }
    }
    bool pairs[kMgMaxLevels] = {};
    for (int l = 0; l < y.L; ++l) pairs[l] = l <= y.lc && pairs_ok(lv[l]);
    const bool mv_pairs = pairs[0] && (reinterpret_cast<uintptr_t>(P) & 7) == 0 &&
                          (reinterpret_cast<uintptr_t>(Q) & 7) == 0;
    const bool pupd4 = n % 4 == 0 && vs % 4 == 0 && (reinterpret_cast<uintptr_t>(P) & 15) == 0 &&
                       (reinterpret_cast<uintptr_t>(lv[0].x) & 15) == 0;
    const dim3 g0((unsigned)nb0, (unsigned)S);
    k_init_sys<<<grid1(S), 256, 0, st>>>(sysst, S, s0, N, fa.skip_first, fa.active, M);
    KC_LAUNCH_CHECK();
    k_setup<<<g0, kT, 0, st>>>(f, sr, ch);
    KC_LAUNCH_CHECK();
    // one V-cycle z = M^{-1} R into x_0, its r.z in partial slots 1 and 2
    auto vcycle = [&]() {
      const int last_streamed = y.lc < y.L ? y.lc - 1 : y.L - 1;
      for (int l = 0; l <= last_streamed; ++l) {
        const dim3 gl((unsigned)y.nb[l], (unsigned)S);
        if (pairs[l])
          k_first_sweep_pairs<<<gl, kT, 0, st>>>(lv[l], ch);
        else
          k_first_sweep<<<gl, kT, 0, st>>>(lv[l], ch);
        KC_LAUNCH_CHECK();
        for (int s = 1; s < sw; ++s) {
          k_half<<<gl, kT, 0, st>>>(lv[l], ch, 0, nullptr, 0, 0, 0, nullptr, 0, 0);
          k_half<<<gl, kT, 0, st>>>(lv[l], ch, 1, nullptr, 0, 0, 0, nullptr, 0, 0);
        }
        KC_LAUNCH_CHECK();
        if (l + 1 < y.L) {
          const dim3 gr((unsigned)y.nb[l + 1], (unsigned)S);
          if (pairs[l])
            k_restrict_pairs<<<gr, kT, 0, st>>>(lv[l], lv[l + 1], ch);
          else
            k_restrict<<<gr, kT, 0, st>>>(lv[l], lv[l + 1], ch);
          KC_LAUNCH_CHECK();
        } else {   // level 0 is the coarsest (n <= 2): the transposed sweeps, r.z on the last
          for (int s = 0; s < sw; ++s) {
            const bool last = s == sw - 1;
            k_half<<<gl, kT, 0, st>>>(lv[l], ch, 1, nullptr, 0, 0, 0, last ? part : nullptr, nb0, 1);
            k_half<<<gl, kT, 0, st>>>(lv[l], ch, 0, nullptr, 0, 0, 0, last ? part : nullptr, nb0, 2);
          }
          KC_LAUNCH_CHECK();
          return;
        }
      }
      if (y.lc < y.L) {
        k_onchip<<<dim3(1, (unsigned)S), kOnChipT, y.lds_bytes, st>>>(oc, coef, y.coef_per_sample, lv[y.lc].b, lv[y.lc].x,
                                                                vs, ch);
        KC_LAUNCH_CHECK();
      }
      for (int l = last_streamed; l >= 0; --l) {
        const dim3 gl((unsigned)y.nb[l], (unsigned)S);
        const float* e = lv[l + 1].x;
        const int mc = y.m[l + 1];
        for (int s = 0; s < sw; ++s) {
          const bool dot = l == 0 && s == sw - 1;
          k_half<<<gl, kT, 0, st>>>(lv[l], ch, 1, e, mc, vs, s == 0 ? 1 : 0, dot ? part : nullptr, nb0, 1);
          k_half<<<gl, kT, 0, st>>>(lv[l], ch, 0, e, mc, vs, s == 0 ? 2 : 0, dot ? part : nullptr, nb0, 2);
        }
        KC_LAUNCH_CHECK();
      }
    };
    for (int step = 0; step < J; ++step) {
      if (step > 0) {
        k_step_start<<<g0, kT, 0, st>>>(f, ch, step);
        KC_LAUNCH_CHECK();
      }
      k_residual<<<g0, kT, 0, st>>>(f, ch, part, nb0);
      KC_LAUNCH_CHECK();
      int refining = counted([&](const Ctl& k) {
        k_decide<<<(unsigned)S, 64, 0, st>>>(ch, part, nb0, PH_RESID, k);
        KC_LAUNCH_CHECK();
      });
      while (refining > 0) {
        k_rhs<<<g0, kT, 0, st>>>(f, X, R, vs, ch, part, nb0);
        KC_LAUNCH_CHECK();
        int incg = counted([&](const Ctl& k) {
          k_decide<<<(unsigned)S, 64, 0, st>>>(ch, part, nb0, PH_R0, k);
          KC_LAUNCH_CHECK();
        });
        bool first = true;
        while (incg > 0) {
          vcycle();
          k_decide<<<(unsigned)S, 64, 0, st>>>(ch, part, nb0, first ? PH_RZ : PH_BETA, k0);
          if (pupd4)
            k_pupd4<<<g0, kT, 0, st>>>(n, y.rb[0], P, lv[0].x, vs, ch, first ? 1 : 0);
          else
            k_pupd<<<g0, kT, 0, st>>>(n, y.rb[0], P, lv[0].x, vs, ch, first ? 1 : 0);
          if (mv_pairs)
            k_matvec_pairs<<<g0, kT, 0, st>>>(lv[0], P, Q, vs, ch, part, nb0);
          else
            k_matvec<<<g0, kT, 0, st>>>(lv[0], P, Q, vs, ch, part, nb0);
          k_decide<<<(unsigned)S, 64, 0, st>>>(ch, part, nb0, PH_ALPHA, k0);
          k_xr<<<g0, kT, 0, st>>>(n, y.rb[0], X, R, P, Q, vs, ch, part, nb0);
          KC_LAUNCH_CHECK();
          incg = counted([&](const Ctl& k) {
            k_decide<<<(unsigned)S, 64, 0, st>>>(ch, part, nb0, PH_RR, k);
            KC_LAUNCH_CHECK();
          });
          first = false;
        }
        k_update64<<<g0, kT, 0, st>>>(f, X, vs, ch, part, nb0);
        KC_LAUNCH_CHECK();
        refining = counted([&](const Ctl& k) {
          k_decide<<<(unsigned)S, 64, 0, st>>>(ch, part, nb0, PH_UPD, k);
          KC_LAUNCH_CHECK();
        });
      }
      k_decide<<<(unsigned)S, 64, 0, st>>>(ch, part, nb0, PH_END, k0);
      KC_LAUNCH_CHECK();
      if (progress_due(last_line))
        progress_line("multigrid fine propagation: systems %lld..%lld of %lld, step %d of %d", (long long)s0,
                      (long long)(s0 + S), (long long)nsys, step + 1, J);
    }
    k_stats<<<grid1(S), 256, 0, st>>>(sysst, S, J, flag, cnt);
    KC_LAUNCH_CHECK();
  }
  return KC_OK;
}

}  // namespace kc
