// Aggregation multigrid V-cycle shared by the float32 Krylov kernels that stream their
// vectors through device memory (the shifted solves of step (b), complex; the implicit
// steps of the fine propagator, real).
//
// Both operate on a Jacobi-scaled 5-point operator L = diag(dg) - C on an m x m grid
// (node p = j m + i): real couplings cw[p] between nodes p-1 and p and cs[p] between
// p-m and p (0 on the boundary), and a diagonal dg of scalar type T (float or float2).
// Level l+1 aggregates 2x2 blocks of level l (a last 1-wide block when m is odd); its
// operator is the Galerkin product P^T L P for the piecewise-constant prolongation P,
// again 5-point: couplings summed across aggregate faces, diagonal summed over the block
// minus twice its internal couplings.  The V-cycle restricts by summation and prolongates
// by injection scaled by kMgScale (aggregation coarse spaces are too stiff by about that
// factor).  Smoother (h.sweeps sweeps per level and direction, default 2, the same on the
// coarsest level of at most 2x2): red-black Gauss-Seidel (default; colour (i + j) mod 2,
// red then black going down, black then red going up, so the post-smoother is the
// transpose of the pre-smoother) or damped Jacobi (the same symmetric operator down and
// up).  Either way the preconditioner is symmetric (complex symmetric for T = float2), as
// CG and COCG require.  All device functions are executed by every thread of the work-
// group and contain work-group barriers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kc {

constexpr int kMgMaxLevels = 12;
constexpr float kMgOmega = 0.7f;
constexpr float kMgScale = 1.8f;
constexpr int kMgSweeps = 2;   // default smoothing sweeps per level and direction
constexpr int kMgGaussSeidel = 0, kMgJacobi = 1;

struct MgLevels {
  int L;
  int sweeps;                  // smoothing sweeps per level and direction (>= 1)
  int smoother;                // kMgGaussSeidel or kMgJacobi
  int m[kMgMaxLevels];
  int64_t off[kMgMaxLevels];   // float offset of each level's block in a system's scratch
  int64_t per_sys;             // floats of scratch per system
};

template <class T>
struct MgT;

template <>
struct MgT<float> {
  static constexpr int words = 1;
  __device__ static float zero() { return 0.f; }
  __device__ static float one() { return 1.f; }
  __device__ static float mul(float a, float b) { return a * b; }
  __device__ static float add(float a, float b) { return a + b; }
  __device__ static float sub(float a, float b) { return a - b; }
  __device__ static float scale(float s, float a) { return s * a; }
  __device__ static float axpy(float s, float x, float y) { return fmaf(s, x, y); }   // s x + y
  __device__ static float recip(float a) { return 1.f / a; }
  __device__ static float sub_real(float a, float c) { return a - c; }
};

template <>
struct MgT<float2> {
  static constexpr int words = 2;
  __device__ static float2 zero() { return make_float2(0.f, 0.f); }
  __device__ static float2 mul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  }
  __device__ static float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
  __device__ static float2 sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
  __device__ static float2 scale(float s, float2 a) { return make_float2(s * a.x, s * a.y); }
  __device__ static float2 axpy(float s, float2 x, float2 y) { return make_float2(fmaf(s, x.x, y.x), fmaf(s, x.y, y.y)); }
  __device__ static float2 recip(float2 a) {
    const float den = a.x * a.x + a.y * a.y;
    return make_float2(a.x / den, -a.y / den);
  }
  __device__ static float2 sub_real(float2 a, float c) { return make_float2(a.x - c, a.y); }
};

// Level table for an n x n grid; `head` floats of Krylov vectors precede the levels in a
// system's scratch.  Level block (m = m_l): cw[m^2], cs[m^2] (float), then dg, di, xa,
// xb, b (T each).
inline MgLevels mg_levels(int n, int words, int64_t head, int sweeps, int smoother) {
  MgLevels h{};
  h.sweeps = sweeps >= 1 ? sweeps : kMgSweeps;
  h.smoother = smoother == kMgJacobi ? kMgJacobi : kMgGaussSeidel;
  int m = n, L = 0;
  int64_t off = head;
  while (true) {
    h.m[L] = m;
    h.off[L] = off;
    off += (2 + 5 * (int64_t)words) * m * m;
    off = (off + 1) / 2 * 2;   // keep float2 blocks 8-byte aligned
    ++L;
    if (m <= 2 || L == kMgMaxLevels) break;
    m = (m + 1) / 2;
  }
  h.L = L;
  h.per_sys = off;
  return h;
}

template <class T>
struct MgLv {
  int m;
  float *cw, *cs;
  T *dg, *di, *xa, *xb, *b;
};

template <class T>
__device__ __forceinline__ MgLv<T> mg_lv(float* base, const MgLevels& h, int l) {
  MgLv<T> v;
  v.m = h.m[l];
  const int64_t mm = (int64_t)v.m * v.m;
  float* p = base + h.off[l];
  v.cw = p;
  v.cs = p + mm;
  v.dg = (T*)(p + 2 * mm);
  v.di = v.dg + mm;
  v.xa = v.di + mm;
  v.xb = v.xa + mm;
  v.b = v.xb + mm;
  return v;
}

// (L x)_p on a level; X(q, i, j) yields x at node q = j m + i
template <class T, class XF>
__device__ __forceinline__ T mg_apply(const MgLv<T>& v, int64_t p, int i, int j, XF X) {
  using O = MgT<T>;
  const int m = v.m;
  T acc = O::mul(v.dg[p], X(p, i, j));
  if (i > 0) acc = O::axpy(-v.cw[p], X(p - 1, i - 1, j), acc);
  if (i < m - 1) acc = O::axpy(-v.cw[p + 1], X(p + 1, i + 1, j), acc);
  if (j > 0) acc = O::axpy(-v.cs[p], X(p - m, i, j - 1), acc);
  if (j < m - 1) acc = O::axpy(-v.cs[p + m], X(p + m, i, j + 1), acc);
  return acc;
}

// Coarse levels 1..L-1 from level 0 (whose cw, cs, dg must be complete and visible).
template <class T>
__device__ void mg_build_coarse(float* base, const MgLevels& h) {
  using O = MgT<T>;
  for (int l = 1; l < h.L; ++l) {
    const MgLv<T> f = mg_lv<T>(base, h, l - 1);
    const MgLv<T> c = mg_lv<T>(base, h, l);
    const int mf = f.m, mc = c.m;
    for (int64_t Pn = threadIdx.x; Pn < (int64_t)mc * mc; Pn += blockDim.x) {
      const int I = (int)(Pn % mc), J = (int)(Pn / mc);
      const int i0 = 2 * I, j0 = 2 * J;
      const bool two_i = i0 + 1 < mf, two_j = j0 + 1 < mf;
      T dg = O::zero();
      float cwc = 0.f, csc = 0.f, inner = 0.f;
      for (int dj = 0; dj < (two_j ? 2 : 1); ++dj)
        for (int di = 0; di < (two_i ? 2 : 1); ++di) {
          const int64_t p = (int64_t)(j0 + dj) * mf + (i0 + di);
          dg = O::add(dg, f.dg[p]);
          if (di == 1) inner += f.cw[p];            // coupling inside the block (x)
          if (dj == 1) inner += f.cs[p];            // coupling inside the block (y)
          if (di == 0 && I > 0) cwc += f.cw[p];     // couplings across the west face
          if (dj == 0 && J > 0) csc += f.cs[p];     // couplings across the south face
        }
      dg = O::sub_real(dg, 2.f * inner);
      c.dg[Pn] = dg;
      c.di[Pn] = O::recip(dg);
      c.cw[Pn] = cwc;
      c.cs[Pn] = csc;
    }
    __syncthreads();
  }
}

// One red-black Gauss-Seidel half sweep on a level: the nodes of colour col take
// x_p += di_p (b_p - (L x)_p); their neighbours all have the other colour, so the update
// is exact Gauss-Seidel.  Work items run over the nodes of that colour only (row j holds
// them at i = 2k + ((col + j) & 1)).  With DOT, the work item also adds b_p x_p of its
// updated nodes to dot.  Ends with a barrier.
template <class T, bool DOT = false>
__device__ __forceinline__ void mg_gs_half(const MgLv<T>& v, const T* b, T* x, int col, T* dot = nullptr) {
  using O = MgT<T>;
  const int m = v.m, hw = (m + 1) / 2;
  for (int64_t q = threadIdx.x; q < (int64_t)m * hw; q += blockDim.x) {
    const int j = (int)(q / hw);
    const int i = 2 * (int)(q % hw) + ((col + j) & 1);
    if (i < m) {
      const int64_t p = (int64_t)j * m + i;
      // the diagonal's reciprocal from the diagonal mg_apply reads anyway (the kernel is
      // bound by memory traffic, not by the few extra operations)
      const T dgp = v.dg[p];
      const T xp = x[p];
      T acc = O::mul(dgp, xp);
      if (i > 0) acc = O::axpy(-v.cw[p], x[p - 1], acc);
      if (i < m - 1) acc = O::axpy(-v.cw[p + 1], x[p + 1], acc);
      if (j > 0) acc = O::axpy(-v.cs[p], x[p - m], acc);
      if (j < m - 1) acc = O::axpy(-v.cs[p + m], x[p + m], acc);
      const T bp = b[p];
      const T xn = O::add(xp, O::mul(O::recip(dgp), O::sub(bp, acc)));
      x[p] = xn;
      if constexpr (DOT) *dot = O::add(*dot, O::mul(bp, xn));
    }
  }
  __syncthreads();
}

// Red-black Gauss-Seidel V-cycle; the iterate of every level lives in its xa buffer.  With
// dot non-null the work item's share of sum_p rhs0_p z_p is added to *dot (every level-0
// node takes its final value in one of the last two half sweeps, which read rhs0_p anyway).
template <class T>
__device__ T* mg_vcycle_gs(float* base, const MgLevels& h, const T* rhs0, T* dot = nullptr) {
  using O = MgT<T>;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int l = 0; l < h.L; ++l) {
    const MgLv<T> v = mg_lv<T>(base, h, l);
    const T* b = l == 0 ? rhs0 : v.b;
    const int m = v.m;
    const int64_t mm = (int64_t)m * m;
    // first sweep from x = 0: the red half is x_r = di_r b_r, the black nodes start at 0
    for (int64_t p = tid; p < mm; p += nt) {
      const int i = (int)(p % m), j = (int)(p / m);
      v.xa[p] = ((i + j) & 1) == 0 ? O::mul(O::recip(v.dg[p]), b[p]) : O::zero();
    }
    __syncthreads();
    mg_gs_half<T>(v, b, v.xa, 1);
    for (int s = 1; s < h.sweeps; ++s) {
      mg_gs_half<T>(v, b, v.xa, 0);
      mg_gs_half<T>(v, b, v.xa, 1);
    }
    if (l + 1 < h.L) {   // restrict the residual: b_{l+1}[I,J] = sum over the block of (b - L x)
      const MgLv<T> c = mg_lv<T>(base, h, l + 1);
      const int mc = c.m;
      const T* xc = v.xa;
      for (int64_t P = tid; P < (int64_t)mc * mc; P += nt) {
        const int I = (int)(P % mc), J = (int)(P / mc);
        T sum = O::zero();
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) {
            const int i = 2 * I + di, j = 2 * J + dj;
            if (i < m && j < m) {
              const int64_t p = (int64_t)j * m + i;
              const T lx = mg_apply<T>(v, p, i, j, [&](int64_t q, int, int) { return xc[q]; });
              sum = O::add(sum, O::sub(b[p], lx));
            }
          }
        c.b[P] = sum;
      }
      __syncthreads();
    } else {             // coarsest level: the transposed sweeps complete its smoothing
      for (int s = 0; s < h.sweeps; ++s) {
        if (l == 0 && dot && s == h.sweeps - 1) {   // a one-level hierarchy ends here
          mg_gs_half<T, true>(v, b, v.xa, 1, dot);
          mg_gs_half<T, true>(v, b, v.xa, 0, dot);
        } else {
          mg_gs_half<T>(v, b, v.xa, 1);
          mg_gs_half<T>(v, b, v.xa, 0);
        }
      }
    }
  }
  for (int l = h.L - 2; l >= 0; --l) {
    const MgLv<T> v = mg_lv<T>(base, h, l);
    const MgLv<T> c = mg_lv<T>(base, h, l + 1);
    const T* b = l == 0 ? rhs0 : v.b;
    const int m = v.m, mc = c.m;
    const int64_t mm = (int64_t)m * m;
    for (int64_t p = tid; p < mm; p += nt) {   // x += s P e
      const int i = (int)(p % m), j = (int)(p / m);
      v.xa[p] = O::axpy(kMgScale, c.xa[(int64_t)(j >> 1) * mc + (i >> 1)], v.xa[p]);
    }
    __syncthreads();
    for (int s = 0; s < h.sweeps; ++s) {
      if (l == 0 && dot && s == h.sweeps - 1) {
        mg_gs_half<T, true>(v, b, v.xa, 1, dot);
        mg_gs_half<T, true>(v, b, v.xa, 0, dot);
      } else {
        mg_gs_half<T>(v, b, v.xa, 1);
        mg_gs_half<T>(v, b, v.xa, 0);
      }
    }
  }
  return mg_lv<T>(base, h, 0).xa;
}

// z = V-cycle applied to rhs0 (level 0); returns the level-0 buffer holding z.
// rhs0 must be visible to the whole work-group; z is visible on return.
template <class T>
__device__ T* mg_vcycle(float* base, const MgLevels& h, const T* rhs0) {
  if (h.smoother == kMgGaussSeidel) return mg_vcycle_gs<T>(base, h, rhs0);
  using O = MgT<T>;
  int cur[kMgMaxLevels];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int l = 0; l < h.L; ++l) {
    const MgLv<T> v = mg_lv<T>(base, h, l);
    const T* b = l == 0 ? rhs0 : v.b;
    const int m = v.m;
    const int64_t mm = (int64_t)m * m;
    for (int64_t p = tid; p < mm; p += nt) v.xa[p] = O::scale(kMgOmega, O::mul(v.di[p], b[p]));
    __syncthreads();
    T* xc = v.xa;
    T* xn = v.xb;
    for (int s = 1; s < h.sweeps; ++s) {
      for (int64_t p = tid; p < mm; p += nt) {
        const int i = (int)(p % m), j = (int)(p / m);
        const T lx = mg_apply<T>(v, p, i, j, [&](int64_t q, int, int) { return xc[q]; });
        xn[p] = O::add(xc[p], O::scale(kMgOmega, O::mul(v.di[p], O::sub(b[p], lx))));
      }
      __syncthreads();
      T* tmp = xc;
      xc = xn;
      xn = tmp;
    }
    cur[l] = xc == v.xa ? 0 : 1;
    if (l + 1 < h.L) {   // restrict the residual: b_{l+1}[I,J] = sum over the block of (b - L x)
      const MgLv<T> c = mg_lv<T>(base, h, l + 1);
      const int mc = c.m;
      for (int64_t P = tid; P < (int64_t)mc * mc; P += nt) {
        const int I = (int)(P % mc), J = (int)(P / mc);
        T sum = O::zero();
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) {
            const int i = 2 * I + di, j = 2 * J + dj;
            if (i < m && j < m) {
              const int64_t p = (int64_t)j * m + i;
              const T lx = mg_apply<T>(v, p, i, j, [&](int64_t q, int, int) { return xc[q]; });
              sum = O::add(sum, O::sub(b[p], lx));
            }
          }
        c.b[P] = sum;
      }
      __syncthreads();
    }
  }
  for (int l = h.L - 2; l >= 0; --l) {
    const MgLv<T> v = mg_lv<T>(base, h, l);
    const MgLv<T> c = mg_lv<T>(base, h, l + 1);
    const T* ec = cur[l + 1] ? c.xb : c.xa;
    const T* b = l == 0 ? rhs0 : v.b;
    const int m = v.m, mc = c.m;
    const int64_t mm = (int64_t)m * m;
    T* xc = cur[l] ? v.xb : v.xa;
    T* xn = cur[l] ? v.xa : v.xb;
    // first post-smoothing sweep on x + s P e (the prolongated correction folded in)
    auto xp = [&](int64_t q, int qi, int qj) {
      return O::axpy(kMgScale, ec[(int64_t)(qj >> 1) * mc + (qi >> 1)], xc[q]);
    };
    for (int64_t p = tid; p < mm; p += nt) {
      const int i = (int)(p % m), j = (int)(p / m);
      const T lx = mg_apply<T>(v, p, i, j, xp);
      xn[p] = O::add(xp(p, i, j), O::scale(kMgOmega, O::mul(v.di[p], O::sub(b[p], lx))));
    }
    __syncthreads();
    T* tmp = xc;
    xc = xn;
    xn = tmp;
    for (int s = 1; s < h.sweeps; ++s) {
      for (int64_t p = tid; p < mm; p += nt) {
        const int i = (int)(p % m), j = (int)(p / m);
        const T lx = mg_apply<T>(v, p, i, j, [&](int64_t q, int, int) { return xc[q]; });
        xn[p] = O::add(xc[p], O::scale(kMgOmega, O::mul(v.di[p], O::sub(b[p], lx))));
      }
      __syncthreads();
      tmp = xc;
      xc = xn;
      xn = tmp;
    }
    cur[l] = xc == v.xa ? 0 : 1;
  }
  const MgLv<T> v0 = mg_lv<T>(base, h, 0);
  return cur[0] ? v0.xb : v0.xa;
}

}  // namespace kc
