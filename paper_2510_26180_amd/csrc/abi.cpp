// C ABI entry points: argument validation, stream/device binding, error capture, and
// the host-side orchestration of the KL / gPC stages and of the parareal iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#include "common.h"
#include "models.h"

namespace kc {

void field_kl_host(int dim, int n, int d, double corr_len, double sigma, std::vector<double>& lam,
                   std::vector<double>& phi);
void launch_dgemm_nt(hipStream_t s, int64_t Mr, int64_t Nc, int64_t K, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                     double alpha);

bool progress_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("KLECGC_PROGRESS");
    return v && v[0] && v[0] != '0';
  }();
  return on;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool progress_due(double& last_s) {
  if (!progress_enabled()) return false;
  const double t = now_s();
  if (t - last_s < 10.0) return false;
  last_s = t;
  return true;
}

void progress_line(const char* fmt, ...) {
  if (!progress_enabled()) return;
  std::va_list ap;
  va_start(ap, fmt);
  std::fputs("[klecgc] ", stderr);
  std::vfprintf(stderr, fmt, ap);
  std::fputc('\n', stderr);
  std::fflush(stderr);
  va_end(ap);
}

void* Workspace::get(int slot, size_t bytes) {
  if ((int)ptr.size() < WS_COUNT) {
    ptr.resize(WS_COUNT, nullptr);
    cap.resize(WS_COUNT, 0);
  }
  if (bytes == 0) bytes = 1;
  if (arena) {
    if (cap[slot] >= bytes) return ptr[slot];
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (need > arena_left())
      throw Error{KC_EINVAL, "allocation-free call: its workspace exceeds the " + std::to_string(arena_bytes) +
                                 "-byte device scratch array (" + std::to_string(arena_used) +
                                 " bytes taken, " + std::to_string(bytes) + " more requested)"};
    ptr[slot] = arena + arena_used;
    cap[slot] = bytes;
    arena_used += need;
    return ptr[slot];
  }
  if (cap[slot] < bytes) {
    if (ptr[slot]) {
      KC_TRY_HIP(hipDeviceSynchronize());
      KC_TRY_HIP(hipFree(ptr[slot]));
      ptr[slot] = nullptr;
      cap[slot] = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{KC_ENOMEM, "device workspace allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    ptr[slot] = p;
    cap[slot] = bytes;
  }
  return ptr[slot];
}

void Workspace::release() {
  if (arena) return;   // the arena is not the workspace's
  for (auto& p : ptr)
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
  std::fill(cap.begin(), cap.end(), 0);
}

DevStatus status_block(klecgc_ctx* ctx, int slot) {
  char* b = (char*)ctx->ws.get(slot, kStatusBytes);
  return DevStatus{(int*)b, (unsigned long long*)(b + 8)};
}

void status_reset(klecgc_ctx* ctx, const DevStatus& st) {
  if (ctx->capturing) return;
  launch_zero_bytes(ctx->stream, st.flag, kStatusBytes);
}

int status_collect(klecgc_ctx* ctx, const DevStatus& st, int base) {
  if (ctx->capturing) return 0;
  unsigned char h[kStatusBytes];
  KC_TRY_HIP(hipMemcpyAsync(h, st.flag, kStatusBytes, hipMemcpyDeviceToHost, ctx->stream));
  KC_TRY_HIP(hipStreamSynchronize(ctx->stream));
  int flag;
  unsigned long long c[10];
  std::memcpy(&flag, h, sizeof(int));
  std::memcpy(c, h + 8, sizeof(c));
  ctx->stats[base == 0 ? 10 : 11] += (int64_t)c[5];   // solves that missed their target
  if (base == 0) {
    ctx->stats[8] += (int64_t)c[8];
    ctx->stats[9] += (int64_t)c[9];
  }
  ctx->stats[base + 0] += (int64_t)c[0];
  ctx->stats[base + 1] += (int64_t)c[1];
  ctx->stats[base + 2] += (int64_t)c[2];
  ctx->stats[base + 3] = std::max<int64_t>(ctx->stats[base + 3], (int64_t)c[3]);
  return flag;
}

void validate_problem(const klecgc_problem& p) {
  KC_REQUIRE(p.dim == 1 || p.dim == 2, KC_EINVAL, "dim must be 1 or 2");
  KC_REQUIRE(p.n >= 1, KC_EINVAL, "n must be >= 1");
  KC_REQUIRE(p.T > 0 && std::isfinite(p.T), KC_EINVAL, "T must be positive");
  KC_REQUIRE(p.N >= 2 && p.N <= 256 && (p.N & (p.N - 1)) == 0, KC_EINVAL,
             "N must be a power of two in [2, 256]");
  KC_REQUIRE(p.J >= 1, KC_EINVAL, "J must be >= 1");
  KC_REQUIRE(p.alpha > 0 && p.alpha < 1, KC_EINVAL, "alpha must lie in (0, 1)");
  KC_REQUIRE(std::isfinite(p.forcing), KC_EINVAL, "forcing must be finite");
  KC_REQUIRE(p.precision == KC_PREC_F64 || p.precision == KC_PREC_F32_REFINED, KC_EINVAL,
             "unknown precision");
  KC_REQUIRE(p.tol > 0, KC_EINVAL, "tol must be positive");
  KC_REQUIRE(p.max_iter >= 1, KC_EINVAL, "max_iter must be >= 1");
  KC_REQUIRE(p.inner_rtol >= 0 && p.cgc_rtol >= 0, KC_EINVAL, "tolerances must be >= 0");
  KC_REQUIRE(p.inner_max_iter >= 0 && p.cgc_max_iter >= 0, KC_EINVAL, "iteration caps must be >= 0");
  if (p.dim == 1)
    KC_REQUIRE(p.precision == KC_PREC_F64, KC_EUNSUPPORTED, "1D supports only KC_PREC_F64");
  if (p.dim == 2) KC_REQUIRE(p.n <= 4096, KC_EUNSUPPORTED, "2D grids above 4096^2 unsupported");
}

static std::vector<std::vector<int>> index_set(int d, int p) {
  // total-order multi-indices, degree ascending then lexicographic ascending
  std::vector<std::vector<int>> out;
  std::vector<int> cur(d, 0);
  for (int deg = 0; deg <= p; ++deg) {
    // enumerate compositions of deg into d parts in lexicographic order
    std::function<void(int, int)> rec = [&](int pos, int left) {
      if (pos == d - 1) {
        cur[pos] = left;
        out.push_back(cur);
        return;
      }
      for (int v = 0; v <= left; ++v) {
        cur[pos] = v;
        rec(pos + 1, left - v);
      }
    };
    rec(0, deg);
  }
  return out;
}

int gpc_predict_impl(klecgc_ctx* ctx, const klecgc_gpc* g, const double* xi, int64_t M, double* U0) {
  hipStream_t st = ctx->stream;
  double* Psi = (double*)ctx->ws.get(WS_GEMM_A, sizeof(double) * M * g->P);
  double* Z = (double*)ctx->ws.get(WS_GEMM_B, sizeof(double) * M * g->n_modes);
  launch_gpc_basis(st, xi, M, g->d, g->idx, g->P, g->basis, Psi);
  launch_dgemm(st, M, g->n_modes, g->P, Psi, g->P, g->H, g->n_modes, Z, g->n_modes, nullptr, 1.0);
  timed(ctx, KT_GEMM, [&] { launch_dgemm(st, M, g->L, g->n_modes, Z, g->n_modes, g->W, g->L, U0, g->L, g->mean, 1.0); });
  return KC_OK;
}

}  // namespace kc

using namespace kc;

namespace {

// device allocation released when the scope ends (also on an error)
struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

template <class F>
int guarded(klecgc_ctx* ctx, F&& f) {
  if (!ctx) return KC_EINVAL;
  ctx->err.clear();
  for (auto& v : ctx->stats) v = 0;
  for (auto& v : ctx->ktime) v = 0;
  for (auto& v : ctx->kcount) v = 0;
  try {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) throw Error{KC_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e)};
    return f();
  } catch (const Error& e) {
    ctx->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return KC_ENOMEM;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return KC_EINVAL;
  }
}

}  // namespace

extern "C" {

const char* klecgc_version(void) { return "klecgc 0.1 (gfx950)"; }

int klecgc_create(klecgc_ctx** out, int device, void* hip_stream) {
  if (!out) return KC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return KC_EHIP;
  if (hipSetDevice(device) != hipSuccess) return KC_EHIP;
  auto* c = new (std::nothrow) klecgc_ctx;
  if (!c) return KC_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->num_cus = cus;
  if (hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess) {
    delete c;
    return KC_EHIP;
  }
  // the device's copy of the allocation-free scratch array (resolved once per device); a
  // failure leaves it unset and only the allocation-free entry point reports it
  if (kc::scratch_resolve(device, &c->scratch) != hipSuccess) {
    (void)hipGetLastError();
    c->scratch = nullptr;
  }
  *out = c;
  return KC_OK;
}

void klecgc_destroy(klecgc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  kc::release_blas(ctx);
  ctx->ws.release();
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

int klecgc_set_stream(klecgc_ctx* ctx, void* s) {
  return guarded(ctx, [&] {
    ctx->stream = (hipStream_t)s;
    return KC_OK;
  });
}

const char* klecgc_last_error(const klecgc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int klecgc_last_times(const klecgc_ctx* ctx, double* ms8, int64_t* count8) {
  if (!ctx || !ms8) return KC_EINVAL;
  for (int i = 0; i < 8; ++i) {
    ms8[i] = ctx->ktime[i];
    if (count8) count8[i] = ctx->kcount[i];
  }
  return KC_OK;
}

int klecgc_set_tuning(klecgc_ctx* ctx, int32_t n, const klecgc_tuning* t) {
  return guarded(ctx, [&] {
    KC_REQUIRE(t, KC_EINVAL, "null argument");
    KC_REQUIRE(n >= 1, KC_EINVAL, "n must be >= 1");
    KC_REQUIRE(t->fine_variant == -1 || fine_variant_fits(t->fine_variant, n), KC_EINVAL,
               "fine variant does not fit this grid size");
    KC_REQUIRE(t->cgc_variant == -1 || cgc_variant_fits(t->cgc_variant, n), KC_EINVAL,
               "shifted-solve variant does not fit this grid size");
    KC_REQUIRE(t->fine_pcg_rtol > 0.f && t->fine_pcg_rtol < 0.5f && t->cgc_inner_rtol > 0.f &&
                   t->cgc_inner_rtol < 0.5f,
               KC_EINVAL, "per-pass reductions must lie in (0, 0.5)");
    KC_REQUIRE(t->mg_sweeps >= 0 && t->mg_sweeps <= 4, KC_EINVAL, "mg_sweeps must lie in [0, 4]");
    KC_REQUIRE(t->mg_smoother == 0 || t->mg_smoother == 1, KC_EINVAL, "mg_smoother must be 0 or 1");
    KcTuning k;
    k.fine_variant = t->fine_variant;
    k.fine_pcg_rtol = t->fine_pcg_rtol;
    k.cgc_variant = t->cgc_variant;
    k.cgc_inner_rtol = t->cgc_inner_rtol;
    k.mg_sweeps = t->mg_sweeps;
    k.mg_smoother = t->mg_smoother;
    ctx->tuning[n] = k;
    return KC_OK;
  });
}

int klecgc_get_tuning(const klecgc_ctx* ctx, int32_t n, klecgc_tuning* t) {
  if (!ctx || !t) return KC_EINVAL;
  const KcTuning k = tuning_for(ctx, n);
  t->fine_variant = k.fine_variant;
  t->fine_pcg_rtol = k.fine_pcg_rtol;
  t->cgc_variant = k.cgc_variant;
  t->cgc_inner_rtol = k.cgc_inner_rtol;
  t->mg_sweeps = k.mg_sweeps;
  t->mg_smoother = k.mg_smoother;
  return KC_OK;
}

int klecgc_autotune(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev, int64_t M, klecgc_tuning* out,
                    double* ms_out) {
  return guarded(ctx, [&] {
    KC_REQUIRE(prob && a_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_problem(*prob);
    return autotune_impl(ctx, *prob, a_dev, M, out, ms_out);
  });
}

int klecgc_last_stats(const klecgc_ctx* ctx, int64_t* out16) {
  if (!ctx || !out16) return KC_EINVAL;
  for (int i = 0; i < 16; ++i) out16[i] = ctx->stats[i];
  return KC_OK;
}

void klecgc_kle_free(klecgc_kle* h) {
  if (!h) return;
  (void)hipFree(h->phi);
  (void)hipFree(h->sqrt_lam);
  (void)hipFree(h->mean);
  (void)hipFree(h->W);
  (void)hipFree(h->lam);
  delete h;
}

void klecgc_gpc_free(klecgc_gpc* h) {
  if (!h) return;
  (void)hipFree(h->idx);
  (void)hipFree(h->H);
  delete h;
}

int kle_build(klecgc_ctx* ctx, const klecgc_kle_desc* desc, const double* S_dev, int64_t n_t,
              klecgc_kle** out, int32_t* n_modes) {
  return guarded(ctx, [&] {
    KC_REQUIRE(desc && out, KC_EINVAL, "null argument");
    *out = nullptr;
    hipStream_t st = ctx->stream;
    auto* h = new klecgc_kle;
    h->kind = desc->kind;
    try {
      if (desc->kind == KC_KLE_FIELD_EXP) {
        KC_REQUIRE(desc->dim == 1 || desc->dim == 2, KC_EINVAL, "dim must be 1 or 2");
        KC_REQUIRE(desc->n >= 1 && desc->d >= 1 && desc->d <= 256, KC_EINVAL, "bad n or d");
        KC_REQUIRE(desc->corr_len > 0 && desc->sigma >= 0, KC_EINVAL, "bad corr_len or sigma");
        h->dim = desc->dim;
        h->n = desc->n;
        h->d = desc->d;
        h->nfaces = n_faces(desc->dim, desc->n);
        std::vector<double> lam, phi;
        field_kl_host(desc->dim, desc->n, desc->d, desc->corr_len, desc->sigma, lam, phi);
        std::vector<double> sl(desc->d);
        for (int k = 0; k < desc->d; ++k) sl[k] = std::sqrt(lam[k]);
        h->lam_host = lam;
        KC_TRY_HIP(hipMalloc(&h->phi, sizeof(double) * phi.size()));
        KC_TRY_HIP(hipMalloc(&h->sqrt_lam, sizeof(double) * sl.size()));
        KC_TRY_HIP(hipMemcpyAsync(h->phi, phi.data(), sizeof(double) * phi.size(), hipMemcpyHostToDevice, st));
        KC_TRY_HIP(hipMemcpyAsync(h->sqrt_lam, sl.data(), sizeof(double) * sl.size(), hipMemcpyHostToDevice, st));
        KC_TRY_HIP(hipStreamSynchronize(st));
        if (n_modes) *n_modes = desc->d;
      } else if (desc->kind == KC_KLE_SNAPSHOT) {
        KC_REQUIRE(S_dev, KC_EINVAL, "S_dev required");
        KC_REQUIRE(n_t >= 2 && desc->L >= 1, KC_EINVAL, "need n_t >= 2 and L >= 1");
        KC_REQUIRE(desc->eps_kl >= 0 && desc->eps_kl < 1, KC_EINVAL, "eps_kl must lie in [0, 1)");
        const int64_t L = desc->L;
        h->L = L;
        h->n_t = n_t;
        DevBuf sc_buf, cd_buf, e_buf;
        KC_TRY_HIP(hipMalloc(&h->mean, sizeof(double) * L));
        KC_TRY_HIP(hipMalloc(&sc_buf.p, sizeof(double) * L * n_t));
        KC_TRY_HIP(hipMalloc(&cd_buf.p, sizeof(double) * n_t * n_t));
        double* Sc = (double*)sc_buf.p;
        double* Cd = (double*)cd_buf.p;
        launch_col_mean_center(st, S_dev, n_t, L, h->mean, Sc);
        launch_dgemm_nt(st, n_t, n_t, L, Sc, L, Sc, L, Cd, n_t, 1.0 / (double)n_t);
        std::vector<double> C, w;
        gram_eig(ctx, (int)n_t, Cd, C, w);
        for (auto& x : w) x = std::max(x, 0.0);
        double total = 0.0;
        for (double x : w) total += x;
        KC_REQUIRE(total > 0, KC_ERANK, "snapshots have zero variance");
        int MQ = 0;
        double cum = 0.0;
        for (int64_t i = 0; i < n_t; ++i) {
          cum += w[i];
          MQ = (int)i + 1;
          if (cum / total >= 1.0 - desc->eps_kl) break;
        }
        int rank = 0;
        for (int64_t i = 0; i < n_t; ++i)
          if (w[i] > (double)n_t * 2.220446049250313e-16 * w[0]) ++rank;
        MQ = std::max(1, std::min(MQ, rank));
        h->n_modes = MQ;
        // E [n_t][MQ]; W = E^T S~ / sqrt(n_t)  (= diag(sqrt(lam)) g)
        std::vector<double> E((size_t)n_t * MQ);
        h->zeta_train.resize((size_t)n_t * MQ);
        for (int64_t r = 0; r < n_t; ++r)
          for (int c = 0; c < MQ; ++c) {
            E[r * MQ + c] = C[r * n_t + c];
            h->zeta_train[r * MQ + c] = std::sqrt((double)n_t) * C[r * n_t + c];
          }
        KC_TRY_HIP(hipMalloc(&e_buf.p, sizeof(double) * E.size()));
        double* Ed = (double*)e_buf.p;
        KC_TRY_HIP(hipMalloc(&h->W, sizeof(double) * MQ * L));
        KC_TRY_HIP(hipMalloc(&h->lam, sizeof(double) * MQ));
        KC_TRY_HIP(hipMemcpyAsync(Ed, E.data(), sizeof(double) * E.size(), hipMemcpyHostToDevice, st));
        KC_TRY_HIP(hipMemcpyAsync(h->lam, w.data(), sizeof(double) * MQ, hipMemcpyHostToDevice, st));
        launch_dgemm_tn(st, MQ, L, n_t, Ed, MQ, Sc, L, h->W, L, 1.0 / std::sqrt((double)n_t));
        KC_TRY_HIP(hipStreamSynchronize(st));
        h->lam_host.assign(w.begin(), w.begin() + MQ);
        if (n_modes) *n_modes = MQ;
      } else {
        throw Error{KC_EINVAL, "unknown KL kind"};
      }
    } catch (...) {
      klecgc_kle_free(h);
      throw;
    }
    *out = h;
    return KC_OK;
  });
}

int kle_synthesize(klecgc_ctx* ctx, const klecgc_kle* f, const double* xi_dev, int64_t M, double* a_dev,
                   float* a32_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(f && xi_dev && a_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(f->kind == KC_KLE_FIELD_EXP, KC_EINVAL, "handle is not a FIELD_EXP KL");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    launch_field_synth(ctx->stream, f->phi, f->sqrt_lam, f->d, f->nfaces, xi_dev, M, a_dev, a32_dev);
    return KC_OK;
  });
}

int kle_export(klecgc_ctx* ctx, const klecgc_kle* h, double* mean_dev, double* W_dev, double* lam_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(h && h->kind == KC_KLE_SNAPSHOT, KC_EINVAL, "handle is not a SNAPSHOT KL");
    hipStream_t st = ctx->stream;
    if (mean_dev) KC_TRY_HIP(hipMemcpyAsync(mean_dev, h->mean, sizeof(double) * h->L, hipMemcpyDeviceToDevice, st));
    if (W_dev)
      KC_TRY_HIP(hipMemcpyAsync(W_dev, h->W, sizeof(double) * h->L * h->n_modes, hipMemcpyDeviceToDevice, st));
    if (lam_dev) KC_TRY_HIP(hipMemcpyAsync(lam_dev, h->lam, sizeof(double) * h->n_modes, hipMemcpyDeviceToDevice, st));
    return KC_OK;
  });
}

int gpc_fit(klecgc_ctx* ctx, const klecgc_kle* snap, const double* xi_train_dev, int64_t n_t,
            int32_t d, int32_t p, int32_t basis, klecgc_gpc** out, int32_t* P) {
  return guarded(ctx, [&] {
    KC_REQUIRE(snap && xi_train_dev && out, KC_EINVAL, "null argument");
    KC_REQUIRE(snap->kind == KC_KLE_SNAPSHOT, KC_EINVAL, "handle is not a SNAPSHOT KL");
    KC_REQUIRE(n_t == snap->n_t, KC_EINVAL, "n_t differs from the snapshot count");
    KC_REQUIRE(d >= 1 && p >= 0 && p <= 16, KC_EINVAL, "bad d or p");
    KC_REQUIRE(basis == KC_GPC_HERMITE || basis == KC_GPC_LEGENDRE, KC_EINVAL, "unknown gPC basis");
    *out = nullptr;
    hipStream_t st = ctx->stream;
    auto idx = index_set(d, p);
    const int Pn = (int)idx.size();
    if (P) *P = Pn;
    KC_REQUIRE(n_t >= Pn, KC_ERANK, "n_t < P: least-squares problem under-determined");
    auto* g = new klecgc_gpc;
    try {
      g->d = d;
      g->p = p;
      g->basis = basis;
      g->P = Pn;
      g->n_modes = snap->n_modes;
      g->L = snap->L;
      g->kl = snap;
      g->mean = snap->mean;
      g->W = snap->W;
      std::vector<int32_t> flat((size_t)Pn * d);
      for (int i = 0; i < Pn; ++i)
        for (int l = 0; l < d; ++l) flat[(size_t)i * d + l] = idx[i][l];
      KC_TRY_HIP(hipMalloc(&g->idx, sizeof(int32_t) * flat.size()));
      KC_TRY_HIP(hipMemcpyAsync(g->idx, flat.data(), sizeof(int32_t) * flat.size(), hipMemcpyHostToDevice, st));
      double* Bd = (double*)ctx->ws.get(WS_GEMM_A, sizeof(double) * n_t * Pn);
      launch_gpc_basis(st, xi_train_dev, n_t, d, g->idx, Pn, basis, Bd);
      std::vector<double> B((size_t)n_t * Pn);
      KC_TRY_HIP(hipMemcpyAsync(B.data(), Bd, sizeof(double) * B.size(), hipMemcpyDeviceToHost, st));
      KC_TRY_HIP(hipStreamSynchronize(st));
      std::vector<double> Dm = snap->zeta_train, X;
      int r = householder_lstsq((int)n_t, Pn, snap->n_modes, B, Dm, X);
      KC_REQUIRE(r == KC_OK, KC_ERANK, "gPC design matrix is rank-deficient");
      KC_TRY_HIP(hipMalloc(&g->H, sizeof(double) * X.size()));
      KC_TRY_HIP(hipMemcpyAsync(g->H, X.data(), sizeof(double) * X.size(), hipMemcpyHostToDevice, st));
      KC_TRY_HIP(hipStreamSynchronize(st));
    } catch (...) {
      klecgc_gpc_free(g);
      throw;
    }
    *out = g;
    return KC_OK;
  });
}

int gpc_predict(klecgc_ctx* ctx, const klecgc_gpc* g, const double* xi_dev, int64_t M, double* U0_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(g && xi_dev && U0_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    return gpc_predict_impl(ctx, g, xi_dev, M, U0_dev);
  });
}

int fine_propagate(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                   const double* start_dev, int64_t M, double* end_dev, const uint8_t* active_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(prob && a_dev && start_dev && end_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_problem(*prob);
    KC_REQUIRE(start_dev != end_dev, KC_EINVAL, "start_dev and end_dev may not alias");
    FineArgs fa{a_dev, start_dev, nullptr, false, 0, active_dev, end_dev, M};
    return fine_propagate_impl(ctx, *prob, fa);
  });
}

int fine_propagate_noalloc(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                           const double* start_dev, int64_t M, double* end_dev, const uint8_t* active_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(prob && a_dev && start_dev && end_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_problem(*prob);
    KC_REQUIRE(start_dev != end_dev, KC_EINVAL, "start_dev and end_dev may not alias");
    KC_REQUIRE(ctx->scratch, KC_EHIP, "the device scratch array could not be resolved on this device");
    // the context's own workspace is set aside for the call; every slot comes from the scratch array
    struct ArenaScope {
      klecgc_ctx* c;
      Workspace saved;
      ArenaScope(klecgc_ctx* c_, void* base, size_t bytes) : c(c_) {
        saved = std::move(c->ws);
        c->ws = Workspace{};
        c->ws.arena = (char*)base;
        c->ws.arena_bytes = bytes;
      }
      ~ArenaScope() { c->ws = std::move(saved); }
    } scope(ctx, ctx->scratch, scratch_bytes());
    FineArgs fa{a_dev, start_dev, nullptr, false, 0, active_dev, end_dev, M};
    return fine_propagate_impl(ctx, *prob, fa);
  });
}

int cgc_diag_solve(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev, const double* r_dev,
                   int64_t M, double* u_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(prob && a_dev && r_dev && u_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_problem(*prob);
    const int64_t Nx = n_unknowns(*prob);
    const int K = prob->N / 2 + 1;
    double* spec = (double*)ctx->ws.get(WS_SPEC, sizeof(double) * 2 * M * K * Nx);
    timed(ctx, KT_FFT_FWD, [&] { launch_fft_forward(ctx->stream, *prob, r_dev, nullptr, M, spec); });
    int rc = shifted_solve_impl(ctx, *prob, a_dev, nullptr, M, spec);
    timed(ctx, KT_FFT_INV, [&] { launch_fft_inverse(ctx->stream, *prob, spec, nullptr, M, u_dev, false, nullptr); });
    return rc;
  });
}

int coarse_propagate(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev, const double* u0_dev,
                     int64_t M, double* U_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(prob && a_dev && U_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_problem(*prob);
    return coarse_sweep_impl(ctx, *prob, a_dev, u0_dev, M, U_dev);
  });
}

int serial_fine_propagate(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                          const double* u0_dev, int64_t M, double* U_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(prob && a_dev && U_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_problem(*prob);
    return serial_fine_impl(ctx, *prob, a_dev, u0_dev, M, U_dev);
  });
}

int parareal_solve_batch(klecgc_ctx* ctx, const klecgc_problem* base, const klecgc_task* tasks, int64_t M,
                         const double* a_dev, int32_t init, double* U_dev, int32_t flags, int32_t* iters_host,
                         int32_t* status_host, double* latency_ms_host, double* total_ms_host) {
  return guarded(ctx, [&] {
    KC_REQUIRE(base && tasks && a_dev && U_dev && iters_host && status_host, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    KC_REQUIRE((flags & ~(KC_BATCH_GRAPH | KC_BATCH_PROGRESS | KC_BATCH_PERSISTENT)) == 0, KC_EINVAL, "unknown flags");
    return parareal_batch_impl(ctx, *base, tasks, M, a_dev, init, U_dev, flags, iters_host, status_host,
                               latency_ms_host, total_ms_host);
  });
}

int parareal_solve(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev, const double* u0_dev,
                   int64_t M, int32_t init, const double* init_dev, const klecgc_gpc* gpc, klecgc_mlp* mlp,
                   const double* xi_dev, uint64_t seed, double* U_dev, int32_t* iters_host, int32_t* status_host,
                   double* delta_hist_host, int32_t* guess_host) {
  return guarded(ctx, [&] {
    KC_REQUIRE(prob && a_dev && U_dev && iters_host && status_host, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_problem(*prob);
    GuessArgs g{init, init_dev, gpc, mlp, xi_dev, seed};
    return parareal_impl(ctx, *prob, a_dev, u0_dev, M, g, U_dev, iters_host, status_host, delta_hist_host,
                         guess_host);
  });
}

int parareal_solve_sequential(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                              const double* u0_dev, int64_t M, int32_t init, const double* init_dev,
                              const klecgc_gpc* gpc, klecgc_mlp* mlp, const double* xi_dev, uint64_t seed,
                              double* U_dev, int32_t* iters_host, int32_t* status_host, double* delta_hist_host) {
  return guarded(ctx, [&] {
    KC_REQUIRE(prob && a_dev && U_dev && iters_host && status_host, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_problem(*prob);
    GuessArgs g{init, init_dev, gpc, mlp, xi_dev, seed};
    return parareal_seq_impl(ctx, *prob, a_dev, u0_dev, M, g, U_dev, iters_host, status_host, delta_hist_host);
  });
}

int model_fine_propagate(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev, const double* start_dev,
                         int64_t M, double* end_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(mp && c_dev && start_dev && end_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_model(*mp);
    KC_REQUIRE(start_dev != end_dev, KC_EINVAL, "start_dev and end_dev may not alias");
    return model_fine_impl(ctx, *mp, c_dev, start_dev, M, end_dev);
  });
}

int model_coarse_propagate(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev, const double* u0_dev,
                           int64_t M, double* U_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(mp && c_dev && U_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_model(*mp);
    return model_coarse_impl(ctx, *mp, c_dev, u0_dev, M, U_dev);
  });
}

int model_serial_fine(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev, const double* u0_dev, int64_t M,
                      double* U_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(mp && c_dev && U_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_model(*mp);
    return model_serial_fine_impl(ctx, *mp, c_dev, u0_dev, M, U_dev);
  });
}

int model_cgc_solve(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev, const double* Uk_dev,
                    const double* F_dev, int64_t M, double* Unew_dev, int32_t* newton_its_host) {
  return guarded(ctx, [&] {
    KC_REQUIRE(mp && c_dev && Uk_dev && F_dev && Unew_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_model(*mp);
    KC_REQUIRE(F_dev != Unew_dev, KC_EINVAL, "F_dev and Unew_dev may not alias");
    return model_cgc_impl(ctx, *mp, c_dev, Uk_dev, F_dev, M, Unew_dev, newton_its_host);
  });
}

static int model_solve_common(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev, const double* u0_dev,
                              int64_t M, int32_t init, const double* init_dev, const klecgc_gpc* gpc,
                              const double* xi_dev, uint64_t seed, const double* ref_dev, double* U_dev,
                              int32_t* iters_host, int32_t* status_host, double* delta_hist_host,
                              double* err_hist_host, bool sequential) {
  return guarded(ctx, [&] {
    KC_REQUIRE(mp && c_dev && U_dev && iters_host && status_host, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    validate_model(*mp);
    KC_REQUIRE(!err_hist_host || ref_dev, KC_EINVAL, "err_hist_host needs ref_dev");
    KC_REQUIRE(init != KC_INIT_GIVEN || init_dev, KC_EINVAL, "KC_INIT_GIVEN needs init_dev");
    ModelSolveArgs a{c_dev, u0_dev, M, GuessArgs{init, init_dev, gpc, nullptr, xi_dev, seed}, ref_dev, U_dev,
                     iters_host, status_host, delta_hist_host, err_hist_host, sequential};
    return model_parareal_impl(ctx, *mp, a);
  });
}

int model_parareal_solve(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev, const double* u0_dev,
                         int64_t M, int32_t init, const double* init_dev, const klecgc_gpc* gpc, const double* xi_dev,
                         uint64_t seed, const double* ref_dev, double* U_dev, int32_t* iters_host,
                         int32_t* status_host, double* delta_hist_host, double* err_hist_host) {
  return model_solve_common(ctx, mp, c_dev, u0_dev, M, init, init_dev, gpc, xi_dev, seed, ref_dev, U_dev, iters_host,
                            status_host, delta_hist_host, err_hist_host, false);
}

int model_parareal_solve_sequential(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev,
                                    const double* u0_dev, int64_t M, int32_t init, const double* init_dev,
                                    const klecgc_gpc* gpc, const double* xi_dev, uint64_t seed,
                                    const double* ref_dev, double* U_dev, int32_t* iters_host,
                                    int32_t* status_host, double* delta_hist_host, double* err_hist_host) {
  return model_solve_common(ctx, mp, c_dev, u0_dev, M, init, init_dev, gpc, xi_dev, seed, ref_dev, U_dev, iters_host,
                            status_host, delta_hist_host, err_hist_host, true);
}

int mlp_create(klecgc_ctx* ctx, int32_t n_in, int32_t hidden, int64_t n_out, klecgc_mlp** out, int64_t* n_params) {
  return guarded(ctx, [&] {
    KC_REQUIRE(out, KC_EINVAL, "null argument");
    *out = nullptr;
    int rc = mlp_create_impl(ctx, n_in, hidden, n_out, out);
    if (n_params) *n_params = mlp_param_count(*out);
    return rc;
  });
}

int mlp_set_params(klecgc_ctx* ctx, klecgc_mlp* h, const float* params_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(h && params_dev, KC_EINVAL, "null argument");
    return mlp_set_params_impl(ctx, h, params_dev);
  });
}

int mlp_get_params(klecgc_ctx* ctx, const klecgc_mlp* h, float* params_dev, float* mean_dev, float* std_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(h, KC_EINVAL, "null argument");
    int rc = mlp_get_params_impl(ctx, h, params_dev, mean_dev, std_dev);
    KC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    return rc;
  });
}

int mlp_normalize_targets(klecgc_ctx* ctx, klecgc_mlp* h, float* Y_dev, int64_t n) {
  return guarded(ctx, [&] {
    KC_REQUIRE(h && Y_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(n >= 1, KC_EINVAL, "n must be >= 1");
    return mlp_normalize_impl(ctx, h, Y_dev, n);
  });
}

int mlp_train(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi_dev, const float* Y_dev, int64_t n, int32_t epochs,
              int32_t batch, float lr, float lr_final, const int32_t* perm_dev, float* loss_host) {
  return guarded(ctx, [&] {
    KC_REQUIRE(h && xi_dev && Y_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(n >= 1, KC_EINVAL, "n must be >= 1");
    return mlp_train_impl(ctx, h, xi_dev, Y_dev, n, epochs, batch, lr, lr_final, perm_dev, loss_host);
  });
}

int mlp_predict(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi_dev, int64_t M, float* Y_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(h && xi_dev && Y_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(M >= 1, KC_EINVAL, "M must be >= 1");
    return mlp_predict_impl(ctx, h, xi_dev, M, Y_dev);
  });
}

int mlp_grad(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi_dev, const float* Y_dev, int64_t n, float* grads_dev,
             double* loss_host) {
  return guarded(ctx, [&] {
    KC_REQUIRE(h && xi_dev && Y_dev, KC_EINVAL, "null argument");
    return mlp_grad_impl(ctx, h, xi_dev, Y_dev, n, grads_dev, loss_host);
  });
}

int grid_restrict(klecgc_ctx* ctx, int32_t n, int32_t nc, const double* U_dev, int64_t R, float* Yc_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(U_dev && Yc_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(n >= 1 && nc >= 1 && R >= 1, KC_EINVAL, "n, nc and R must be >= 1");
    return grid_restrict_impl(ctx, n, nc, U_dev, R, Yc_dev);
  });
}

int mlp_initial_guess(klecgc_ctx* ctx, klecgc_mlp* h, int32_t n, int32_t nc, int32_t N, const double* xi_dev,
                      int64_t M, double* U0_dev) {
  return guarded(ctx, [&] {
    KC_REQUIRE(h && xi_dev && U0_dev, KC_EINVAL, "null argument");
    KC_REQUIRE(n >= 1 && nc >= 1 && N >= 1 && M >= 1, KC_EINVAL, "n, nc, N and M must be >= 1");
    return mlp_initial_guess_impl(ctx, h, n, nc, N, xi_dev, M, U0_dev);
  });
}

}  // extern "C"
