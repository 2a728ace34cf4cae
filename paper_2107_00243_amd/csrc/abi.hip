// C-ABI entry points: argument validation, workspace carving and launch
// sequencing of the preconditioned log-likelihood estimator (Algorithms 1 and 2).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "gpmll_impl.h"

namespace gpmll {

hipError_t launch_stage_x(const Ctx& c, const Hyper& h);
hipError_t launch_stage_x_bwd(const Ctx& c, const Hyper& h);
hipError_t launch_cg_after_product(const Ctx& c, const Hyper& h, int it, double tol);
hipError_t launch_slq_logp(const Ctx& c, const Hyper& h, const double* y, double* logp);
hipError_t launch_backward(const Ctx& c, const Hyper& h, int ard, int precond_grad, int precond_kind, double* grad);

static size_t al(size_t x) { return (x + 255) / 256 * 256; }
static int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

Layout make_layout(int64_t n, int d, int ard, int num_probes, int max_iters, int rank, int prec, int probe_mode) {
  Layout L{};
  L.n = n;
  L.n_pad = rup(n, kRowBlock);
  L.d = d;
  L.p = ard ? d : 1;
  L.ell = num_probes;
  L.t = 1 + num_probes;
  {
    // tile counts with compiled tile kernels
    static const int ntts[] = {1, 2, 3, 4, 5, 6, 8, 12, 16};
    int need = (L.t + 15) / 16, ntt = 16;
    for (int v : ntts)
      if (v >= need) {
        ntt = v;
        break;
      }
    L.tp = 16 * ntt;
  }
  L.k = rank;
  L.max_iters = max_iters;
  L.prec = prec;
  L.bprec = prec == GP_PREC_FP64 ? GP_PREC_FP64 : GP_PREC_FP32;
  if (prec == GP_PREC_BF16X3 || prec == GP_PREC_FP16X3) {
    const int dq = (d + 7) / 8 * 8;
    L.kd = (int)rup(4 * dq, 32);
  } else {
    const int nk4 = (d + 3) / 4;
    L.kd = 4 * (nk4 <= 1 ? 1 : nk4 <= 2 ? 2 : nk4 <= 4 ? 4 : 8);
  }
  L.bkd = (int)rup(d, 4);
  L.bow = (2 * d + 1 + 15) / 16 * 16 + 16;
  L.nrb = (int)(L.n_pad / kRowBlock);
  // Column splits: the tile grid (row blocks x splits) runs in rounds of
  // kWgSlots resident workgroups (two per CU on the 256 CUs); take the fewest
  // splits that give at least two rounds with the last round >= 95 % full, else
  // the best-filled count (every split non-empty, >= 256 columns).
  const int ntt_full = L.tp / 16;
  const int64_t rows_wg = (prec == GP_PREC_BF16X3 || prec == GP_PREC_FP16X3)
                              ? kRowBlock
                              : 64 * fp_row_groups(prec == GP_PREC_FP64 ? 8 : 4, ntt_full);
  const int64_t nrbk = L.n_pad / rows_wg;
  const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(32, L.n_pad / 256));
  int64_t want = smax;
  double best = -1.0;
  for (int64_t s = 1; s <= smax; ++s) {
    const double rounds = (double)(nrbk * s) / kWgSlots;
    const double eff = rounds / std::ceil(rounds);
    if (rounds >= 2.0 && eff >= 0.95) {
      want = s;
      break;
    }
    if (eff > best + 1e-12 && rounds >= 1.0) {
      best = eff;
      want = s;
    }
  }
  int64_t cps = rup((L.n_pad + want - 1) / want, 256);
  if (cps < 256) cps = 256;
  L.cols_per_split = cps;
  L.nsplit = (int)((L.n_pad + cps - 1) / cps);
  L.nchunk = (int)((n + kChunkRows - 1) / kChunkRows);
  // L^T R: about 512 row chunks (two workgroups per CU per l-group), >= 64 rows each
  L.ltr_rows = std::max<int64_t>(64, rup((n + 511) / 512, 16));
  L.nchunk_ltr = (int)((n + L.ltr_rows - 1) / L.ltr_rows);
  // row-parallel reductions: about 128 rows per workgroup, at most 1024 workgroups
  L.nred = (int)std::min<int64_t>(1024, (n + 127) / 128);

  const int64_t np = L.n_pad, tp = L.tp, k = rank;
  const int64_t kk = std::max<int64_t>(k, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += al(bytes ? bytes : 1);
    return o;
  };
  const bool split16 = prec == GP_PREC_BF16X3 || prec == GP_PREC_FP16X3;
  const size_t esz = prec == GP_PREC_FP64 ? 8 : (prec == GP_PREC_FP32 ? 4 : 2);
  const size_t bsz = L.bprec == GP_PREC_FP64 ? 8 : 4;
  // preconditioner block: offsets depend on (n, d, rank) only, so a preconditioner
  // built by gp_precond_build sits where every later call expects it
  L.xs = take(np * d * 8);
  L.mean = take(GP_MAX_D * 8);
  L.mean_part = take((size_t)L.nred * GP_MAX_D * 8);
  L.L = take(n * k * 8);
  L.diag = take(n * 8);
  L.ispiv = take(n);
  L.piv = take(kk * 4);
  L.amax = take(2 * ((n + 255) / 256) * 16);
  L.C = take(kk * kk * 8);
  L.Rc = take(kk * kk * 8);
  L.Rinv = take(kk * kk * 8);
  L.Cinv = take(kk * kk * 8);
  L.logdetP = take(8);
  L.scal_small = take(64);
  L.flags = take(64);
  L.ltr_part = take((size_t)L.nchunk * kk * kk * 8);
  L.freq = take((size_t)(kk / 2 + 1) * GP_MAX_D * 8);
  L.landmarks = take(kk * 4);
  L.famp = take((kk / 2 + 1) * 8);
  L.lf_ltr = take(k > 0 ? rup(n, 64) * rup(k, 16) * 8 : 0);
  L.precond_end = off;
  // estimator block
  L.xfa = take(np * L.kd * esz);
  L.xfb = take(np * L.kd * esz);
  L.rowterm = take(np * (prec == GP_PREC_FP64 ? 8 : 4));
  L.colterm = take(np * (prec == GP_PREC_FP64 ? 8 : 4));
  L.H = take(kk * num_probes * 8);
  L.Y = take(rup(kk, 64) * tp * 8);  // rows past k zero (whole LDS chunks in the z-apply)
  L.ltr = take(kk * tp * 8);
  L.ltr_raw = take(kk * tp * 8);
  L.ltr_part2 = take((size_t)L.nchunk_ltr * rup(kk, 16) * tp * 8);
  L.Xs = take(np * tp * 8);
  L.R = take(np * tp * 8);
  L.Z0 = take(np * tp * 8);
  L.Pd = take(np * tp * 8);
  L.W = take(np * tp * 8);
  L.vfrag = take(np * tp * (split16 ? 6 : esz));  // up to three 16-bit pieces
  L.vx = take(split16 ? np * 4 : 0);
  L.vscale = take(2 * tp * 4);
  L.wpart = take((size_t)L.nsplit * np * std::max<int64_t>(tp * (prec == GP_PREC_FP64 ? 8 : 4), L.bow * bsz));
  L.rho = take(tp * 8);
  L.rho0 = take(tp * 8);
  L.bnorm = take(tp * 8);
  L.rnorm2 = take(tp * 8);
  L.pw = take(2 * tp * 8);
  L.active = take(tp * 4);
  L.nactive = take(16);
  L.iters = take(tp * 4);
  L.colmap = take(tp * 4);
  L.alog = take(tp * max_iters * 8);
  L.blog = take(tp * max_iters * 8);
  const int64_t nb64 = (n + 63) / 64, nb256 = (n + 255) / 256;
  L.dot_part = take((L.nred + 2 * nb64 + nb256) * tp * 8);
  L.gamma = take((num_probes + 4) * 8);
  L.slq_work = take((size_t)num_probes * 3 * max_iters * 8);
  L.cprime = take(np * tp * 8);
  L.bxa = take(np * L.bkd * bsz);
  L.bxb = take(np * L.bkd * bsz);
  L.brt = take(np * bsz);
  L.bct = take(np * bsz);
  const size_t frag_row = std::max<size_t>(tp * bsz, (size_t)bwd_nkm(L.t) * 64);  // bytes per row
  L.bafrag = take(np * frag_row);
  L.bcfrag = take(np * frag_row);
  L.bxaug = take(np * ((2 * d + 1 + 15) / 16 * 16) * bsz);
  L.bwd_part = take(nb256 * (GP_MAX_D + 1) * 8);
  L.pg_small = take((4 * kk * kk + kk * tp) * 8);
  L.omega = take(n * k * 8);
  L.pg_part = take(((n + k + 255) / 256 + 1) * (GP_MAX_D + 1) * 8);
  L.sqrt_work = take(probe_mode == 1 ? 6 * kk * kk * 8 : 0);
  L.total = off;
  return L;
}

}  // namespace gpmll

using namespace gpmll;

struct gp_precond {
  Layout lay;
  char* ws;
  std::vector<double> theta;
  gp_problem prob;
  int kind = kPivChol;
};

static thread_local int g_last_hip = 0;

#define HIPCHK(expr)                    \
  do {                                  \
    hipError_t _e = (expr);             \
    if (_e != hipSuccess) {             \
      g_last_hip = (int)_e;             \
      return GP_EHIP;                   \
    }                                   \
  } while (0)

static int check_device() {
  static std::mutex mu;
  static std::vector<int> ok;  // per device: 0 unknown, 1 gfx950, -1 other
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)ok.size() <= dev) ok.resize(dev + 1, 0);
  if (ok[dev] == 0) {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    ok[dev] = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
  }
  return ok[dev] == 1 ? GP_OK : GP_EUNSUPPORTED;
}

int gpmll::gpmll_check_device() { return check_device(); }
void gpmll::gpmll_set_hip_error(int e) { g_last_hip = e; }

static int check_problem(const gp_problem* prob) {
  if (!prob || !prob->X_dev || !prob->y_dev) return GP_EINVAL;
  if (prob->n < 1 || prob->d < 1 || prob->d > GP_MAX_D) return GP_EINVAL;
  if (prob->kernel < 0 || prob->kernel > 3) return GP_EINVAL;
  if (prob->kernel == GP_KERNEL_RATQUAD && !(prob->kernel_shape > 0.0 && std::isfinite(prob->kernel_shape)))
    return GP_EINVAL;
  if (prob->ard != 0 && prob->ard != 1) return GP_EINVAL;
  if (prob->n > ((int64_t)1 << 31) - 256) return GP_EINVAL;
  return GP_OK;
}

static int check_options(const gp_options* o) {
  if (!o) return GP_EINVAL;
  if (o->precision < 0 || o->precision > 3) return GP_EINVAL;
  if (o->num_probes < 1 || o->num_probes > GP_MAX_PROBES) return GP_EINVAL;
  if (o->max_iters < 1 || o->max_iters > 100000) return GP_EINVAL;
  if (!(o->cg_tol >= 0.0) || !std::isfinite(o->cg_tol)) return GP_EINVAL;
  if (o->precond_grad != 0 && o->precond_grad != 1) return GP_EINVAL;
  if (o->sync_every < 0) return GP_EINVAL;
  if (o->probe_mode != 0 && o->probe_mode != 1) return GP_EINVAL;
  return GP_OK;
}

static int check_rank(const gp_problem* prob, int32_t rank) {
  if (rank < 0 || rank > GP_MAX_RANK || (int64_t)rank > prob->n) return GP_EINVAL;
  return GP_OK;
}

static int make_hyper(const gp_problem* prob, const double* theta, Hyper* h) {
  if (!theta) return GP_EINVAL;
  const int p = prob->ard ? prob->d : 1;
  for (int i = 0; i < p + 2; ++i)
    if (!(theta[i] > 0.0) || !std::isfinite(theta[i])) return GP_EINVAL;
  std::memset(h, 0, sizeof(*h));
  h->kind = prob->kernel;
  h->d = prob->d;
  for (int j = 0; j < prob->d; ++j) h->inv_ls[j] = 1.0 / theta[prob->ard ? j : 0];
  h->s = theta[p];
  h->s2 = theta[p + 1];
  h->log2s = std::log2(h->s);
  h->alpha = prob->kernel == GP_KERNEL_RATQUAD ? prob->kernel_shape : 1.0;
  return GP_OK;
}

static int check_ws(void* ws, size_t ws_bytes, const Layout& L) {
  if (!ws) return GP_EINVAL;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return GP_EINVAL;
  if (ws_bytes < L.total) return GP_EWORKSPACE;
  return GP_OK;
}

#define RET_IF(x)            \
  do {                       \
    int _r = (x);            \
    if (_r != GP_OK) return _r; \
  } while (0)

extern "C" int gp_workspace_size(const gp_problem* prob, const gp_options* opt, int32_t rank, size_t* bytes) {
  if (!bytes) return GP_EINVAL;
  if (!prob || prob->n < 1 || prob->d < 1 || prob->d > GP_MAX_D) return GP_EINVAL;
  RET_IF(check_options(opt));
  RET_IF(check_rank(prob, rank));
  Layout L = make_layout(prob->n, prob->d, prob->ard, opt->num_probes, opt->max_iters, rank, opt->precision,
                         opt->probe_mode);
  *bytes = L.total;
  return GP_OK;
}

static int build_precond(const gp_problem* prob, const Hyper& h, const Ctx& c) {
  HIPCHK(launch_prep(c, prob->X_dev, h));
  HIPCHK(launch_pivchol(c, h));
  HIPCHK(launch_precond_finish(c, h));
  return GP_OK;
}

extern "C" int gp_precond_build(const gp_problem* prob, const double* theta_host, int32_t rank, void* ws_dev,
                                size_t ws_bytes, hipStream_t stream, gp_precond** out) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  RET_IF(check_problem(prob));
  RET_IF(check_rank(prob, rank));
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  RET_IF(check_device());
  // the preconditioner block of the layout does not depend on the estimator options
  Layout L = make_layout(prob->n, prob->d, prob->ard, 1, 1, rank, GP_PREC_FP64);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 255) != 0) return GP_EINVAL;
  if (ws_bytes < L.precond_end) return GP_EWORKSPACE;
  Ctx c{&L, (char*)ws_dev, stream};
  gpmll_forget_forward(ws_dev);
  HIPCHK(hipMemsetAsync(c.at<int>(L.flags), 0, 64, stream));
  RET_IF(build_precond(prob, h, c));
  gp_precond* P = new gp_precond;
  P->lay = L;
  P->ws = (char*)ws_dev;
  P->prob = *prob;
  const int p = prob->ard ? prob->d : 1;
  P->theta.assign(theta_host, theta_host + p + 2);
  *out = P;
  return GP_OK;
}

extern "C" int gp_precond_build_rff(const gp_problem* prob, const double* theta_host, int32_t rank,
                                    const double* freq_dev, void* ws_dev, size_t ws_bytes, hipStream_t stream,
                                    gp_precond** out) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  RET_IF(check_problem(prob));
  RET_IF(check_rank(prob, rank));
  if (rank < 2 || rank % 2 != 0 || !freq_dev) return GP_EINVAL;
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  RET_IF(check_device());
  Layout L = make_layout(prob->n, prob->d, prob->ard, 1, 1, rank, GP_PREC_FP64);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 255) != 0) return GP_EINVAL;
  if (ws_bytes < L.precond_end) return GP_EWORKSPACE;
  Ctx c{&L, (char*)ws_dev, stream};
  gpmll_forget_forward(ws_dev);
  HIPCHK(hipMemsetAsync(c.at<int>(L.flags), 0, 64, stream));
  // the samples are copied into the workspace, so the handle does not keep freq_dev
  HIPCHK(hipMemcpyAsync(c.at<double>(L.freq), freq_dev, (size_t)(rank / 2) * prob->d * sizeof(double),
                        hipMemcpyDeviceToDevice, stream));
  HIPCHK(launch_prep(c, prob->X_dev, h));
  HIPCHK(launch_rff(c, h));
  HIPCHK(launch_precond_finish(c, h));
  gp_precond* P = new gp_precond;
  P->lay = L;
  P->ws = (char*)ws_dev;
  P->prob = *prob;
  P->kind = kRff;
  const int p = prob->ard ? prob->d : 1;
  P->theta.assign(theta_host, theta_host + p + 2);
  *out = P;
  return GP_OK;
}

extern "C" int gp_precond_build_nystrom(const gp_problem* prob, const double* theta_host, int32_t rank,
                                        const int32_t* landmarks_host, void* ws_dev, size_t ws_bytes,
                                        hipStream_t stream, gp_precond** out) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  RET_IF(check_problem(prob));
  RET_IF(check_rank(prob, rank));
  if (rank < 1 || !landmarks_host) return GP_EINVAL;
  {
    std::vector<int32_t> s(landmarks_host, landmarks_host + rank);
    std::sort(s.begin(), s.end());
    if (s.front() < 0 || (int64_t)s.back() >= prob->n) return GP_EINVAL;
    if (std::adjacent_find(s.begin(), s.end()) != s.end()) return GP_EINVAL;
  }
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  RET_IF(check_device());
  Layout L = make_layout(prob->n, prob->d, prob->ard, 1, 1, rank, GP_PREC_FP64);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 255) != 0) return GP_EINVAL;
  if (ws_bytes < L.precond_end) return GP_EWORKSPACE;
  Ctx c{&L, (char*)ws_dev, stream};
  gpmll_forget_forward(ws_dev);
  HIPCHK(hipMemsetAsync(c.at<int>(L.flags), 0, 64, stream));
  // the landmark table comes from pageable host memory: wait for the copy once
  HIPCHK(hipMemcpyAsync(c.at<int32_t>(L.landmarks), landmarks_host, (size_t)rank * sizeof(int32_t),
                        hipMemcpyHostToDevice, stream));
  HIPCHK(hipStreamSynchronize(stream));
  HIPCHK(launch_prep(c, prob->X_dev, h));
  HIPCHK(launch_pivchol(c, h, c.at<int32_t>(L.landmarks)));
  HIPCHK(launch_precond_finish(c, h));
  gp_precond* P = new gp_precond;
  P->lay = L;
  P->ws = (char*)ws_dev;
  P->prob = *prob;
  const int p = prob->ard ? prob->d : 1;
  P->theta.assign(theta_host, theta_host + p + 2);
  *out = P;
  return GP_OK;
}

// Gauss rule of the standard normal with q points (probabilists' Hermite
// polynomials He_0 = 1, He_1 = x, He_{k+1} = x He_k - k He_{k-1}): nodes are the
// eigenvalues of the Jacobi matrix (zero diagonal, off-diagonal sqrt(k)), found by
// Sturm-sequence bisection and polished by Newton steps on He_q; weights
// q! / (q He_{q-1}(x))^2 (Christoffel numbers, summing to 1).  Nodes ascending.
static void hermite_pair(int q, double x, double* hq, double* hq1) {
  double a = 1.0, b = x;  // He_0, He_1
  for (int k = 1; k < q; ++k) {
    const double c = x * b - k * a;
    a = b;
    b = c;
  }
  *hq = b;   // He_q
  *hq1 = a;  // He_{q-1}
}

static void gauss_hermite_normal(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  // eigenvalues below t = negative pivots of the LDL^T factorisation of J - t I
  // (an exact zero pivot is taken as -0, i.e. t as slightly larger)
  auto below = [q](double t) {
    int cnt = 0;
    double dk = -t;
    for (int k = 0;; ++k) {
      if (dk == 0.0) dk = -1e-300;
      if (dk < 0.0) ++cnt;
      if (k + 1 == q) break;
      dk = -t - (double)(k + 1) / dk;
    }
    return cnt;
  };
  const double bound = 2.0 * std::sqrt((double)q) + 2.0;
  for (int i = 0; i < q; ++i) {
    double lo = -bound, hi = bound;  // below(lo) <= i < below(hi)
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo)); ++it) {
      const double mid = 0.5 * (lo + hi);
      if (below(mid) <= i) lo = mid;
      else hi = mid;
    }
    double xi = 0.5 * (lo + hi);
    for (int it = 0; it < 3; ++it) {
      double hq, hq1;
      hermite_pair(q, xi, &hq, &hq1);
      if (hq1 != 0.0) xi -= hq / (q * hq1);
    }
    double hq, hq1;
    hermite_pair(q, xi, &hq, &hq1);
    x[i] = xi;
    w[i] = std::exp(std::lgamma(q + 1.0) - 2.0 * std::log((double)q) - 2.0 * std::log(std::fabs(hq1)));
  }
}

extern "C" int gp_precond_build_qff(const gp_problem* prob, const double* theta_host, int32_t nodes_per_dim,
                                    void* ws_dev, size_t ws_bytes, hipStream_t stream, gp_precond** out) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  RET_IF(check_problem(prob));
  const int q = nodes_per_dim;
  if (q < 2 || q % 2 != 0 || q > 64) return GP_EINVAL;  // He_{q-1} stays in range up to q = 64
  int64_t rank64 = 1;
  for (int j = 0; j < prob->d; ++j) {
    rank64 *= q;
    if (rank64 > GP_MAX_RANK) return GP_EINVAL;
  }
  const int rank = (int)rank64;
  RET_IF(check_rank(prob, rank));
  if (prob->kernel != GP_KERNEL_RBF) return GP_EUNSUPPORTED;
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  RET_IF(check_device());
  Layout L = make_layout(prob->n, prob->d, prob->ard, 1, 1, rank, GP_PREC_FP64);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 255) != 0) return GP_EINVAL;
  if (ws_bytes < L.precond_end) return GP_EWORKSPACE;
  // tensor grid, first coordinate over the q/2 negative nodes (one of each +- pair,
  // weight doubled), lexicographic with the first coordinate slowest
  std::vector<double> gx, gw;
  gauss_hermite_normal(q, gx, gw);
  const int m = rank / 2, d = prob->d;
  std::vector<double> W((size_t)m * d), amp(m);
  for (int r = 0; r < m; ++r) {
    int rem = r;
    double wt = 2.0;
    for (int j = d - 1; j >= 0; --j) {
      const int base = (j == 0) ? q / 2 : q;
      const int idx = rem % base;
      rem /= base;
      W[(size_t)r * d + j] = gx[idx];
      wt *= gw[idx];
    }
    amp[r] = std::sqrt(h.s * wt);
  }
  Ctx c{&L, (char*)ws_dev, stream};
  gpmll_forget_forward(ws_dev);
  HIPCHK(hipMemsetAsync(c.at<int>(L.flags), 0, 64, stream));
  HIPCHK(hipMemcpyAsync(c.at<double>(L.freq), W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(c.at<double>(L.famp), amp.data(), amp.size() * sizeof(double), hipMemcpyHostToDevice,
                        stream));
  HIPCHK(hipStreamSynchronize(stream));  // the host tables are locals
  HIPCHK(launch_prep(c, prob->X_dev, h));
  HIPCHK(launch_rff(c, h, true));
  HIPCHK(launch_precond_finish(c, h));
  gp_precond* P = new gp_precond;
  P->lay = L;
  P->ws = (char*)ws_dev;
  P->prob = *prob;
  P->kind = kRff;
  const int p = prob->ard ? prob->d : 1;
  P->theta.assign(theta_host, theta_host + p + 2);
  *out = P;
  return GP_OK;
}

extern "C" int gp_precond_view_of(const gp_precond* P, gp_precond_view* view) {
  if (!P || !view) return GP_EINVAL;
  view->L_dev = reinterpret_cast<const double*>(P->ws + P->lay.L);
  view->pivots_dev = reinterpret_cast<const int32_t*>(P->ws + P->lay.piv);
  view->logdet_dev = reinterpret_cast<const double*>(P->ws + P->lay.logdetP);
  view->n = P->lay.n;
  view->rank = P->lay.k;
  return GP_OK;
}

extern "C" void gp_precond_free(gp_precond* P) {
  if (P) gpmll_forget_forward(P->ws);  // a forward pass made with this handle is not reused after it
  delete P;
}

// The CG iterations of one call on the right-hand sides already in R (one CG run
// with many right-hand sides, footnote to Section 4.4).  With the host polling the
// active-column count, the product of an iteration runs only over the active
// columns, packed to the fewest 16-column tiles (the count read last is an upper
// bound: columns only ever stop).
static int run_cg(const Ctx& c, const Hyper& h, const gp_options* opt) {
  const Layout& L = *c.lay;
  int* nact = c.at<int>(L.nactive);
  const int q = opt->sync_every;
  int host_nact = L.t;
  for (int it = 0; it < opt->max_iters; ++it) {
    if (q > 0 && it > 0 && it % q == 0) {
      HIPCHK(hipMemcpyAsync(&host_nact, nact, sizeof(int), hipMemcpyDeviceToHost, c.st));
      HIPCHK(hipStreamSynchronize(c.st));
      if (host_nact == 0) break;
    }
    TilePlan plan = tile_plan(L, L.t);
    const int* cmap = nullptr;
    if (q > 0) {
      plan = tile_plan(L, host_nact);
      HIPCHK(launch_colmap(c));
      cmap = c.at<int>(L.colmap);
    }
    if (L.prec == GP_PREC_BF16X3 && it < kBf16V3Iters && bf16_v3_fits(plan.ntt)) plan.vp = 3;
    const int nstaged = 16 * plan.ntt + plan.xc;
    HIPCHK(launch_stage_v(c, c.at<double>(L.Pd), L.tp, nstaged, h, cmap, plan));
    HIPCHK(launch_khat_tiles(c, h, nact, plan));
    HIPCHK(launch_khat_reduce(c, c.at<double>(L.Pd), L.tp, c.at<double>(L.W), L.tp, nstaged, h,
                              c.at<double>(L.dot_part), nact, cmap, L.tp));
    HIPCHK(launch_cg_after_product(c, h, it, opt->cg_tol));
  }
  return GP_OK;
}

// A prebuilt preconditioner must come from the same problem, theta, rank and
// workspace; then only the per-evaluation flags are cleared.  Otherwise the
// pivoted Cholesky preconditioner is built in the workspace.
static int check_precond_handle(const gp_problem* prob, const double* theta_host, int32_t rank, const gp_precond* P,
                                const Ctx& c) {
  const Layout& L = *c.lay;
  const int p = prob->ard ? prob->d : 1;
  if (P->ws != c.ws || P->lay.k != rank || P->lay.n != prob->n || P->lay.d != prob->d || P->lay.L != L.L ||
      P->lay.Cinv != L.Cinv || P->prob.X_dev != prob->X_dev)
    return GP_EINVAL;
  for (int i = 0; i < p + 2; ++i)
    if (P->theta[i] != theta_host[i]) return GP_EINVAL;
  return GP_OK;
}

static int use_or_build_precond(const gp_problem* prob, const double* theta_host, int32_t rank, gp_precond* P,
                                const Hyper& h, const Ctx& c) {
  const Layout& L = *c.lay;
  if (P) {
    RET_IF(check_precond_handle(prob, theta_host, rank, P, c));
    // keep flags[1] (a build-time status); clear the per-evaluation flags
    HIPCHK(hipMemsetAsync(c.at<int>(L.flags), 0, 4, c.st));
    HIPCHK(hipMemsetAsync(c.at<int>(L.flags) + 2, 0, 56, c.st));
    return GP_OK;
  }
  HIPCHK(hipMemsetAsync(c.at<int>(L.flags), 0, 64, c.st));
  return build_precond(prob, h, c);
}

// The last forward-only pass (gp_mll_eval) completed on each workspace (host-side
// record).  A gp_mll_grad with the same problem, theta, options, rank,
// preconditioner handle and stream finds the solves, the CG coefficients and the
// preconditioner still in the workspace and runs only the derivative part.  Every
// other call that writes into a workspace forgets its record first.
namespace {
struct ForwardRecord {
  gp_problem prob;
  std::vector<double> theta;
  gp_options opt;
  int32_t rank;
  const gp_precond* P;
  hipStream_t stream;
};
std::mutex g_fwd_mu;
std::map<const void*, ForwardRecord> g_fwd;

bool same_options(const gp_options& a, const gp_options& b) {
  return a.precision == b.precision && a.num_probes == b.num_probes && a.max_iters == b.max_iters &&
         a.cg_tol == b.cg_tol && a.seed == b.seed && a.precond_grad == b.precond_grad &&
         a.sync_every == b.sync_every && a.probe_mode == b.probe_mode;
}

bool same_problem(const gp_problem& a, const gp_problem& b) {
  return a.X_dev == b.X_dev && a.y_dev == b.y_dev && a.n == b.n && a.d == b.d && a.kernel == b.kernel &&
         a.ard == b.ard && (a.kernel != GP_KERNEL_RATQUAD || a.kernel_shape == b.kernel_shape);
}

bool forward_matches(const void* ws, const gp_problem* prob, const double* theta, const gp_options* opt,
                     int32_t rank, const gp_precond* P, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_fwd_mu);
  auto it = g_fwd.find(ws);
  if (it == g_fwd.end()) return false;
  const ForwardRecord& r = it->second;
  if (!same_problem(r.prob, *prob) || !same_options(r.opt, *opt) || r.rank != rank || r.P != P ||
      r.stream != stream)
    return false;
  for (size_t i = 0; i < r.theta.size(); ++i)
    if (r.theta[i] != theta[i]) return false;
  return true;
}

void forward_remember(const void* ws, const gp_problem* prob, const double* theta, const gp_options* opt,
                      int32_t rank, const gp_precond* P, hipStream_t stream) {
  const int p = prob->ard ? prob->d : 1;
  std::lock_guard<std::mutex> lk(g_fwd_mu);
  g_fwd[ws] = ForwardRecord{*prob, std::vector<double>(theta, theta + p + 2), *opt, rank, P, stream};
}
}  // namespace

void gpmll::gpmll_forget_forward(const void* ws) {
  std::lock_guard<std::mutex> lk(g_fwd_mu);
  g_fwd.erase(ws);
}

static int run_estimator(const gp_problem* prob, const double* theta_host, const gp_options* opt, int32_t rank,
                         gp_precond* P, void* ws_dev, size_t ws_bytes, hipStream_t stream, double* logp_dev,
                         double* grad_dev, gp_stats* stats) {
  RET_IF(check_problem(prob));
  RET_IF(check_options(opt));
  RET_IF(check_rank(prob, rank));
  if (!logp_dev) return GP_EINVAL;
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  RET_IF(check_device());
  Layout L = make_layout(prob->n, prob->d, prob->ard, opt->num_probes, opt->max_iters, rank, opt->precision,
                         opt->probe_mode);
  RET_IF(check_ws(ws_dev, ws_bytes, L));
  Ctx c{&L, (char*)ws_dev, stream};
  if (P) RET_IF(check_precond_handle(prob, theta_host, rank, P, c));
  const bool resume = grad_dev && forward_matches(ws_dev, prob, theta_host, opt, rank, P, stream);
  gpmll_forget_forward(ws_dev);
  if (!resume) {
    RET_IF(use_or_build_precond(prob, theta_host, rank, P, h, c));
    HIPCHK(launch_stage_x(c, h));
    if (opt->probe_mode == 1) HIPCHK(launch_probes_sqrt(c, prob->y_dev, h, opt->seed));
    else HIPCHK(launch_probes(c, prob->y_dev, h, opt->seed));
    HIPCHK(launch_cg_init(c, h));
    RET_IF(run_cg(c, h, opt));
  }
  // (after a matching forward pass only log p is rewritten from the stored coefficients)
  if (resume) HIPCHK(hipMemsetAsync(c.at<int>(L.flags) + 2, 0, 4, stream));  // the Ritz clamps are recounted
  HIPCHK(launch_slq_logp(c, h, prob->y_dev, logp_dev));
  if (grad_dev) {
    HIPCHK(launch_stage_x_bwd(c, h));
    HIPCHK(launch_backward(c, h, prob->ard, opt->precond_grad, P ? P->kind : kPivChol, grad_dev));
  }
  if (stats) {
    int flags[4];
    HIPCHK(hipMemcpyAsync(flags, c.at<int>(L.flags), sizeof(flags), hipMemcpyDeviceToHost, stream));
    int small[2];
    HIPCHK(hipMemcpyAsync(small, c.at<int>(L.scal_small), sizeof(small), hipMemcpyDeviceToHost, stream));
    std::vector<int> it(L.tp);
    HIPCHK(hipMemcpyAsync(it.data(), c.at<int>(L.iters), L.tp * sizeof(int), hipMemcpyDeviceToHost, stream));
    std::vector<double> sl(L.ell + 2);
    HIPCHK(hipMemcpyAsync(sl.data(), c.at<double>(L.gamma), sl.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
    double ldp = 0.0;
    HIPCHK(hipMemcpyAsync(&ldp, c.at<double>(L.logdetP), sizeof(double), hipMemcpyDeviceToHost, stream));
    std::vector<double> rn(L.tp), bn(L.tp);
    HIPCHK(hipMemcpyAsync(rn.data(), c.at<double>(L.rnorm2), L.tp * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipMemcpyAsync(bn.data(), c.at<double>(L.bnorm), L.tp * sizeof(double), hipMemcpyDeviceToHost, stream));
    std::vector<int32_t> pv(std::max(1, rank));
    if (rank > 0)
      HIPCHK(hipMemcpyAsync(pv.data(), c.at<int32_t>(L.piv), rank * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (flags[1] != 0) return flags[1];
    stats->num_columns = L.t;
    int mx = 0;
    for (int i = 0; i < L.t; ++i) mx = std::max(mx, it[i]);
    stats->iters_max = mx;
    stats->rank_achieved = rank > 0 ? small[1] : 0;
    stats->flags = flags[0];
    stats->ritz_clamped = flags[2];
    stats->logdet_precond = ldp;
    stats->datafit = sl[L.ell];
    stats->logdet_estimate = sl[L.ell + 1];
    if (stats->col_iters_host)
      for (int i = 0; i < L.t; ++i) stats->col_iters_host[i] = it[i];
    if (stats->gammas_host)
      for (int i = 0; i < L.ell; ++i) stats->gammas_host[i] = sl[i];
    if (stats->rel_residual_host)
      for (int i = 0; i < L.t; ++i) stats->rel_residual_host[i] = bn[i] > 0.0 ? rn[i] / bn[i] : 0.0;
    if (stats->pivots_host)
      for (int i = 0; i < rank; ++i) stats->pivots_host[i] = pv[i];
  }
  // only a forward-only call leaves a record: a gp_mll_grad always recomputes after
  // another gp_mll_grad, so repeated identical calls each do the whole evaluation
  if (!grad_dev) forward_remember(ws_dev, prob, theta_host, opt, rank, P, stream);
  return GP_OK;
}

extern "C" int gp_mll_eval(const gp_problem* prob, const double* theta_host, const gp_options* opt, int32_t rank,
                           gp_precond* P, void* ws_dev, size_t ws_bytes, hipStream_t stream, double* logp_dev,
                           gp_stats* stats) {
  return run_estimator(prob, theta_host, opt, rank, P, ws_dev, ws_bytes, stream, logp_dev, nullptr, stats);
}

extern "C" int gp_mll_grad(const gp_problem* prob, const double* theta_host, const gp_options* opt, int32_t rank,
                           gp_precond* P, void* ws_dev, size_t ws_bytes, hipStream_t stream, double* logp_dev,
                           double* grad_dev, gp_stats* stats) {
  if (!grad_dev) return GP_EINVAL;
  return run_estimator(prob, theta_host, opt, rank, P, ws_dev, ws_bytes, stream, logp_dev, grad_dev, stats);
}

extern "C" int gp_predict(const gp_problem* prob, const double* theta_host, const gp_options* opt, int32_t rank,
                          gp_precond* P, const double* Xstar_dev, int64_t nstar, void* ws_dev, size_t ws_bytes,
                          hipStream_t stream, double* mean_dev, double* var_dev) {
  RET_IF(check_problem(prob));
  RET_IF(check_options(opt));
  RET_IF(check_rank(prob, rank));
  if (!Xstar_dev || !mean_dev || nstar < 1 || nstar > ((int64_t)1 << 31)) return GP_EINVAL;
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  RET_IF(check_device());
  Layout L = make_layout(prob->n, prob->d, prob->ard, opt->num_probes, opt->max_iters, rank, opt->precision);
  RET_IF(check_ws(ws_dev, ws_bytes, L));
  Ctx c{&L, (char*)ws_dev, stream};
  gpmll_forget_forward(ws_dev);
  RET_IF(use_or_build_precond(prob, theta_host, rank, P, h, c));
  HIPCHK(launch_stage_x(c, h));
  // test points in chunks of num_probes: one CG call on [y | k(X, x*_j)] per chunk
  for (int64_t j0 = 0; j0 < nstar; j0 += L.ell) {
    const int m = (int)std::min<int64_t>(L.ell, nstar - j0);
    HIPCHK(launch_pred_rhs(c, h, prob->y_dev, Xstar_dev + j0 * prob->d, m));
    HIPCHK(launch_cg_init(c, h));
    RET_IF(run_cg(c, h, opt));
    HIPCHK(launch_pred_finish(c, h, m, mean_dev + j0, var_dev ? var_dev + j0 : nullptr));
  }
  int flags[2];
  HIPCHK(hipMemcpyAsync(flags, c.at<int>(L.flags), sizeof(flags), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (flags[1] != 0) return flags[1];
  return GP_OK;
}

extern "C" int gp_khat_matvec(const gp_problem* prob, const double* theta_host, int32_t precision, const double* V_dev,
                              int32_t num_rhs, double* W_dev, void* ws_dev, size_t ws_bytes, hipStream_t stream) {
  RET_IF(check_problem(prob));
  if (!V_dev || !W_dev) return GP_EINVAL;
  if (num_rhs < 1 || num_rhs > 1 + GP_MAX_PROBES) return GP_EINVAL;
  if (precision < 0 || precision > 3) return GP_EINVAL;
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  RET_IF(check_device());
  Layout L = make_layout(prob->n, prob->d, prob->ard, std::max(1, num_rhs - 1), 1, 0, precision);
  RET_IF(check_ws(ws_dev, ws_bytes, L));
  Ctx c{&L, (char*)ws_dev, stream};
  gpmll_forget_forward(ws_dev);
  HIPCHK(launch_prep(c, prob->X_dev, h));
  HIPCHK(launch_stage_x(c, h));
  const TilePlan plan = tile_plan(L, num_rhs);
  HIPCHK(launch_stage_v(c, V_dev, num_rhs, num_rhs, h, nullptr, plan));
  HIPCHK(launch_khat_tiles(c, h, nullptr, plan));
  HIPCHK(launch_khat_reduce(c, V_dev, num_rhs, W_dev, num_rhs, num_rhs, h, nullptr, nullptr));
  return GP_OK;
}

namespace gpmll {
__global__ void k_fill_pattern(double* P, int64_t n, int64_t n_pad, int tp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_pad * tp) return;
  const int64_t i = e / tp;
  const int c = (int)(e % tp);
  // deterministic values in [-1, 1): a Weyl sequence of the element index
  const double v = (i < n) ? 2.0 * (double)((e * 2654435761ull) % 1000003ull) / 1000003.0 - 1.0 : 0.0;
  P[e] = (c < 1 << 30) ? v : 0.0;
}
}  // namespace gpmll

extern "C" int gp_khat_profile(const gp_problem* prob, const double* theta_host, const gp_options* opt, int32_t reps,
                               void* ws_dev, size_t ws_bytes, hipStream_t stream, double* ms_per_launch,
                               int64_t* grid_x, int64_t* grid_y) {
  RET_IF(check_problem(prob));
  RET_IF(check_options(opt));
  if (reps < 1 || !ms_per_launch) return GP_EINVAL;
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  RET_IF(check_device());
  Layout L = make_layout(prob->n, prob->d, prob->ard, opt->num_probes, opt->max_iters, 0, opt->precision);
  RET_IF(check_ws(ws_dev, ws_bytes, L));
  Ctx c{&L, (char*)ws_dev, stream};
  gpmll_forget_forward(ws_dev);
  HIPCHK(launch_prep(c, prob->X_dev, h));
  HIPCHK(launch_stage_x(c, h));
  const int64_t cnt = L.n_pad * L.tp;
  hipLaunchKernelGGL(k_fill_pattern, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, c.at<double>(L.Pd),
                     L.n, L.n_pad, L.tp);
  HIPCHK(hipGetLastError());
  // the products of CG iterations 0 .. reps-1 with every column of [y | probes]
  // active: split-BF16 tiles take the three-piece search directions for the first
  // kBf16V3Iters iterations, as run_cg does; each run of launches with one split is
  // staged and warmed up outside its own pair of events
  const TilePlan plan = tile_plan(L, L.t);
  TilePlan plan3 = plan;
  int n3 = 0;
  if (L.prec == GP_PREC_BF16X3 && bf16_v3_fits(plan.ntt)) {
    plan3.vp = 3;
    n3 = reps < kBf16V3Iters ? reps : kBf16V3Iters;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipError_t err = hipSuccess;
  float ms = 0.f;
  for (int part = 0; part < 2 && err == hipSuccess; ++part) {
    const TilePlan& pl = part == 0 ? plan3 : plan;
    const int count = part == 0 ? n3 : reps - n3;
    if (count == 0) continue;
    err = launch_stage_v(c, c.at<double>(L.Pd), L.tp, L.tp, h, nullptr, pl);
    if (err == hipSuccess) err = launch_khat_tiles(c, h, nullptr, pl);  // warm-up launch
    if (err == hipSuccess) err = hipEventRecord(e0, stream);
    for (int r = 0; r < count && err == hipSuccess; ++r) err = launch_khat_tiles(c, h, nullptr, pl);
    if (err == hipSuccess) err = hipEventRecord(e1, stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float part_ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&part_ms, e0, e1);
    ms += part_ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(err);
  *ms_per_launch = (double)ms / reps;
  const int ntt = L.tp / 16;
  int rows_per_wg;
  if (L.prec == GP_PREC_FP64) rows_per_wg = 64 * (ntt <= 4 ? 2 : 1);
  else if (L.prec == GP_PREC_BF16X3 || L.prec == GP_PREC_FP16X3) rows_per_wg = 256;
  else rows_per_wg = 64 * (ntt <= 5 ? 4 : (ntt <= 8 ? 2 : 1));
  if (grid_x) *grid_x = L.n_pad / rows_per_wg;
  if (grid_y) *grid_y = L.nsplit;
  return GP_OK;
}

extern "C" const char* gp_strerror(int status) {
  switch (status) {
    case GP_OK: return "ok";
    case GP_EINVAL: return "invalid argument (null pointer, size out of range, or non-positive/NaN hyperparameter)";
    case GP_EWORKSPACE: return "workspace smaller than gp_workspace_size";
    case GP_ENOTSPD: return "matrix not positive definite (p^T K_hat p <= 0 or Woodbury matrix not SPD)";
    case GP_EHIP: return "HIP runtime error (see gp_last_hip_error)";
    case GP_EUNSUPPORTED: return "unsupported device (gfx950 required) or option";
  }
  return "unknown status";
}

extern "C" int gp_last_hip_error(void) { return g_last_hip; }

// ---------------------------------------------------------------------------
// gp_khat_matvec_noalloc: the product of gp_khat_matvec with its staging arrays
// in a file-scope device array instead of a caller workspace, for callers that
// cannot allocate device memory.  Each device holds its own copy of the array
// (from the library's load until the process ends); its device address is taken
// once per device with hipGetSymbolAddress and used for every kernel argument.
// Calls that overlap on one device race on the array.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = GP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

// device address of `scratch` on the current device (taken on first use there)
static int scratch_on_current_device(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return GP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr || (reinterpret_cast<uintptr_t>(p) & 255) != 0) return GP_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GP_OK;
}

// The arrays one K_hat V product touches (centring and scaling of X, staged
// distance operands, staged right-hand sides, split-K partial sums), carved back
// to back.  The partial sums grow with the column splits: fewer splits are taken
// while they would not fit in `cap` bytes.  total = 0: nothing fits.
static Layout matvec_layout(const Layout& full, size_t cap) {
  for (int want = full.nsplit; want >= 1; --want) {
    Layout L = full;
    if (want != full.nsplit) {
      L.cols_per_split = std::max<int64_t>(256, rup((L.n_pad + want - 1) / want, 256));
      L.nsplit = (int)((L.n_pad + L.cols_per_split - 1) / L.cols_per_split);
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
      size_t o = off;
      off += al(bytes ? bytes : 1);
      return o;
    };
    const int64_t np = L.n_pad, tp = L.tp;
    const bool split16 = L.prec == GP_PREC_BF16X3 || L.prec == GP_PREC_FP16X3;
    const size_t esz = L.prec == GP_PREC_FP64 ? 8 : (L.prec == GP_PREC_FP32 ? 4 : 2);
    const size_t wsz = L.prec == GP_PREC_FP64 ? 8 : 4;
    L.xs = take(np * L.d * 8);
    L.mean = take(GP_MAX_D * 8);
    L.mean_part = take((size_t)L.nred * GP_MAX_D * 8);
    L.xfa = take(np * L.kd * esz);
    L.xfb = take(np * L.kd * esz);
    L.rowterm = take(np * wsz);
    L.colterm = take(np * wsz);
    L.vfrag = take(np * tp * (split16 ? 6 : esz));  // up to three 16-bit pieces
    L.vx = take(split16 ? np * 4 : 0);
    L.vscale = take(2 * tp * 4);
    L.wpart = take((size_t)L.nsplit * np * tp * wsz);
    L.total = off;
    if (L.total <= cap) return L;
  }
  Layout none = full;
  none.total = 0;
  return none;
}

extern "C" int gp_khat_matvec_noalloc(const gp_problem* prob, const double* theta_host, int32_t precision,
                                      const double* V_dev, int32_t num_rhs, double* W_dev, hipStream_t stream) {
  RET_IF(check_problem(prob));
  if (!V_dev || !W_dev) return GP_EINVAL;
  if (num_rhs < 1 || num_rhs > 1 + GP_MAX_PROBES) return GP_EINVAL;
  if (precision < 0 || precision > 3) return GP_EINVAL;
  Hyper h;
  RET_IF(make_hyper(prob, theta_host, &h));
  const Layout full = make_layout(prob->n, prob->d, prob->ard, std::max(1, num_rhs - 1), 1, 0, precision);
  const Layout L = matvec_layout(full, kScratchBytes);
  if (L.total == 0) return GP_EWORKSPACE;
  RET_IF(check_device());
  void* ws = nullptr;
  RET_IF(scratch_on_current_device(&ws));
  Ctx c{&L, (char*)ws, stream};
  // every array below is fully rewritten by this call (the FP16X3 column maxima
  // are cleared by a kernel), so nothing left by an earlier call is read
  HIPCHK(launch_prep(c, prob->X_dev, h));
  HIPCHK(launch_stage_x(c, h));
  const TilePlan plan = tile_plan(L, num_rhs);
  HIPCHK(launch_stage_v(c, V_dev, num_rhs, num_rhs, h, nullptr, plan));
  HIPCHK(launch_khat_tiles(c, h, nullptr, plan));
  HIPCHK(launch_khat_reduce(c, V_dev, num_rhs, W_dev, num_rhs, num_rhs, h, nullptr, nullptr));
  return GP_OK;
}
