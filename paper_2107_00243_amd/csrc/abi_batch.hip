// Host side of the batched entry points (gp_batch_*): validation, the batched
// workspace layout and its small tables (per-problem descriptors, tile and
// derivative-sweep work items, block -> problem map), and the launch sequence,
// one launch per phase for all problems.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch_impl.h"

namespace gpmll {
namespace {

size_t al256(size_t x) { return (x + 255) / 256 * 256; }
int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct HostTables {
  std::vector<BDesc> desc;
  std::vector<int4> items, bitems;
  std::vector<int32_t> item_prob;
  std::vector<int32_t> blkprob;
};

int check_batch(const gp_batch* bp) {
  if (!bp || !bp->offsets_host) return GP_EINVAL;
  if (bp->batch < 1 || bp->batch > 65536) return GP_EINVAL;
  if (bp->d < 1 || bp->d > GP_MAX_D) return GP_EINVAL;
  if (bp->kernel == GP_KERNEL_RATQUAD) return GP_EUNSUPPORTED;  // batches: RBF and Matern kernels
  if (bp->kernel < 0 || bp->kernel > 2) return GP_EINVAL;
  if (bp->ard != 0 && bp->ard != 1) return GP_EINVAL;
  if (bp->offsets_host[0] != 0) return GP_EINVAL;
  int64_t padded = 0;
  for (int b = 0; b < bp->batch; ++b) {
    const int64_t n = bp->offsets_host[b + 1] - bp->offsets_host[b];
    if (n < 1) return GP_EINVAL;
    padded += rup(n, kBRows);
  }
  if (padded > ((int64_t)1 << 31) - 256) return GP_EINVAL;
  return GP_OK;
}

int check_batch_options(const gp_options* o, int32_t rank) {
  if (!o) return GP_EINVAL;
  if (o->precision < 0 || o->precision > 3) return GP_EINVAL;
  if (o->num_probes < 1 || o->num_probes > GP_MAX_PROBES) return GP_EINVAL;
  if (o->max_iters < 1 || o->max_iters > 2645) return GP_EINVAL;  // tridiagonal + 256 doubles in 64 KB of LDS
  if (!(o->cg_tol >= 0.0) || !std::isfinite(o->cg_tol)) return GP_EINVAL;
  if (o->precond_grad != 0 && o->precond_grad != 1) return GP_EINVAL;
  if (o->sync_every < 0) return GP_EINVAL;
  if (o->probe_mode != 0 && o->probe_mode != 1) return GP_EINVAL;
  if (rank < 0) return GP_EINVAL;
  if (o->probe_mode != 0) return GP_EUNSUPPORTED;
  if (o->precision != GP_PREC_FP64 && o->precision != GP_PREC_FP32) return GP_EUNSUPPORTED;
  if (o->num_probes > GP_BATCH_MAX_PROBES || rank > GP_BATCH_MAX_RANK) return GP_EUNSUPPORTED;
  return GP_OK;
}

int pick4(int d) { return d <= 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : 32; }

// Layout of the batch; with ht != NULL also the host tables (theta required).
BLayout make_blayout(const gp_batch* bp, const gp_options* o, int32_t rank, const double* theta, HostTables* ht) {
  BLayout L;
  std::memset(&L, 0, sizeof(L));
  L.B = bp->batch;
  L.d = bp->d;
  L.kind = bp->kernel;
  L.ard = bp->ard;
  L.p = bp->ard ? bp->d : 1;
  L.ell = o->num_probes;
  L.t = 1 + L.ell;
  L.tp = (int)rup(L.t, 16);
  L.K = rank;
  L.max_iters = o->max_iters;
  L.prec = o->precision;
  L.dm = pick4(L.d);
  const int ntt = L.tp / 16;
  const size_t elem = L.prec == GP_PREC_FP64 ? 8 : 4;
  const int rows_wg = 64 * fp_row_groups(elem, ntt);

  int64_t off = 0, loff = 0;
  int nblk = 0, maxsplit = 1, nitems = 0, nbitems = 0;
  if (ht) {
    ht->desc.resize(L.B);
    ht->items.clear();
    ht->item_prob.clear();
    ht->bitems.clear();
    ht->blkprob.clear();
  }
  for (int b = 0; b < L.B; ++b) {
    const int64_t n = bp->offsets_host[b + 1] - bp->offsets_host[b];
    const int64_t np = rup(n, kBRows);
    const int64_t ncol = rup(n, 16);
    const int nsplit = (int)((ncol + kBColsPerSplit - 1) / kBColsPerSplit);
    maxsplit = std::max(maxsplit, nsplit);
    const int nrow_items = (int)((n + rows_wg - 1) / rows_wg);
    const int nb_rows = (int)((n + kBRows - 1) / kBRows);
    const int nb_cols = (int)((n + kBBwdCols - 1) / kBBwdCols);
    if (ht) {
      BDesc& D = ht->desc[b];
      std::memset(&D, 0, sizeof(D));
      D.xoff = bp->offsets_host[b];
      D.off = off;
      D.n = n;
      D.n_pad = np;
      D.loff = loff;
      D.blk0 = nblk;
      D.nblk = (int32_t)(np / kBRows);
      D.nsplit = nsplit;
      D.k = (int32_t)std::min<int64_t>(rank, n);
      D.bitem0 = nbitems;
      D.nbitem = nb_rows * nb_cols;
      const double* th = theta + (size_t)b * (L.p + 2);
      for (int j = 0; j < L.d; ++j) D.inv_ls[j] = 1.0 / th[L.ard ? j : 0];
      D.s = th[L.p];
      D.s2 = th[L.p + 1];
      D.sigma = std::sqrt(D.s2);
      D.seed = o->seed + (uint64_t)b;
      for (int r = 0; r < nrow_items; ++r)
        for (int s = 0; s < nsplit; ++s) {
          const int64_t c0 = off + (int64_t)s * kBColsPerSplit;
          const int64_t c1 = std::min(off + ncol, c0 + kBColsPerSplit);
          ht->items.push_back(int4{(int)(off + (int64_t)r * rows_wg), (int)c0, (int)c1, s});
          ht->item_prob.push_back(b);
        }
      for (int r = 0; r < nb_rows; ++r)
        for (int q = 0; q < nb_cols; ++q) {
          const int64_t c0 = off + (int64_t)q * kBBwdCols;
          const int64_t c1 = std::min(off + n, c0 + kBBwdCols);
          ht->bitems.push_back(int4{(int)(off + (int64_t)r * kBRows), (int)c0, (int)c1, b});
        }
      for (int q = 0; q < (int)(np / kBRows); ++q) ht->blkprob.push_back(b);
    }
    nitems += nrow_items * nsplit;
    nbitems += nb_rows * nb_cols;
    nblk += (int)(np / kBRows);
    off += np;
    loff += np * rank;
  }
  L.N = off;
  L.nblk = nblk;
  L.maxsplit = maxsplit;
  L.nitems = nitems;
  L.nbitems = nbitems;

  const int64_t N = L.N, B = L.B, K = std::max(1, L.K), tp = L.tp;
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    size_t o2 = cur;
    cur += al256(std::max<size_t>(bytes, 8));
    return o2;
  };
  L.desc = take(B * sizeof(BDesc));
  L.items = take((size_t)nitems * sizeof(int4));
  L.item_prob = take((size_t)nitems * 4);
  L.bitems = take((size_t)nbitems * sizeof(int4));
  L.blkprob = take((size_t)nblk * 4);
  L.xs = take(N * L.d * 8);
  L.L = take((size_t)std::max<int64_t>(loff, 1) * 8);
  L.diag = take(N * 8);
  L.ispiv = take(N);
  L.piv = take(B * K * 4);
  L.kach = take(2 * B * 4);
  L.stop = L.kach + B * 4;
  L.C = take(B * K * K * 8);
  L.Rc = take(B * K * K * 8);
  L.Rinv = take(B * K * K * 8);
  L.Cinv = take(B * K * K * 8);
  L.logdetP = take(B * 8);
  L.H = take(B * K * L.ell * 8);
  L.Tb = take(B * K * tp * 8);
  L.Y = take(B * K * tp * 8);
  L.ltr_part = take((size_t)nblk * rup(K, 16) * tp * 8);
  L.R = take(N * tp * 8);
  L.Xs = take(N * tp * 8);
  L.Z0 = take(N * tp * 8);
  L.Pd = take(N * tp * 8);
  L.W = take(N * tp * 8);
  L.rho = take(B * tp * 8);
  L.rho0 = take(B * tp * 8);
  L.bnorm = take(B * tp * 8);
  L.rnorm = take(B * tp * 8);
  L.alpha = take(B * tp * 8);
  L.beta = take(B * tp * 8);
  L.active = take(B * tp * 4);
  L.iters = take(B * tp * 4);
  L.nactive = take(2 * 4);
  L.pact = take(B * 4);
  L.alog = take(B * tp * L.max_iters * 8);
  L.blog = take(B * tp * L.max_iters * 8);
  L.part = take((size_t)nblk * tp * 8);
  L.part2 = take((size_t)nblk * tp * 8);
  L.gamma = take(B * L.ell * 8);
  L.flags = take(4 * B * 4);
  L.logp_aux = take(2 * B * 8);
  L.cprime = take(N * tp * 8);
  L.bwd_part = take((size_t)nbitems * (GP_MAX_D + 1) * 8);
  L.pgs = take(B * (4 * K * K + K * tp) * 8);
  L.pg_psi = take(B * (GP_MAX_D + 1) * 8);
  L.pg_part = take((size_t)nblk * (GP_MAX_D + 1) * 8);

  // tile-kernel view of the concatenation
  Layout& V = L.view;
  V.n = N;
  V.n_pad = N;
  V.d = L.d;
  V.p = L.p;
  V.t = L.t;
  V.tp = L.tp;
  V.k = L.K;
  V.ell = L.ell;
  V.max_iters = L.max_iters;
  V.prec = L.prec;
  V.bprec = GP_PREC_FP64;
  V.kd = pick4(L.d);
  V.nsplit = maxsplit;
  V.cols_per_split = kBColsPerSplit;
  V.xs = L.xs;
  const int nk4 = V.kd / 4;
  V.xfa = take((size_t)(N / 16) * nk4 * 64 * elem);
  V.xfb = take((size_t)(N / 16) * nk4 * 64 * elem);
  V.rowterm = take(N * elem);
  V.colterm = take(N * elem);
  V.vfrag = take(N * tp * elem);
  V.wpart = take((size_t)maxsplit * N * tp * elem);
  L.total = cur;
  V.total = cur;
  return L;
}

#define BHIP(expr)                  \
  do {                              \
    hipError_t _e = (expr);         \
    if (_e != hipSuccess) {         \
      gpmll_set_hip_error((int)_e); \
      return GP_EHIP;               \
    }                               \
  } while (0)

#define BRET(x)                    \
  do {                             \
    int _r = (x);                  \
    if (_r != GP_OK) return _r;    \
  } while (0)

int run_batch(const gp_batch* bp, const double* theta_host, const gp_options* opt, int32_t rank, void* ws_dev,
              size_t ws_bytes, hipStream_t stream, double* logp_dev, double* grad_dev, gp_batch_stats* stats) {
  BRET(check_batch(bp));
  BRET(check_batch_options(opt, rank));
  if (!bp->X_dev || !bp->y_dev || !theta_host || !logp_dev) return GP_EINVAL;
  const int p = bp->ard ? bp->d : 1;
  for (int64_t e = 0; e < (int64_t)bp->batch * (p + 2); ++e)
    if (!(theta_host[e] > 0.0) || !std::isfinite(theta_host[e])) return GP_EINVAL;
  BRET(gpmll_check_device());
  HostTables ht;
  BLayout L = make_blayout(bp, opt, rank, theta_host, &ht);
  if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 255) != 0) return GP_EINVAL;
  if (ws_bytes < L.total) return GP_EWORKSPACE;
  char* ws = (char*)ws_dev;
  BHIP(hipMemcpyAsync(ws + L.desc, ht.desc.data(), ht.desc.size() * sizeof(BDesc), hipMemcpyHostToDevice, stream));
  BHIP(hipMemcpyAsync(ws + L.items, ht.items.data(), ht.items.size() * sizeof(int4), hipMemcpyHostToDevice, stream));
  BHIP(hipMemcpyAsync(ws + L.item_prob, ht.item_prob.data(), ht.item_prob.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice, stream));
  BHIP(hipMemcpyAsync(ws + L.bitems, ht.bitems.data(), ht.bitems.size() * sizeof(int4), hipMemcpyHostToDevice,
                      stream));
  BHIP(hipMemcpyAsync(ws + L.blkprob, ht.blkprob.data(), ht.blkprob.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                      stream));
  // the host tables go out of scope with this call
  BHIP(hipStreamSynchronize(stream));

  Ctx c{&L.view, ws, stream};
  gpmll_forget_forward(ws);
  Hyper h;
  std::memset(&h, 0, sizeof(h));
  h.kind = bp->kernel;
  h.d = bp->d;
  h.s = 1.0;
  h.log2s = 0.0;
  h.alpha = 1.0;
  BHIP(bl_zero_flags(L, ws, stream));
  BHIP(bl_prep(L, ws, stream, bp->X_dev));
  BHIP(bl_precond(L, ws, stream));
  BHIP(launch_stage_x(c, h));
  BHIP(bl_probes(L, ws, stream, bp->y_dev));
  BHIP(bl_cg_init(L, ws, stream));
  int* nact = reinterpret_cast<int*>(ws + L.nactive);
  ItemTable items;
  items.items = reinterpret_cast<const int4*>(ws + L.items);
  items.nitems = L.nitems;
  items.gate = reinterpret_cast<const int*>(ws + L.item_prob);
  items.gate_count = reinterpret_cast<const int*>(ws + L.pact);
  const int q = opt->sync_every;
  for (int it = 0; it < opt->max_iters; ++it) {
    if (q > 0 && it > 0 && it % q == 0) {
      int host_nact = 0;
      BHIP(hipMemcpyAsync(&host_nact, nact, sizeof(int), hipMemcpyDeviceToHost, stream));
      BHIP(hipStreamSynchronize(stream));
      if (host_nact == 0) break;
    }
    BHIP(launch_stage_v(c, reinterpret_cast<double*>(ws + L.Pd), L.tp, L.tp, h));
    BHIP(launch_khat_tiles_items(c, h, items, nact));
    BHIP(bl_reduce(L, ws, stream));
    BHIP(bl_cg_after_product(L, ws, stream, it, opt->cg_tol));
  }
  BHIP(bl_slq_logp(L, ws, stream, bp->y_dev, logp_dev));
  if (grad_dev) BHIP(bl_backward(L, ws, stream, opt->precond_grad, grad_dev));
  if (stats) {
    std::vector<int> flags(4 * L.B), iters((size_t)L.B * L.tp), kach(L.B);
    BHIP(hipMemcpyAsync(flags.data(), ws + L.flags, flags.size() * sizeof(int), hipMemcpyDeviceToHost, stream));
    BHIP(hipMemcpyAsync(iters.data(), ws + L.iters, iters.size() * sizeof(int), hipMemcpyDeviceToHost, stream));
    BHIP(hipMemcpyAsync(kach.data(), ws + L.kach, kach.size() * sizeof(int), hipMemcpyDeviceToHost, stream));
    BHIP(hipStreamSynchronize(stream));
    int mx_all = 0, f_all = 0;
    for (int b = 0; b < L.B; ++b) {
      if (flags[4 * b + 1] != 0) return flags[4 * b + 1];
      int mx = 0;
      for (int cc = 0; cc < L.t; ++cc) mx = std::max(mx, iters[(size_t)b * L.tp + cc]);
      mx_all = std::max(mx_all, mx);
      f_all |= flags[4 * b];
      if (stats->iters_host) stats->iters_host[b] = mx;
      if (stats->flags_host) stats->flags_host[b] = flags[4 * b];
      if (stats->rank_host) stats->rank_host[b] = rank > 0 ? kach[b] : 0;
    }
    stats->iters_max = mx_all;
    stats->flags_any = f_all;
  }
  return GP_OK;
}

}  // namespace
}  // namespace gpmll

using namespace gpmll;

extern "C" int gp_batch_workspace_size(const gp_batch* bp, const gp_options* opt, int32_t rank, size_t* bytes) {
  if (!bytes) return GP_EINVAL;
  BRET(check_batch(bp));
  BRET(check_batch_options(opt, rank));
  BLayout L = make_blayout(bp, opt, rank, nullptr, nullptr);
  *bytes = L.total;
  return GP_OK;
}

extern "C" int gp_batch_mll_eval(const gp_batch* bp, const double* theta_host, const gp_options* opt, int32_t rank,
                                 void* ws_dev, size_t ws_bytes, hipStream_t stream, double* logp_dev,
                                 gp_batch_stats* stats) {
  return run_batch(bp, theta_host, opt, rank, ws_dev, ws_bytes, stream, logp_dev, nullptr, stats);
}

extern "C" int gp_batch_mll_grad(const gp_batch* bp, const double* theta_host, const gp_options* opt, int32_t rank,
                                 void* ws_dev, size_t ws_bytes, hipStream_t stream, double* logp_dev, double* grad_dev,
                                 gp_batch_stats* stats) {
  if (!grad_dev) return GP_EINVAL;
  return run_batch(bp, theta_host, opt, rank, ws_dev, ws_bytes, stream, logp_dev, grad_dev, stats);
}
