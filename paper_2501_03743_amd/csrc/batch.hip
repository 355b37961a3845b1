// Batched persistent solves (ssp_solve_batch) and their autotuner
// (ssp_autotune_batch).  One launch of k_batch<S> runs every system's
// mixed-precision s-step solve to completion; see batch.hpp.
#include <chrono>
#include <fstream>
#include <sstream>

#include "batch.hpp"
#include "engine.hpp"

using namespace ssp;

namespace {

constexpr int kBatchSMax = 8;
constexpr int kBatchMaxSys = 4096;
constexpr unsigned kDefaultSpin = 1u << 20;  // idle polls without progress before giving up

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

template <int... Ss>
struct BatchTable {
  static int launch(int s, int grid, hipStream_t st, const BatchSys *sys, BatchSched *sched,
                    BatchGlobal *glob, int nsys, const int *order_arr, int order, unsigned spin,
                    int run) {
    int done = 0;
    ((s == Ss ? (k_batch<Ss><<<grid, kWG, 0, st>>>(sys, sched, glob, nsys, order_arr, order, spin,
                                                    run),
                 done = 1, 0)
              : 0),
     ...);
    return done;
  }
};
using BT = BatchTable<1, 2, 3, 4, 5, 6, 7, 8>;

template <int... Ss>
struct StepTable {
  static int launch(int s, int ntiles, int nsys, hipStream_t st, const BatchSys *sys,
                    BatchSched *sched, BatchGlobal *glob, const int *tsys, const int *tidx) {
    int done = 0;
    ((s == Ss ? (k_batch_tiles<Ss><<<ntiles, kWG, 0, st>>>(sys, sched, tsys, tidx),
                 k_batch_step<Ss><<<nsys, kWG, 0, st>>>(sys, sched, glob), done = 1, 0)
              : 0),
     ...);
    return done;
  }
};
using ST = StepTable<1, 2, 3, 4, 5, 6, 7, 8>;

struct Layout {
  int64_t n, ld, tile_rows;
  int ntiles;
  size_t off_q1, off_q2, off_r32, off_d32, off_part, off_hist, off_state;
};

}  // namespace

extern "C" {

int ssp_solve_batch(ssp_handle *h, int nsys, const ssp_matrix *const *A, const double *const *b,
                    double *const *x, int s, double rtol, int maxit, const ssp_opts *opts,
                    const ssp_tune *tune, int *status_out, int *outer_out, double *true_rel_out) {
  if (!h) return SSP_EINVAL;
  if (nsys < 1 || nsys > kBatchMaxSys || !A || !b || !x)
    return fail(h, SSP_EINVAL, "ssp_solve_batch: need 1..4096 systems and their arrays");
  if (s < 1 || s > kBatchSMax)
    return fail(h, SSP_EINVAL, "ssp_solve_batch: s must be in 1..8");
  if (!(rtol >= 0.0) || maxit < 0) return fail(h, SSP_EINVAL, "ssp_solve_batch: bad rtol/maxit");
  if (opts && opts->precision != SSP_PRECISION_MIXED_IR && opts->precision != SSP_PRECISION_FP64)
    return fail(h, SSP_EINVAL, "ssp_solve_batch: unknown precision");
  for (int i = 0; i < nsys; ++i) {
    if (!A[i] || A[i]->h != h || !b[i] || !x[i])
      return fail(h, SSP_EINVAL, "ssp_solve_batch: system " + std::to_string(i) + " is invalid");
    if (s > A[i]->n) return fail(h, SSP_EINVAL, "ssp_solve_batch: s exceeds a system size");
    if (A[i]->prec == SSP_PREC_AMG)
      return fail(h, SSP_EUNSUPPORTED, "ssp_solve_batch: the AMG preconditioner is not batched");
  }
  HIPCHK(h, hipSetDevice(h->device));
  const double inner_rtol = (opts && opts->inner_rtol > 0.0) ? opts->inner_rtol : 1e-5;
  const int max_refine = (opts && opts->max_refine > 0) ? opts->max_refine : 10;
  const int inner_max = (int)((maxit + (int64_t)s - 1) / s);
  const int grid = (tune && tune->grid > 0) ? tune->grid : 512;
  const int order = tune ? tune->order : 0;
  const unsigned spin = (tune && tune->spin_limit > 0) ? (unsigned)tune->spin_limit : kDefaultSpin;
  const int64_t trq = tune ? tune->tile_rows : 0;
  const int schedule = tune ? tune->schedule : 0;
  const int run = (tune && tune->run > 0) ? tune->run : 1;
  if (run > (1 << 20)) return fail(h, SSP_EINVAL, "ssp_solve_batch: run must be <= 2^20");
  if (schedule != 0 && schedule != 1) return fail(h, SSP_EINVAL, "ssp_solve_batch: bad schedule");

  // layout of the per-system arrays in one device buffer
  std::vector<Layout> L(nsys);
  size_t bytes = 0;
  for (int i = 0; i < nsys; ++i) {
    int rc = ensure_fp32(h, const_cast<ssp_matrix *>(A[i]));
    if (rc) return rc;
    Layout &l = L[i];
    l.n = A[i]->n;
    l.ld = (l.n + 63) / 64 * 64 + kColumnStagger / (int64_t)sizeof(float);
    if (trq <= 0) {
      // the partition of a single solve: results equal ssp_solve's bit for bit
      const int G = grid_rows(l.n);
      l.tile_rows = (l.n + G - 1) / G;
      l.ntiles = G;
    } else {
      int64_t T = (trq + kWG - 1) / kWG * kWG;
      if ((l.n + T - 1) / T > kGridMax) T = ((l.n + kGridMax - 1) / kGridMax + kWG - 1) / kWG * kWG;
      l.tile_rows = T;
      l.ntiles = (int)((l.n + T - 1) / T);
    }
    const int np = std::max(2 * s, 3);
    l.off_q1 = bytes; bytes = align256(bytes + sizeof(float) * l.ld * 2 * s);
    l.off_q2 = bytes; bytes = align256(bytes + sizeof(float) * l.ld * 2 * s);
    l.off_r32 = bytes; bytes = align256(bytes + sizeof(float) * l.ld);
    l.off_d32 = bytes; bytes = align256(bytes + sizeof(float) * l.ld);
    l.off_part = bytes; bytes = align256(bytes + sizeof(double) * np * l.ntiles);
    l.off_hist = bytes; bytes = align256(bytes + sizeof(double) * (max_refine + 1));
    l.off_state = bytes; bytes = align256(bytes + sizeof(DevState));
  }
  const size_t off_sys = bytes;
  bytes = align256(bytes + sizeof(BatchSys) * nsys);
  const size_t off_sched = bytes;
  bytes = align256(bytes + sizeof(BatchSched) * nsys);
  const size_t off_glob = bytes;
  bytes = align256(bytes + sizeof(BatchGlobal));
  const size_t off_order = bytes;
  bytes = align256(bytes + sizeof(int) * nsys);
  int64_t total_tiles = 0;
  for (int i = 0; i < nsys; ++i) total_tiles += L[i].ntiles;
  if (schedule == 1 && total_tiles > (int64_t)INT32_MAX / 2)
    return fail(h, SSP_EINVAL, "ssp_solve_batch: too many tiles for the stepped schedule");
  const size_t off_tsys = bytes;
  bytes = align256(bytes + (schedule == 1 ? sizeof(int) * total_tiles : 0));
  const size_t off_tidx = bytes;
  bytes = align256(bytes + (schedule == 1 ? sizeof(int) * total_tiles : 0));
  if (bytes > h->batch_bytes) {
    if (h->batch_mem) (void)hipFree(h->batch_mem);
    h->batch_mem = nullptr;
    h->batch_bytes = 0;
    if (hipMalloc(&h->batch_mem, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, SSP_ENOMEM, "ssp_solve_batch: workspace allocation failed");
    }
    h->batch_bytes = bytes;
  }
  char *base = (char *)h->batch_mem;

  // host images of the descriptors, control blocks and scheduling words
  std::vector<BatchSys> sys(nsys);
  std::vector<BatchSched> sched(nsys);
  std::vector<DevState> hdr(nsys);
  std::vector<int> ord(nsys);
  for (int i = 0; i < nsys; ++i) {
    const ssp_matrix *M = A[i];
    const Layout &l = L[i];
    BatchSys &y = sys[i];
    memset(&y, 0, sizeof(y));
    y.kind = M->kind;
    y.c64 = M->csr;
    y.c32 = M->csr32;
    y.s64 = M->sten;
    y.s32 = M->sten32;
    double *t64 = nullptr;
    float *t32 = nullptr;
    y.pc64 = prec_of(M, t64);
    y.pc32 = prec_of(M, t32);
    y.b = b[i];
    y.x = x[i];
    y.Q1 = (float *)(base + l.off_q1);
    y.Q2 = (float *)(base + l.off_q2);
    y.r32 = (float *)(base + l.off_r32);
    y.d32 = (float *)(base + l.off_d32);
    y.ld = l.ld;
    y.partials = (double *)(base + l.off_part);
    y.hist = (double *)(base + l.off_hist);
    y.st = (DevState *)(base + l.off_state);
    y.n = l.n;
    y.tile_rows = l.tile_rows;
    y.ntiles = l.ntiles;
    y.single = trq <= 0;
    DevState &c = hdr[i];
    memset(&c, 0, sizeof(c));
    c.status = ST_RUNNING;
    c.outer_max = inner_max;
    c.s = s;
    c.rtol = inner_rtol;
    c.ir_max_refine = max_refine;
    c.ir_hist_cap = max_refine + 1;
    c.ir_rtol = rtol;
    c.ir_inner_rtol = inner_rtol;
    BatchSched &q = sched[i];
    memset(&q, 0, sizeof(q));
    q.claim = 1ull << 32;   // sequence 1, tile 0
    q.phase = PH_RESID;
    q.j = 1;
    ord[i] = i;
  }
  if (order == 0)
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return L[a].n > L[c].n; });
  BatchGlobal g;
  memset(&g, 0, sizeof(g));
  for (int i = 0; i < nsys; ++i)
    HIPCHK(h, hipMemcpyAsync(base + L[i].off_state, &hdr[i], sizeof(DevState),
                             hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(base + off_sys, sys.data(), sizeof(BatchSys) * nsys,
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(base + off_sched, sched.data(), sizeof(BatchSched) * nsys,
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(base + off_glob, &g, sizeof(g), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(base + off_order, ord.data(), sizeof(int) * nsys,
                           hipMemcpyHostToDevice, h->stream));
  if (schedule == 0) {
    if (!BT::launch(s, grid, h->stream, (const BatchSys *)(base + off_sys),
                    (BatchSched *)(base + off_sched), (BatchGlobal *)(base + off_glob), nsys,
                    (const int *)(base + off_order), order, spin, run))
      return fail(h, SSP_EINVAL, "ssp_solve_batch: no kernel for s");
    LAUNCHCHK(h);
  } else {
    // work-item map (largest systems first), then launch pairs until every
    // system is done; the host reads the done counter every few steps
    std::vector<int> tsys, tidx;
    tsys.reserve(total_tiles);
    tidx.reserve(total_tiles);
    std::vector<int> big(nsys);
    for (int i = 0; i < nsys; ++i) big[i] = i;
    std::stable_sort(big.begin(), big.end(), [&](int a, int c) { return L[a].n > L[c].n; });
    for (int i : big)
      for (int t = 0; t < L[i].ntiles; ++t) {
        tsys.push_back(i);
        tidx.push_back(t);
      }
    HIPCHK(h, hipMemcpyAsync(base + off_tsys, tsys.data(), sizeof(int) * total_tiles,
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(base + off_tidx, tidx.data(), sizeof(int) * total_tiles,
                             hipMemcpyHostToDevice, h->stream));
    // a system needs at most (max_refine + 1) * (2 + inner_max * (s + 1)) steps
    const int64_t max_steps = (int64_t)(max_refine + 1) * (2 + (int64_t)inner_max * (s + 1)) + 1;
    const int every = 8;
    BatchGlobal gp;
    for (int64_t step = 0;;) {
      for (int q = 0; q < every; ++q, ++step)
        if (!ST::launch(s, (int)total_tiles, nsys, h->stream, (const BatchSys *)(base + off_sys),
                        (BatchSched *)(base + off_sched), (BatchGlobal *)(base + off_glob),
                        (const int *)(base + off_tsys), (const int *)(base + off_tidx)))
          return fail(h, SSP_EINVAL, "ssp_solve_batch: no kernel for s");
      LAUNCHCHK(h);
      HIPCHK(h, hipMemcpyAsync(&gp, base + off_glob, sizeof(gp), hipMemcpyDeviceToHost,
                               h->stream));
      HIPCHK(h, hipStreamSynchronize(h->stream));
      if (gp.ndone >= (unsigned)nsys) break;
      if (step > max_steps)
        return fail(h, SSP_EHIP, "ssp_solve_batch: stepped schedule exceeded its step bound");
    }
  }
  HIPCHK(h, hipMemcpyAsync(&g, base + off_glob, sizeof(g), hipMemcpyDeviceToHost, h->stream));
  for (int i = 0; i < nsys; ++i)
    HIPCHK(h, hipMemcpyAsync(&hdr[i], base + L[i].off_state, sizeof(DevState),
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (g.error || g.ndone != (unsigned)nsys)
    return fail(h, SSP_EHIP, "ssp_solve_batch: the scheduler stalled (" +
                                 std::to_string(g.ndone) + " of " + std::to_string(nsys) +
                                 " systems finished)");
  int worst = SSP_OK;
  for (int i = 0; i < nsys; ++i) {
    const DevState &d = hdr[i];
    if (d.status == ST_ZERO_RHS)
      HIPCHK(h, hipMemsetAsync(x[i], 0, sizeof(double) * A[i]->n, h->stream));
    const int code = status_code(d.status);
    if (code > worst) worst = code;
    if (status_out) status_out[i] = code;
    if (outer_out) outer_out[i] = d.ir_inner_total;
    if (true_rel_out) {
      const double bn = std::sqrt(d.ir_bb);
      true_rel_out[i] = (d.status == ST_ZERO_RHS || bn == 0.0) ? 0.0 : std::sqrt(d.true_rr) / bn;
    }
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return worst;
}

int ssp_autotune_batch(ssp_handle *h, int nsys, const ssp_matrix *const *A,
                       const double *const *b, int s, const char *cache_path, ssp_tune *out) {
  if (!h || !out) return SSP_EINVAL;
  if (nsys < 1 || nsys > kBatchMaxSys || !A || !b || s < 1 || s > kBatchSMax)
    return fail(h, SSP_EINVAL, "ssp_autotune_batch: invalid arguments");
  int64_t total = 0, largest = 0;
  unsigned kinds = 0;
  for (int i = 0; i < nsys; ++i) {
    if (!A[i] || A[i]->h != h) return fail(h, SSP_EINVAL, "ssp_autotune_batch: invalid matrix");
    total += A[i]->n;
    largest = std::max<int64_t>(largest, A[i]->n);
    kinds |= 1u << A[i]->kind;
  }
  int lg = 0;
  while ((int64_t)1 << (lg + 1) <= total) ++lg;
  std::ostringstream key;
  key << "gfx950 nsys=" << nsys << " rows_log2=" << lg << " s=" << s << " kinds=" << kinds;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      if (line.rfind(key.str() + " ", 0) == 0) {
        std::istringstream f(line.substr(key.str().size()));
        std::string tag;
        ssp_tune t{0, 0, 0, 0, 0, 0};
        while (f >> tag) {
          if (tag.rfind("tile_rows=", 0) == 0) t.tile_rows = std::stoi(tag.substr(10));
          else if (tag.rfind("grid=", 0) == 0) t.grid = std::stoi(tag.substr(5));
          else if (tag.rfind("order=", 0) == 0) t.order = std::stoi(tag.substr(6));
          else if (tag.rfind("schedule=", 0) == 0) t.schedule = std::stoi(tag.substr(9));
          else if (tag.rfind("run=", 0) == 0) t.run = std::stoi(tag.substr(4));
        }
        if (t.grid > 0 || t.schedule == 1) {
          *out = t;
          return SSP_OK;
        }
      }
    }
  }
  // scratch iterates; short solves (two refinements of at most 4 outer
  // iterations) measure the throughput of each candidate
  std::vector<double *> xs(nsys, nullptr);
  for (int i = 0; i < nsys; ++i) {
    if (hipMalloc(&xs[i], sizeof(double) * A[i]->n) != hipSuccess) {
      (void)hipGetLastError();
      for (double *p : xs)
        if (p) (void)hipFree(p);
      return fail(h, SSP_ENOMEM, "ssp_autotune_batch: scratch allocation failed");
    }
  }
  ssp_opts o;
  memset(&o, 0, sizeof(o));
  o.precision = SSP_PRECISION_MIXED_IR;
  o.max_refine = 2;
  o.inner_rtol = 1e-30;   // run the full inner budget
  const int tiles[] = {0, 16384, 65536, 262144};
  const int grids[] = {256, 512, 1024, 2048};
  double best = 1e300;
  ssp_tune bt{0, 512, 0, 0, 0, 0};
  int rc = SSP_OK;
  auto trial = [&](const ssp_tune &t) {
    double ms = 0.0;
    for (int rep = 0; rep < 2 && rc >= 0; ++rep) {
      for (int i = 0; i < nsys; ++i)
        (void)hipMemsetAsync(xs[i], 0, sizeof(double) * A[i]->n, h->stream);
      (void)hipStreamSynchronize(h->stream);
      auto t0 = std::chrono::steady_clock::now();
      rc = ssp_solve_batch(h, nsys, A, b, xs.data(), s, 0.0, 4 * s, &o, &t, nullptr, nullptr,
                           nullptr);
      auto t1 = std::chrono::steady_clock::now();
      if (rep == 1) ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (rc >= 0 && ms < best) {
      best = ms;
      bt = t;
    }
    return rc >= 0 ? ms : 1e300;
  };
  ssp_tune bp{0, 512, 0, 0, 0, 0};   // the best persistent candidate
  double bp_ms = 1e300;
  for (int ti : tiles) {
    for (int gi : grids)
      for (int oi = 0; oi < 2 && rc >= 0; ++oi) {
        const ssp_tune t{ti, gi, oi, 0, 0, 0};
        const double ms = trial(t);
        if (ms < bp_ms) {
          bp = t;
          bp_ms = ms;
        }
      }
    if (rc >= 0) trial(ssp_tune{ti, 0, 0, 0, 1, 0});
  }
  // then the best persistent candidate with longer runs of tiles per claim
  for (int ru : {2, 4, 8, 16})
    if (rc >= 0) trial(ssp_tune{bp.tile_rows, bp.grid, bp.order, 0, 0, ru});
  for (double *p : xs) (void)hipFree(p);
  if (rc < 0) return rc;
  *out = bt;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << key.str() << " tile_rows=" << bt.tile_rows << " grid=" << bt.grid
      << " order=" << bt.order << " schedule=" << bt.schedule << " run=" << bt.run
      << " ms=" << best << "\n";
  }
  return SSP_OK;
}

}  // extern "C"
