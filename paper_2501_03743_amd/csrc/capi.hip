// libsstep: the C ABI declared in include/sstep.h, on top of the gfx950
// kernels.  Host code only orders launches on the handle's stream, polls the
// device status word every few outer iterations and copies results back;
// every arithmetic step of a solve runs in the kernels.
#include <mutex>

#include "engine.hpp"
#include "measure.hpp"
#include "setup_kernels.hpp"

using namespace ssp;

namespace ssp {

int status_code(int st) {
  switch (st) {
    case ST_CONVERGED:
    case ST_ZERO_RHS:
      return SSP_OK;
    case ST_BREAKDOWN:
      return SSP_BREAKDOWN;
    default:
      return SSP_NOT_CONVERGED;
  }
}

// Builds the FP32 copy of a matrix (values, coefficients, Jacobi vector).
int ensure_fp32(ssp_handle *h, ssp_matrix *A) {
  if (A->has32) return SSP_OK;
  const unsigned nb = (unsigned)((A->n + kWG - 1) / kWG);
  if (A->kind == 0) {
    if (hipMalloc(&A->val32, sizeof(float) * A->nnz) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, SSP_ENOMEM, "FP32 matrix allocation failed");
    }
    const unsigned nbz = (unsigned)((A->nnz + kWG - 1) / kWG);
    k_to_float<<<nbz, kWG, 0, h->stream>>>(A->nnz, A->csr.val, A->val32);
    LAUNCHCHK(h);
    A->csr32 = CsrArgs<float>{A->csr.n, A->csr.rowptr, A->csr.colind, A->val32,
                              A->csr.rows_per_rb, A->csr.nrb, A->csr.variant,
                              A->csr.sell_col, nullptr, A->csr.slice_off, A->csr.slice_w,
                              A->csr.nslices,
                              A->sell_entries * (int64_t)(sizeof(float) + sizeof(int32_t)) >
                                  kInfinityCache,
                              A->csr.sell_wmax};
    if (A->sell_val) {
      const int64_t ne = A->sell_entries;
      if (hipMalloc(&A->sell_val32, sizeof(float) * (ne + kSellPad * kWave)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, SSP_ENOMEM, "FP32 sliced-ELL allocation failed");
      }
      k_to_float<<<(unsigned)((ne + kWG - 1) / kWG), kWG, 0, h->stream>>>(ne, A->sell_val,
                                                                           A->sell_val32);
      HIPCHK(h, hipMemsetAsync(A->sell_val32 + ne, 0, sizeof(float) * kSellPad * kWave, h->stream));
      LAUNCHCHK(h);
      A->csr32.sell_val = A->sell_val32;
    }
  } else {
    const StencilArgs<double> &S = A->sten;
    A->sten32 = StencilArgs<float>{S.n, S.nx, S.ny, S.nz, S.fx, S.fy, (float)S.diag,
                                   (float)S.off, nullptr};
    if (A->kind == SSP_STENCIL_3D7_VARK) {
      if (hipMalloc(&A->k32, sizeof(float) * A->n) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, SSP_ENOMEM, "FP32 coefficient allocation failed");
      }
      k_to_float<<<nb, kWG, 0, h->stream>>>(A->n, S.k, A->k32);
      LAUNCHCHK(h);
      A->sten32.k = A->k32;
    }
  }
  if (A->dinv) {
    if (hipMalloc(&A->dinv32, sizeof(float) * A->n) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, SSP_ENOMEM, "FP32 Jacobi allocation failed");
    }
    k_to_float<<<nb, kWG, 0, h->stream>>>(A->n, A->dinv, A->dinv32);
    LAUNCHCHK(h);
  }
  A->has32 = true;
  return SSP_OK;
}

}  // namespace ssp

namespace {

// Scratch of the allocation-free entry point (ssp_mpk_noalloc): the control
// block of the call, then the per-workgroup partial sums of the moments
// (at most kGridMax workgroups x 2 kSMax values).  One copy per GPU, held
// until the process ends.  Host code never names the array in a launch or a
// copy: it uses the device address that hipGetSymbolAddress returned for the
// current device at ssp_create (scratch_addr below).
constexpr size_t kScratchState = (sizeof(DevState) + 255) / 256 * 256;
constexpr size_t kScratchPartials = (size_t)kGridMax * 2 * kSMax;   // doubles
constexpr size_t kScratchBytes = kScratchState + kScratchPartials * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), looked up
// once per device.
int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return SSP_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_addr[device]) return SSP_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return SSP_EHIP;
  }
  scratch_addr[device] = p;
  return SSP_OK;
}

void hfree(void *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <typename P>
void hfree_t(P *&p) {
  void *q = (void *)p;
  hfree(q);
  p = nullptr;
}

// Leading dimension of the n x 2s blocks: n rounded up to `align` entries
// plus a stagger of 17 x 256 bytes.  Columns whose starts differ by a large
// power of two fall on the same HBM channels row for row; the block update
// streams 4s + 2 such columns at once and ran 30 % slower without the
// stagger (128^3 7-point, s = 4).
int64_t block_ld(int64_t n, int64_t align, int64_t elem_bytes) {
  return (n + align - 1) / align * align + kColumnStagger / elem_bytes;
}

int ensure_workspace(ssp_handle *h, int64_t n, int s, int hist_need, bool pcg,
                     bool gram = false) {
  Workspace &w = h->ws;
  if (!w.partials) HIPCHK(h, hipMalloc(&w.partials, sizeof(double) * kGridMax * 2 * kSMax));
  if (!w.partials_rr) HIPCHK(h, hipMalloc(&w.partials_rr, sizeof(double) * kGridMax));
  if (gram && !w.partials_gram)
    HIPCHK(h, hipMalloc(&w.partials_gram,
                        sizeof(double) * kGramGrid * kSMax * (2 * kSMax + 1)));
  if (n > w.n || s > w.s) {
    hfree_t(w.P1);
    hfree_t(w.P2);
    hfree_t(w.r);
    hfree_t(w.pcg_p);
    hfree_t(w.pcg_s);
    const int64_t nn = std::max(n, w.n);
    const int ss = std::max(s, w.s);
    const int64_t ld = block_ld(nn, 32, sizeof(double));  // 256-byte column alignment
    if (hipMalloc(&w.P1, sizeof(double) * ld * 2 * ss) != hipSuccess ||
        hipMalloc(&w.P2, sizeof(double) * ld * 2 * ss) != hipSuccess ||
        hipMalloc(&w.r, sizeof(double) * ld) != hipSuccess) {
      (void)hipGetLastError();
      hfree_t(w.P1);
      hfree_t(w.P2);
      hfree_t(w.r);
      w.n = w.s = 0;
      return fail(h, SSP_ENOMEM, "workspace allocation failed (n=" + std::to_string(n) + ")");
    }
    w.n = nn;
    w.s = ss;
    w.ld = ld;
  }
  if (pcg && !w.pcg_p) {
    if (hipMalloc(&w.pcg_p, sizeof(double) * w.ld) != hipSuccess ||
        hipMalloc(&w.pcg_s, sizeof(double) * w.ld) != hipSuccess) {
      (void)hipGetLastError();
      hfree_t(w.pcg_p);
      hfree_t(w.pcg_s);
      return fail(h, SSP_ENOMEM, "workspace allocation failed (n=" + std::to_string(n) + ")");
    }
  }
  if (hist_need > w.hist_cap) {
    hfree_t(w.hist);
    const int cap = std::max(hist_need, 1024);
    if (hipMalloc(&w.hist, sizeof(double) * cap) != hipSuccess) {
      (void)hipGetLastError();
      w.hist_cap = 0;
      return fail(h, SSP_ENOMEM, "history allocation failed");
    }
    w.hist_cap = cap;
  }
  return SSP_OK;
}

// FP32 blocks and vectors of the inner solves of mixed-precision refinement.
int ensure_workspace32(ssp_handle *h, int64_t n, int s) {
  Workspace &w = h->ws;
  if (n <= w.n32 && s <= w.s32) return SSP_OK;
  hfree_t(w.Q1);
  hfree_t(w.Q2);
  hfree_t(w.r32);
  hfree_t(w.d32);
  const int64_t nn = std::max(n, w.n32);
  const int ss = std::max(s, w.s32);
  const int64_t ld = block_ld(nn, 64, sizeof(float));
  if (hipMalloc(&w.Q1, sizeof(float) * ld * 2 * ss) != hipSuccess ||
      hipMalloc(&w.Q2, sizeof(float) * ld * 2 * ss) != hipSuccess ||
      hipMalloc(&w.r32, sizeof(float) * ld) != hipSuccess ||
      hipMalloc(&w.d32, sizeof(float) * ld) != hipSuccess) {
    (void)hipGetLastError();
    hfree_t(w.Q1);
    hfree_t(w.Q2);
    hfree_t(w.r32);
    hfree_t(w.d32);
    w.n32 = w.s32 = 0;
    return fail(h, SSP_ENOMEM, "FP32 workspace allocation failed (n=" + std::to_string(n) + ")");
  }
  w.n32 = nn;
  w.s32 = ss;
  w.ld32 = ld;
  return SSP_OK;
}

// Writes the header of the device control block (status, options): the
// handle's, or `dst` when given.
int state_init(ssp_handle *h, int s, int outer_max, int fixed, double rtol, int hist_cap,
               DevState *dst = nullptr) {
  DevState *c = h->h_init;
  HIPCHK(h, hipStreamSynchronize(h->stream));  // staging buffer reuse
  memset(c, 0, offsetof(DevState, vm));
  c->status = ST_RUNNING;
  c->k = 0;
  c->outer_max = outer_max;
  c->fixed = fixed;
  c->s = s;
  c->hist_cap = hist_cap;
  c->rtol = rtol;
  HIPCHK(h, hipMemcpyAsync(dst ? dst : h->st, c, offsetof(DevState, vm), hipMemcpyHostToDevice,
                           h->stream));
  return SSP_OK;
}

int read_state(ssp_handle *h, bool whole, const DevState *src = nullptr) {
  const size_t bytes = whole ? sizeof(DevState) : offsetof(DevState, vm);
  HIPCHK(h, hipMemcpyAsync(h->h_read, src ? src : h->st, bytes, hipMemcpyDeviceToHost,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return SSP_OK;
}

int check_matrix(ssp_handle *h, const ssp_matrix *A) {
  if (!A || A->h != h) return fail(h, SSP_EINVAL, "matrix is NULL or belongs to another handle");
  return SSP_OK;
}

// The true residual of the returned iterate and the results of the solve.
int finish_solve(ssp_handle *h, const ssp_matrix *A, const double *b, double *x, int s) {
  int rc = read_state(h, false);
  if (rc) return rc;
  const int status = h->h_read->status;
  if (status == ST_ZERO_RHS) HIPCHK(h, hipMemsetAsync(x, 0, sizeof(double) * A->n, h->stream));
  rc = launch_op<double>(h, A, x, EpiTrueRes{b}, 3);
  if (rc) return rc;
  rc = read_state(h, true);
  if (rc) return rc;
  const DevState &d = *h->h_read;
  // the iteration that broke down ran its matrix powers as well
  prof_collect(h, d.k + (status == ST_BREAKDOWN ? 1 : 0));
  h->prof_iter = -1;
  h->last_s = s;
  h->last_outer = (status == ST_ZERO_RHS) ? 0 : d.k;
  const double bn = std::sqrt(d.bb);
  h->last_true_rel = (status == ST_ZERO_RHS || bn == 0.0) ? 0.0 : std::sqrt(d.true_rr) / bn;
  const int len = std::min(h->last_outer + 1, h->ws.hist_cap);
  h->last_hist.assign(len, 0.0);
  if (status != ST_ZERO_RHS && len > 0)
    HIPCHK(h, hipMemcpy(h->last_hist.data(), h->ws.hist, sizeof(double) * len,
                        hipMemcpyDeviceToHost));
  return status_code(status);
}

// The three CSR kernel forms give bitwise-identical products; pick one for
// this matrix by timing four back-to-back products of each, alternating,
// best of three (SSP_CSR_VARIANT=0/1/2 forces one).  Preference order sliced ELL, row,
// staged: a later form is taken only if it is faster by more than 10 %, so
// that timing noise (a profiler's per-dispatch overhead, for instance)
// cannot flip the choice between runs.
int csr_pick_variant(ssp_handle *h, ssp_matrix *A) {
  const char *env = getenv("SSP_CSR_VARIANT");
  if (env && env[0] >= '0' && env[0] <= '2' && (env[0] != '2' || A->sell_col)) {
    A->csr.variant = env[0] - '0';
    return SSP_OK;
  }
  h->prof_on = false;
  int rc = ensure_workspace(h, 1, 1, 1, false);
  if (rc) return rc;
  double *y = nullptr, *xv = nullptr;
  HIPCHK(h, hipMalloc(&y, sizeof(double) * A->n));
  HIPCHK(h, hipMalloc(&xv, sizeof(double) * A->n));
  HIPCHK(h, hipMemsetAsync(xv, 0, sizeof(double) * A->n, h->stream));
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  const int nv = A->sell_col ? 3 : 2;
  float best[3] = {1e30f, 1e30f, 1e30f};
  for (int v = 0; v < nv && rc == SSP_OK; ++v) {   // warm-up
    A->csr.variant = v;
    rc = launch_op<double>(h, A, xv, EpiStore<double>{y}, 0);
  }
  for (int rep = 0; rep < 3 && rc == SSP_OK; ++rep)
    for (int v = 0; v < nv && rc == SSP_OK; ++v) {
      A->csr.variant = v;
      (void)hipEventRecord(e0, h->stream);
      for (int q = 0; q < 4 && rc == SSP_OK; ++q)
        rc = launch_op<double>(h, A, xv, EpiStore<double>{y}, 0);
      (void)hipEventRecord(e1, h->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best[v]) best[v] = ms;
    }
  int pick = (nv == 3) ? CSR_SELL : CSR_ROW;
  if (nv == 3 && best[CSR_ROW] < 0.9f * best[pick]) pick = CSR_ROW;
  if (best[CSR_STAGED] < 0.9f * best[pick]) pick = CSR_STAGED;
  A->csr.variant = pick;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(y);
  (void)hipFree(xv);
  return rc;
}

// Sliced ELL copy of a CSR matrix (slices of 64 rows, padded to the longest
// row of each slice).  Skipped (the form is then not offered) when padding
// would more than double the stored entries.
int csr_build_sell(ssp_handle *h, ssp_matrix *A) {
  const int64_t ns = (A->n + kWave - 1) / kWave;
  int32_t *w = nullptr;
  HIPCHK(h, hipMalloc(&w, sizeof(int32_t) * ns));
  k_sell_width<<<(unsigned)((ns + kWG - 1) / kWG), kWG, 0, h->stream>>>(A->n, ns, A->csr.rowptr,
                                                                        w);
  LAUNCHCHK(h);
  std::vector<int32_t> hw(ns);
  std::vector<int64_t> off(ns);
  HIPCHK(h, hipMemcpyAsync(hw.data(), w, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int64_t tot = 0;
  for (int64_t i = 0; i < ns; ++i) {
    off[i] = tot;
    tot += (int64_t)kWave * hw[i];
  }
  if (tot > 2 * std::max<int64_t>(A->nnz, 1) + kWave) {
    (void)hipFree(w);
    return SSP_OK;
  }
  // padding of kSellPad entries per lane after the last slice: the
  // narrow-slice kernel reads as many entries of every slice as the widest has
  const int64_t alloc = tot + kSellPad * kWave;
  if (hipMalloc(&A->slice_off, sizeof(int64_t) * ns) != hipSuccess ||
      hipMalloc(&A->sell_col, sizeof(int32_t) * alloc) != hipSuccess ||
      hipMalloc(&A->sell_val, sizeof(double) * alloc) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(w);
    hfree_t(A->slice_off);
    hfree_t(A->sell_col);
    hfree_t(A->sell_val);
    return SSP_OK;   // the form is optional
  }
  A->slice_w = w;
  A->sell_entries = tot;
  HIPCHK(h, hipMemsetAsync(A->sell_col + tot, 0, sizeof(int32_t) * kSellPad * kWave, h->stream));
  HIPCHK(h, hipMemsetAsync(A->sell_val + tot, 0, sizeof(double) * kSellPad * kWave, h->stream));
  HIPCHK(h, hipMemcpyAsync(A->slice_off, off.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice,
                           h->stream));
  k_sell_fill<<<(unsigned)((ns * kWave + kWG - 1) / kWG), kWG, 0, h->stream>>>(
      A->n, ns, A->csr.rowptr, A->csr.colind, A->csr.val, A->slice_off, A->slice_w, A->sell_col,
      A->sell_val);
  LAUNCHCHK(h);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  A->csr.sell_col = A->sell_col;
  A->csr.sell_val = A->sell_val;
  A->csr.slice_off = A->slice_off;
  A->csr.slice_w = A->slice_w;
  A->csr.nslices = ns;
  A->csr.sell_xcd = tot * (int64_t)(sizeof(double) + sizeof(int32_t)) > kInfinityCache;
  A->csr.sell_wmax = 0;
  for (int64_t i = 0; i < ns; ++i) A->csr.sell_wmax = std::max(A->csr.sell_wmax, (int)hw[i]);
  return SSP_OK;
}

int csr_finish_setup(ssp_handle *h, ssp_matrix *A) {
  // longest row -> rows per LDS block; Jacobi vector; kernel form
  int *d_max = nullptr;
  HIPCHK(h, hipMalloc(&d_max, sizeof(int)));
  HIPCHK(h, hipMemsetAsync(d_max, 0, sizeof(int), h->stream));
  const int64_t nb = (A->n + kWG - 1) / kWG;
  k_csr_maxrow<<<(unsigned)nb, kWG, 0, h->stream>>>(A->n, A->csr.rowptr, d_max);
  LAUNCHCHK(h);
  int maxrow = 0;
  HIPCHK(h, hipMemcpyAsync(&maxrow, d_max, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  (void)hipFree(d_max);
  int R = maxrow > 0 ? kCsrLds / maxrow : kCsrRowsMax;
  if (R > kCsrRowsMax) R = kCsrRowsMax;
  if (R < 1) R = 1;
  A->csr.rows_per_rb = R;
  A->csr.nrb = (A->n + R - 1) / R;
  HIPCHK(h, hipMalloc(&A->dinv, sizeof(double) * A->n));
  k_csr_dinv<<<(unsigned)nb, kWG, 0, h->stream>>>(A->n, A->csr.rowptr, A->csr.colind,
                                                  A->csr.val, A->dinv);
  LAUNCHCHK(h);
  // a constant diagonal needs no Jacobi vector (same values, less traffic)
  int *d_diff = nullptr;
  HIPCHK(h, hipMalloc(&d_diff, sizeof(int)));
  HIPCHK(h, hipMemsetAsync(d_diff, 0, sizeof(int), h->stream));
  k_all_equal<<<(unsigned)nb, kWG, 0, h->stream>>>(A->n, A->dinv, d_diff);
  LAUNCHCHK(h);
  int differs = 1;
  double d0 = 0.0;
  HIPCHK(h, hipMemcpyAsync(&differs, d_diff, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(&d0, A->dinv, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  (void)hipFree(d_diff);
  if (!differs && std::isfinite(d0) && d0 > 0.0) {
    A->dconst = d0;
    (void)hipFree(A->dinv);
    A->dinv = nullptr;
  }
  const int rc = csr_build_sell(h, A);
  if (rc) return rc;
  return csr_pick_variant(h, A);
}

int stencil_args(ssp_handle *h, int kind, int nx, int ny, int nz, const double *coef,
                 ssp_matrix *A) {
  if (nx < 1 || ny < 1 || nz < 1 || (kind == SSP_STENCIL_2D5 && nz != 1) ||
      kind < SSP_STENCIL_2D5 || kind > SSP_STENCIL_3D7_VARK)
    return fail(h, SSP_EINVAL, "invalid stencil kind or grid (kind=" + std::to_string(kind) + ")");
  const int64_t n = (int64_t)nx * ny * nz;
  if (n >= (int64_t)1 << 31) return fail(h, SSP_EINVAL, "grid too large (n=" + std::to_string(n) + ")");
  StencilArgs<double> &S = A->sten;
  S.n = n;
  S.nx = nx;
  S.ny = ny;
  S.nz = nz;
  S.fx = FastDiv{nx, 1.0 / nx};
  S.fy = FastDiv{ny, 1.0 / ny};
  S.k = nullptr;
  A->n = n;
  // SSP_MPK_TEMPORAL=0: one launch per matrix power everywhere; =2: the
  // temporally blocked launches wherever they apply, also on grids too small
  // to fill the GPU (for comparisons and tests)
  const char *tb = getenv("SSP_MPK_TEMPORAL");
  A->tb = (tb && tb[0] == '0') ? 0 : (tb && tb[0] == '2') ? 2 : 1;
  if (kind == SSP_STENCIL_3D7_VARK) {
    if (!coef) return fail(h, SSP_EINVAL, "3D7_VARK needs the device coefficient array");
    S.k = coef;
    S.diag = S.off = 0.0;
  } else {
    const double dflt[4][2] = {{0, 0}, {4.0, -1.0}, {6.0, -1.0}, {26.0, -1.0}};
    S.diag = coef ? coef[0] : dflt[kind][0];
    S.off = coef ? coef[1] : dflt[kind][1];
  }
  A->nnz = (kind == SSP_STENCIL_3D27) ? (int64_t)(3 * nx - 2) * (3 * ny - 2) * (3 * nz - 2)
           : (kind == SSP_STENCIL_2D5)
               ? 5LL * nx * ny - 2LL * nx - 2LL * ny
               : 7LL * nx * ny * nz - 2LL * nx * ny - 2LL * ny * nz - 2LL * nx * nz;
  return SSP_OK;
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------

// The true-residual judge of a predicted initial guess: optional damped
// Jacobi sweeps, then x is kept only if ||b - A x|| < ||b|| (a non-finite
// residual also falls back), else x = 0.
int warm_start_judge(ssp_handle *h, const ssp_matrix *A, const double *b, double *x,
                     const ssp_opts *o) {
  int rc = ensure_workspace(h, A->n, 1, 1, false);
  if (rc) return rc;
  Workspace &w = h->ws;
  const int sweeps = o->warm_sweeps > 0 ? o->warm_sweeps : 0;
  const double omega = o->warm_omega > 0.0 ? o->warm_omega : 2.0 / 3.0;
  double *tag = nullptr;
  const Prec<double> pc = prec_of(A, tag);
  double *cur = x, *nxt = w.r;
  for (int i = 0; i < sweeps; ++i) {
    rc = launch_op<double>(h, A, cur, EpiJacobiSweep{b, cur, nxt, pc, omega}, 3);
    if (rc) return rc;
    std::swap(cur, nxt);
  }
  if (cur != x)
    HIPCHK(h, hipMemcpyAsync(x, cur, sizeof(double) * A->n, hipMemcpyDeviceToDevice, h->stream));
  rc = launch_op<double>(h, A, x, EpiWarmCheck{b}, 3);
  if (rc) return rc;
  rc = read_state(h, false);
  if (rc) return rc;
  const double bb = h->h_read->bb, rr = h->h_read->true_rr;
  h->last_warm_rel0 = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
  const bool keep = bb > 0.0 && rr < bb;
  h->last_warm_kept = keep ? 1 : 0;
  if (!keep) HIPCHK(h, hipMemsetAsync(x, 0, sizeof(double) * A->n, h->stream));
  return SSP_OK;
}

// Largest diagonal entry of A, from the Jacobi data built at set-up (the
// default Chebyshev interval without a preconditioner).
int max_diagonal(ssp_handle *h, const ssp_matrix *A, double &dmax) {
  if (A->kind != 0 && A->kind != SSP_STENCIL_3D7_VARK) {
    dmax = A->sten.diag;
    return SSP_OK;
  }
  if (!A->dinv) {
    dmax = 1.0 / A->dconst;
    return SSP_OK;
  }
  // the first word of the (idle) partial-sum buffer holds the maximum's bits
  unsigned long long *d = reinterpret_cast<unsigned long long *>(h->ws.partials);
  HIPCHK(h, hipMemsetAsync(d, 0, sizeof(unsigned long long), h->stream));
  const unsigned nb = (unsigned)std::min<int64_t>((A->n + kWG - 1) / kWG, kGridMax);
  k_max_recip<<<nb, kWG, 0, h->stream>>>(A->n, A->dinv, d);
  LAUNCHCHK(h);
  unsigned long long bits = 0;
  HIPCHK(h, hipMemcpyAsync(&bits, d, sizeof(bits), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  memcpy(&dmax, &bits, sizeof(dmax));
  return SSP_OK;
}

// Centre c and inverse half-width g of the Chebyshev basis interval.
int cheb_params(ssp_handle *h, const ssp_matrix *A, const ssp_opts *o, double &c, double &g) {
  double lo = o ? o->basis_lo : 0.0, hi = o ? o->basis_hi : 0.0;
  if (!(hi > lo)) {
    lo = 0.0;
    if (A->prec == SSP_PREC_JACOBI) {
      hi = 2.0;
    } else {
      double dmax = 0.0;
      const int rc = max_diagonal(h, A, dmax);
      if (rc) return rc;
      hi = 2.0 * dmax;
    }
  }
  if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo))
    return fail(h, SSP_EINVAL, "Chebyshev basis: invalid interval");
  c = 0.5 * (hi + lo);
  g = 1.0 / (0.5 * (hi - lo));
  return SSP_OK;
}

int solve_sstep(ssp_handle *h, const ssp_matrix *A, const double *b, double *x, int s,
                double rtol, int maxit, const ssp_opts *o) {
  const int fixed = (o && o->fixed_outer > 0) ? o->fixed_outer : 0;
  const int outer_max = fixed ? fixed : (int)((maxit + (int64_t)s - 1) / s);
  const bool cheb = o && o->basis == SSP_BASIS_CHEBYSHEV;
  int rc = ensure_workspace(h, A->n, s, outer_max + 1, false, cheb);
  if (rc) return rc;
  double cc = 0.0, cg = 0.0;
  if (cheb) {
    rc = cheb_params(h, A, o, cc, cg);
    if (rc) return rc;
  }
  Workspace &w = h->ws;
  rc = state_init(h, s, outer_max, fixed ? 1 : 0, rtol, w.hist_cap);
  if (rc) return rc;
  double *tag = nullptr;
  // r = b - A x0 and z1 = B^-1 r into column 1 of the block used at k = 0
  rc = launch_op<double>(h, A, x, EpiInit{b, w.r, w.P2, prec_of(A, tag), w.hist}, 3);
  if (rc) return rc;
  if (A->prec == SSP_PREC_AMG) {   // z1 = B^-1 r by a V-cycle
    rc = amg_vcycle(h, A, w.r, w.P2);
    if (rc) return rc;
  }
  const iter_fn<double> step = cheb ? cheb_iteration_f64(s) : iteration_f64(s);
  const IterBufs<double> B{w.P1, w.P2, w.ld, x, w.r, cc, cg};
  const int trace_cap = (o && o->trace_cap > 0 && o->trace_vm && o->trace_alpha &&
                         o->trace_beta && o->trace_W) ? o->trace_cap : 0;
  int every = (o && o->check_every > 0) ? o->check_every : std::max(1, 32 / s);
  if (trace_cap) every = 1;
  int k = 0;
  rc = read_state(h, false);
  if (rc) return rc;
  while (k < outer_max && h->h_read->status == ST_RUNNING) {
    const int m = std::min(every, outer_max - k);
    for (int i = 0; i < m; ++i, ++k) {
      h->prof_iter = k;
      rc = step(h, A, B, k, i == 0, i == m - 1);
      if (rc) return rc;
    }
    h->prof_iter = -1;
    rc = read_state(h, trace_cap > 0);
    if (rc) return rc;
    if (trace_cap) {
      const DevState &d = *h->h_read;
      const int it = d.k - 1;  // iteration whose coefficients are in the block
      if (d.k == k && it < trace_cap) {
        memcpy(o->trace_vm + (size_t)it * 2 * s, d.vm, sizeof(double) * 2 * s);
        memcpy(o->trace_alpha + (size_t)it * s, d.alpha, sizeof(double) * s);
        memcpy(o->trace_beta + (size_t)it * s * s, d.beta, sizeof(double) * s * s);
        memcpy(o->trace_W + (size_t)it * s * s, d.W, sizeof(double) * s * s);
      }
    }
  }
  return finish_solve(h, A, b, x, s);
}

int solve_pcg(ssp_handle *h, const ssp_matrix *A, const double *b, double *x, double rtol,
              int maxit, const ssp_opts *o) {
  const int fixed = (o && o->fixed_outer > 0) ? o->fixed_outer : 0;
  const int outer_max = fixed ? fixed : maxit;
  int rc = ensure_workspace(h, A->n, 1, outer_max + 1, true);
  if (rc) return rc;
  Workspace &w = h->ws;
  rc = state_init(h, 1, outer_max, fixed ? 1 : 0, rtol, w.hist_cap);
  if (rc) return rc;
  double *tag = nullptr;
  const Prec<double> pc = prec_of(A, tag);
  rc = launch_op<double>(h, A, x, EpiPcgInit{b, w.r, w.pcg_p, pc, w.hist}, 3);
  if (rc) return rc;
  const int every = (o && o->check_every > 0) ? o->check_every : 32;
  const int G = grid_rows(A->n);
  int k = 0;
  rc = read_state(h, false);
  if (rc) return rc;
  while (k < outer_max && h->h_read->status == ST_RUNNING) {
    const int m = std::min(every, outer_max - k);
    for (int i = 0; i < m; ++i, ++k) {
      h->prof_iter = k;
      rc = launch_op<double>(h, A, w.pcg_p, EpiPcgSpmv{w.pcg_p, w.pcg_s}, 0);
      if (rc) return rc;
      prof_begin(h, 2);
      k_pcg_update<<<G, kWG, 0, h->stream>>>(A->n, x, w.r, w.pcg_p, w.pcg_s, pc, h->st,
                                             w.partials);
      k_finalize<FinPcgUpdate><<<1, kWG, 0, h->stream>>>(FinPcgUpdate{w.hist}, h->st, w.partials,
                                                         G);
      prof_end(h);
      LAUNCHCHK(h);
      prof_begin(h, 2);
      k_pcg_direction<<<G, kWG, 0, h->stream>>>(A->n, w.r, w.pcg_p, pc, h->st);
      prof_end(h);
      LAUNCHCHK(h);
    }
    h->prof_iter = -1;
    rc = read_state(h, false);
    if (rc) return rc;
  }
  return finish_solve(h, A, b, x, 1);
}

// Alg. 2 (PFCG): per step one operator pass with the three coupled dot
// products (one reduction) and one fused update with ||r||^2.  p and s live
// in the first block's two columns, w and the stored B^-1 r (Jacobi vector
// only) in the second block's.
int solve_pfcg(ssp_handle *h, const ssp_matrix *A, const double *b, double *x, double rtol,
               int maxit, const ssp_opts *o) {
  const int fixed = (o && o->fixed_outer > 0) ? o->fixed_outer : 0;
  const int outer_max = fixed ? fixed : maxit;
  int rc = ensure_workspace(h, A->n, 1, outer_max + 1, false);
  if (rc) return rc;
  Workspace &w = h->ws;
  rc = state_init(h, 1, outer_max, fixed ? 1 : 0, rtol, w.hist_cap);
  if (rc) return rc;
  double *tag = nullptr;
  const Prec<double> pc = prec_of(A, tag);
  double *p = w.P1, *sv = w.P1 + w.ld, *wv = w.P2;
  double *u = pc.dinv ? w.P2 + w.ld : nullptr;
  HIPCHK(h, hipMemsetAsync(p, 0, sizeof(double) * A->n, h->stream));
  HIPCHK(h, hipMemsetAsync(sv, 0, sizeof(double) * A->n, h->stream));
  rc = launch_op<double>(h, A, x, EpiPfcgInit{b, w.r, u, pc, w.hist}, 3);
  if (rc) return rc;
  const int every = (o && o->check_every > 0) ? o->check_every : 32;
  const int G = grid_rows(A->n);
  int k = 0;
  rc = read_state(h, false);
  if (rc) return rc;
  while (k < outer_max && h->h_read->status == ST_RUNNING) {
    const int m = std::min(every, outer_max - k);
    // within a batch, a step's stopping test runs in the next step's
    // operator-pass finalisation; the batch's last step has its own
    for (int i = 0; i < m; ++i, ++k) {
      h->prof_iter = k;
      rc = launch_op<double>(
          h, A, u ? u : w.r,
          EpiPfcgSpmv{w.r, u, sv, wv, pc.dc, i == 0 ? nullptr : w.partials_rr, G, w.hist}, 0,
          u ? 1.0 : pc.dc);
      if (rc) return rc;
      prof_begin(h, 2);
      k_pfcg_update<<<G, kWG, 0, h->stream>>>(A->n, x, w.r, p, sv, wv, u, pc, h->st,
                                              w.partials_rr);
      if (i == m - 1)
        k_finalize<FinUpdate><<<1, kWG, 0, h->stream>>>(FinUpdate{w.hist}, h->st, w.partials_rr,
                                                        G);
      prof_end(h);
      LAUNCHCHK(h);
    }
    h->prof_iter = -1;
    rc = read_state(h, false);
    if (rc) return rc;
  }
  return finish_solve(h, A, b, x, 1);
}

// Mixed precision: FP32 inner s-step solves (matrix powers and block updates
// in FP32; moments, s x s solves and the inner stopping test in FP64) of
// A d = r inside FP64 iterative refinement x += d, r = b - A x.
int solve_mixed(ssp_handle *h, ssp_matrix *A, const double *b, double *x, int s, double rtol,
                int maxit, const ssp_opts *o) {
  if (s > kSMaxF32)
    return fail(h, SSP_EUNSUPPORTED, "mixed precision supports s <= " + std::to_string(kSMaxF32));
  const double inner_rtol = (o && o->inner_rtol > 0.0) ? o->inner_rtol : 1e-5;
  const int max_refine = (o && o->max_refine > 0) ? o->max_refine : 10;
  const int inner_max = (int)((maxit + (int64_t)s - 1) / s);
  const bool cheb = o && o->basis == SSP_BASIS_CHEBYSHEV;
  int rc = ensure_workspace(h, A->n, 1, std::max(max_refine + 1, inner_max + 1), false, cheb);
  if (rc) return rc;
  double cc = 0.0, cg = 0.0;
  if (cheb) {
    rc = cheb_params(h, A, o, cc, cg);
    if (rc) return rc;
  }
  rc = ensure_workspace32(h, A->n, s);
  if (rc) return rc;
  rc = ensure_fp32(h, A);
  if (rc) return rc;
  Workspace &w = h->ws;
  // control block: inner-solve options plus the refinement loop's
  rc = state_init(h, s, inner_max, 0, inner_rtol, 0);
  if (rc) return rc;
  {
    DevState *c = h->h_init;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    c->ir_refine = 0;
    c->ir_max_refine = max_refine;
    c->ir_hist_cap = w.hist_cap;
    c->ir_rtol = rtol;
    c->ir_inner_rtol = inner_rtol;
    HIPCHK(h, hipMemcpyAsync(h->st, c, offsetof(DevState, vm), hipMemcpyHostToDevice, h->stream));
  }
  float *tag32 = nullptr;
  const Prec<float> pc32 = prec_of(A, tag32);
  const iter_fn<float> step = cheb ? cheb_iteration_f32(s) : iteration_f32(s);
  const IterBufs<float> B{w.Q1, w.Q2, w.ld32, w.d32, w.r32, cc, cg};
  const int every = (o && o->check_every > 0) ? o->check_every : std::max(1, 32 / s);
  int total_outer = 0, refine = 0, final_status = ST_MAXIT;
  for (refine = 0; refine <= max_refine; ++refine) {
    if (refine > 0) {
      // x += d, then the next outer step
      const int G = grid_rows(A->n);
      k_ir_add<<<G, kWG, 0, h->stream>>>(A->n, x, w.d32);
      LAUNCHCHK(h);
      h->h_init->ir_refine = refine;  // only this field changes
      HIPCHK(h, hipMemcpyAsync(&h->st->ir_refine, &h->h_init->ir_refine, sizeof(int),
                               hipMemcpyHostToDevice, h->stream));
      // the inner-solve fields the previous inner solve changed
      HIPCHK(h, hipMemcpyAsync(&h->st->outer_max, &h->h_init->outer_max, sizeof(int),
                               hipMemcpyHostToDevice, h->stream));
    }
    rc = launch_op<double>(h, A, x, EpiIrResidual{b, w.r32, w.Q2, w.d32, pc32, w.hist}, 3);
    if (rc) return rc;
    rc = read_state(h, false);
    if (rc) return rc;
    const int st = h->h_read->status;
    if (st != ST_RUNNING) {
      final_status = st;
      break;
    }
    int k = 0;
    while (k < inner_max && h->h_read->status == ST_RUNNING) {
      const int m = std::min(every, inner_max - k);
      for (int i = 0; i < m; ++i, ++k) {
        rc = step(h, A, B, k, i == 0, i == m - 1);
        if (rc) return rc;
      }
      rc = read_state(h, false);
      if (rc) return rc;
    }
    const int inner_k = h->h_read->k;
    total_outer += inner_k;
    if (h->h_read->status == ST_BREAKDOWN && inner_k == 0) {
      final_status = ST_BREAKDOWN;   // no progress possible
      break;
    }
  }
  h->prof_on = false;
  // final FP64 true residual, history of the outer (true) residuals
  if (final_status == ST_ZERO_RHS) HIPCHK(h, hipMemsetAsync(x, 0, sizeof(double) * A->n, h->stream));
  rc = launch_op<double>(h, A, x, EpiTrueRes{b}, 3);
  if (rc) return rc;
  rc = read_state(h, true);
  if (rc) return rc;
  const DevState &d = *h->h_read;
  h->last_s = s;
  h->last_outer = total_outer;
  const double bn = std::sqrt(d.ir_bb);
  h->last_true_rel = (final_status == ST_ZERO_RHS || bn == 0.0) ? 0.0 : std::sqrt(d.true_rr) / bn;
  const int len = std::min(std::min(refine, max_refine) + 1, w.hist_cap);
  h->last_hist.assign(len, 0.0);
  if (final_status != ST_ZERO_RHS && len > 0)
    HIPCHK(h, hipMemcpy(h->last_hist.data(), w.hist, sizeof(double) * len, hipMemcpyDeviceToHost));
  return status_code(final_status);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int ssp_create(ssp_handle **out, int device, void *stream) {
  if (!out) return SSP_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return SSP_EINVAL;
  }
  ssp_handle *h = new (std::nothrow) ssp_handle();
  if (!h) return SSP_ENOMEM;
  h->device = device;
  h->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess || hipMalloc(&h->st, sizeof(DevState)) != hipSuccess ||
      hipMemset(h->st, 0, sizeof(DevState)) != hipSuccess ||
      hipHostMalloc((void **)&h->h_init, sizeof(DevState), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&h->h_read, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ssp_destroy(h);
    return SSP_EHIP;
  }
  const int rc = scratch_setup(device);
  if (rc) {
    ssp_destroy(h);
    return rc;
  }
  *out = h;
  return SSP_OK;
}

int ssp_destroy(ssp_handle *h) {
  if (!h) return SSP_OK;
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  Workspace &w = h->ws;
  hfree_t(w.P1);
  hfree_t(w.P2);
  hfree_t(w.r);
  hfree_t(w.pcg_p);
  hfree_t(w.pcg_s);
  hfree_t(w.Q1);
  hfree_t(w.Q2);
  hfree_t(w.r32);
  hfree_t(w.d32);
  hfree_t(w.partials);
  hfree_t(w.partials_rr);
  hfree_t(w.partials_gram);
  hfree_t(w.hist);
  hfree_t(h->st);
  if (h->batch_mem) (void)hipFree(h->batch_mem);
  if (h->h_init) (void)hipHostFree(h->h_init);
  if (h->h_read) (void)hipHostFree(h->h_read);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  delete h;
  return SSP_OK;
}

const char *ssp_last_error(const ssp_handle *h) {
  static const char none[] = "";
  return h ? h->err.c_str() : none;
}

const char *ssp_status_string(int status) {
  switch (status) {
    case SSP_OK: return "converged";
    case SSP_NOT_CONVERGED: return "iteration limit reached before convergence";
    case SSP_BREAKDOWN: return "breakdown (non-SPD moment matrix, alpha(s) ~ 0 or non-finite value)";
    case SSP_EINVAL: return "invalid argument";
    case SSP_ENOMEM: return "out of device memory";
    case SSP_EHIP: return "HIP runtime error";
    case SSP_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
  }
}

int ssp_matrix_csr(ssp_handle *h, int64_t n, int64_t nnz, const int32_t *rowptr,
                   const int32_t *colind, const double *val, unsigned flags, ssp_matrix **out) {
  if (!h || !out) return SSP_EINVAL;
  *out = nullptr;
  if (n < 1 || nnz < n || nnz >= (int64_t)1 << 31 || !rowptr || !colind || !val)
    return fail(h, SSP_EINVAL, "ssp_matrix_csr: invalid sizes or pointers (n=" + std::to_string(n) + ")");
  HIPCHK(h, hipSetDevice(h->device));
  ssp_matrix *A = new (std::nothrow) ssp_matrix();
  if (!A) return SSP_ENOMEM;
  A->h = h;
  A->kind = 0;
  A->n = n;
  A->nnz = nnz;
  if (flags & SSP_COPY) {
    if (hipMalloc(&A->own_rowptr, sizeof(int32_t) * (n + 1)) != hipSuccess ||
        hipMalloc(&A->own_colind, sizeof(int32_t) * nnz) != hipSuccess ||
        hipMalloc(&A->own_val, sizeof(double) * nnz) != hipSuccess) {
      (void)hipGetLastError();
      ssp_matrix_destroy(A);
      return fail(h, SSP_ENOMEM, "ssp_matrix_csr: copy allocation failed");
    }
    (void)hipMemcpyAsync(A->own_rowptr, rowptr, sizeof(int32_t) * (n + 1),
                         hipMemcpyDeviceToDevice, h->stream);
    (void)hipMemcpyAsync(A->own_colind, colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice,
                         h->stream);
    (void)hipMemcpyAsync(A->own_val, val, sizeof(double) * nnz, hipMemcpyDeviceToDevice,
                         h->stream);
    rowptr = A->own_rowptr;
    colind = A->own_colind;
    val = A->own_val;
  }
  A->csr.n = n;
  A->csr.rowptr = rowptr;
  A->csr.colind = colind;
  A->csr.val = val;
  if (flags & SSP_VALIDATE) {
    int *d_bad = nullptr;
    int bad = 0;
    if (hipMalloc(&d_bad, sizeof(int)) != hipSuccess) {
      ssp_matrix_destroy(A);
      return fail(h, SSP_ENOMEM, "validation flag allocation failed");
    }
    (void)hipMemsetAsync(d_bad, 0, sizeof(int), h->stream);
    k_csr_validate<<<(unsigned)((n + kWG - 1) / kWG), kWG, 0, h->stream>>>(n, nnz, rowptr, colind,
                                                                           val, d_bad);
    (void)hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(d_bad);
    if (bad) {
      ssp_matrix_destroy(A);
      return fail(h, SSP_EINVAL, "ssp_matrix_csr: validation failed");
    }
  }
  int rc = csr_finish_setup(h, A);
  if (rc) {
    ssp_matrix_destroy(A);
    return rc;
  }
  *out = A;
  return SSP_OK;
}

int ssp_matrix_stencil(ssp_handle *h, int kind, int nx, int ny, int nz, const double *coef,
                       ssp_matrix **out) {
  if (!h || !out) return SSP_EINVAL;
  *out = nullptr;
  HIPCHK(h, hipSetDevice(h->device));
  ssp_matrix *A = new (std::nothrow) ssp_matrix();
  if (!A) return SSP_ENOMEM;
  A->h = h;
  A->kind = kind;
  int rc = stencil_args(h, kind, nx, ny, nz, coef, A);
  if (rc) {
    delete A;
    return rc;
  }
  if (kind == SSP_STENCIL_3D7_VARK) {
    if (hipMalloc(&A->dinv, sizeof(double) * A->n) != hipSuccess) {
      (void)hipGetLastError();
      delete A;
      return fail(h, SSP_ENOMEM, "Jacobi vector allocation failed");
    }
    k_vark_dinv<<<(unsigned)((A->n + kWG - 1) / kWG), kWG, 0, h->stream>>>(A->sten, A->dinv);
    LAUNCHCHK(h);
  } else {
    A->dconst = 1.0 / A->sten.diag;
  }
  *out = A;
  return SSP_OK;
}

int ssp_matrix_csr_from_stencil(ssp_handle *h, int kind, int nx, int ny, int nz,
                                const double *coef, ssp_matrix **out) {
  if (!h || !out) return SSP_EINVAL;
  *out = nullptr;
  HIPCHK(h, hipSetDevice(h->device));
  ssp_matrix tmp;
  int rc = stencil_args(h, kind, nx, ny, nz, coef, &tmp);
  if (rc) return rc;
  const int64_t n = tmp.n;
  // row pointer on the host from the row lengths of the grid (set-up only)
  std::vector<int32_t> rp(n + 1);
  rp[0] = 0;
  int64_t e = 0, p = 0;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x, ++p) {
        const int cx = 1 + (x > 0) + (x < nx - 1);
        const int cy = 1 + (y > 0) + (y < ny - 1);
        const int cz = (kind == SSP_STENCIL_2D5) ? 1 : 1 + (z > 0) + (z < nz - 1);
        e += (kind == SSP_STENCIL_3D27) ? cx * cy * cz : 1 + (cx - 1) + (cy - 1) + (cz - 1);
        if (e >= ((int64_t)1 << 31)) return fail(h, SSP_EINVAL, "nnz exceeds int32 indexing");
        rp[p + 1] = (int32_t)e;
      }
  ssp_matrix *A = new (std::nothrow) ssp_matrix();
  if (!A) return SSP_ENOMEM;
  A->h = h;
  A->kind = 0;
  A->n = n;
  A->nnz = e;
  if (hipMalloc(&A->own_rowptr, sizeof(int32_t) * (n + 1)) != hipSuccess ||
      hipMalloc(&A->own_colind, sizeof(int32_t) * e) != hipSuccess ||
      hipMalloc(&A->own_val, sizeof(double) * e) != hipSuccess) {
    (void)hipGetLastError();
    ssp_matrix_destroy(A);
    return fail(h, SSP_ENOMEM, "CSR allocation failed (nnz=" + std::to_string(e) + ")");
  }
  HIPCHK(h, hipMemcpy(A->own_rowptr, rp.data(), sizeof(int32_t) * (n + 1),
                      hipMemcpyHostToDevice));
  const unsigned nb = (unsigned)((n + kWG - 1) / kWG);
  switch (kind) {
    case SSP_STENCIL_2D5:
      k_stencil_fill<K_2D5><<<nb, kWG, 0, h->stream>>>(tmp.sten, A->own_rowptr, A->own_colind, A->own_val);
      break;
    case SSP_STENCIL_3D7:
      k_stencil_fill<K_3D7><<<nb, kWG, 0, h->stream>>>(tmp.sten, A->own_rowptr, A->own_colind, A->own_val);
      break;
    case SSP_STENCIL_3D27:
      k_stencil_fill<K_3D27><<<nb, kWG, 0, h->stream>>>(tmp.sten, A->own_rowptr, A->own_colind, A->own_val);
      break;
    default:
      k_stencil_fill<K_VARK><<<nb, kWG, 0, h->stream>>>(tmp.sten, A->own_rowptr, A->own_colind, A->own_val);
      break;
  }
  LAUNCHCHK(h);
  A->csr.n = n;
  A->csr.rowptr = A->own_rowptr;
  A->csr.colind = A->own_colind;
  A->csr.val = A->own_val;
  rc = csr_finish_setup(h, A);
  if (rc) {
    ssp_matrix_destroy(A);
    return rc;
  }
  *out = A;
  return SSP_OK;
}

int ssp_matrix_info(const ssp_matrix *A, int64_t *n, int64_t *nnz) {
  if (!A) return SSP_EINVAL;
  if (n) *n = A->n;
  if (nnz) *nnz = A->nnz;
  return SSP_OK;
}

int ssp_matrix_csr_arrays(const ssp_matrix *A, const int32_t **rowptr, const int32_t **colind,
                          const double **val) {
  if (!A || A->kind != 0) return SSP_EINVAL;
  if (rowptr) *rowptr = A->csr.rowptr;
  if (colind) *colind = A->csr.colind;
  if (val) *val = A->csr.val;
  return SSP_OK;
}

int ssp_matrix_csr_form(const ssp_matrix *A, int *form) {
  if (!A || !form) return SSP_EINVAL;
  *form = A->kind == 0 ? A->csr.variant : -1;
  return SSP_OK;
}

int ssp_matrix_destroy(ssp_matrix *A) {
  if (!A) return SSP_OK;
  if (A->h) {
    (void)hipSetDevice(A->h->device);
    (void)hipStreamSynchronize(A->h->stream);
  }
  hfree_t(A->own_rowptr);
  hfree_t(A->own_colind);
  hfree_t(A->own_val);
  hfree_t(A->val32);
  hfree_t(A->sell_col);
  hfree_t(A->sell_val);
  hfree_t(A->sell_val32);
  hfree_t(A->slice_off);
  hfree_t(A->slice_w);
  hfree_t(A->k32);
  hfree_t(A->dinv);
  hfree_t(A->dinv32);
  amg_free(A);
  delete A;
  return SSP_OK;
}

int ssp_set_preconditioner(ssp_matrix *A, int kind) {
  if (!A || (kind != SSP_PREC_NONE && kind != SSP_PREC_JACOBI && kind != SSP_PREC_AMG))
    return SSP_EINVAL;
  if (kind == SSP_PREC_AMG && !A->amg) return SSP_EINVAL;
  A->prec = kind;
  return SSP_OK;
}

int ssp_spmv(ssp_handle *h, const ssp_matrix *A, const double *x, double *y) {
  if (!h) return SSP_EINVAL;
  int rc = check_matrix(h, A);
  if (rc) return rc;
  if (!x || !y) return fail(h, SSP_EINVAL, "ssp_spmv: NULL vector");
  HIPCHK(h, hipSetDevice(h->device));
  rc = ensure_workspace(h, 1, 1, 1, false);
  if (rc) return rc;
  return launch_op<double>(h, A, x, EpiStore<double>{y}, 0);
}

int ssp_mpk(ssp_handle *h, const ssp_matrix *A, const double *r, int s, double *P, int64_t ld,
            double *vm) {
  if (!h) return SSP_EINVAL;
  int rc = check_matrix(h, A);
  if (rc) return rc;
  if (!r || !P || s < 1 || s > SSP_SMAX || s > A->n || ld < A->n)
    return fail(h, SSP_EINVAL, "ssp_mpk: invalid arguments (s=" + std::to_string(s) + ")");
  HIPCHK(h, hipSetDevice(h->device));
  rc = ensure_workspace(h, 1, 1, 1, false);
  if (rc) return rc;
  rc = state_init(h, s, 1, 1, 0.0, 0);
  if (rc) return rc;
  rc = mpk_f64(s)(h, A, r, P, ld, nullptr);
  if (rc) return rc;
  if (vm) {
    rc = read_state(h, true);
    if (rc) return rc;
    memcpy(vm, h->h_read->vm, sizeof(double) * 2 * s);
  }
  return SSP_OK;
}

int ssp_cheb_basis(ssp_handle *h, const ssp_matrix *A, const double *r, int s, double lo,
                   double hi, double *P, int64_t ld, double *gram) {
  if (!h) return SSP_EINVAL;
  int rc = check_matrix(h, A);
  if (rc) return rc;
  if (!r || !P || s < 1 || s > SSP_SMAX || s > A->n || ld < A->n || (ld % 2) != 0)
    return fail(h, SSP_EINVAL, "ssp_cheb_basis: invalid arguments (s=" + std::to_string(s) + ")");
  if (((uintptr_t)P % 16) != 0 || ((uintptr_t)r % 16) != 0)
    return fail(h, SSP_EINVAL, "ssp_cheb_basis: P and r must be 16-byte aligned");
  HIPCHK(h, hipSetDevice(h->device));
  rc = ensure_workspace(h, 1, 1, 1, false, true);
  if (rc) return rc;
  ssp_opts o{};
  o.basis_lo = lo;
  o.basis_hi = hi;
  double c = 0.0, g = 0.0;
  rc = cheb_params(h, A, &o, c, g);
  if (rc) return rc;
  rc = state_init(h, s, 1, 1, 0.0, 0);
  if (rc) return rc;
  double *out = h->ws.partials_rr;   // s (2s+1) <= kGridMax totals
  rc = cheb_basis_f64(s)(h, A, r, P, ld, c, g, out);
  if (rc) return rc;
  if (gram) {
    std::vector<double> t((size_t)s * (2 * s + 1));
    HIPCHK(h, hipMemcpyAsync(t.data(), out, sizeof(double) * t.size(), hipMemcpyDeviceToHost,
                             h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int a = 0; a < s; ++a) {
      for (int q = 0; q < s; ++q) gram[a * (s + 1) + q] = t[(size_t)a * (2 * s + 1) + q];
      gram[a * (s + 1) + s] = t[(size_t)a * (2 * s + 1) + 2 * s];
    }
  }
  return SSP_OK;
}

int ssp_mpk_noalloc(ssp_handle *h, const ssp_matrix *A, const double *r, int s, double *P,
                    int64_t ld, double *vm) {
  if (!h) return SSP_EINVAL;
  int rc = check_matrix(h, A);
  if (rc) return rc;
  if (!r || !P || s < 1 || s > SSP_SMAX || s > A->n || ld < A->n)
    return fail(h, SSP_EINVAL, "ssp_mpk_noalloc: invalid arguments (s=" + std::to_string(s) + ")");
  const int G = grid_of(A);
  if ((size_t)G * 2 * s > kScratchPartials)
    return fail(h, SSP_EINVAL, "ssp_mpk_noalloc: " + std::to_string(G) + " workgroups x 2s = " +
                                   std::to_string(2 * s) + " partial sums exceed the scratch (" +
                                   std::to_string(kScratchPartials) + ")");
  HIPCHK(h, hipSetDevice(h->device));
  unsigned char *base = h->device < kMaxDevices ? (unsigned char *)scratch_addr[h->device] : nullptr;
  if (!base) return fail(h, SSP_EHIP, "ssp_mpk_noalloc: no scratch address for this device");
  const Ctl ctl{(DevState *)base, (double *)(base + kScratchState)};
  // no event objects may be created here: profiling is off for this call
  const bool prof = h->prof_on;
  h->prof_on = false;
  rc = state_init(h, s, 1, 1, 0.0, 0, ctl.st);
  if (!rc) rc = mpk_f64(s)(h, A, r, P, ld, &ctl);
  if (!rc && vm) {
    rc = read_state(h, true, ctl.st);
    if (!rc) memcpy(vm, h->h_read->vm, sizeof(double) * 2 * s);
  }
  h->prof_on = prof;
  return rc;
}

int ssp_solve(ssp_handle *h, const ssp_matrix *A, const double *b, double *x, int s, double rtol,
              int maxit, const ssp_opts *opts) {
  if (!h) return SSP_EINVAL;
  int rc = check_matrix(h, A);
  if (rc) return rc;
  const int method = opts ? opts->method : SSP_METHOD_SSTEP;
  const int precision = opts ? opts->precision : SSP_PRECISION_FP64;
  if (!b || !x) return fail(h, SSP_EINVAL, "ssp_solve: NULL vector");
  if (!(rtol >= 0.0) || maxit < 0) return fail(h, SSP_EINVAL, "ssp_solve: rtol must be >= 0 and maxit >= 0");
  if (method == SSP_METHOD_SSTEP && (s < 1 || s > SSP_SMAX || s > A->n))
    return fail(h, SSP_EINVAL, "ssp_solve: s out of range (s=" + std::to_string(s) + ")");
  if (method != SSP_METHOD_SSTEP && method != SSP_METHOD_PCG && method != SSP_METHOD_PFCG)
    return fail(h, SSP_EINVAL, "ssp_solve: unknown method " + std::to_string(method));
  if (precision != SSP_PRECISION_FP64 && precision != SSP_PRECISION_MIXED_IR)
    return fail(h, SSP_EINVAL, "ssp_solve: unknown precision " + std::to_string(precision));
  if (precision == SSP_PRECISION_MIXED_IR && method != SSP_METHOD_SSTEP)
    return fail(h, SSP_EUNSUPPORTED, "ssp_solve: mixed precision is implemented for the s-step method");
  const int restarts = opts ? opts->restarts : 0;
  if (restarts < 0) return fail(h, SSP_EINVAL, "ssp_solve: restarts must be >= 0");
  const int basis = opts ? opts->basis : SSP_BASIS_MONOMIAL;
  if (basis != SSP_BASIS_MONOMIAL && basis != SSP_BASIS_CHEBYSHEV)
    return fail(h, SSP_EINVAL, "ssp_solve: unknown basis " + std::to_string(basis));
  if (basis == SSP_BASIS_CHEBYSHEV && method != SSP_METHOD_SSTEP)
    return fail(h, SSP_EUNSUPPORTED, "ssp_solve: the Chebyshev basis is for the s-step method");
  if (A->prec == SSP_PREC_AMG &&
      (method != SSP_METHOD_SSTEP || precision != SSP_PRECISION_FP64 ||
       basis != SSP_BASIS_MONOMIAL || (opts && opts->warm_start)))
    return fail(h, SSP_EUNSUPPORTED,
                "ssp_solve: the AMG preconditioner runs with the FP64 s-step method on the "
                "monomial basis without a warm start");
  HIPCHK(h, hipSetDevice(h->device));
  h->prof_on = opts && opts->profile;
  h->ev_used = 0;
  for (int c = 0; c < SSP_PROFILE_CLASSES; ++c) {
    h->prof_launch[c] = 0;
    h->prof_ms[c] = 0.0;
  }
  h->last_warm_kept = -1;
  h->last_warm_rel0 = NAN;
  h->last_restarts = 0;
  if (opts && opts->warm_start) {
    if (opts->warm_sweeps < 0 || opts->warm_omega < 0.0 || opts->warm_omega >= 2.0)
      return fail(h, SSP_EINVAL, "ssp_solve: warm_sweeps must be >= 0 and 0 <= warm_omega < 2");
    rc = warm_start_judge(h, A, b, x, opts);
    if (rc) return rc;
  }
  if (precision == SSP_PRECISION_MIXED_IR)
    return solve_mixed(h, const_cast<ssp_matrix *>(A), b, x, s, rtol, maxit, opts);
  const int sm = method == SSP_METHOD_SSTEP ? s : 1;   // CG-equivalent steps per outer iteration
  auto run = [&](int budget) {
    if (method == SSP_METHOD_PCG) return solve_pcg(h, A, b, x, rtol, budget, opts);
    if (method == SSP_METHOD_PFCG) return solve_pfcg(h, A, b, x, rtol, budget, opts);
    return solve_sstep(h, A, b, x, s, rtol, budget, opts);
  };
  rc = run(maxit);
  if (restarts > 0 && !(opts && opts->fixed_outer > 0)) {
    // residual replacement: the recursive test held, the true residual did
    // not; run again from the current x, whose first residual is the true one
    int outer = h->last_outer;
    std::vector<double> hist = h->last_hist;
    while (rc == SSP_OK && h->last_restarts < restarts && h->last_true_rel > rtol) {
      const int64_t left = (int64_t)maxit - (int64_t)outer * sm;
      if (left <= 0) break;
      rc = run((int)left);
      if (rc < 0) return rc;
      h->last_restarts++;
      outer += h->last_outer;
      hist.insert(hist.end(), h->last_hist.begin(), h->last_hist.end());
    }
    h->last_outer = outer;
    h->last_hist = hist;
  }
  return rc;
}

int ssp_get_iterations(const ssp_handle *h, int *outer, int *cg_equiv) {
  if (!h) return SSP_EINVAL;
  if (outer) *outer = h->last_outer;
  if (cg_equiv) *cg_equiv = h->last_outer * h->last_s;
  return SSP_OK;
}

int ssp_get_restarts(const ssp_handle *h, int *restarts) {
  if (!h) return SSP_EINVAL;
  if (restarts) *restarts = h->last_restarts;
  return SSP_OK;
}

int ssp_get_warm_start(const ssp_handle *h, int *kept, double *rel0) {
  if (!h) return SSP_EINVAL;
  if (kept) *kept = h->last_warm_kept;
  if (rel0) *rel0 = h->last_warm_rel0;
  return SSP_OK;
}

int ssp_get_residual_history(const ssp_handle *h, double *buf, int cap, int *len) {
  if (!h || cap < 0 || (cap > 0 && !buf)) return SSP_EINVAL;
  const int n = (int)h->last_hist.size();
  for (int i = 0; i < std::min(n, cap); ++i) buf[i] = h->last_hist[i];
  if (len) *len = n;
  return SSP_OK;
}

int ssp_get_true_residual(const ssp_handle *h, double *rel) {
  if (!h || !rel) return SSP_EINVAL;
  *rel = h->last_true_rel;
  return SSP_OK;
}

int ssp_stream_probe(ssp_handle *h, int mode, const double *src, double *dst, int64_t n,
                     int reps, double *ms) {
  if (!h || !src || !ms || n < 2 || (n % 2) != 0 || reps < 1 || (mode != 0 && mode != 1) ||
      (mode == 1 && !dst) || ((uintptr_t)src % 16) != 0 || (dst && ((uintptr_t)dst % 16) != 0))
    return h ? fail(h, SSP_EINVAL, "ssp_stream_probe: invalid arguments") : SSP_EINVAL;
  HIPCHK(h, hipSetDevice(h->device));
  int rc = ensure_workspace(h, 1, 1, 1, false);
  if (rc) return rc;
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(h, SSP_EHIP, "ssp_stream_probe: event creation failed");
  }
  auto launch = [&]() {
    if (mode == 0) k_stream_read<<<kGridMax, kWG, 0, h->stream>>>(n, src, h->ws.partials);
    else k_stream_copy<<<kGridMax, kWG, 0, h->stream>>>(n, src, dst);
  };
  launch();   // warm-up
  (void)hipEventRecord(e0, h->stream);
  for (int i = 0; i < reps; ++i) launch();
  (void)hipEventRecord(e1, h->stream);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(h, SSP_EHIP, std::string("ssp_stream_probe: ") + hipGetErrorString(e));
  *ms = (double)t / reps;
  return SSP_OK;
}

int ssp_get_profile(const ssp_handle *h, int *launches, double *ms) {
  if (!h) return SSP_EINVAL;
  for (int c = 0; c < SSP_PROFILE_CLASSES; ++c) {
    if (launches) launches[c] = h->prof_launch[c];
    if (ms) ms[c] = h->prof_ms[c];
  }
  return SSP_OK;
}

}  // extern "C"
