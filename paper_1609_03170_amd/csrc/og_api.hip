// Host side of the open-GRAPE library: operator preparation, workspace
// layout, the forward / checkpoint / adjoint orchestration and the C ABI
// declared in opengrape.h.
//
// Method (Boutin et al., Sec. III): rho is integrated slice by slice with
// classical RK4 (Eq. (14)); lambda is integrated backward with L^dag from
// sigma (Eqs. (11), (15)); the gradient of every slice is contracted from
// the pair of states (Eq. (13)).  Every RK4 step is evaluated in the
// nested (Horner) form
//     Z1 = rho + h/4 L(rho),  Z2 = rho + h/3 L(Z1),  Z3 = rho + h/2 L(Z2),
//     rho' = rho + h L(Z3),
// which equals rho + h L rho + h^2/2 L^2 rho + h^3/6 L^3 rho + h^4/24 L^4 rho
// exactly for the linear, slice-wise constant L, and needs one stage buffer
// less than the k1..k4 form.
//
// Memory: forward states are stored every S = ckpt_stride slices (default
// ceil(sqrt(N_t))); the backward sweep recomputes one segment of S states at
// a time, so the workspace grows as sqrt(N_t) d^2, not N_t d^2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/opengrape.h"
#include "og_device.h"

using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

og_status fail(og_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define OG_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(OG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define OG_CHECK_LAUNCH()                                                                     \
  do {                                                                                        \
    hipError_t e_ = hipGetLastError();                                                        \
    if (e_ != hipSuccess)                                                                     \
      return fail(OG_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e_));     \
  } while (0)

#define OG_TRY(expr)                 \
  do {                               \
    og_status s_ = (expr);           \
    if (s_ != OG_OK) return s_;      \
  } while (0)

// ---------------------------------------------------------------------------
// Host-side operator algebra (float64 complex, row-major d x d)
// ---------------------------------------------------------------------------
struct Mat {
  int d = 0;
  std::vector<cd> a;
  Mat() {}
  explicit Mat(int n) : d(n), a((size_t)n * n, cd(0, 0)) {}
  cd& operator()(int i, int j) { return a[(size_t)i * d + j]; }
  cd operator()(int i, int j) const { return a[(size_t)i * d + j]; }
};

Mat from_ptr(const void* p, int d, size_t index) {
  Mat m(d);
  const double* x = static_cast<const double*>(p) + 2 * (size_t)d * d * index;
  for (size_t e = 0; e < (size_t)d * d; ++e) m.a[e] = cd(x[2 * e], x[2 * e + 1]);
  return m;
}

Mat dagger(const Mat& m) {
  Mat r(m.d);
  for (int i = 0; i < m.d; ++i)
    for (int j = 0; j < m.d; ++j) r(i, j) = std::conj(m(j, i));
  return r;
}

Mat matmul(const Mat& x, const Mat& y) {
  Mat r(x.d);
  for (int i = 0; i < x.d; ++i)
    for (int k = 0; k < x.d; ++k) {
      const cd v = x(i, k);
      if (v == cd(0, 0)) continue;
      for (int j = 0; j < x.d; ++j) r(i, j) += v * y(k, j);
    }
  return r;
}

Mat axpy(const Mat& x, cd s, const Mat& y) {  // x + s*y
  Mat r = x;
  for (size_t e = 0; e < r.a.size(); ++e) r.a[e] += s * y.a[e];
  return r;
}

Mat scaled(cd s, const Mat& y) {
  Mat r(y.d);
  for (size_t e = 0; e < r.a.size(); ++e) r.a[e] = s * y.a[e];
  return r;
}

Mat transpose(const Mat& m) {
  Mat r(m.d);
  for (int i = 0; i < m.d; ++i)
    for (int j = 0; j < m.d; ++j) r(i, j) = m(j, i);
  return r;
}

double herm_defect(const Mat& m) {
  double worst = 0, scale = 0;
  for (int i = 0; i < m.d; ++i)
    for (int j = 0; j < m.d; ++j) {
      worst = std::max(worst, std::abs(m(i, j) - std::conj(m(j, i))));
      scale = std::max(scale, std::abs(m(i, j)));
    }
  return scale > 0 ? worst / scale : 0.0;
}

// Nonzero diagonals of m (offset o holds m[i, i + o]).
void collect_offsets(const Mat& m, std::vector<int>& offs) {
  for (int o = -(m.d - 1); o <= m.d - 1; ++o) {
    bool nz = false;
    for (int i = 0; i < m.d && !nz; ++i) {
      const int j = i + o;
      if (j >= 0 && j < m.d && m(i, j) != cd(0, 0)) nz = true;
    }
    if (nz && std::find(offs.begin(), offs.end(), o) == offs.end()) offs.push_back(o);
  }
  std::sort(offs.begin(), offs.end());
}

std::vector<cd> dia_values(const Mat& m, const std::vector<int>& offs, cd scale = cd(1, 0)) {
  std::vector<cd> v(offs.size() * (size_t)m.d, cd(0, 0));
  for (size_t t = 0; t < offs.size(); ++t)
    for (int i = 0; i < m.d; ++i) {
      const int j = i + offs[t];
      if (j >= 0 && j < m.d) v[t * m.d + i] = scale * m(i, j);
    }
  return v;
}

// Ladder order of the banded taps: diagonals 0, +1, -1 first, then the
// others; dissipator taps (0, 0) and (s, s) with s = +1 or -1 first.  Taps
// the operators lack enter with zero coefficients.  Applied (and *lad set)
// only when the result holds at most 5 diagonals and 3 dissipator taps, the
// compiled bounds of the ladder stage kernel; otherwise nothing changes.
void ladder_order(std::vector<int>& offs, std::vector<int>& tp, std::vector<int>& tq,
                  std::vector<std::vector<cd>>& dl, std::vector<std::vector<cd>>& dr, int d, int* lad) {
  std::vector<int> o2{0, 1, -1};
  for (int o : offs)
    if (o < -1 || o > 1) o2.push_back(o);
  if (o2.size() > 5) return;
  int iz = -1, iu = -1;
  for (size_t t = 0; t < tp.size(); ++t) {
    if (iz < 0 && tp[t] == 0 && tq[t] == 0) iz = (int)t;
    if (iu < 0 && tp[t] == tq[t] && (tp[t] == 1 || tp[t] == -1)) iu = (int)t;
  }
  const size_t n2 = tp.size() + (iz < 0) + (iu < 0);
  if (n2 > 3) return;
  const std::vector<cd> zero((size_t)d, cd(0, 0));
  std::vector<int> p2, q2;
  std::vector<std::vector<cd>> l2, r2;
  auto take = [&](int t, int p, int q) {
    p2.push_back(p);
    q2.push_back(q);
    l2.push_back(t >= 0 ? dl[t] : zero);
    r2.push_back(t >= 0 ? dr[t] : zero);
  };
  take(iz, 0, 0);
  take(iu, iu >= 0 ? tp[iu] : 1, iu >= 0 ? tq[iu] : 1);
  for (size_t t = 0; t < tp.size(); ++t)
    if ((int)t != iz && (int)t != iu) take((int)t, tp[t], tq[t]);
  offs = o2;
  tp = p2;
  tq = q2;
  dl = l2;
  dr = r2;
  *lad = 1;
}

// Upload a host complex128 vector converted to the working precision.
template <typename T>
og_status upload(const std::vector<cd>& h, og::cpx<T>** dptr) {
  std::vector<og::cpx<T>> tmp(h.size());
  for (size_t e = 0; e < h.size(); ++e) {
    tmp[e].re = (T)h[e].real();
    tmp[e].im = (T)h[e].imag();
  }
  const size_t bytes = std::max<size_t>(1, tmp.size()) * sizeof(og::cpx<T>);
  OG_HIP(hipMalloc((void**)dptr, bytes));
  if (!tmp.empty()) OG_HIP(hipMemcpy(*dptr, tmp.data(), tmp.size() * sizeof(og::cpx<T>), hipMemcpyHostToDevice));
  return OG_OK;
}

std::vector<cd> concat(const std::vector<std::vector<cd>>& parts) {
  std::vector<cd> r;
  for (auto& p : parts) r.insert(r.end(), p.begin(), p.end());
  return r;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kUmaxBlocks = 64;  // blocks of the max|u| reduction

// Workspace of og_evaluate_static: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never uses its name as an
// address (that is a host-side stand-in); the device address of each GPU's
// copy is resolved once per device with hipGetSymbolAddress (at og_create,
// or at the first og_evaluate_static on a device) and kept in
// g_scratch_ptr.
constexpr size_t kStaticWsBytes = size_t(OG_STATIC_WS_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (nullptr on error).
void* scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// ---------------------------------------------------------------------------
// Operator data of one direction of propagation
//   forward : A = G = -i H - 1/2 sum gamma c^dag c,  C_m = c_m
//   adjoint : A = G^dag,                              C_m = c_m^dag
// ---------------------------------------------------------------------------
struct DirHost {
  Mat A0;                 // u-independent part of A
  std::vector<Mat> Ak;    // d A / d u_k
  std::vector<Mat> C;     // collapse operators of this direction
  std::vector<double> g;  // their rates
};

enum Dir { FWD = 0, ADJ = 1 };

}  // namespace

// ---------------------------------------------------------------------------
// Engine (one per working precision)
// ---------------------------------------------------------------------------
struct EngineBase {
  virtual ~EngineBase() {}
  virtual size_t ws_bytes(int B, int n_t) const = 0;
  virtual og_status forward(int B, int n_t, double dt, const double* u, const void* rho0, void* rhoT, void* ws,
                            size_t ws_bytes, hipStream_t st) = 0;
  virtual og_status cost(const void* sigma, double* phi, hipStream_t st) = 0;
  virtual og_status adjoint(const void* sigma, hipStream_t st) = 0;
  virtual og_status gradient(double* grad, hipStream_t st) = 0;
  virtual og_status gradient_sum(double* grad, int accumulate, hipStream_t st) = 0;
  virtual og_status adaptive_stats(long* counts) = 0;
  virtual int fused_used() const = 0;
  // continuous batching (og_server_*)
  virtual og_status serve_submit(const og_request& r, hipStream_t st) = 0;
  virtual og_status serve_step(int max_slices, hipStream_t st, std::vector<long>& done) = 0;
  virtual int serve_active() const = 0;
  virtual void serve_clear() = 0;
};

struct og_server {
  og_ctx* ctx = nullptr;
  int max_active = 0;
  std::vector<long> completed;
};

struct og_ctx {
  int d = 0, K = 0, J = 0;
  og_options opt{};
  int path = OG_PATH_DENSE;
  int phase = 0;  // 0: nothing, 1: forward done, 2: adjoint done
  unsigned long long generation = 0;  // successful og_forward calls
  EngineBase* eng = nullptr;
  // host data for the stability estimate
  std::vector<double> h0_diag, h0_rad, hk_gersh, hk_frob;
  double h0_frob = 0, diss_bound = 0;
  int* status_dev = nullptr;
  double* umax_dev = nullptr;
  // observable penalty (og_set_penalty): Phi -= beta dt sum_n Tr(A rho_n)
  double pen_beta = 0.0;
  og::CooEntry* pen_coo = nullptr;
  int pen_nnz = 0;
  // adaptive steps (og_set_adaptive): relative / absolute tolerances, 0 = fixed steps
  double ad_rtol = 0.0, ad_atol = 0.0;
  // og_set_resident: final slices of the forward sweep whose states stay in
  // device memory (no checkpoint recompute for them)
  int resident = 0;
  int fused_on = 1;          // og_set_fused: fused RK4 steps where the structure allows
  int* host_flag = nullptr;  // pinned: problems still active after an attempt
  // kernel timing samples (og_profile)
  int prof_every = 0;
  long prof_counter = 0;
  std::vector<hipEvent_t> prof_ev;  // start, stop pairs
  size_t prof_used = 0;             // pairs recorded

  // Record the start event of a sampled launch; returns the pair index or -1.
  long prof_begin(hipStream_t st) {
    if (prof_every <= 0) return -1;
    if ((prof_counter++ % prof_every) != 0) return -1;
    if (prof_used >= 65536) return -1;
    if (prof_ev.size() < 2 * (prof_used + 1)) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return -1;
      if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1;
      }
      prof_ev.push_back(a);
      prof_ev.push_back(b);
    }
    if (hipEventRecord(prof_ev[2 * prof_used], st) != hipSuccess) return -1;
    return (long)prof_used++;
  }
  void prof_end(long idx, hipStream_t st) {
    if (idx >= 0) (void)hipEventRecord(prof_ev[2 * idx + 1], st);
  }
};

namespace {

template <typename T>
struct DirDev {
  // banded
  og::BandOps<T> band{};
  og::cpx<T>* bA0 = nullptr;
  og::cpx<T>* bAk = nullptr;
  og::cpx<T>* bDl = nullptr;
  og::cpx<T>* bDr = nullptr;
  // dense
  og::cpx<T>* A0 = nullptr;    // d x d
  og::cpx<T>* Ak = nullptr;    // K x d x d
  og::cpx<T>* C = nullptr;     // J x d x d
  og::cpx<T>* Chat = nullptr;  // (J d) x d: rows m d .. : gamma_m / 2 * C_m^dag
};

template <typename T>
struct Engine : EngineBase {
  og_ctx* ctx;
  int d, K, J;
  bool banded;
  long E;   // elements per matrix
  long EH;  // elements of a packed Hermitian half, d (d + 1) / 2
  DirDev<T> dir[2];
  og::HBand<T> hband{};
  og::cpx<T>* hHd = nullptr;   // banded H_k diagonals
  // weights of the Hermitian-half contraction (band_contract_half_kernel)
  // by kind of offset o in (0, +1, -1, +N, -N): fhw[a][k][kind] =
  // H_k[a - o, a]; half_ok when the H_k allow that contraction
  og::cpx<T>* fhw = nullptr;
  bool half_ok = false;
  int half_k0 = 0;  // some H_k has a diagonal term
  // fused RK4 step (rk4_fused_kernel) per direction, when the operators have
  // the multi-level x oscillator structure it needs
  bool fused[2] = {false, false};
  og::FusedGeo fgeo[2]{};
  size_t fused_lds[2] = {0, 0};
  size_t fused_lds_slots[2] = {0, 0};  // serving launches: + the coefficient rows of the window
  // the same step on smaller tiles (two more n-blocks per axis) for the
  // smallest grids: more, shorter blocks
  og::FusedGeo fgeo_s[2];
  size_t fused_lds_s[2] = {0, 0};
  size_t fused_lds_slots_s[2] = {0, 0};
  // waves per fused-step block: 8 in float64; in float32 4 (four blocks per
  // CU), or 8 for grids of fewer than kFusedSmall blocks, which fill less
  // than one round of the chip and wait on each block's own latency; grids
  // of fewer than kFusedTiny blocks also take the smaller tiles of fgeo_s
  // (measured at d = 240: 20.3 instead of 22.1 us at 21 blocks, 33.5
  // instead of 27.0 at 336)
  // (measured at d = 240: 8 waves 22 / 27 / 40 us at 21 / 336 / 672 blocks
  // against 32 / 34 / 40 us with 4; 4 waves ahead from 1008 blocks on)
  static constexpr int kFusedSmall = 768;
  static constexpr int kFusedTiny = 128;
  // fused-step coefficient data per direction: A0 and A_k on the five
  // diagonals (0, +1, -1, -N, +N) row by row (d x 5, K x d x 5), the row
  // (d x 3) and column (d x FDR) factors of the dissipator taps
  og::cpx<T>*fa0[2] = {nullptr, nullptr}, *fak[2] = {nullptr, nullptr};
  og::cpx<T>*fdl[2] = {nullptr, nullptr}, *fdr[2] = {nullptr, nullptr};
  og::cpx<T>* fcoef[2] = {nullptr, nullptr};  // ring of rows of FSLOT coefficients per slice
  int fc0[2] = {0, 0}, fc1[2] = {0, 0};
  og::cpx<T>* HT = nullptr;    // dense: transposes of H_k, K x d x d
  int ntile = 0;
  static constexpr bool comp = sizeof(T) == 4;  // compensated states in float32

  // evaluation state
  int B = 0, n_t = 0, S = 1, n_seg = 0;
  double dt = 0;
  const double* u = nullptr;
  // workspace views
  og::cpx<T>*cur_hi, *cur_lo, *lam_hi, *lam_lo, *Za, *Zb;
  og::cpx<T>* cur_base = nullptr;  // the buffer cur_hi is bound to (the fused step swaps buffers)
  og::cpx<T>*ck_hi, *ck_lo, *sg_hi, *sg_lo;
  og::cpx<T>* tail = nullptr;  // resident states rho_{n_t - n_tail} .. rho_{n_t}
  int n_tail = 0;
  og::cpx<T>*Z1, *Z2, *Z3, *Zb1, *Zb2, *Zb3;
  og::cpx<T>*st_hi, *st_lo;  // substep start states (EXACT, n_sub > 1)
  og::cpx<T>*Aj[2], *X, *W, *Wp, *Ps;
  // banded: diagonal coefficients of a chunk of up to kCoefChunk slices per
  // direction, [slice - cc0[dr]][problem][diagonal][i]; a sweep refills the
  // chunk in the order it walks the slices (coef_hint)
  static constexpr int kCoefChunk = 64;
  // Stage launches of fewer blocks than this take the serving launch shape
  // (one or two rows per thread): their blocks finish sooner, which is what
  // a grid that does not fill the chip waits on.  Measured at d = 240: in
  // float32 the small shape is 1.4-1.5x faster at 36 and 144 blocks and 3 %
  // slower at 576; in float64 1.3x faster at 36 and 144, 10 % at 576, even
  // at 1152.
  static constexpr long kSmallStageGrid = sizeof(T) == 4 ? 384 : 1024;
  // Float32 launches of fewer blocks than this (and at least
  // kSmallStageGrid) run two rows per thread, 512 threads: measured at
  // d = 240, 9 % faster than four rows at 576 blocks, 5 % at 1152, 3 % at
  // 2304; 3 % slower at 3456 and 4 % at 4608.
  static constexpr long kMidStageGrid = 2880;
  og::cpx<T>* acoef[2];
  int cc0[2] = {0, 0}, cc1[2] = {0, 0};  // slices [cc0, cc1) held; empty when cc1 <= cc0
  struct CoefHint {
    int lo, hi;
    bool asc;
  } chint[2] = {{0, 0, true}, {0, 0, true}};
  void coef_hint(int dr, int lo, int hi, bool asc) { chint[dr] = CoefHint{lo, hi, asc}; }
  void coef_reset() { cc0[0] = cc1[0] = cc0[1] = cc1[1] = fc0[0] = fc1[0] = fc0[1] = fc1[1] = 0; }
  int max_nA() const { return std::max(dir[0].band.nA, dir[1].band.nA); }
  const og::cpx<T>* coef_ptr(int dr, int j) const {
    return acoef[dr] + (size_t)(j - cc0[dr]) * B * dir[dr].band.nA * d;
  }
  double* grad;
  double* pen;  // per-problem penalty traces Tr(A rho_n), n = 0..N_t

  Engine(og_ctx* c) : ctx(c), d(c->d), K(c->K), J(c->J), banded(c->path == OG_PATH_BANDED), E((long)c->d * c->d),
                         EH((long)c->d * (c->d + 1) / 2) {}

  // Dense GEMMs: float32/float64 matrix-core GEMM, or for the split
  // precisions the 16-bit three-product split GEMM (float32 storage).
  // One launch of up to GM products (GemmArgs holds GM operand sets).
  void launch_gemm(const og::GemmArgs<T>& g, dim3 grid) {
    if (g.nm < 1 || g.nm > og::GM) return;  // callers split larger sets (launch_gemm_set)
    if constexpr (sizeof(T) == 4) {
      if (ctx->opt.prec == OG_F32_SPLIT_BF16) {
        og::zgemm_split_kernel<og::SPLIT_BF16><<<grid, 256, 0, st>>>(g);
        return;
      }
      if (ctx->opt.prec == OG_F32_SPLIT_F16) {
        og::zgemm_split_kernel<og::SPLIT_F16><<<grid, 256, 0, st>>>(g);
        return;
      }
    }
    // float32 grids of at least four blocks per CU take the double-buffered
    // variant at four waves per SIMD (all blocks resident at once); measured
    // with d = 240, B = 16: 1024 blocks 76.6 -> 70.2 us, while a d = 512
    // product of 320 blocks took 69.2 -> 83.4 us, so smaller grids keep one
    // buffer and the unrestricted register count
    const long nblk = (long)grid.x * grid.y * grid.z;
    if (sizeof(T) == 4 && nblk >= 4L * 256)
      og::zgemm_kernel<T, 2><<<grid, 256, 0, st>>>(g);
    else
      og::zgemm_kernel<T, 1><<<grid, 256, 0, st>>>(g);
  }

  ~Engine() override {
    for (int s = 0; s < 2; ++s) {
      void* ps[] = {dir[s].bA0, dir[s].bAk, dir[s].bDl, dir[s].bDr, dir[s].A0, dir[s].Ak, dir[s].C, dir[s].Chat};
      for (void* p : ps)
        if (p) (void)hipFree(p);
    }
    if (hHd) (void)hipFree(hHd);
    if (fhw) (void)hipFree(fhw);
    if (HT) (void)hipFree(HT);
    for (int s = 0; s < 2; ++s)
      for (void* p : {(void*)fa0[s], (void*)fak[s], (void*)fdl[s], (void*)fdr[s]})
        if (p) (void)hipFree(p);
  }

  // Structure test of the fused RK4 step (rk4_fused_kernel) for direction
  // s of the operators h, on the dissipator taps (tp, tq, values dl, dr) of
  // the banded setup: diagonals of A(u) only at 0, +-1 and +-N with
  // d = nq N, taps (0, 0), (s, s) with s = +-1 and (t N, t N) with t = +-1
  // of one sign, with real factors;
  // the +-1 couplings must vanish between blocks of N (rows n = N - 1 for +1,
  // n = 0 for -1); nq <= 4 and a tile edge T with nq (T + 6) <= 64 whose LDS
  // needs fit in 64 KiB.  Then the coefficient data of the fused step are
  // uploaded; otherwise the four-launch stage kernels run.
  og_status fused_setup(int s, const DirHost& h, const std::vector<int>& tp, const std::vector<int>& tq,
                        const std::vector<std::vector<cd>>& dl, const std::vector<std::vector<cd>>& dr) {
    fused[s] = false;
    std::vector<int> offs;
    collect_offsets(h.A0, offs);
    for (auto& m : h.Ak) collect_offsets(m, offs);
    int N = 0;  // block length from the diagonals beyond 0, +-1 and the taps beyond (0, 0), (+-1, +-1)
    auto take = [&](int o) {
      const int a = o < 0 ? -o : o;
      if (N == 0) N = a;
      return a == N;
    };
    for (int o : offs)
      if (o < -1 || o > 1)
        if (!take(o)) return OG_OK;
    int s1 = 0, t2 = 0, i0 = -1, i1 = -1, i2 = -1;
    for (size_t t = 0; t < tp.size(); ++t) {
      if (tp[t] != tq[t]) return OG_OK;
      const int p = tp[t];
      if (p == 0) {
        if (i0 >= 0) return OG_OK;
        i0 = (int)t;
      } else if (p == 1 || p == -1) {
        if (i1 >= 0) return OG_OK;
        i1 = (int)t;
        s1 = p;
      } else {
        if (i2 >= 0 || !take(p)) return OG_OK;
        i2 = (int)t;
        t2 = p > 0 ? 1 : -1;
      }
    }
    if (N == 0) N = d;
    if (N < 2 || d % N != 0) return OG_OK;
    const int nq = d / N;
    if (nq > 4 || (nq == 1 && i2 >= 0)) return OG_OK;
    for (int t : {i0, i1, i2})  // the kernel takes the dissipator factors as real
      if (t >= 0)
        for (int i = 0; i < d; ++i)
          if (dl[t][i].imag() != 0.0 || dr[t][i].imag() != 0.0) return OG_OK;
    if (s1 == 0) s1 = t2 != 0 ? t2 : 1;  // no (+-1, +-1) tap: a zero one
    if (t2 != 0 && t2 != s1) return OG_OK;  // compiled for taps (s, s), (s N, s N) of one sign
    if (t2 == 0 && nq > 1) t2 = s1;         // no (t N, t N) tap: a zero one
    const int slot_off[5] = {0, 1, -1, -N, N};
    std::vector<std::vector<cd>> a5;  // A0 and A_k on the five slots
    a5.push_back(dia_values(h.A0, std::vector<int>(slot_off, slot_off + 5)));
    for (auto& m : h.Ak) a5.push_back(dia_values(m, std::vector<int>(slot_off, slot_off + 5)));
    // no +-1 coupling across a block boundary, for any u; none for the (s, s) tap
    for (int i = 0; i < d; ++i) {
      const int n = i % N;
      for (auto& v : a5) {
        if (n == N - 1 && v[(size_t)1 * d + i] != cd(0, 0)) return OG_OK;
        if (n == 0 && v[(size_t)2 * d + i] != cd(0, 0)) return OG_OK;
      }
      if (i1 >= 0 && ((s1 > 0 && n == N - 1) || (s1 < 0 && n == 0)))
        if (dl[i1][i] != cd(0, 0) || dr[i1][i] != cd(0, 0)) return OG_OK;
    }
    // tile edge: the widest that fits the lanes (nq (T + 6) <= 64), the
    // compiled LDS stride (window edge min(T + 8, N) <= WS) and 64 KiB of LDS
    const int ws = nq == 1 ? og::fused_ws<T, 1>() : nq == 2 ? og::fused_ws<T, 2>()
                 : nq == 3 ? og::fused_ws<T, 3>() : og::fused_ws<T, 4>();
    const int tlane = 64 / nq - 6;
    int nb = (N + tlane - 1) / tlane;
    size_t bytes = 0;
    size_t bytes_lc = 0;
    for (; nb <= N; ++nb) {
      const int tmax = (N + nb - 1) / nb;
      bytes = (size_t)og::fused_lds_elems(nq, ws, tmax) * sizeof(og::cpx<T>);
      bytes_lc = (size_t)og::fused_lds_elems(nq, ws, tmax, true) * sizeof(og::cpx<T>);
      if (std::min(tmax + 8, N) <= ws && bytes <= 65536) break;
    }
    if (nb > N || (N + nb - 1) / nb < 2) return OG_OK;
    // coefficient data, row by row
    std::vector<cd> a0t((size_t)d * 5), akt((size_t)K * d * 5), dlt((size_t)d * 3, cd(0, 0));
    std::vector<cd> drt((size_t)d * og::FDR, cd(0, 0));
    for (size_t m = 0; m < a5.size(); ++m)
      for (int i = 0; i < d; ++i)
        for (int a = 0; a < 5; ++a) {
          const cd v = a5[m][(size_t)a * d + i];
          if (m == 0)
            a0t[(size_t)i * 5 + a] = v;
          else
            akt[((m - 1) * (size_t)d + i) * 5 + a] = v;
        }
    const int idx[3] = {i0, i1, i2};
    for (int t = 0; t < 3; ++t)
      if (idx[t] >= 0)
        for (int i = 0; i < d; ++i) {
          dlt[(size_t)i * 3 + t] = dl[idx[t]][i];
          drt[(size_t)i * og::FDR + t] = dr[idx[t]][i];
        }
    OG_TRY(upload<T>(a0t, &fa0[s]));
    OG_TRY(upload<T>(akt, &fak[s]));
    OG_TRY(upload<T>(dlt, &fdl[s]));
    OG_TRY(upload<T>(drt, &fdr[s]));
    og::FusedGeo& g = fgeo[s];
    g = og::FusedGeo{};
    g.N = N;
    g.nq = nq;
    g.nb = nb;
    g.ntile = nb * (nb + 1) / 2;
    g.s1 = s1;
    g.t2 = t2;
    fused_lds[s] = bytes;
    fused_lds_slots[s] = bytes_lc;
    {
      const int nbs = std::max(nb, std::min(nb + 2, N / 2));
      const int tmax = (N + nbs - 1) / nbs;
      og::FusedGeo& gs = fgeo_s[s];
      gs = g;
      gs.nb = nbs;
      gs.ntile = nbs * (nbs + 1) / 2;
      fused_lds_s[s] = (size_t)og::fused_lds_elems(nq, ws, tmax) * sizeof(og::cpx<T>);
      fused_lds_slots_s[s] = (size_t)og::fused_lds_elems(nq, ws, tmax, true) * sizeof(og::cpx<T>);
    }
    fused[s] = true;
    return OG_OK;
  }

  og_status init(const DirHost host[2], const std::vector<Mat>& Hk) {
    // upper-triangular tiles (the kernels compute a tile's position from its index)
    const int nt = (d + og::TS - 1) / og::TS;
    ntile = nt * (nt + 1) / 2;
    for (int s = 0; s < 2; ++s) {
      const DirHost& h = host[s];
      DirDev<T>& dv = dir[s];
      if (banded) {
        std::vector<int> offs;
        collect_offsets(h.A0, offs);
        for (auto& m : h.Ak) collect_offsets(m, offs);
        if (offs.empty()) offs.push_back(0);
        std::vector<std::vector<cd>> dl, dr;
        std::vector<int> tp, tq;
        for (size_t m = 0; m < h.C.size(); ++m) {
          if (h.g[m] == 0.0) continue;
          std::vector<int> co;
          collect_offsets(h.C[m], co);
          for (int p : co)
            for (int q : co) {
              tp.push_back(p);
              tq.push_back(q);
              std::vector<int> one_p{p}, one_q{q};
              dl.push_back(dia_values(h.C[m], one_p, cd(h.g[m], 0)));
              dr.push_back(dia_values(h.C[m], one_q));
            }
        }
        // ladder order when it fits the (5, 3) ladder kernel
        dv.band.lad = 0;
        ladder_order(offs, tp, tq, dl, dr, d, &dv.band.lad);
        dv.band.nA = (int)offs.size();
        for (size_t t = 0; t < offs.size(); ++t) dv.band.offA[t] = offs[t];
        std::vector<std::vector<cd>> ak;
        for (auto& m : h.Ak) ak.push_back(dia_values(m, offs));
        OG_TRY(upload<T>(dia_values(h.A0, offs), &dv.bA0));
        OG_TRY(upload<T>(concat(ak), &dv.bAk));
        const int nD = (int)tp.size();
        for (int t = 0; t < nD; ++t) {
          dv.band.dp[t] = tp[t];
          dv.band.dq[t] = tq[t];
        }
        dv.band.nD = nD;
        OG_TRY(upload<T>(concat(dl), &dv.bDl));
        OG_TRY(upload<T>(concat(dr), &dv.bDr));
        dv.band.A0 = dv.bA0;
        dv.band.Ak = dv.bAk;
        dv.band.Dl = dv.bDl;
        dv.band.Dr = dv.bDr;
        OG_TRY(fused_setup(s, h, tp, tq, dl, dr));
      } else {
        OG_TRY(upload<T>(h.A0.a, &dv.A0));
        std::vector<std::vector<cd>> ak, cc, ch;
        for (auto& m : h.Ak) ak.push_back(m.a);
        OG_TRY(upload<T>(concat(ak), &dv.Ak));
        for (size_t m = 0; m < h.C.size(); ++m) {
          cc.push_back(h.C[m].a);
          ch.push_back(scaled(cd(0.5 * h.g[m], 0), dagger(h.C[m])).a);
        }
        OG_TRY(upload<T>(concat(cc), &dv.C));
        OG_TRY(upload<T>(concat(ch), &dv.Chat));
      }
    }
    if (banded) {
      std::vector<int> offs;
      for (auto& m : Hk) collect_offsets(m, offs);
      if (offs.empty()) offs.push_back(0);
      hband.nH = (int)offs.size();
      for (size_t t = 0; t < offs.size(); ++t) hband.offH[t] = offs[t];
      std::vector<std::vector<cd>> hv;
      for (auto& m : Hk) hv.push_back(dia_values(m, offs));
      OG_TRY(upload<T>(concat(hv), &hHd));
      hband.Hd = hHd;
      OG_TRY(half_setup(offs, hv));
    } else {
      std::vector<std::vector<cd>> ht;
      for (auto& m : Hk) ht.push_back(transpose(m).a);
      OG_TRY(upload<T>(concat(ht), &HT));
    }
    return OG_OK;
  }

  // The Hermitian-half contraction needs both directions fused (their level
  // count nq and level size N), K <= FCK, every diagonal offset of the H_k
  // one of 0, +1, -1, +N, -N and the +-1 diagonals zero where they cross
  // from one level block to the next.
  og_status half_setup(const std::vector<int>& offs, const std::vector<std::vector<cd>>& hv) {
    half_ok = false;
    if (!(fused[FWD] && fused[ADJ]) || K < 1 || K > og::FCK) return OG_OK;
    const int Nn = fgeo[ADJ].N, nq = fgeo[ADJ].nq;
    const int ko[5] = {0, 1, -1, Nn, -Nn};
    std::vector<int> kind(offs.size(), -1);
    for (size_t t = 0; t < offs.size(); ++t) {
      for (int a = 0; a < (nq > 1 ? 5 : 3); ++a)
        if (offs[t] == ko[a]) kind[t] = a;
      if (kind[t] < 0) return OG_OK;
    }
    for (int k = 0; k < K; ++k)
      for (size_t t = 0; t < offs.size(); ++t)
        for (int a = 0; a < d; ++a) {
          const int b = a + offs[t];
          const bool cross = (offs[t] == 1 || offs[t] == -1) && b >= 0 && b < d && (a / Nn) != (b / Nn);
          if (cross && hv[k][t * d + a] != cd(0, 0)) return OG_OK;
        }
    // h(k, kind, a) = H_k[a, a + o_kind]
    auto h = [&](int k, int a5, int a) {
      cd v(0, 0);
      if (a < 0 || a >= d) return v;
      for (size_t t = 0; t < offs.size(); ++t)
        if (kind[t] == a5) v += hv[k][t * d + a];
      return v;
    };
    std::vector<cd> hw((size_t)d * og::FCK * 5, cd(0, 0));
    for (int i = 0; i < d; ++i)
      for (int k = 0; k < K; ++k)
        for (int a5 = 0; a5 < 5; ++a5) hw[((size_t)i * og::FCK + k) * 5 + a5] = h(k, a5, i - ko[a5]);
    OG_TRY(upload<T>(hw, &fhw));
    half_k0 = 0;
    for (size_t t = 0; t < offs.size(); ++t) half_k0 |= kind[t] == 0 ? 1 : 0;
    half_ok = true;
    return OG_OK;
  }

  // ----- workspace layout -----
  static constexpr int kMaxRegions = 48;
  struct Layout {
    size_t off[kMaxRegions];
    size_t total;
  };
  enum {
    L_CUR_HI, L_CUR_LO, L_LAM_HI, L_LAM_LO, L_ZA, L_ZB, L_CK_HI, L_CK_LO, L_SG_HI, L_SG_LO,
    L_Z1, L_Z2, L_Z3, L_ZB1, L_ZB2, L_ZB3, L_ST_HI, L_ST_LO, L_AJF, L_AJA, L_X, L_W, L_WP, L_PS, L_COEF, L_GRAD, L_PEN,
    L_DPK, L_DPY, L_DPD, L_DPP, L_DPC, L_DPCK, L_TAIL, L_FCOEF, L_N
  };
  static_assert(L_N <= kMaxRegions, "workspace layout has more regions than Layout holds");

  int stride_for(int nt) const {
    int s = ctx->opt.ckpt_stride;
    if (s <= 0) s = (int)std::ceil(std::sqrt((double)nt));
    return std::max(1, std::min(s, std::max(nt, 1)));
  }

  // Resident tail: the last n_tail slices keep their states rho_j (working
  // precision, no compensation term) from the forward sweep, so that the
  // backward sweep recomputes only the slices before them.  Fixed steps
  // only, and for the exact gradient one substep (whose backward pass reads
  // no compensation term of the stored state).
  int tail_len(int nt) const {
    const bool ok = ctx->resident > 0 && !(ctx->ad_rtol > 0.0) &&
                    (ctx->opt.gmode != OG_GRAD_EXACT || ctx->opt.n_sub == 1);
    return ok ? std::min(ctx->resident, nt) : 0;
  }

  Layout layout(int b, int nt) const {
    Layout L{};
    const int ntail = tail_len(nt);
    const int s = stride_for(nt - ntail);
    const int nseg = (nt - ntail + s - 1) / s;
    const size_t m = (size_t)b * E * sizeof(og::cpx<T>);  // one matrix per problem
    const bool exact = ctx->opt.gmode == OG_GRAD_EXACT;
    const int nsub = ctx->opt.n_sub;
    size_t sz[L_N] = {};
    sz[L_CUR_HI] = m;
    sz[L_CUR_LO] = comp ? m : 0;
    sz[L_LAM_HI] = m;
    sz[L_LAM_LO] = comp ? m : 0;
    sz[L_ZA] = m;
    sz[L_ZB] = m;
    sz[L_CK_HI] = (size_t)nseg * m;
    sz[L_CK_LO] = comp ? (size_t)nseg * m : 0;
    sz[L_SG_HI] = (size_t)(s + 1) * m;
    sz[L_SG_LO] = comp ? (size_t)(s + 1) * m : 0;
    if (exact) {
      sz[L_Z1] = sz[L_Z2] = sz[L_Z3] = m;
      sz[L_ZB1] = sz[L_ZB2] = sz[L_ZB3] = m;
      sz[L_ST_HI] = (size_t)(nsub > 1 ? nsub - 1 : 0) * m;
      sz[L_ST_LO] = comp ? sz[L_ST_HI] : 0;
    }
    if (!banded) {
      sz[L_AJF] = m;
      sz[L_AJA] = exact ? m : 0;
      sz[L_X] = m;
      sz[L_W] = (size_t)std::max(J, 1) * m;
      sz[L_WP] = (exact ? 4 : 1) * m;
      sz[L_PS] = (J > 0 && J <= og::GM) ? (size_t)J * m : 0;
    } else {
      sz[L_COEF] = 2 * (size_t)kCoefChunk * b * max_nA() * d * sizeof(og::cpx<T>);
    }
    // per-slice gradient partial sums, one per row chunk of the contraction
    sz[L_GRAD] = (size_t)b * nt * og::NCH * std::max(K, 1) * sizeof(double);
    sz[L_PEN] = (size_t)b * (nt + 1) * sizeof(double);
    if (ctx->ad_rtol > 0.0) {
      sz[L_DPK] = 7 * m;
      sz[L_DPY] = m;
      sz[L_DPD] = m;
      sz[L_DPP] = (size_t)b * og::NCH * sizeof(double);
      sz[L_DPC] = kDpCtl * dpctl_bytes(b);
      sz[L_DPCK] = (size_t)nseg * b * 2 * sizeof(double);
    }
    // the packed Hermitian half of every state when the contraction reads that
    sz[L_TAIL] = ntail > 0 ? (size_t)(ntail + 1) * (half_contract() ? (size_t)b * EH * sizeof(og::cpx<T>) : m) : 0;
    if (banded && (fused[0] || fused[1]))
      sz[L_FCOEF] = 2 * (size_t)kCoefChunk * b * og::FSLOT * d * sizeof(og::cpx<T>);
    size_t pos = 0;
    for (int i = 0; i < L_N; ++i) {
      L.off[i] = pos;
      pos += align256(sz[i]);
    }
    L.total = pos;
    return L;
  }

  size_t ws_bytes(int b, int nt) const override { return layout(b, nt).total; }

  // ----- launch helpers -----
  hipStream_t st = nullptr;

  dim3 stage_grid() const { return dim3((unsigned)(B * ntile)); }

  og::StageIO<T> io_base() const {
    og::StageIO<T> io{};
    io.in_s = E;
    io.s_s = E;
    io.o_s = E;
    io.ex_s = E;
    io.status = ctx->status_dev;
    io.active = stage_active;
    return io;
  }

  // The stage kernel is compiled for a few upper bounds of the number of
  // diagonals (NA) and dissipator taps (ND): the ladder-order kernel (5, 3)
  // when the operators were put in that order, else 8 diagonals / 4 taps or
  // the library maxima.
  template <int MODE, int NA, int ND, bool LAD = false>
  void launch_band_v(const og::BandOps<T>& ops, const og::StageIO<T>& io, const og::cpx<T>* coef) {
    const long blocks = (long)B * ntile;
    if (blocks < kSmallStageGrid)
      og::band_stage_kernel<T, MODE, NA, ND, LAD, og::SlotCfg<T>::NQ><<<stage_grid(), og::slot_threads<T>(), 0, st>>>(
          ops, io, ntile, d, coef);
    else if (sizeof(T) == 4 && blocks < kMidStageGrid)
      og::band_stage_kernel<T, MODE, NA, ND, LAD, 2><<<stage_grid(), og::TS * og::TS / 2, 0, st>>>(ops, io, ntile, d,
                                                                                                coef);
    else
      og::band_stage_kernel<T, MODE, NA, ND, LAD><<<stage_grid(), og::stage_threads<T>(), 0, st>>>(
          ops, io, ntile, d, coef);
  }
  template <int MODE>
  void launch_band(const og::BandOps<T>& ops, const og::StageIO<T>& io, const og::cpx<T>* coef) {
    const int na = ops.nA, nd = ops.nD;
    if (ops.lad)
      launch_band_v<MODE, 5, 3, true>(ops, io, coef);
    else if (na <= 8 && nd <= 4)
      launch_band_v<MODE, 8, 4>(ops, io, coef);
    else
      launch_band_v<MODE, og::MAXA, og::MAXD>(ops, io, coef);
  }

  // One Runge-Kutta stage for the whole batch: out = f(L_dir(in)).
  og_status stage(int dr, int mode, int jslice, const og::cpx<T>* in, const og::cpx<T>* shi,
                  const og::cpx<T>* slo, og::cpx<T>* ohi, og::cpx<T>* olo, T coef,
                  const og::cpx<T>* ex0 = nullptr, const og::cpx<T>* ex1 = nullptr,
                  const og::cpx<T>* ex2 = nullptr) {
    og::StageIO<T> io = io_base();
    io.in = in;
    io.shi = shi;
    io.slo = slo;
    io.ohi = ohi;
    io.olo = olo;
    io.coef = coef;
    io.ex[0] = ex0;
    io.ex[1] = ex1;
    io.ex[2] = ex2;
    io.nex = ex2 ? 3 : (ex1 ? 2 : (ex0 ? 1 : 0));
    if (banded) {
      const og::BandOps<T>& ops = dir[dr].band;
      OG_TRY(assemble(dr, jslice));  // no launch when slice jslice is held
      const long pidx = ctx->prof_begin(st);
      if (mode == og::SM_STAGE)
        launch_band<og::SM_STAGE>(ops, io, coef_ptr(dr, jslice));
      else if (mode == og::SM_FINAL)
        launch_band<og::SM_FINAL>(ops, io, coef_ptr(dr, jslice));
      else
        launch_band<og::SM_SCALE>(ops, io, coef_ptr(dr, jslice));
      OG_CHECK_LAUNCH();
      ctx->prof_end(pidx, st);
      return OG_OK;
    }
    // dense: X = A_j in + 1/2 sum gamma C (C in)^dag ... via two GEMMs, then X + X^dag.
    // First the 1 + J products A_j Y and C_m Y, in launches of at most GM
    // operand sets.
    const DirDev<T>& dv = dir[dr];
    const long pidx = ctx->prof_begin(st);
    for (int m0 = 0; m0 <= J; m0 += og::GM) {
      og::GemmArgs<T> g{};
      g.nm = std::min(og::GM, J + 1 - m0);
      g.M = g.N = g.Kd = d;
      g.alpha.re = 1;
      for (int q = 0; q < g.nm; ++q) {
        const int m = m0 + q;  // 0: A_j Y; m >= 1: C_m Y into column block m - 1 of W
        g.A[q] = m == 0 ? Aj[dr] : dv.C + (long)(m - 1) * E;
        g.sA[q] = m == 0 ? E : 0;
        g.lda[q] = d;
        g.C[q] = m == 0 ? X : W + (long)(m - 1) * d;
        g.sC[q] = m == 0 ? E : (long)J * E;
        g.ldc[q] = m == 0 ? d : J * d;
        g.B[q] = in;
        g.sB[q] = E;
        g.ldb[q] = d;
      }
      const dim3 gg((d + 63) / 64, (d + 63) / 64, (unsigned)(B * g.nm));
      launch_gemm(g, gg);
      OG_CHECK_LAUNCH();
    }
    ctx->prof_end(pidx, st);
    // sum_m (C_m Y) (gamma_m / 2 C_m^dag): one product per m into its own
    // buffer (J times the blocks of a single product with inner size J d),
    // each Hermitian and formed on and above the block diagonal only, summed
    // in the epilogue; beyond GM collapse operators one full product
    // accumulates into X.
    int np = 0;
    if (J > 0 && J <= og::GM) {
      og::GemmArgs<T> h{};
      h.nm = J;
      h.M = h.N = h.Kd = d;
      h.alpha.re = 1;
      for (int m = 0; m < J; ++m) {
        h.A[m] = W + (long)m * d;
        h.sA[m] = (long)J * E;
        h.lda[m] = J * d;
        h.B[m] = dv.Chat + (long)m * E;
        h.sB[m] = 0;
        h.ldb[m] = d;
        h.C[m] = Ps + (long)m * E;
        h.sC[m] = (long)J * E;
        h.ldc[m] = d;
      }
      h.upper = 1;
      const int nt = (d + 63) / 64;
      const dim3 hg((unsigned)(nt * (nt + 1) / 2), 1, (unsigned)(B * J));
      launch_gemm(h, hg);
      OG_CHECK_LAUNCH();
      np = J;
    } else if (J > 0) {
      og::GemmArgs<T> h{};
      h.nm = 1;
      h.M = d;
      h.N = d;
      h.Kd = J * d;
      h.alpha.re = 1;
      h.beta.re = 1;
      h.A[0] = W;
      h.sA[0] = (long)J * E;
      h.lda[0] = J * d;
      h.B[0] = dv.Chat;
      h.sB[0] = 0;
      h.ldb[0] = d;
      h.C[0] = X;
      h.sC[0] = E;
      h.ldc[0] = d;
      const dim3 hg((d + 63) / 64, (d + 63) / 64, (unsigned)B);
      launch_gemm(h, hg);
      OG_CHECK_LAUNCH();
    }
    const long ps = (long)J * E;
    if (mode == og::SM_STAGE)
      og::dense_stage_kernel<T, og::SM_STAGE><<<stage_grid(), 256, 0, st>>>(X, E, Ps, ps, np, io, ntile, d);
    else if (mode == og::SM_FINAL)
      og::dense_stage_kernel<T, og::SM_FINAL><<<stage_grid(), 256, 0, st>>>(X, E, Ps, ps, np, io, ntile, d);
    else
      og::dense_stage_kernel<T, og::SM_SCALE><<<stage_grid(), 256, 0, st>>>(X, E, Ps, ps, np, io, ntile, d);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }

  // Slice generator assembly A(u_j) (Eq. (1)) for direction dr: diagonal
  // coefficients (banded) or the dense matrix, for every problem.  Banded:
  // when slice j is not in the held chunk, the next kCoefChunk slices in the
  // direction of the current sweep (within its range) are computed at once.
  og_status assemble(int dr, int jslice) {
    const DirDev<T>& dv = dir[dr];
    if (banded) {
      if (jslice >= cc0[dr] && jslice < cc1[dr]) return OG_OK;
      const CoefHint& hn = chint[dr];
      const int lo = std::max(0, std::min(hn.lo, jslice)), hi = std::min(n_t, std::max(hn.hi, jslice + 1));
      const int c0 = hn.asc ? jslice : std::max(lo, jslice - kCoefChunk + 1);
      const int c1 = hn.asc ? std::min(hi, jslice + kCoefChunk) : jslice + 1;
      const int n = dv.band.nA * d;
      const unsigned gx = (unsigned)std::max(1, std::min((n + 255) / 256, 64));
      og::band_coef_kernel<T><<<dim3(gx, (unsigned)B, (unsigned)(c1 - c0)), 256, 0, st>>>(dv.band, d, K, u, (long)n_t * K,
                                                                                         c0, acoef[dr]);
      OG_CHECK_LAUNCH();
      cc0[dr] = c0;
      cc1[dr] = c1;
      return OG_OK;
    }
    const unsigned gx = (unsigned)std::min<long>((E + 255) / 256, 1024);
    og::assemble_kernel<T><<<dim3(gx, (unsigned)B), 256, 0, st>>>(dv.A0, dv.Ak, K, E, u, (long)n_t * K, jslice, Aj[dr]);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }

  bool use_fused(int dr) const { return banded && fused[dr] && ctx->fused_on; }
  // serving launches form the coefficients in LDS as well: fused only if that still fits
  bool use_fused_slots(int dr) const { return use_fused(dr) && fused_lds_slots[dr] <= 65536; }
  og::FusedOps<T> fops(int dr) const {
    og::FusedOps<T> f;
    f.a0 = fa0[dr];
    f.ak = fak[dr];
    f.dl = fdl[dr];
    f.K = K;
    return f;
  }

  // Call f(levels, sign) with the compile-time level count (1..4) and tap
  // sign (+-1) of direction dr's fused step.
  template <typename F>
  void fused_dispatch(int dr, long blocks, F&& f) {
    using std::integral_constant;
    if (sizeof(T) == 4 && blocks >= kFusedSmall)
      fused_dispatch_nw(dr, f, integral_constant<int, 4>{});
    else
      fused_dispatch_nw(dr, f, integral_constant<int, 8>{});
  }
  template <typename F, typename NW>
  void fused_dispatch_nw(int dr, F& f, NW nw) {
    using std::integral_constant;
    const int nq = fgeo[dr].nq, sg = fgeo[dr].s1;
    if (sg > 0) {
      if (nq == 1) f(integral_constant<int, 1>{}, integral_constant<int, 1>{}, nw);
      else if (nq == 2) f(integral_constant<int, 2>{}, integral_constant<int, 1>{}, nw);
      else if (nq == 3) f(integral_constant<int, 3>{}, integral_constant<int, 1>{}, nw);
      else f(integral_constant<int, 4>{}, integral_constant<int, 1>{}, nw);
    } else {
      if (nq == 1) f(integral_constant<int, 1>{}, integral_constant<int, -1>{}, nw);
      else if (nq == 2) f(integral_constant<int, 2>{}, integral_constant<int, -1>{}, nw);
      else if (nq == 3) f(integral_constant<int, 3>{}, integral_constant<int, -1>{}, nw);
      else f(integral_constant<int, 4>{}, integral_constant<int, -1>{}, nw);
    }
  }
  int fused_used() const override { return use_fused(FWD) && use_fused(ADJ) ? 1 : 0; }
  // First-order gradient with fused steps in both directions: the slice
  // contraction reads the Hermitian half of rho_{j+1} in the fused step's
  // level-interleaved order (band_contract_half_kernel), and the resident
  // tail keeps only that half, packed, written by the forward steps.
  bool half_contract() const { return fused_used() && ctx->opt.gmode != OG_GRAD_EXACT && half_ok; }
  og::cpx<T>* hslot(og::cpx<T>* base, int idx) const { return base + (long)idx * B * EH; }


  // One fused RK4 step (the four nested stages in one launch) for the whole
  // batch: (ihi, ilo) -> (ohi, olo).  ohi must differ from ihi (other tiles
  // read the halo of the input while the output is written); olo may equal
  // ilo (every element's compensation term is read and written by one block).
  og_status fused_step(int dr, int jslice, const og::cpx<T>* ihi, const og::cpx<T>* ilo, og::cpx<T>* ohi,
                       og::cpx<T>* olo, T h, og::cpx<T>* pk = nullptr) {
    OG_TRY(assemble_fused(dr, jslice));
    og::StageIO<T> io = io_base();
    io.in = ihi;
    io.shi = ihi;
    io.slo = ilo;
    io.ohi = ohi;
    io.olo = olo;
    io.pk = pk;  // the packed Hermitian half of the output as well
    io.pk_s = EH;
    const og::cpx<T>* cf = fcoef[dr] + (size_t)(jslice - fc0[dr]) * B * og::FSLOT * d;
    const long blocks = (long)B * fgeo[dr].ntile;
    const bool small = blocks < kFusedTiny;
    const og::FusedGeo& geo = small ? fgeo_s[dr] : fgeo[dr];
    const dim3 grid((unsigned)(B * geo.ntile));
    const size_t lds = small ? fused_lds_s[dr] : fused_lds[dr];
    const long pidx = ctx->prof_begin(st);
    fused_dispatch(dr, blocks, [&](auto nq, auto sg, auto nw) {
      constexpr int NW = decltype(nw)::value;
      og::rk4_fused_kernel<T, decltype(nq)::value, NW, decltype(sg)::value>
          <<<grid, NW * 64, lds, st>>>(geo, io, d, cf, fdr[dr], h);
    });
    OG_CHECK_LAUNCH();
    ctx->prof_end(pidx, st);
    return OG_OK;
  }

  // Coefficients of the fused step (rows of FSLOT) for slice j of direction
  // dr: when j is not in the held chunk, the next kCoefChunk slices in the
  // direction of the current sweep (the same hints as the stage kernels'
  // coefficients) are computed at once.
  og_status assemble_fused(int dr, int jslice) {
    if (jslice >= fc0[dr] && jslice < fc1[dr]) return OG_OK;
    const CoefHint& hn = chint[dr];
    const int lo = std::max(0, std::min(hn.lo, jslice)), hi = std::min(n_t, std::max(hn.hi, jslice + 1));
    const int c0 = hn.asc ? jslice : std::max(lo, jslice - kCoefChunk + 1);
    const int c1 = hn.asc ? std::min(hi, jslice + kCoefChunk) : jslice + 1;
    const int n = og::FSLOT * d;
    const unsigned gx = (unsigned)std::max(1, std::min((n + 255) / 256, 64));
    og::fused_coef_kernel<T><<<dim3(gx, (unsigned)B, (unsigned)(c1 - c0)), 256, 0, st>>>(
        fops(dr), d, u, (long)n_t * K, c0, fcoef[dr]);
    OG_CHECK_LAUNCH();
    fc0[dr] = c0;
    fc1[dr] = c1;
    return OG_OK;
  }

  // n_sub RK4 steps of slice j in direction dr on the state (hi, lo) "in
  // place": with the fused step every step writes the other buffer of the
  // pair (hi, alt) and the two pointers are swapped, so hi holds the result.
  // pk (fused steps only): the last step also writes the packed Hermitian
  // half of the result there.
  og_status advance(int dr, int jslice, og::cpx<T>*& hi, og::cpx<T>* lo, og::cpx<T>*& alt,
                    og::cpx<T>* pk = nullptr) {
    if (!use_fused(dr)) {
      if (pk) return fail(OG_ERR_ARG, "internal: packed output without the fused step");
      return rk_slice(dr, jslice, hi, lo, hi, lo);
    }
    const int nsub = ctx->opt.n_sub;
    const T h = (T)(dt / nsub);
    for (int s = 0; s < nsub; ++s) {
      OG_TRY(fused_step(dr, jslice, hi, lo, alt, lo, h, s == nsub - 1 ? pk : nullptr));
      std::swap(hi, alt);
    }
    return OG_OK;
  }

  // n_sub RK4 steps of slice j in direction dr: (in) -> (out).  in == out is
  // allowed for the four-launch stages only (callers use advance() for
  // in-place steps); with the fused step several substeps alternate between
  // out and Zb so that the last one writes out.
  og_status rk_slice(int dr, int jslice, const og::cpx<T>* ihi, const og::cpx<T>* ilo, og::cpx<T>* ohi,
                     og::cpx<T>* olo) {
    const int nsub = ctx->opt.n_sub;
    const T h = (T)(dt / nsub);
    if (use_fused(dr)) {
      if (ihi == ohi) return fail(OG_ERR_ARG, "internal: fused RK4 step in place");
      const og::cpx<T>* src = ihi;
      const og::cpx<T>* slo = ilo;
      for (int s = 0; s < nsub; ++s) {
        og::cpx<T>* dst = ((nsub - 1 - s) % 2 == 0) ? ohi : Zb;
        OG_TRY(fused_step(dr, jslice, src, slo, dst, olo, h));
        src = dst;
        slo = olo;
      }
      return OG_OK;
    }
    OG_TRY(assemble(dr, jslice));
    for (int s = 0; s < nsub; ++s) {
      const og::cpx<T>* shi = s == 0 ? ihi : ohi;
      const og::cpx<T>* slo = s == 0 ? ilo : olo;
      OG_TRY(stage(dr, og::SM_STAGE, jslice, shi, shi, slo, Za, nullptr, h / T(4)));
      OG_TRY(stage(dr, og::SM_STAGE, jslice, Za, shi, slo, Zb, nullptr, h / T(3)));
      OG_TRY(stage(dr, og::SM_STAGE, jslice, Zb, shi, slo, Za, nullptr, h / T(2)));
      OG_TRY(stage(dr, og::SM_FINAL, jslice, Za, shi, slo, ohi, olo, h));
    }
    return OG_OK;
  }

  // g[:, j, :] = coef * 2 Im Tr(H_k X L) from the Hermitian half of X (packed
  // or full) and the full L, in the fused step's level order.
  og_status contract_half(int jslice, const og::cpx<T>* X, bool x_packed, const og::cpx<T>* Lm, double coef) {
    if (K == 0) return OG_OK;
    og::HalfPair<T> hp{};
    hp.X = X;
    hp.x_s = x_packed ? EH : E;
    hp.x_packed = x_packed ? 1 : 0;
    hp.L = Lm;
    hp.l_s = E;
    hp.coef = coef;
    hp.hw = fhw;
    hp.K = K;
    hp.k0 = half_k0;
    const int nblk = std::min(og::half_units<T>(d), og::NCH);  // blocks per problem: one unit each if they fit
    const dim3 cg((unsigned)(nblk * B));
    const int N = fgeo[FWD].N;
    switch (fgeo[FWD].nq) {
      case 1: og::band_contract_half_kernel<T, 1><<<cg, 256, 0, st>>>(hp, N, d, nblk, grad, n_t, jslice); break;
      case 2: og::band_contract_half_kernel<T, 2><<<cg, 256, 0, st>>>(hp, N, d, nblk, grad, n_t, jslice); break;
      case 3: og::band_contract_half_kernel<T, 3><<<cg, 256, 0, st>>>(hp, N, d, nblk, grad, n_t, jslice); break;
      case 4: og::band_contract_half_kernel<T, 4><<<cg, 256, 0, st>>>(hp, N, d, nblk, grad, n_t, jslice); break;
      default: return fail(OG_ERR_ARG, "internal: Hermitian-half contraction without its level count");
    }
    OG_CHECK_LAUNCH();
    return OG_OK;
  }

  // g[:, j, :] (+)= sum_p coef_p * 2 Im Tr(H_k X_p L_p)
  og_status contract(int jslice, int np, const og::cpx<T>* const* Xs, const og::cpx<T>* const* Ls,
                     const double* coefs, int accumulate) {
    if (K == 0) return OG_OK;
    const dim3 cg((unsigned)og::NCH, (unsigned)B);
    const dim3 cg1((unsigned)(og::NCH * B));
    if (banded) {
      og::PairArgs<T> pa{};
      pa.np = np;
      pa.x_s = E;
      pa.l_s = E;
      for (int p = 0; p < np; ++p) {
        pa.X[p] = Xs[p];
        pa.L[p] = Ls[p];
        pa.coef[p] = coefs[p];
      }
      if (hband.nH <= 4 && K <= 4)
        og::band_contract_kernel<T, 4, 4><<<cg1, 256, 0, st>>>(pa, hband, K, d, grad, n_t, jslice, accumulate);
      else if (hband.nH <= 4)
        og::band_contract_kernel<T, 4><<<cg1, 256, 0, st>>>(pa, hband, K, d, grad, n_t, jslice, accumulate);
      else if (hband.nH <= 8)
        og::band_contract_kernel<T, 8><<<cg1, 256, 0, st>>>(pa, hband, K, d, grad, n_t, jslice, accumulate);
      else
        og::band_contract_kernel<T, og::MAXH><<<cg1, 256, 0, st>>>(pa, hband, K, d, grad, n_t, jslice, accumulate);
      OG_CHECK_LAUNCH();
      return OG_OK;
    }
    // dense: W_p = X_p L_p for every pair, then the Frobenius products
    og::GemmArgs<T> g{};
    g.nm = np;
    g.M = g.N = g.Kd = d;
    g.alpha.re = 1;
    for (int p = 0; p < np; ++p) {
      g.A[p] = Xs[p];
      g.sA[p] = E;
      g.lda[p] = d;
      g.B[p] = Ls[p];
      g.sB[p] = E;
      g.ldb[p] = d;
      g.C[p] = Wp + (long)p * E;
      g.sC[p] = (long)np * E;
      g.ldc[p] = d;
    }
    const dim3 gg((d + 63) / 64, (d + 63) / 64, (unsigned)(B * np));
    launch_gemm(g, gg);
    OG_CHECK_LAUNCH();
    double c[4] = {0, 0, 0, 0};
    for (int p = 0; p < np; ++p) c[p] = coefs[p];
    og::dense_contract_kernel<T><<<cg, 256, 0, st>>>(Wp, E, (long)np * E, np, c[0], c[1], c[2], c[3], HT, K, E,
                                                    grad, n_t, jslice, accumulate);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }

  og::cpx<T>* slot(og::cpx<T>* base, int idx) const { return base ? base + (long)idx * B * E : nullptr; }

  // ----- adaptive steps (og_set_adaptive) -----
  // Controllers: the forward sweep, its checkpoint recompute (restarted from
  // the controller state stored with every checkpoint) and the adjoint.
  enum { DP_FWD = 0, DP_REC = 1, DP_ADJ = 2, kDpCtl = 3 };
  static constexpr int kMaxAttempts = 100000;  // per slice
  og::cpx<T>* dpk = nullptr;  // k_1..k_7, B matrices each
  og::cpx<T>* dpy = nullptr;  // stage input Y_i
  og::cpx<T>* dpd = nullptr;  // increment of the attempt
  double* dpp = nullptr;      // error partial sums, B x NCH
  og::DpCtl dpc[kDpCtl]{};
  double* dpck = nullptr;     // (h, rejected) per checkpoint and problem
  const int* stage_active = nullptr;  // gate of the banded stage launches

  static size_t dpctl_bytes(int b) {
    return align256((size_t)b * (5 * sizeof(double) + 3 * sizeof(int)) + sizeof(int));
  }
  static og::DpCtl carve_ctl(char* p, int b) {
    og::DpCtl c{};
    c.h = reinterpret_cast<double*>(p);
    c.t_rem = c.h + b;
    c.hu = c.t_rem + b;
    c.n_acc = reinterpret_cast<long long*>(c.hu + b);
    c.n_rej = c.n_acc + b;
    c.act = reinterpret_cast<int*>(c.n_rej + b);
    c.acc = c.act + b;
    c.rej = c.acc + b;
    c.n_active = c.rej + b;
    return c;
  }

  // One slice of the adaptive integrator (Dormand-Prince 5(4) with step
  // control) on the state (hi, lo) in place, for every problem.
  og_status adaptive_slice(int dr, int jslice, og::cpx<T>* hi, og::cpx<T>* lo, const og::DpCtl& c) {
    static const double A[7][6] = {
        {0, 0, 0, 0, 0, 0},
        {1.0 / 5, 0, 0, 0, 0, 0},
        {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
        {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
        {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
        {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
        {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
    static const double Bw[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
    static const double Bh[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100,
                                 1.0 / 40};
    og::DpRow bw{}, ew{};
    for (int i = 0; i < 7; ++i) {
      bw.c[i] = Bw[i];
      ew.c[i] = Bw[i] - Bh[i];
    }
    const long mst = (long)B * E;
    const unsigned gx = (unsigned)std::min<long>((E + 255) / 256, 1024);
    OG_TRY(assemble(dr, jslice));
    og::dp_begin_kernel<<<1, 256, 0, st>>>(c, B, dt);
    OG_CHECK_LAUNCH();
    stage_active = c.act;
    for (int attempt = 0;; ++attempt) {
      if (attempt >= kMaxAttempts) {
        stage_active = nullptr;
        return fail(OG_ERR_UNSTABLE_DT, "adaptive step control did not finish slice " + std::to_string(jslice));
      }
      og_status s_ = stage(dr, og::SM_SCALE, jslice, hi, nullptr, nullptr, dpk, nullptr, T(1));
      for (int i = 1; i < 7 && s_ == OG_OK; ++i) {
        og::DpRow a{};
        for (int l = 0; l < i; ++l) a.c[l] = A[i][l];
        og::dp_combine_kernel<T><<<dim3(gx, (unsigned)B), 256, 0, st>>>(hi, dpk, mst, E, i, a, c.hu, c.act, dpy, E);
        if (hipGetLastError() != hipSuccess) s_ = fail(OG_ERR_DEVICE, "combine launch failed");
        if (s_ == OG_OK) s_ = stage(dr, og::SM_SCALE, jslice, dpy, nullptr, nullptr, dpk + i * mst, nullptr, T(1));
      }
      if (s_ != OG_OK) {
        stage_active = nullptr;
        return s_;
      }
      og::dp_error_kernel<T><<<dim3((unsigned)og::NCH, (unsigned)B), 256, 0, st>>>(
          hi, dpk, mst, E, bw, ew, c.hu, c.act, ctx->ad_rtol, ctx->ad_atol, dpd, dpp, E);
      OG_CHECK_LAUNCH();
      og::dp_control_kernel<<<1, 256, 0, st>>>(c, dpp, B, 2.0 * (double)E);
      OG_CHECK_LAUNCH();
      og::StageIO<T> io = io_base();
      io.in = dpd;
      io.shi = hi;
      io.slo = lo;
      io.ohi = hi;
      io.olo = lo;
      og::dp_accept_kernel<T><<<stage_grid(), 256, 0, st>>>(io, c.acc, ntile, d);
      OG_CHECK_LAUNCH();
      OG_HIP(hipMemcpyAsync(ctx->host_flag, c.n_active, sizeof(int), hipMemcpyDeviceToHost, st));
      OG_HIP(hipStreamSynchronize(st));
      if (*ctx->host_flag == 0) break;
    }
    stage_active = nullptr;
    return OG_OK;
  }

  og_status adaptive_stats(long* counts) override {
    if (ctx->ad_rtol <= 0.0 || !dpk) return fail(OG_ERR_ORDER, "no adaptive evaluation has run");
    std::vector<long long> v((size_t)4 * B);
    OG_HIP(hipMemcpy(v.data(), dpc[DP_FWD].n_acc, B * sizeof(long long), hipMemcpyDeviceToHost));
    OG_HIP(hipMemcpy(v.data() + B, dpc[DP_FWD].n_rej, B * sizeof(long long), hipMemcpyDeviceToHost));
    OG_HIP(hipMemcpy(v.data() + 2 * B, dpc[DP_ADJ].n_acc, B * sizeof(long long), hipMemcpyDeviceToHost));
    OG_HIP(hipMemcpy(v.data() + 3 * B, dpc[DP_ADJ].n_rej, B * sizeof(long long), hipMemcpyDeviceToHost));
    for (int b = 0; b < B; ++b)
      for (int q = 0; q < 4; ++q) counts[4 * b + q] = (long)v[(size_t)q * B + b];
    return OG_OK;
  }

  og_status bind(void* ws, int b, int nt) {
    const Layout L = layout(b, nt);
    char* p = static_cast<char*>(ws);
    auto at = [&](int i) { return reinterpret_cast<og::cpx<T>*>(p + L.off[i]); };
    auto opt_at = [&](int i, bool use) { return use ? at(i) : nullptr; };
    const bool exact = ctx->opt.gmode == OG_GRAD_EXACT;
    cur_hi = cur_base = at(L_CUR_HI);
    cur_lo = opt_at(L_CUR_LO, comp);
    lam_hi = at(L_LAM_HI);
    lam_lo = opt_at(L_LAM_LO, comp);
    Za = at(L_ZA);
    Zb = at(L_ZB);
    ck_hi = at(L_CK_HI);
    ck_lo = opt_at(L_CK_LO, comp);
    sg_hi = at(L_SG_HI);
    sg_lo = opt_at(L_SG_LO, comp);
    n_tail = tail_len(nt);
    tail = opt_at(L_TAIL, n_tail > 0);
    Z1 = opt_at(L_Z1, exact);
    Z2 = opt_at(L_Z2, exact);
    Z3 = opt_at(L_Z3, exact);
    Zb1 = opt_at(L_ZB1, exact);
    Zb2 = opt_at(L_ZB2, exact);
    Zb3 = opt_at(L_ZB3, exact);
    st_hi = opt_at(L_ST_HI, exact && ctx->opt.n_sub > 1);
    st_lo = opt_at(L_ST_LO, exact && ctx->opt.n_sub > 1 && comp);
    Aj[0] = opt_at(L_AJF, !banded);
    Aj[1] = opt_at(L_AJA, !banded && exact);
    if (!banded && !exact) Aj[1] = Aj[0];
    X = opt_at(L_X, !banded);
    W = opt_at(L_W, !banded);
    Wp = opt_at(L_WP, !banded);
    Ps = opt_at(L_PS, !banded && J > 0 && J <= og::GM);
    acoef[0] = opt_at(L_COEF, banded);
    acoef[1] = banded ? acoef[0] + (size_t)kCoefChunk * b * max_nA() * d : nullptr;
    fcoef[0] = opt_at(L_FCOEF, banded && (fused[0] || fused[1]));
    fcoef[1] = fcoef[0] ? fcoef[0] + (size_t)kCoefChunk * b * og::FSLOT * d : nullptr;
    grad = reinterpret_cast<double*>(p + L.off[L_GRAD]);
    if (ctx->ad_rtol > 0.0) {
      dpk = at(L_DPK);
      dpy = at(L_DPY);
      dpd = at(L_DPD);
      dpp = reinterpret_cast<double*>(p + L.off[L_DPP]);
      char* c = p + L.off[L_DPC];
      for (int i = 0; i < kDpCtl; ++i) dpc[i] = carve_ctl(c + (size_t)i * dpctl_bytes(b), b);
      dpck = reinterpret_cast<double*>(p + L.off[L_DPCK]);
    }
    pen = reinterpret_cast<double*>(p + L.off[L_PEN]);
    return OG_OK;
  }

  og_status copy_hi(og::cpx<T>* dhi, const og::cpx<T>* shi) {
    OG_HIP(hipMemcpyAsync(dhi, shi, (size_t)B * E * sizeof(og::cpx<T>), hipMemcpyDeviceToDevice, st));
    return OG_OK;
  }

  og_status copy_state(og::cpx<T>* dhi, og::cpx<T>* dlo, const og::cpx<T>* shi, const og::cpx<T>* slo) {
    const size_t bytes = (size_t)B * E * sizeof(og::cpx<T>);
    OG_HIP(hipMemcpyAsync(dhi, shi, bytes, hipMemcpyDeviceToDevice, st));
    if (comp) OG_HIP(hipMemcpyAsync(dlo, slo, bytes, hipMemcpyDeviceToDevice, st));
    return OG_OK;
  }

  og_status load(const void* src, long src_s, og::cpx<T>* hi, og::cpx<T>* lo) {
    const unsigned gx = (unsigned)std::min<long>((E + 255) / 256, 1024);
    og::load_state_kernel<T><<<dim3(gx, (unsigned)B), 256, 0, st>>>(static_cast<const double*>(src), src_s, E, hi, lo, E);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }

  og_status forward(int b, int nt, double dt_, const double* u_, const void* rho0, void* rhoT, void* ws,
                    size_t wsb, hipStream_t s) override {
    if (wsb < ws_bytes(b, nt)) return fail(OG_ERR_WORKSPACE, "workspace smaller than og_workspace_bytes()");
    st = s;
    B = b;
    n_t = nt;
    dt = dt_;
    u = u_;
    OG_TRY(bind(ws, b, nt));
    coef_reset();
    coef_hint(FWD, 0, nt, true);
    const int jt = nt - n_tail;  // first slice of the resident tail
    S = stride_for(jt);
    n_seg = (jt + S - 1) / S;
    OG_TRY(load(rho0, E, cur_hi, cur_lo));
    OG_TRY(penalty_trace(0));
    const bool ad = ctx->ad_rtol > 0.0;
    if (ad) {
      og::dp_init_kernel<<<1, 256, 0, st>>>(dpc[DP_FWD], B, dt);
      OG_CHECK_LAUNCH();
    }
    for (int j = 0; j < jt; ++j) {
      if (j % S == 0) {
        OG_TRY(copy_state(slot(ck_hi, j / S), slot(ck_lo, j / S), cur_hi, cur_lo));
        if (ad) {
          og::dp_save_kernel<<<1, 256, 0, st>>>(dpc[DP_FWD], B, dpck + (size_t)(j / S) * B * 2);
          OG_CHECK_LAUNCH();
        }
      }
      if (ad)
        OG_TRY(adaptive_slice(FWD, j, cur_hi, cur_lo, dpc[DP_FWD]));
      else
        OG_TRY(advance(FWD, j, cur_hi, cur_lo, Za));
      OG_TRY(penalty_trace(j + 1));
    }
    const bool half = half_contract();
    if (n_tail > 0 && half) {
      // packed tail: the steps go on in the state buffers and also write the
      // Hermitian half of rho_{j+1} to its slot
      for (int k = 0; k < n_tail; ++k) {
        OG_TRY(advance(FWD, jt + k, cur_hi, cur_lo, Za, hslot(tail, k + 1)));
        OG_TRY(penalty_trace(jt + k + 1));
      }
    }
    if (cur_hi != cur_base) {  // the fused step left the state in the other buffer
      OG_TRY(copy_hi(cur_base, cur_hi));
      Za = cur_hi;
      cur_hi = cur_base;
    }
    if (n_tail > 0 && !half) {
      // the tail runs on the stored states; the compensation term stays in
      // cur_lo (read and written at the same elements by the final stage)
      OG_TRY(copy_hi(slot(tail, 0), cur_hi));
      for (int k = 0; k < n_tail; ++k) {
        OG_TRY(rk_slice(FWD, jt + k, slot(tail, k), cur_lo, slot(tail, k + 1), cur_lo));
        OG_TRY(penalty_trace(jt + k + 1, slot(tail, k + 1)));
      }
      OG_TRY(copy_hi(cur_hi, slot(tail, n_tail)));
    }
    if (rhoT) {
      const unsigned gx = (unsigned)std::min<long>((E + 255) / 256, 1024);
      og::store_state_kernel<T><<<dim3(gx, (unsigned)B), 256, 0, st>>>(cur_hi, cur_lo, E, d, static_cast<double*>(rhoT));
      OG_CHECK_LAUNCH();
    }
    return OG_OK;
  }

  // Penalty (Eqs. (24)-(25), App. B): Tr(A rho_n) after every slice in the
  // forward sweep, Phi -= beta dt sum_n, and lambda -= beta dt A at every
  // slice boundary of the backward sweep (the combined adjoint).
  og_status penalty_trace(int n, const og::cpx<T>* hi = nullptr) {
    if (ctx->pen_beta == 0.0 || !ctx->pen_coo) return OG_OK;
    og::penalty_trace_kernel<T><<<dim3((unsigned)B), 256, 0, st>>>(ctx->pen_coo, ctx->pen_nnz, hi ? hi : cur_hi, cur_lo,
                                                                   E, d, pen + n, (long)n_t + 1);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }
  og_status penalty_inject() {
    if (ctx->pen_beta == 0.0 || !ctx->pen_coo) return OG_OK;
    const unsigned gx = (unsigned)std::max(1, std::min((ctx->pen_nnz + 255) / 256, 64));
    og::inject_kernel<T><<<dim3(gx, (unsigned)B), 256, 0, st>>>(ctx->pen_coo, ctx->pen_nnz, -ctx->pen_beta * dt,
                                                                lam_hi, E, d);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }

  og_status cost(const void* sigma, double* phi, hipStream_t s) override {
    og::cost_kernel<T><<<dim3((unsigned)B), 256, 0, s>>>(static_cast<const double*>(sigma), cur_hi, cur_lo, E, d, phi);
    OG_CHECK_LAUNCH();
    if (ctx->pen_beta != 0.0 && ctx->pen_coo) {
      og::penalty_sum_kernel<<<dim3((unsigned)B), 256, 0, s>>>(pen, (long)n_t + 1, ctx->pen_beta * dt, phi);
      OG_CHECK_LAUNCH();
    }
    return OG_OK;
  }

  og_status adjoint(const void* sigma, hipStream_t s) override {
    st = s;
    OG_TRY(load(sigma, 0, lam_hi, lam_lo));
    OG_TRY(penalty_inject());
    const bool ad = ctx->ad_rtol > 0.0;
    if (ad) {
      og::dp_init_kernel<<<1, 256, 0, st>>>(dpc[DP_ADJ], B, dt);
      OG_CHECK_LAUNCH();
      og::dp_init_kernel<<<1, 256, 0, st>>>(dpc[DP_REC], B, dt);
      OG_CHECK_LAUNCH();
    }
    // resident tail: its states are stored, nothing to recompute
    const int jt = n_t - n_tail;
    coef_reset();
    coef_hint(ADJ, 0, n_t, false);
    coef_hint(FWD, jt, n_t, false);
    if (half_contract())
      for (int k = n_tail - 1; k >= 0; --k) OG_TRY(back_slice(jt + k, nullptr, nullptr, hslot(tail, k + 1), true));
    else
      for (int k = n_tail - 1; k >= 0; --k) OG_TRY(back_slice(jt + k, slot(tail, k), nullptr, slot(tail, k + 1)));
    for (int seg = n_seg - 1; seg >= 0; --seg) {
      const int j0 = seg * S, j1 = std::min(jt, j0 + S), n = j1 - j0;
      coef_hint(FWD, j0, j1, true);
      OG_TRY(copy_state(slot(sg_hi, 0), slot(sg_lo, 0), slot(ck_hi, seg), slot(ck_lo, seg)));
      if (ad) {
        // the recompute restarts from the controller state stored with the
        // checkpoint, so it takes the forward sweep's steps exactly
        og::dp_load_kernel<<<1, 256, 0, st>>>(dpc[DP_REC], B, dpck + (size_t)seg * B * 2);
        OG_CHECK_LAUNCH();
        for (int jj = 0; jj < n; ++jj) {
          OG_TRY(copy_state(slot(sg_hi, jj + 1), slot(sg_lo, jj + 1), slot(sg_hi, jj), slot(sg_lo, jj)));
          OG_TRY(adaptive_slice(FWD, j0 + jj, slot(sg_hi, jj + 1), slot(sg_lo, jj + 1), dpc[DP_REC]));
        }
      } else {
        for (int jj = 0; jj < n; ++jj)
          OG_TRY(rk_slice(FWD, j0 + jj, slot(sg_hi, jj), slot(sg_lo, jj), slot(sg_hi, jj + 1), slot(sg_lo, jj + 1)));
      }
      coef_hint(FWD, j0, j1, false);
      for (int jj = n - 1; jj >= 0; --jj)
        OG_TRY(back_slice(j0 + jj, slot(sg_hi, jj), slot(sg_lo, jj), slot(sg_hi, jj + 1)));
    }
    return OG_OK;
  }

  // One slice j of the backward sweep: the gradient contraction and the
  // adjoint step, from rho_j (r_hi, r_lo) and rho_{j+1} (r1_hi; its packed
  // Hermitian half when r1_packed).
  og_status back_slice(int j, const og::cpx<T>* r_hi, const og::cpx<T>* r_lo, const og::cpx<T>* r1_hi,
                       bool r1_packed = false) {
    const bool exact = ctx->opt.gmode == OG_GRAD_EXACT;
    const int nsub = ctx->opt.n_sub;
    const T h = (T)(dt / nsub);
    const bool ad = ctx->ad_rtol > 0.0;
    if (!exact) {
      if (half_contract()) {
        OG_TRY(contract_half(j, r1_hi, r1_packed, lam_hi, dt));
      } else {
        if (r1_packed) return fail(OG_ERR_ARG, "internal: packed state without the half contraction");
        const og::cpx<T>* Xs[1] = {r1_hi};
        const og::cpx<T>* Ls[1] = {lam_hi};
        const double cf[1] = {dt};
        OG_TRY(contract(j, 1, Xs, Ls, cf, 0));
      }
      if (ad)
        OG_TRY(adaptive_slice(ADJ, j, lam_hi, lam_lo, dpc[DP_ADJ]));
      else
        OG_TRY(advance(ADJ, j, lam_hi, lam_lo, Za));
      return penalty_inject();
    }
    // exact derivative of the RK4-discretised Phi: reverse through the
    // nested stages Z1..Z3 of every substep of slice j.
    OG_TRY(assemble(FWD, j));
    OG_TRY(assemble(ADJ, j));
    for (int sub = 1; sub < nsub; ++sub) {
      const og::cpx<T>* phi_ = sub == 1 ? r_hi : slot(st_hi, sub - 2);
      const og::cpx<T>* plo = sub == 1 ? r_lo : slot(st_lo, sub - 2);
      og::cpx<T>* ohi = slot(st_hi, sub - 1);
      og::cpx<T>* olo = slot(st_lo, sub - 1);
      OG_TRY(stage(FWD, og::SM_STAGE, j, phi_, phi_, plo, Za, nullptr, h / T(4)));
      OG_TRY(stage(FWD, og::SM_STAGE, j, Za, phi_, plo, Zb, nullptr, h / T(3)));
      OG_TRY(stage(FWD, og::SM_STAGE, j, Zb, phi_, plo, Za, nullptr, h / T(2)));
      OG_TRY(stage(FWD, og::SM_FINAL, j, Za, phi_, plo, ohi, olo, h));
    }
    for (int sub = nsub - 1; sub >= 0; --sub) {
      const og::cpx<T>* s_hi = sub == 0 ? r_hi : slot(st_hi, sub - 1);
      const og::cpx<T>* s_lo = sub == 0 ? r_lo : slot(st_lo, sub - 1);
      OG_TRY(stage(FWD, og::SM_STAGE, j, s_hi, s_hi, s_lo, Z1, nullptr, h / T(4)));
      OG_TRY(stage(FWD, og::SM_STAGE, j, Z1, s_hi, s_lo, Z2, nullptr, h / T(3)));
      OG_TRY(stage(FWD, og::SM_STAGE, j, Z2, s_hi, s_lo, Z3, nullptr, h / T(2)));
      OG_TRY(stage(ADJ, og::SM_SCALE, j, lam_hi, nullptr, nullptr, Zb3, nullptr, h));
      OG_TRY(stage(ADJ, og::SM_SCALE, j, Zb3, nullptr, nullptr, Zb2, nullptr, h / T(2)));
      OG_TRY(stage(ADJ, og::SM_SCALE, j, Zb2, nullptr, nullptr, Zb1, nullptr, h / T(3)));
      const og::cpx<T>* Xs[4] = {Z3, Z2, Z1, s_hi};
      const og::cpx<T>* Ls[4] = {lam_hi, Zb3, Zb2, Zb1};
      const double hd = dt / nsub;
      const double cf[4] = {hd, hd / 2, hd / 3, hd / 4};
      OG_TRY(contract(j, 4, Xs, Ls, cf, sub != nsub - 1));
      OG_TRY(stage(ADJ, og::SM_FINAL, j, Zb1, lam_hi, lam_lo, lam_hi, lam_lo, h / T(4), Zb1, Zb2, Zb3));
    }
    return penalty_inject();
  }

  og_status gradient_sum(double* out, int accumulate, hipStream_t s) override {
    if (K == 0) return OG_OK;
    const long n = (long)n_t * K;
    og::reduce_partials_sum_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(grad, B, n_t, K, accumulate,
                                                                                    out);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }

  og_status gradient(double* out, hipStream_t s) override {
    if (K == 0) return OG_OK;
    const long n = (long)B * n_t * K;
    og::reduce_partials_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(grad, (long)B * n_t, K, out);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }

  // -------------------------------------------------------------------------
  // Continuous batching.  Every request runs the same sequence as a batch of
  // one through forward() / cost() / adjoint() / gradient(): forward slices
  // with a checkpoint every S slices, the cost, then per segment (last
  // first) the recompute and the adjoint slices with the first-order
  // contraction.  Requests at the same kind of slice operation share the
  // launches of one step.
  // -------------------------------------------------------------------------
  enum { PH_FWD = 1, PH_RECOMP = 2, PH_ADJ = 3, PH_DONE = 4, PH_TAIL = 5 };
  struct Slot {
    og_request r;
    int S = 1, n_seg = 1;
    og::cpx<T>*cur_hi, *cur_lo, *lam_hi, *lam_lo, *za, *zb, *ck_hi, *ck_lo, *sg_hi, *sg_lo, *coefF, *coefA;
    double* part;
    // resident states (packed Hermitian halves) of the slices jt .. n_t - 1
    og::cpx<T>* tail = nullptr;
    int n_tail = 0, jt = 0;
    long ctxEH = 0;
    og::cpx<T>* tl(int i) const { return tail + (long)i * ctxEH; }
    int phase = 0, j = 0, seg = 0, jj = 0, n = 0;
    bool inited = false;
    og::cpx<T>* ck(int i) const { return ck_hi + (long)i * ctxE; }
    og::cpx<T>* ckl(int i) const { return ck_lo ? ck_lo + (long)i * ctxE : nullptr; }
    og::cpx<T>* sg(int i) const { return sg_hi + (long)i * ctxE; }
    og::cpx<T>* sgl(int i) const { return sg_lo ? sg_lo + (long)i * ctxE : nullptr; }
    long ctxE = 0;
  };
  std::vector<Slot> slots;

  og_status serve_submit(const og_request& r, hipStream_t s) override {
    if (!banded) return fail(OG_ERR_SHAPE, "serving needs the banded path");
    if (ctx->ad_rtol > 0.0) return fail(OG_ERR_ARG, "serving runs fixed steps; disable adaptive steps");
    if (ctx->resident > 0 && !(half_contract() && use_fused_slots(FWD) && use_fused_slots(ADJ)))
      return fail(OG_ERR_ARG,
                  "serving keeps resident states only as packed halves of fused steps; og_set_resident(ctx, 0)");
    if (r.ws_bytes < ws_bytes(1, r.n_t)) return fail(OG_ERR_WORKSPACE, "request workspace too small");
    Slot sl;
    sl.r = r;
    sl.ctxE = E;
    sl.ctxEH = EH;
    sl.n_tail = tail_len(r.n_t);
    sl.jt = r.n_t - sl.n_tail;
    sl.S = stride_for(sl.jt);
    sl.n_seg = (sl.jt + sl.S - 1) / sl.S;
    const Layout L = layout(1, r.n_t);
    char* p = static_cast<char*>(r.ws);
    auto at = [&](int i) { return reinterpret_cast<og::cpx<T>*>(p + L.off[i]); };
    sl.cur_hi = at(L_CUR_HI);
    sl.cur_lo = comp ? at(L_CUR_LO) : nullptr;
    sl.lam_hi = at(L_LAM_HI);
    sl.lam_lo = comp ? at(L_LAM_LO) : nullptr;
    sl.za = at(L_ZA);
    sl.zb = at(L_ZB);
    sl.ck_hi = at(L_CK_HI);
    sl.ck_lo = comp ? at(L_CK_LO) : nullptr;
    sl.sg_hi = at(L_SG_HI);
    sl.sg_lo = comp ? at(L_SG_LO) : nullptr;
    sl.coefF = at(L_COEF);
    sl.coefA = sl.coefF + (size_t)og::MAXA * d;
    sl.part = reinterpret_cast<double*>(p + L.off[L_GRAD]);
    sl.tail = sl.n_tail > 0 ? at(L_TAIL) : nullptr;
    (void)s;
    slots.push_back(sl);
    return OG_OK;
  }

  int serve_active() const override { return (int)slots.size(); }
  void serve_clear() override { slots.clear(); }

  og_status load1(const void* src, long src_s, og::cpx<T>* hi, og::cpx<T>* lo, hipStream_t s) {
    const unsigned gx = (unsigned)std::min<long>((E + 255) / 256, 1024);
    og::load_state_kernel<T><<<dim3(gx, 1), 256, 0, s>>>(static_cast<const double*>(src), src_s, E, hi, lo, E);
    OG_CHECK_LAUNCH();
    return OG_OK;
  }
  og_status copy1(og::cpx<T>* dhi, og::cpx<T>* dlo, const og::cpx<T>* shi, const og::cpx<T>* slo, hipStream_t s) {
    OG_HIP(hipMemcpyAsync(dhi, shi, (size_t)E * sizeof(og::cpx<T>), hipMemcpyDeviceToDevice, s));
    if (comp) OG_HIP(hipMemcpyAsync(dlo, slo, (size_t)E * sizeof(og::cpx<T>), hipMemcpyDeviceToDevice, s));
    return OG_OK;
  }
  og_status start_segment(Slot& sl, hipStream_t s) {
    const int j0 = sl.seg * sl.S;
    sl.n = std::min(sl.jt, j0 + sl.S) - j0;
    sl.jj = 0;
    sl.phase = PH_RECOMP;
    return copy1(sl.sg(0), sl.sgl(0), sl.ck(sl.seg), sl.ckl(sl.seg), s);
  }

  struct Op {
    int slot;
    int slice;
    const og::cpx<T>*ihi, *ilo;
    og::cpx<T>*ohi, *olo;
    const og::cpx<T>* pairX;
    og::cpx<T>* pk = nullptr;  // forward: the packed half of the result as well
    bool xpacked = false;      // adjoint: pairX is a packed half
  };

  template <int MODE, int NA, int ND, bool LAD = false>
  void launch_slots_v(int dr, const og::SlotTable<T>& tab, int n, int in_role, int out_role, T coef) {
    og::band_stage_slots_kernel<T, MODE, NA, ND, LAD>
        <<<dim3((unsigned)(n * ntile)), og::slot_threads<T>(), 0, st>>>(dir[dr].band, tab, in_role, out_role,
                                                                         coef, ctx->status_dev, ntile, d);
  }
  template <int MODE>
  og_status launch_slots(int dr, const og::SlotTable<T>& tab, int n, int in_role, int out_role, T coef) {
    const og::BandOps<T>& ops = dir[dr].band;
    const long pidx = ctx->prof_begin(st);
    if (ops.lad)
      launch_slots_v<MODE, 5, 3, true>(dr, tab, n, in_role, out_role, coef);
    else if (ops.nA <= 8 && ops.nD <= 4)
      launch_slots_v<MODE, 8, 4>(dr, tab, n, in_role, out_role, coef);
    else
      launch_slots_v<MODE, og::MAXA, og::MAXD>(dr, tab, n, in_role, out_role, coef);
    OG_CHECK_LAUNCH();
    ctx->prof_end(pidx, st);
    return OG_OK;
  }

  // One slice operation (n_sub RK4 steps) for up to MAXSLOT requests of the
  // same direction and slice length (MAXFSLOT with the fused step); adjoint
  // operations first contract the first-order gradient of their slice.
  og_status run_chunk(int dr, const std::vector<Op>& ops, size_t i0, size_t i1, double dtv) {
    const int n = (int)(i1 - i0);
    // contraction and coefficients: sub-launches of at most MAXPSLOT requests
    // (MAXSLOT with the stage kernels' coefficient table)
    const int per = use_fused_slots(dr) ? og::MAXPSLOT : og::MAXSLOT;
    for (int q0 = 0; q0 < n; q0 += per) {
      const int m = std::min(per, n - q0);
      if (dr == ADJ && K > 0) {
        og::PairSlots<T> ps{};
        for (int q = 0; q < m; ++q) {
          const Op& o = ops[i0 + q0 + q];
          const Slot& sl = slots[o.slot];
          ps.X[q] = o.pairX;
          ps.xp[q] = o.xpacked ? 1 : 0;
          ps.L[q] = sl.lam_hi;
          ps.out[q] = sl.part + (long)o.slice * og::NCH * K;
        }
        const dim3 cg((unsigned)(og::NCH * m));
        const int hN = fgeo[FWD].N;
        if (half_contract()) {  // the same arithmetic as the batch entry points
          const int nb = std::min(og::half_units<T>(d), og::NCH);
          const dim3 hg((unsigned)(nb * m));
          switch (fgeo[FWD].nq) {
            case 1: og::band_contract_half_slots_kernel<T, 1><<<hg, 256, 0, st>>>(ps, dtv, fhw, half_k0, K, hN, d, nb); break;
            case 2: og::band_contract_half_slots_kernel<T, 2><<<hg, 256, 0, st>>>(ps, dtv, fhw, half_k0, K, hN, d, nb); break;
            case 3: og::band_contract_half_slots_kernel<T, 3><<<hg, 256, 0, st>>>(ps, dtv, fhw, half_k0, K, hN, d, nb); break;
            default: og::band_contract_half_slots_kernel<T, 4><<<hg, 256, 0, st>>>(ps, dtv, fhw, half_k0, K, hN, d, nb); break;
          }
        } else if (hband.nH <= 4)
          og::band_contract_slots_kernel<T, 4><<<cg, 256, 0, st>>>(ps, dtv, hband, K, d);
        else if (hband.nH <= 8)
          og::band_contract_slots_kernel<T, 8><<<cg, 256, 0, st>>>(ps, dtv, hband, K, d);
        else
          og::band_contract_slots_kernel<T, og::MAXH><<<cg, 256, 0, st>>>(ps, dtv, hband, K, d);
        OG_CHECK_LAUNCH();
      }
      if (use_fused_slots(dr)) {
        // the fused serving kernel forms its coefficients itself
      } else {
        og::SlotTable<T> ct{};
        for (int q = 0; q < m; ++q) {
          const Op& o = ops[i0 + q0 + q];
          const Slot& sl = slots[o.slot];
          ct.e[q].coef = dr == FWD ? sl.coefF : sl.coefA;
          ct.e[q].urow = sl.r.u + (long)o.slice * K;
        }
        const int na = dir[dr].band.nA * d;
        const unsigned gx = (unsigned)std::max(1, std::min((na + 255) / 256, 64));
        og::band_coef_slots_kernel<T><<<dim3(gx, (unsigned)m), 256, 0, st>>>(dir[dr].band, ct, d, K);
      }
      OG_CHECK_LAUNCH();
    }
    const int nsub = ctx->opt.n_sub;
    const T h = (T)(dtv / nsub);
    if (use_fused_slots(dr)) {
      // In-place operations (the forward state, lambda) write the request's
      // other buffer (za for the state, zb for lambda) and swap the two;
      // the segment recompute (sg[jj] -> sg[jj + 1]) chains several substeps
      // through za so that the last one writes sg[jj + 1].
      std::vector<const og::cpx<T>*> prev((size_t)n);
      for (int sub = 0; sub < nsub; ++sub) {
        og::FusedSlotTable<T> ft{};
        for (int q = 0; q < n; ++q) {
          const Op& o = ops[i0 + q];
          Slot& sl = slots[o.slot];
          og::FusedSlot<T>& e = ft.e[q];
          e.urow = sl.r.u + (long)o.slice * K;
          if (o.ihi == o.ohi) {
            og::cpx<T>*& cur = dr == FWD ? sl.cur_hi : sl.lam_hi;
            og::cpx<T>*& alt = dr == FWD ? sl.za : sl.zb;
            e.s_hi = cur;
            e.o_hi = alt;
            e.pk = sub == nsub - 1 ? o.pk : nullptr;
            e.s_lo = e.o_lo = dr == FWD ? sl.cur_lo : sl.lam_lo;
            std::swap(cur, alt);
          } else {
            e.s_hi = sub == 0 ? o.ihi : prev[q];
            e.s_lo = sub == 0 ? o.ilo : o.olo;
            e.o_hi = ((nsub - 1 - sub) % 2 == 0) ? o.ohi : sl.za;
            e.o_lo = o.olo;
            prev[q] = e.o_hi;
          }
        }
        const long blocks = (long)n * fgeo[dr].ntile;
        const bool small = blocks < kFusedTiny;
        const og::FusedGeo& geo = small ? fgeo_s[dr] : fgeo[dr];
        const dim3 grid((unsigned)(n * geo.ntile));
        const size_t lds = small ? fused_lds_slots_s[dr] : fused_lds_slots[dr];
        const long pidx = ctx->prof_begin(st);
        fused_dispatch(dr, blocks, [&](auto nq, auto sg, auto nw) {
          constexpr int NW = decltype(nw)::value;
          og::rk4_fused_slots_kernel<T, decltype(nq)::value, NW, decltype(sg)::value>
              <<<grid, NW * 64, lds, st>>>(geo, ft, fops(dr), fdr[dr], h, ctx->status_dev, d);
        });
        OG_CHECK_LAUNCH();
        ctx->prof_end(pidx, st);
      }
      return OG_OK;
    }
    og::SlotTable<T> tab{};
    for (int q = 0; q < n; ++q) {
      const Op& o = ops[i0 + q];
      const Slot& sl = slots[o.slot];
      og::SlotEntry<T>& e = tab.e[q];
      e.s_hi = o.ihi;
      e.s_lo = o.ilo;
      e.o_hi = o.ohi;
      e.o_lo = o.olo;
      e.za = sl.za;
      e.zb = sl.zb;
      e.coef = dr == FWD ? sl.coefF : sl.coefA;
      e.urow = sl.r.u + (long)o.slice * K;
    }
    for (int sub = 0; sub < nsub; ++sub) {
      if (sub == 1)
        for (int q = 0; q < n; ++q) {
          tab.e[q].s_hi = tab.e[q].o_hi;
          tab.e[q].s_lo = tab.e[q].o_lo;
        }
      OG_TRY(launch_slots<og::SM_STAGE>(dr, tab, n, og::R_STATE, og::R_ZA, h / T(4)));
      OG_TRY(launch_slots<og::SM_STAGE>(dr, tab, n, og::R_ZA, og::R_ZB, h / T(3)));
      OG_TRY(launch_slots<og::SM_STAGE>(dr, tab, n, og::R_ZB, og::R_ZA, h / T(2)));
      OG_TRY(launch_slots<og::SM_FINAL>(dr, tab, n, og::R_ZA, og::R_OUT, h));
    }
    return OG_OK;
  }

  og_status run_group(int dr, std::vector<Op>& ops) {
    // same slice length in one launch: sort by dt, then chunks of MAXSLOT
    // (MAXFSLOT with the fused step)
    std::stable_sort(ops.begin(), ops.end(),
                     [&](const Op& a, const Op& b) { return slots[a.slot].r.dt < slots[b.slot].r.dt; });
    const size_t cap = use_fused_slots(dr) ? (size_t)og::MAXFSLOT : (size_t)og::MAXSLOT;
    size_t i = 0;
    while (i < ops.size()) {
      const double dtv = slots[ops[i].slot].r.dt;
      size_t k = i;
      while (k < ops.size() && k - i < cap && slots[ops[k].slot].r.dt == dtv) ++k;
      OG_TRY(run_chunk(dr, ops, i, k, dtv));
      i = k;
    }
    return OG_OK;
  }

  // the request's gradient from its partial sums; the request is done
  og_status finish(Slot& sl, hipStream_t s) {
    if (K > 0) {
      const long nn = (long)sl.r.n_t * K;
      og::reduce_partials_kernel<<<dim3((unsigned)((nn + 255) / 256)), 256, 0, s>>>(sl.part, sl.r.n_t, K,
                                                                                    sl.r.grad);
      OG_CHECK_LAUNCH();
    }
    sl.phase = PH_DONE;
    return OG_OK;
  }

  og_status serve_step(int max_slices, hipStream_t s, std::vector<long>& done) override {
    st = s;
    for (int it = 0; it < max_slices && !slots.empty(); ++it) {
      std::vector<Op> fwd, adj;
      for (size_t i = 0; i < slots.size(); ++i) {
        Slot& sl = slots[i];
        for (;;) {
          if (!sl.inited) {
            OG_TRY(load1(sl.r.rho0, E, sl.cur_hi, sl.cur_lo, s));
            sl.inited = true;
            sl.phase = PH_FWD;
            sl.j = 0;
          }
          if (sl.phase == PH_FWD) {
            if (sl.j == sl.r.n_t) {
              og::cost_kernel<T><<<1, 256, 0, s>>>(static_cast<const double*>(sl.r.sigma), sl.cur_hi, sl.cur_lo, E, d,
                                                  sl.r.phi);
              OG_CHECK_LAUNCH();
              OG_TRY(load1(sl.r.sigma, 0, sl.lam_hi, sl.lam_lo, s));
              if (sl.n_tail > 0) {  // the resident slices first, then the recomputed segments
                sl.phase = PH_TAIL;
                sl.jj = sl.n_tail - 1;
                continue;
              }
              sl.seg = sl.n_seg - 1;
              OG_TRY(start_segment(sl, s));
              continue;
            }
            if (sl.j < sl.jt && sl.j % sl.S == 0)
              OG_TRY(copy1(sl.ck(sl.j / sl.S), sl.ckl(sl.j / sl.S), sl.cur_hi, sl.cur_lo, s));
            Op o{(int)i, sl.j, sl.cur_hi, sl.cur_lo, sl.cur_hi, sl.cur_lo, nullptr};
            if (sl.j >= sl.jt) o.pk = sl.tl(sl.j - sl.jt + 1);
            fwd.push_back(o);
            break;
          }
          if (sl.phase == PH_TAIL) {
            if (sl.jj < 0) {
              if (sl.n_seg > 0) {
                sl.seg = sl.n_seg - 1;
                OG_TRY(start_segment(sl, s));
                continue;
              }
              OG_TRY(finish(sl, s));
              break;
            }
            Op o{(int)i, sl.jt + sl.jj, sl.lam_hi, sl.lam_lo, sl.lam_hi, sl.lam_lo, sl.tl(sl.jj + 1)};
            o.xpacked = true;
            adj.push_back(o);
            break;
          }
          if (sl.phase == PH_RECOMP) {
            if (sl.jj == sl.n) {
              sl.phase = PH_ADJ;
              sl.jj = sl.n - 1;
              continue;
            }
            fwd.push_back(Op{(int)i, sl.seg * sl.S + sl.jj, sl.sg(sl.jj), sl.sgl(sl.jj), sl.sg(sl.jj + 1),
                             sl.sgl(sl.jj + 1), nullptr});
            break;
          }
          if (sl.phase == PH_ADJ) {
            if (sl.jj < 0) {
              if (--sl.seg >= 0) {
                OG_TRY(start_segment(sl, s));
                continue;
              }
              OG_TRY(finish(sl, s));
              break;
            }
            adj.push_back(Op{(int)i, sl.seg * sl.S + sl.jj, sl.lam_hi, sl.lam_lo, sl.lam_hi, sl.lam_lo,
                             sl.sg(sl.jj + 1)});
            break;
          }
          break;
        }
      }
      if (!fwd.empty()) OG_TRY(run_group(FWD, fwd));
      if (!adj.empty()) OG_TRY(run_group(ADJ, adj));
      for (const Op& o : fwd) {
        Slot& sl = slots[o.slot];
        if (sl.phase == PH_FWD)
          ++sl.j;
        else
          ++sl.jj;
      }
      for (const Op& o : adj) --slots[o.slot].jj;
      // retire finished requests (order of completion = order of admission within a step)
      std::vector<Slot> keep;
      keep.reserve(slots.size());
      for (Slot& sl : slots) {
        if (sl.phase == PH_DONE)
          done.push_back(sl.r.tag);
        else
          keep.push_back(sl);
      }
      slots.swap(keep);
    }
    return OG_OK;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void og_default_options(og_options* opt) {
  if (!opt) return;
  opt->prec = OG_F64;
  opt->gmode = OG_GRAD_GRAPE1;
  opt->path = OG_PATH_AUTO;
  opt->n_sub = 1;
  opt->ckpt_stride = 0;
  opt->validate = 1;
}

const char* og_status_string(og_status s) {
  switch (s) {
    case OG_OK: return "ok";
    case OG_ERR_ARG: return "invalid argument";
    case OG_ERR_SHAPE: return "unsupported shape or operator structure";
    case OG_ERR_NOT_HERMITIAN: return "operator is not Hermitian";
    case OG_ERR_UNSTABLE_DT: return "time step outside the RK4 stability bound";
    case OG_ERR_WORKSPACE: return "workspace missing or too small";
    case OG_ERR_ORDER: return "call out of order";
    case OG_ERR_NONFINITE: return "non-finite state";
    case OG_ERR_DEVICE: return "HIP device error";
  }
  return "unknown status";
}

const char* og_last_error(void) { return g_err.c_str(); }

int og_path_used(const og_ctx* ctx) { return ctx ? ctx->path : -1; }

og_status og_create(og_ctx** out, int d, int K, int J, const void* H0p, const void* Hkp, const void* cp,
                    const double* gamma, const og_options* optp) {
  g_err.clear();
  if (!out) return fail(OG_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (d < 1 || d > 4096) return fail(OG_ERR_ARG, "d must be in [1, 4096]");
  if (K < 0 || K > og::MAXK) return fail(OG_ERR_ARG, "K must be in [0, 16]");
  if (J < 0 || J > 16) return fail(OG_ERR_ARG, "J must be in [0, 16]");
  if (!H0p) return fail(OG_ERR_ARG, "H0 is NULL");
  if (K > 0 && !Hkp) return fail(OG_ERR_ARG, "Hk is NULL with K > 0");
  if (J > 0 && (!cp || !gamma)) return fail(OG_ERR_ARG, "c_ops or gamma is NULL with J > 0");
  og_options opt;
  og_default_options(&opt);
  if (optp) opt = *optp;
  if (opt.prec < OG_F64 || opt.prec > OG_F32_SPLIT_F16) return fail(OG_ERR_ARG, "unknown precision");
  if (opt.gmode != OG_GRAD_GRAPE1 && opt.gmode != OG_GRAD_EXACT) return fail(OG_ERR_ARG, "unknown gradient mode");
  if (opt.path < OG_PATH_AUTO || opt.path > OG_PATH_BANDED) return fail(OG_ERR_ARG, "unknown path");
  if (opt.n_sub < 1 || opt.n_sub > 64) return fail(OG_ERR_ARG, "n_sub must be in [1, 64]");
  if (opt.ckpt_stride < 0) return fail(OG_ERR_ARG, "ckpt_stride must be >= 0");
  for (int m = 0; m < J; ++m)
    if (!(gamma[m] >= 0.0) || !std::isfinite(gamma[m])) return fail(OG_ERR_ARG, "rates must be finite and >= 0");

  Mat H0 = from_ptr(H0p, d, 0);
  std::vector<Mat> Hk, C;
  for (int k = 0; k < K; ++k) Hk.push_back(from_ptr(Hkp, d, k));
  for (int m = 0; m < J; ++m) C.push_back(from_ptr(cp, d, m));
  for (auto* mp : {&H0})
    for (auto& z : mp->a)
      if (!std::isfinite(z.real()) || !std::isfinite(z.imag())) return fail(OG_ERR_ARG, "non-finite operator entry");
  if (opt.validate) {
    if (herm_defect(H0) > 1e-12) return fail(OG_ERR_NOT_HERMITIAN, "H0 is not Hermitian");
    for (int k = 0; k < K; ++k)
      if (herm_defect(Hk[k]) > 1e-12) return fail(OG_ERR_NOT_HERMITIAN, "H_" + std::to_string(k) + " is not Hermitian");
  }

  // G0 = -i H0 - 1/2 sum_m gamma_m c_m^dag c_m (Eq. (4) folded into the generator)
  const cd mi(0, -1);
  Mat G0 = scaled(mi, H0);
  std::vector<Mat> cdc;
  for (int m = 0; m < J; ++m) {
    cdc.push_back(matmul(dagger(C[m]), C[m]));
    G0 = axpy(G0, cd(-0.5 * gamma[m], 0), cdc.back());
  }
  DirHost host[2];
  host[FWD].A0 = G0;
  host[ADJ].A0 = dagger(G0);
  for (int k = 0; k < K; ++k) {
    host[FWD].Ak.push_back(scaled(mi, Hk[k]));
    host[ADJ].Ak.push_back(scaled(cd(0, 1), Hk[k]));
  }
  for (int m = 0; m < J; ++m) {
    host[FWD].C.push_back(C[m]);
    host[ADJ].C.push_back(dagger(C[m]));
    host[FWD].g.push_back(gamma[m]);
    host[ADJ].g.push_back(gamma[m]);
  }

  // decide the path: diagonal storage when every operator set has few diagonals
  int nA = 0, nD = 0, nH = 0;
  {
    std::vector<int> offs;
    collect_offsets(G0, offs);
    for (auto& m : Hk) collect_offsets(m, offs);
    nA = (int)offs.size();
    for (int m = 0; m < J; ++m) {
      if (gamma[m] == 0.0) continue;
      std::vector<int> co;
      collect_offsets(C[m], co);
      nD += (int)(co.size() * co.size());
    }
    std::vector<int> ho;
    for (auto& m : Hk) collect_offsets(m, ho);
    nH = (int)ho.size();
  }
  const bool band_ok = nA <= og::MAXA && nD <= og::MAXD && nH <= og::MAXH;
  int path = opt.path;
  if (path == OG_PATH_BANDED && !band_ok)
    return fail(OG_ERR_SHAPE, "operators have too many diagonals for the banded path (nA=" + std::to_string(nA) +
                                  ", nD=" + std::to_string(nD) + ", nH=" + std::to_string(nH) + ")");
  if (path == OG_PATH_AUTO) path = (band_ok && 2 * nA + nD <= std::max(8, d / 2)) ? OG_PATH_BANDED : OG_PATH_DENSE;

  og_ctx* ctx = new og_ctx();
  ctx->d = d;
  ctx->K = K;
  ctx->J = J;
  ctx->opt = opt;
  ctx->path = path;
  // Gershgorin data for the stability estimate
  ctx->h0_diag.resize(d);
  ctx->h0_rad.resize(d);
  for (int i = 0; i < d; ++i) {
    double r = 0;
    for (int j = 0; j < d; ++j)
      if (j != i) r += std::abs(H0(i, j));
    ctx->h0_diag[i] = H0(i, i).real();
    ctx->h0_rad[i] = r;
  }
  ctx->hk_gersh.assign((size_t)K * d, 0.0);
  ctx->hk_frob.assign(K, 0.0);
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < d; ++i) {
      double r = 0;
      for (int j = 0; j < d; ++j) {
        r += std::abs(Hk[k](i, j));
        ctx->hk_frob[k] += std::norm(Hk[k](i, j));
      }
      ctx->hk_gersh[(size_t)k * d + i] = r;
    }
  for (int k = 0; k < K; ++k) ctx->hk_frob[k] = std::sqrt(ctx->hk_frob[k]);
  for (auto& z : H0.a) ctx->h0_frob += std::norm(z);
  ctx->h0_frob = std::sqrt(ctx->h0_frob);
  for (int m = 0; m < J; ++m) {
    double worst = 0;
    for (int i = 0; i < d; ++i) {
      double r = 0;
      for (int j = 0; j < d; ++j) r += std::abs(cdc[m](i, j));
      worst = std::max(worst, r);
    }
    ctx->diss_bound += 2.0 * gamma[m] * worst;
  }

  hipError_t e1 = hipMalloc((void**)&ctx->status_dev, 256);
  hipError_t e2 = hipMalloc((void**)&ctx->umax_dev, sizeof(double) * kUmaxBlocks * og::MAXK);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    og_destroy(ctx);
    return fail(OG_ERR_DEVICE, "hipMalloc of context scratch failed");
  }
  if (hipMemset(ctx->status_dev, 0, 256) != hipSuccess) {
    og_destroy(ctx);
    return fail(OG_ERR_DEVICE, "hipMemset failed");
  }
  if (!scratch_ptr()) {  // og_evaluate_static's workspace on this device, resolved once
    og_destroy(ctx);
    return fail(OG_ERR_DEVICE, "hipGetSymbolAddress of the static workspace failed");
  }
  og_status s;
  if (opt.prec == OG_F64) {
    auto* e = new Engine<double>(ctx);
    ctx->eng = e;
    s = e->init(host, Hk);
  } else {
    auto* e = new Engine<float>(ctx);
    ctx->eng = e;
    s = e->init(host, Hk);
  }
  if (s != OG_OK) {
    std::string keep = g_err;
    og_destroy(ctx);
    g_err = keep;
    return s;
  }
  *out = ctx;
  return OG_OK;
}

og_status og_create_banded(og_ctx** out, int d, int K, int J, int n_diag, const int* offsets, const void* H0d,
                           const void* Hkd, const void* cd_, const double* gamma, const og_options* opt) {
  g_err.clear();
  if (!out) return fail(OG_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (d < 1 || d > 4096) return fail(OG_ERR_ARG, "d must be in [1, 4096]");
  if (K < 0 || K > og::MAXK) return fail(OG_ERR_ARG, "K must be in [0, 16]");
  if (J < 0 || J > 16) return fail(OG_ERR_ARG, "J must be in [0, 16]");
  if (n_diag < 1 || n_diag > 2 * d - 1) return fail(OG_ERR_ARG, "n_diag must be in [1, 2 d - 1]");
  if (!offsets || !H0d) return fail(OG_ERR_ARG, "offsets or H0_diags is NULL");
  if (K > 0 && !Hkd) return fail(OG_ERR_ARG, "Hk_diags is NULL with K > 0");
  if (J > 0 && !cd_) return fail(OG_ERR_ARG, "c_diags is NULL with J > 0");
  std::vector<int> seen;
  for (int t = 0; t < n_diag; ++t) {
    const int o = offsets[t];
    if (o <= -d || o >= d) return fail(OG_ERR_ARG, "offset outside (-d, d)");
    if (std::find(seen.begin(), seen.end(), o) != seen.end()) return fail(OG_ERR_ARG, "repeated offset");
    seen.push_back(o);
  }
  // expand operator m of an array of n_ops diagonal sets into dense row-major d x d
  const size_t E = (size_t)d * d;
  auto expand = [&](const void* src, int n_ops, std::vector<cd>& dst) {
    const cd* v = static_cast<const cd*>(src);
    dst.assign((size_t)n_ops * E, cd(0, 0));
    for (int m = 0; m < n_ops; ++m)
      for (int t = 0; t < n_diag; ++t) {
        const int o = offsets[t];
        const cd* row = v + ((size_t)m * n_diag + t) * d;
        for (int i = std::max(0, -o); i < d && i + o < d; ++i) dst[(size_t)m * E + (size_t)i * d + i + o] = row[i];
      }
  };
  std::vector<cd> h0, hk, cc;
  expand(H0d, 1, h0);
  if (K > 0) expand(Hkd, K, hk);
  if (J > 0) expand(cd_, J, cc);
  return og_create(out, d, K, J, h0.data(), K > 0 ? hk.data() : nullptr, J > 0 ? cc.data() : nullptr, gamma, opt);
}

og_status og_destroy(og_ctx* ctx) {
  if (!ctx) return OG_OK;
  (void)hipDeviceSynchronize();
  delete ctx->eng;
  for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
  if (ctx->status_dev) (void)hipFree(ctx->status_dev);
  if (ctx->umax_dev) (void)hipFree(ctx->umax_dev);
  if (ctx->pen_coo) (void)hipFree(ctx->pen_coo);
  if (ctx->host_flag) (void)hipHostFree(ctx->host_flag);
  delete ctx;
  return OG_OK;
}

og_status og_set_adaptive(og_ctx* ctx, double rtol, double atol) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (!(rtol >= 0.0) || !(atol >= 0.0) || !std::isfinite(rtol) || !std::isfinite(atol))
    return fail(OG_ERR_ARG, "tolerances must be finite and >= 0");
  if (rtol > 0.0 && ctx->opt.gmode != OG_GRAD_GRAPE1)
    return fail(OG_ERR_ARG, "adaptive steps support the first-order gradient (OG_GRAD_GRAPE1) only");
  if (rtol > 0.0 && !ctx->host_flag) OG_HIP(hipHostMalloc((void**)&ctx->host_flag, sizeof(int)));
  ctx->ad_rtol = rtol;
  ctx->ad_atol = rtol > 0.0 ? atol : 0.0;
  ctx->phase = 0;
  return OG_OK;
}

og_status og_set_resident(og_ctx* ctx, int n_slices) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (n_slices < 0) return fail(OG_ERR_ARG, "n_slices must be >= 0");
  ctx->resident = n_slices;
  ctx->phase = 0;
  return OG_OK;
}

og_status og_set_fused(og_ctx* ctx, int enable) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (ctx->eng->serve_active() > 0) return fail(OG_ERR_ORDER, "requests are in flight on this context");
  ctx->fused_on = enable ? 1 : 0;
  ctx->phase = 0;
  return OG_OK;
}

int og_fused_used(const og_ctx* ctx) { return ctx && ctx->eng ? ctx->eng->fused_used() : 0; }

og_status og_adaptive_stats(og_ctx* ctx, long* counts) {
  g_err.clear();
  if (!ctx || !ctx->eng || !counts) return fail(OG_ERR_ARG, "ctx or counts is NULL");
  if (ctx->phase < 2) return fail(OG_ERR_ORDER, "og_adaptive_stats before og_adjoint");
  return ctx->eng->adaptive_stats(counts);
}

size_t og_workspace_bytes(const og_ctx* ctx, int B, int n_t) {
  if (!ctx || !ctx->eng || B < 1 || n_t < 1) return 0;
  return ctx->eng->ws_bytes(B, n_t);
}

// RK4 stability of the step h = dt / n_sub for controls u (rows x K): reads
// max|u_k| back (one sync), bounds the spectral span of H = H0 + sum u_k H_k
// by Gershgorin discs (or twice the Frobenius norms) and the dissipative
// extent by 2 sum gamma ||c^dag c||_inf; the imaginary-axis limit of classical
// RK4 is 2 sqrt(2) and the real-axis limit 2.785.
static og_status check_stability(og_ctx* ctx, const double* u, long rows, double dt, hipStream_t st) {
  const int K = ctx->K, d = ctx->d;
  std::vector<double> um(K, 0.0);
  if (K > 0) {
    const int nblk = kUmaxBlocks;
    og::umax_kernel<<<nblk, 256, 0, st>>>(u, rows, K, ctx->umax_dev);
    OG_CHECK_LAUNCH();
    std::vector<double> part((size_t)nblk * K);
    OG_HIP(hipMemcpyAsync(part.data(), ctx->umax_dev, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    OG_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < K; ++k)
      for (int p = 0; p < nblk; ++p) {
        const double v = part[(size_t)p * K + k];
        if (!std::isfinite(v)) return fail(OG_ERR_ARG, "non-finite control");
        um[k] = std::max(um[k], v);
      }
  }
  double hi = -1e300, lo = 1e300, frob = ctx->h0_frob;
  for (int i = 0; i < d; ++i) {
    double r = ctx->h0_rad[i];
    for (int k = 0; k < K; ++k) r += um[k] * ctx->hk_gersh[(size_t)k * d + i];
    hi = std::max(hi, ctx->h0_diag[i] + r);
    lo = std::min(lo, ctx->h0_diag[i] - r);
  }
  for (int k = 0; k < K; ++k) frob += um[k] * ctx->hk_frob[k];
  if (ctx->ad_rtol > 0.0) return OG_OK;  // adaptive steps choose their own size
  const double span = std::min(hi - lo, 2.0 * frob);
  const double h = dt / ctx->opt.n_sub;
  if (h * span > 2.83 || h * ctx->diss_bound > 2.78) {
    char buf[256];
    snprintf(buf, sizeof buf,
             "RK4 step h=%g outside the stability bound: h*span(H)=%.3f (limit 2.83), h*dissipation=%.3f (limit "
             "2.78); raise n_sub",
             h, h * span, h * ctx->diss_bound);
    return fail(OG_ERR_UNSTABLE_DT, buf);
  }
  return OG_OK;
}

og_status og_forward(og_ctx* ctx, int B, int n_t, double dt, const double* u, const void* rho0, void* rhoT,
                     void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (B < 1 || B > (1 << 20)) return fail(OG_ERR_ARG, "B must be >= 1");
  if (n_t < 1) return fail(OG_ERR_ARG, "n_t must be >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(OG_ERR_ARG, "dt must be finite and > 0");
  if ((ctx->K > 0 && !u) || !rho0) return fail(OG_ERR_ARG, "u or rho0 is NULL");
  if (!ws) return fail(OG_ERR_WORKSPACE, "workspace is NULL");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(OG_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  ctx->phase = 0;
  OG_HIP(hipMemsetAsync(ctx->status_dev, 0, sizeof(int), st));
  if (ctx->opt.validate) OG_TRY(check_stability(ctx, u, (long)B * n_t, dt, st));
  OG_TRY(ctx->eng->forward(B, n_t, dt, u, rho0, rhoT, ws, ws_bytes, st));
  ctx->phase = 1;
  ++ctx->generation;
  return OG_OK;
}

unsigned long long og_generation(const og_ctx* ctx) { return ctx ? ctx->generation : 0; }

og_status og_cost(og_ctx* ctx, const void* sigma, double* phi, void* stream) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (!sigma || !phi) return fail(OG_ERR_ARG, "sigma or phi is NULL");
  if (ctx->phase < 1) return fail(OG_ERR_ORDER, "og_cost before og_forward");
  return ctx->eng->cost(sigma, phi, static_cast<hipStream_t>(stream));
}

og_status og_adjoint(og_ctx* ctx, const void* sigma, void* stream) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (!sigma) return fail(OG_ERR_ARG, "sigma is NULL");
  if (ctx->phase < 1) return fail(OG_ERR_ORDER, "og_adjoint before og_forward");
  OG_TRY(ctx->eng->adjoint(sigma, static_cast<hipStream_t>(stream)));
  ctx->phase = 2;
  return OG_OK;
}

og_status og_gradient(og_ctx* ctx, double* grad, void* stream) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (!grad) return fail(OG_ERR_ARG, "grad is NULL");
  if (ctx->phase < 2) return fail(OG_ERR_ORDER, "og_gradient before og_adjoint");
  hipStream_t st = static_cast<hipStream_t>(stream);
  OG_TRY(ctx->eng->gradient(grad, st));
  if (ctx->opt.validate) {
    int flag = 0;
    OG_HIP(hipMemcpyAsync(&flag, ctx->status_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    OG_HIP(hipStreamSynchronize(st));
    if (flag) return fail(OG_ERR_NONFINITE, "a propagated state became non-finite");
  }
  return OG_OK;
}

og_status og_gradient_sum(og_ctx* ctx, double* grad, int accumulate, void* stream) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (!grad) return fail(OG_ERR_ARG, "grad is NULL");
  if (ctx->phase < 2) return fail(OG_ERR_ORDER, "og_gradient_sum before og_adjoint");
  hipStream_t st = static_cast<hipStream_t>(stream);
  OG_TRY(ctx->eng->gradient_sum(grad, accumulate ? 1 : 0, st));
  if (ctx->opt.validate) {
    int flag = 0;
    OG_HIP(hipMemcpyAsync(&flag, ctx->status_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    OG_HIP(hipStreamSynchronize(st));
    if (flag) return fail(OG_ERR_NONFINITE, "a propagated state became non-finite");
  }
  return OG_OK;
}

og_status og_evaluate_static(og_ctx* ctx, int B, int n_t, double dt, const double* u, const void* rho0,
                             const void* sigma, double* phi, double* grad, void* stream) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (B < 1 || B > (1 << 20)) return fail(OG_ERR_ARG, "B must be >= 1");
  if (n_t < 1) return fail(OG_ERR_ARG, "n_t must be >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(OG_ERR_ARG, "dt must be finite and > 0");
  if ((ctx->K > 0 && (!u || !grad)) || !rho0 || !sigma || !phi) return fail(OG_ERR_ARG, "NULL argument");
  if (ctx->ad_rtol > 0.0)
    return fail(OG_ERR_ARG, "adaptive steps read every attempt back to the host; og_evaluate_static runs fixed steps");
  const size_t need = ctx->eng->ws_bytes(B, n_t);
  if (need > kStaticWsBytes) {
    char buf[200];
    snprintf(buf, sizeof buf, "evaluation needs %zu bytes of workspace; the static workspace holds %zu", need,
             kStaticWsBytes);
    return fail(OG_ERR_WORKSPACE, buf);
  }
  void* ws = scratch_ptr();
  if (!ws) return fail(OG_ERR_DEVICE, "hipGetSymbolAddress of the static workspace failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // no event sampling here (it creates events)
  const int prof = ctx->prof_every;
  ctx->prof_every = 0;
  ctx->phase = 0;
  og::clear_status_kernel<<<1, 64, 0, st>>>(ctx->status_dev);
  og_status s = OG_OK;
  if (hipGetLastError() != hipSuccess) s = fail(OG_ERR_DEVICE, "kernel launch failed");
  if (s == OG_OK) s = ctx->eng->forward(B, n_t, dt, u, rho0, nullptr, ws, need, st);
  if (s == OG_OK) {
    ctx->phase = 1;
    ++ctx->generation;
    s = ctx->eng->cost(sigma, phi, st);
  }
  if (s == OG_OK) s = ctx->eng->adjoint(sigma, st);
  if (s == OG_OK) {
    ctx->phase = 2;
    s = ctx->eng->gradient(grad, st);
  }
  ctx->prof_every = prof;
  return s;
}

og_status og_set_penalty(og_ctx* ctx, const void* A, double beta) {
  g_err.clear();
  if (!ctx || !ctx->eng) return fail(OG_ERR_ARG, "ctx is NULL");
  if (!std::isfinite(beta)) return fail(OG_ERR_ARG, "beta must be finite");
  if (ctx->pen_coo) {
    (void)hipFree(ctx->pen_coo);
    ctx->pen_coo = nullptr;
    ctx->pen_nnz = 0;
  }
  ctx->pen_beta = 0.0;
  // the index changes: a forward sweep recorded without (or with another)
  // penalty no longer matches, so cost / adjoint wait for the next og_forward
  ctx->phase = 0;
  if (beta == 0.0 || !A) return OG_OK;
  const int d = ctx->d;
  Mat a = from_ptr(A, d, 0);
  for (auto& z : a.a)
    if (!std::isfinite(z.real()) || !std::isfinite(z.imag())) return fail(OG_ERR_ARG, "non-finite entry of A");
  if (ctx->opt.validate && herm_defect(a) > 1e-12) return fail(OG_ERR_NOT_HERMITIAN, "A is not Hermitian");
  // entries of the upper triangle and their conjugate mirror: exactly Hermitian
  std::vector<og::CooEntry> coo;
  for (int i = 0; i < d; ++i)
    for (int j = i; j < d; ++j) {
      const cd v = a(i, j);
      if (v == cd(0, 0)) continue;
      if (i == j) {
        coo.push_back(og::CooEntry{i, i, v.real(), 0.0});
      } else {
        coo.push_back(og::CooEntry{i, j, v.real(), v.imag()});
        coo.push_back(og::CooEntry{j, i, v.real(), -v.imag()});
      }
    }
  if (coo.empty()) return OG_OK;
  OG_HIP(hipMalloc((void**)&ctx->pen_coo, coo.size() * sizeof(og::CooEntry)));
  OG_HIP(hipMemcpy(ctx->pen_coo, coo.data(), coo.size() * sizeof(og::CooEntry), hipMemcpyHostToDevice));
  ctx->pen_nnz = (int)coo.size();
  ctx->pen_beta = beta;
  return OG_OK;
}

og_status og_filter_apply(int B, int N, int M, int K, double dtu, double dts, double omega0, const double* u,
                          double* s, void* stream) {
  g_err.clear();
  if (B < 1 || N < 1 || M < 1 || K < 1 || K > og::MAXK) return fail(OG_ERR_ARG, "bad sizes");
  if (!(dtu > 0) || !(dts > 0) || !(omega0 > 0) || !std::isfinite(omega0)) return fail(OG_ERR_ARG, "bad grid");
  if (!u || !s) return fail(OG_ERR_ARG, "NULL pointer");
  og::filter_apply_kernel<<<dim3((unsigned)((M + 255) / 256), (unsigned)B), 256, 0,
                            static_cast<hipStream_t>(stream)>>>(N, M, K, dtu, dts, omega0, u, s);
  OG_CHECK_LAUNCH();
  return OG_OK;
}

og_status og_filter_grad(int B, int N, int M, int K, double dtu, double dts, double omega0, int fix_ends,
                         const double* g_s, double* g_u, void* stream) {
  g_err.clear();
  if (B < 1 || N < 1 || M < 1 || K < 1 || K > og::MAXK) return fail(OG_ERR_ARG, "bad sizes");
  if (!(dtu > 0) || !(dts > 0) || !(omega0 > 0) || !std::isfinite(omega0)) return fail(OG_ERR_ARG, "bad grid");
  if (!g_s || !g_u) return fail(OG_ERR_ARG, "NULL pointer");
  og::filter_grad_kernel<<<dim3((unsigned)((N + 255) / 256), (unsigned)B), 256, 0,
                           static_cast<hipStream_t>(stream)>>>(N, M, K, dtu, dts, omega0, fix_ends, g_s, g_u);
  OG_CHECK_LAUNCH();
  return OG_OK;
}

og_status og_server_create(og_server** out, og_ctx* ctx, int max_active) {
  g_err.clear();
  if (!out || !ctx || !ctx->eng) return fail(OG_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (max_active < 1 || max_active > 65536) return fail(OG_ERR_ARG, "max_active must be in [1, 65536]");
  if (ctx->path != OG_PATH_BANDED) return fail(OG_ERR_SHAPE, "serving needs the banded path");
  if (ctx->pen_beta != 0.0) return fail(OG_ERR_ARG, "serving does not support the penalty");
  ctx->eng->serve_clear();
  og_server* s = new og_server();
  s->ctx = ctx;
  s->max_active = max_active;
  *out = s;
  return OG_OK;
}

og_status og_server_submit(og_server* s, const og_request* r, void* stream) {
  g_err.clear();
  if (!s || !r) return fail(OG_ERR_ARG, "NULL argument");
  og_ctx* ctx = s->ctx;
  if (r->n_t < 1) return fail(OG_ERR_ARG, "n_t must be >= 1");
  if (!(r->dt > 0.0) || !std::isfinite(r->dt)) return fail(OG_ERR_ARG, "dt must be finite and > 0");
  if ((ctx->K > 0 && (!r->u || !r->grad)) || !r->rho0 || !r->sigma || !r->phi)
    return fail(OG_ERR_ARG, "request pointer is NULL");
  if (!r->ws || (reinterpret_cast<uintptr_t>(r->ws) & 255) != 0)
    return fail(OG_ERR_WORKSPACE, "request workspace NULL or not 256-byte aligned");
  if (ctx->eng->serve_active() >= s->max_active) return fail(OG_ERR_WORKSPACE, "server full");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ctx->opt.validate) OG_TRY(check_stability(ctx, r->u, r->n_t, r->dt, st));
  return ctx->eng->serve_submit(*r, st);
}

og_status og_server_step(og_server* s, int max_slices, void* stream) {
  g_err.clear();
  if (!s) return fail(OG_ERR_ARG, "NULL server");
  if (max_slices < 1) return fail(OG_ERR_ARG, "max_slices must be >= 1");
  return s->ctx->eng->serve_step(max_slices, static_cast<hipStream_t>(stream), s->completed);
}

int og_server_active(const og_server* s) { return s ? s->ctx->eng->serve_active() : 0; }

int og_server_completed(og_server* s, long* tags, int max_tags) {
  if (!s || !tags || max_tags < 1) return 0;
  const int n = std::min<int>(max_tags, (int)s->completed.size());
  for (int i = 0; i < n; ++i) tags[i] = s->completed[i];
  s->completed.erase(s->completed.begin(), s->completed.begin() + n);
  return n;
}

og_status og_server_destroy(og_server* s) {
  if (!s) return OG_OK;
  s->ctx->eng->serve_clear();
  delete s;
  return OG_OK;
}

og_status og_profile(og_ctx* ctx, int every) {
  g_err.clear();
  if (!ctx) return fail(OG_ERR_ARG, "ctx is NULL");
  if (every < 0) return fail(OG_ERR_ARG, "every must be >= 0");
  ctx->prof_every = every;
  ctx->prof_counter = 0;
  return OG_OK;
}

og_status og_profile_read(og_ctx* ctx, double* mean_us, long* count) {
  g_err.clear();
  if (!ctx || !mean_us || !count) return fail(OG_ERR_ARG, "NULL argument");
  double total = 0;
  long n = 0;
  for (size_t i = 0; i < ctx->prof_used; ++i) {
    OG_HIP(hipEventSynchronize(ctx->prof_ev[2 * i + 1]));
    float ms = 0;
    OG_HIP(hipEventElapsedTime(&ms, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]));
    total += ms;
    ++n;
  }
  *mean_us = n ? 1000.0 * total / n : 0.0;
  *count = n;
  ctx->prof_used = 0;
  ctx->prof_counter = 0;
  return OG_OK;
}

}  // extern "C"
