// Device code of the open-GRAPE library: complex helpers, the Runge-Kutta
// stage kernels (banded stencil and dense epilogue), the batched complex
// GEMM on the matrix cores, the gradient contractions and the reductions.
//
// Storage: every d x d matrix is complex, interleaved (re, im), row-major,
// one matrix per problem of the batch at a fixed element stride.  States
// (rho, lambda and the Runge-Kutta stage inputs) are Hermitian and are kept
// exactly Hermitian: kernels compute only the upper-triangular 32 x 32
// tiles and write every result both at (i, j) and, conjugated, at (j, i)
// through an LDS transpose; diagonal elements are written with a zero
// imaginary part.  A rounding residue in the anti-Hermitian part would
// otherwise be amplified by the X + X^dag form of the right-hand side.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace og {

constexpr int TS = 32;      // tile edge of the stage / epilogue kernels
constexpr int MAXA = 16;    // diagonals of the generator A
constexpr int MAXD = 16;    // dissipator taps
constexpr int MAXH = 16;    // diagonals of the control Hamiltonians
constexpr int MAXK = 16;    // controls
constexpr int MAXP = 4;     // pairs per gradient contraction

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> mkc(T r, T i) {
  cpx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return mkc<T>(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cpx<T> cscale(T s, cpx<T> a) { return mkc<T>(s * a.re, s * a.im); }
template <typename T>
__device__ __forceinline__ cpx<T> conjg(cpx<T> a) { return mkc<T>(a.re, -a.im); }
// acc += a * b
template <typename T>
__device__ __forceinline__ void cfma(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}
// acc += a * conj(b)
template <typename T>
__device__ __forceinline__ void cfmac(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.im * b.re - a.re * b.im;
}
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mkc<T>(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}

// Map the hardware block id to a logical one so that consecutive logical
// blocks (the tiles of one problem) run on the same XCD: blocks are handed
// to the 8 XCDs round-robin, so logical = xcd * (n/8) + slot.
__device__ __forceinline__ int xcd_logical_block(int id, int n) {
  return (n & 7) == 0 ? (id & 7) * (n >> 3) + (id >> 3) : id;
}

// ---------------------------------------------------------------------------
// Runge-Kutta stage input / output description
// ---------------------------------------------------------------------------
enum StageMode : int {
  SM_STAGE = 0,  // out = s_hi + (s_lo + coef * L(in))          Horner stage
  SM_FINAL = 1,  // (o_hi, o_lo) = (s_hi, s_lo) + coef * L(in) + sum(extra)
                 //                 with a compensated (two-sum) update
  SM_SCALE = 2   // out = coef * L(in)                          adjoint chain
};

template <typename T>
struct StageIO {
  const cpx<T>* in;   // stencil / GEMM operand Y (full Hermitian matrix)
  long in_s;          // per-problem stride, elements
  const cpx<T>* shi;  // state, read at own elements only
  const cpx<T>* slo;  // compensation of the state (nullptr in float64)
  long s_s;
  cpx<T>* ohi;        // output (may alias shi in SM_FINAL)
  cpx<T>* olo;        // output compensation (SM_FINAL, float32)
  long o_s;
  const cpx<T>* ex[3];  // extra terms added to the increment (SM_FINAL)
  long ex_s;
  int nex;
  T coef;
  int* status;        // set to 1 when a non-finite value is produced
};

// Diagonal storage of the generator pieces for one direction (forward uses
// A = G = -i H - 1/2 sum gamma c^dag c and C = c; the adjoint uses A = G^dag
// and C = c^dag).  A(u) = A0 + sum_k u_k Ak[k].
//   A0[a*d + i]          = A0[i, i + offA[a]]
//   Ak[(k*nA + a)*d + i] = Ak[k][i, i + offA[a]]
//   dissipator tap t:  gamma * C[i, i + dp[t]] * conj(C[j, j + dq[t]]) * Y[i + dp, j + dq]
//   Dl[t*d + i] = gamma * C[i, i + dp[t]],  Dr[t*d + j] = C[j, j + dq[t]]
template <typename T>
struct BandOps {
  int nA;
  int offA[MAXA];
  const cpx<T>* A0;
  const cpx<T>* Ak;
  int nD;
  int dp[MAXD];
  int dq[MAXD];
  const cpx<T>* Dl;
  const cpx<T>* Dr;
};

// Compensated addition (hi, lo) += delta: Knuth's two-sum of hi and delta,
// the error folded into lo, then a renormalising fast two-sum.
template <typename T>
__device__ __forceinline__ void two_sum_update(T& hi, T& lo, T delta) {
  T s = hi + delta;
  T bp = s - hi;
  T e = (hi - (s - bp)) + (delta - bp);
  T l2 = lo + e;
  T h2 = s + l2;
  lo = l2 - (h2 - s);
  hi = h2;
}

// Write the 32 x 32 tile held in v[4] (rows ty + 8q, column tx) to out at
// (I0, J0) and its conjugate transpose at (J0, I0); on a diagonal tile the
// lower triangle is taken from the conjugated upper one.
template <typename T>
__device__ __forceinline__ void write_herm_tile(cpx<T>* __restrict__ out, int d, int I0, int J0,
                                                const cpx<T> (&v)[4], cpx<T> (*tile)[TS + 1], int tx,
                                                int ty) {
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) tile[ty + 8 * q][tx] = v[q];
  __syncthreads();
  const bool diag = (I0 == J0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int i = I0 + r, j = J0 + tx;
    if (i < d && j < d) {
      cpx<T> z = (!diag || r <= tx) ? tile[r][tx] : conjg(tile[tx][r]);
      out[(long)i * d + j] = z;
    }
  }
  if (!diag) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = ty + 8 * q;
      const int i = J0 + r, j = I0 + tx;
      if (i < d && j < d) out[(long)i * d + j] = conjg(tile[tx][r]);
    }
  }
}

template <typename T, int MODE>
__device__ __forceinline__ void stage_epilogue(const StageIO<T>& io, int d, int b, int I0, int J0,
                                               const cpx<T> (&val)[4], cpx<T> (*tile)[TS + 1], int tx,
                                               int ty) {
  cpx<T> oh[4], ol[4];
  bool bad = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = I0 + ty + 8 * q, j = J0 + tx;
    oh[q] = mkc<T>(0, 0);
    ol[q] = mkc<T>(0, 0);
    if (i < d && j < d) {
      const long e = (long)i * d + j;
      if (MODE == SM_SCALE) {
        oh[q] = cscale(io.coef, val[q]);
      } else if (MODE == SM_STAGE) {
        cpx<T> h = io.shi[(long)b * io.s_s + e];
        cpx<T> l = io.slo ? io.slo[(long)b * io.s_s + e] : mkc<T>(0, 0);
        oh[q] = mkc<T>(h.re + (l.re + io.coef * val[q].re), h.im + (l.im + io.coef * val[q].im));
      } else {  // SM_FINAL
        cpx<T> dl = cscale(io.coef, val[q]);
        for (int x = 0; x < io.nex; ++x) dl = cadd(dl, io.ex[x][(long)b * io.ex_s + e]);
        cpx<T> h = io.shi[(long)b * io.s_s + e];
        if (io.slo) {
          cpx<T> l = io.slo[(long)b * io.s_s + e];
          two_sum_update(h.re, l.re, dl.re);
          two_sum_update(h.im, l.im, dl.im);
          ol[q] = l;
        } else {
          h = cadd(h, dl);
        }
        oh[q] = h;
        bad |= !(isfinite(h.re) && isfinite(h.im));
      }
      if (i == j) {
        oh[q].im = 0;
        ol[q].im = 0;
      }
    }
  }
  if (MODE == SM_FINAL && bad) *io.status = 1;
  write_herm_tile<T>(io.ohi + (long)b * io.o_s, d, I0, J0, oh, tile, tx, ty);
  if (MODE == SM_FINAL && io.olo) write_herm_tile<T>(io.olo + (long)b * io.o_s, d, I0, J0, ol, tile, tx, ty);
}

// ---------------------------------------------------------------------------
// Banded Lindblad right-hand side + Runge-Kutta stage.
//   L(Y)_ij = sum_a A_a(i) Y[i + o_a, j] + sum_a Y[i, j + o_a] conj(A_a(j))
//           + sum_t Dl_t(i) conj(Dr_t(j)) Y[i + dp_t, j + dq_t]
// i.e. A Y + Y A^dag + sum_m gamma_m C_m Y C_m^dag in diagonal storage.
// grid.x = B * ntile (upper-triangular tiles), block = 256 threads, each
// thread owns rows ty, ty+8, ty+16, ty+24 and column tx of the tile.
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(256) void band_stage_kernel(BandOps<T> ops, StageIO<T> io,
                                                         const int2* __restrict__ tiles, int ntile, int d,
                                                         int K, const double* __restrict__ u, long u_bs,
                                                         int jslice) {
  __shared__ cpx<T> cR[MAXA][TS];
  __shared__ cpx<T> cC[MAXA][TS];
  __shared__ cpx<T> tile[TS][TS + 1];
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  const int L = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = L / ntile, t = L - b * ntile;
  const int2 tt = tiles[t];
  const int I0 = tt.x * TS, J0 = tt.y * TS;
  const double* ub = u + (long)b * u_bs + (long)jslice * K;
  const int nA = ops.nA;
  for (int e = tid; e < 2 * nA * TS; e += 256) {
    const int side = e / (nA * TS);
    const int rem = e - side * nA * TS;
    const int a = rem / TS, r = rem - a * TS;
    const int idx = (side ? J0 : I0) + r;
    cpx<T> v = mkc<T>(0, 0);
    if (idx < d) {
      v = ops.A0[(long)a * d + idx];
      for (int k = 0; k < K; ++k) {
        const T uk = (T)ub[k];
        const cpx<T> h = ops.Ak[((long)k * nA + a) * d + idx];
        v.re += uk * h.re;
        v.im += uk * h.im;
      }
    }
    if (side)
      cC[a][r] = v;
    else
      cR[a][r] = v;
  }
  __syncthreads();
  const cpx<T>* __restrict__ Y = io.in + (long)b * io.in_s;
  cpx<T> val[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int i = I0 + r, j = J0 + tx;
    cpx<T> acc = mkc<T>(0, 0);
    if (i < d && j < d) {
      for (int a = 0; a < nA; ++a) {
        const int ii = i + ops.offA[a];
        if ((unsigned)ii < (unsigned)d) cfma(acc, cR[a][r], Y[(long)ii * d + j]);
      }
      for (int a = 0; a < nA; ++a) {
        const int jj = j + ops.offA[a];
        if ((unsigned)jj < (unsigned)d) cfmac(acc, Y[(long)i * d + jj], cC[a][tx]);
      }
      for (int s = 0; s < ops.nD; ++s) {
        const int ii = i + ops.dp[s], jj = j + ops.dq[s];
        if ((unsigned)ii < (unsigned)d && (unsigned)jj < (unsigned)d) {
          const cpx<T> w = cmulc(ops.Dl[(long)s * d + i], ops.Dr[(long)s * d + j]);
          cfma(acc, w, Y[(long)ii * d + jj]);
        }
      }
    }
    val[q] = acc;
  }
  stage_epilogue<T, MODE>(io, d, b, I0, J0, val, tile, tx, ty);
}

// ---------------------------------------------------------------------------
// Dense right-hand side epilogue: L(Y) = X + X^dag with X = A Y + 1/2 sum
// gamma C Y C^dag already formed by the GEMMs; then the Runge-Kutta stage.
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(256) void dense_stage_kernel(const cpx<T>* __restrict__ X, long x_s,
                                                          StageIO<T> io, const int2* __restrict__ tiles,
                                                          int ntile, int d) {
  __shared__ cpx<T> tT[TS][TS + 1];
  __shared__ cpx<T> tile[TS][TS + 1];
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  const int L = xcd_logical_block(blockIdx.x, gridDim.x);
  const int b = L / ntile, t = L - b * ntile;
  const int2 tt = tiles[t];
  const int I0 = tt.x * TS, J0 = tt.y * TS;
  const cpx<T>* __restrict__ Xb = X + (long)b * x_s;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int row = J0 + r, col = I0 + tx;
    tT[r][tx] = (row < d && col < d) ? Xb[(long)row * d + col] : mkc<T>(0, 0);
  }
  __syncthreads();
  cpx<T> val[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int i = I0 + r, j = J0 + tx;
    val[q] = (i < d && j < d) ? cadd(Xb[(long)i * d + j], conjg(tT[tx][r])) : mkc<T>(0, 0);
  }
  stage_epilogue<T, MODE>(io, d, b, I0, J0, val, tile, tx, ty);
}

// ---------------------------------------------------------------------------
// Batched complex GEMM on the matrix cores: C = alpha * A * B + beta * C.
// Real 4M split: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br, each a
// v_mfma_*_16x16x4 on planar re / im tiles staged in LDS.
// Block tile 64 x 64, K step 16, 256 threads (2 x 2 waves of 32 x 32).
// Batch entry z = b * nm + m selects operand set m (up to 8 sets).
// ---------------------------------------------------------------------------
constexpr int GM = 8;
template <typename T>
struct GemmArgs {
  const cpx<T>* A[GM];
  long sA[GM];
  int lda[GM];
  const cpx<T>* B[GM];
  long sB[GM];
  int ldb[GM];
  cpx<T>* C[GM];
  long sC[GM];
  int ldc[GM];
  int nm;
  int M, N, Kd;
  cpx<T> alpha, beta;
};

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element v of lane l sits at row 4*(l/16) + v, column l%16
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element v of lane l sits at row (l/16) + 4*v, column l%16
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <typename T>
__global__ __launch_bounds__(256) void zgemm_kernel(GemmArgs<T> g) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int BM = 64, BN = 64, BK = 16, PAD = 4;
  __shared__ T Ar[BK][BM + PAD], Ai[BK][BM + PAD];
  __shared__ T Br[BK][BN + PAD], Bi[BK][BN + PAD];
  const int z = blockIdx.z;
  const int b = z / g.nm, m = z - b * g.nm;
  const cpx<T>* __restrict__ A = g.A[m] + (long)b * g.sA[m];
  const cpx<T>* __restrict__ Bm = g.B[m] + (long)b * g.sB[m];
  cpx<T>* __restrict__ C = g.C[m] + (long)b * g.sC[m];
  const int lda = g.lda[m], ldb = g.ldb[m], ldc = g.ldc[m];
  const int M = g.M, N = g.N, Kd = g.Kd;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  acc_t cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      cr[a][c] = acc_t{0, 0, 0, 0};
      ci[a][c] = acc_t{0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < Kd; k0 += BK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int r = e >> 4, kk = e & 15;
      const int gm = m0 + r, gk = k0 + kk;
      cpx<T> v = (gm < M && gk < Kd) ? A[(long)gm * lda + gk] : mkc<T>(0, 0);
      Ar[kk][r] = v.re;
      Ai[kk][r] = v.im;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int kk = e >> 6, c = e & 63;
      const int gk = k0 + kk, gn = n0 + c;
      cpx<T> v = (gk < Kd && gn < N) ? Bm[(long)gk * ldb + gn] : mkc<T>(0, 0);
      Br[kk][c] = v.re;
      Bi[kk][c] = v.im;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = Ar[kk][wm + a * 16 + (lane & 15)];
        ai[a] = Ai[kk][wm + a * 16 + (lane & 15)];
        br[a] = Br[kk][wn + a * 16 + (lane & 15)];
        bi[a] = Bi[kk][wn + a * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          cr[a][c] = Mfma<T>::mma(ar[a], br[c], cr[a][c]);
          cr[a][c] = Mfma<T>::mma(-ai[a], bi[c], cr[a][c]);
          ci[a][c] = Mfma<T>::mma(ar[a], bi[c], ci[a][c]);
          ci[a][c] = Mfma<T>::mma(ai[a], br[c], ci[a][c]);
        }
    }
    __syncthreads();
  }
  const cpx<T> al = g.alpha, be = g.beta;
  const bool use_beta = (be.re != T(0) || be.im != T(0));
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + a * 16 + Mfma<T>::row(lane, v);
        const int col = n0 + wn + c * 16 + (lane & 15);
        if (row < M && col < N) {
          const T xr = cr[a][c][v], xi = ci[a][c][v];
          cpx<T> o = mkc<T>(al.re * xr - al.im * xi, al.re * xi + al.im * xr);
          if (use_beta) cfma(o, be, C[(long)row * ldc + col]);
          C[(long)row * ldc + col] = o;
        }
      }
}

// ---------------------------------------------------------------------------
// Dense generator assembly A_b = A0 + sum_k u[b, j, k] Ak[k]  (Eq. (1)).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(const cpx<T>* __restrict__ A0,
                                                       const cpx<T>* __restrict__ Ak, int K, long n,
                                                       const double* __restrict__ u, long u_bs, int jslice,
                                                       cpx<T>* __restrict__ out) {
  const int b = blockIdx.y;
  const double* ub = u + (long)b * u_bs + (long)jslice * K;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    cpx<T> v = A0[e];
    for (int k = 0; k < K; ++k) {
      const T uk = (T)ub[k];
      const cpx<T> h = Ak[(long)k * n + e];
      v.re += uk * h.re;
      v.im += uk * h.im;
    }
    out[(long)b * n + e] = v;
  }
}

// ---------------------------------------------------------------------------
// Reductions (float64, fixed order: per-thread strided sums, then a tree
// over the block).  One block of 256 threads per problem.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  const int tid = threadIdx.x;
  __syncthreads();
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  return sh[0];
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// phi[b] = Re Tr(sigma rho_b) = sum_e Re(sigma_e conj(rho_e)) (rho Hermitian).
template <typename T>
__global__ __launch_bounds__(256) void cost_kernel(const double* __restrict__ sigma, const cpx<T>* __restrict__ hi,
                                                   const cpx<T>* __restrict__ lo, long s_s, long n,
                                                   double* __restrict__ phi) {
  __shared__ double sh[256];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (long e = threadIdx.x; e < n; e += 256) {
    const cpx<T> h = hi[(long)b * s_s + e];
    double rr = (double)h.re, ri = (double)h.im;
    if (lo) {
      const cpx<T> l = lo[(long)b * s_s + e];
      rr += (double)l.re;
      ri += (double)l.im;
    }
    acc += sigma[2 * e] * rr + sigma[2 * e + 1] * ri;
  }
  const double s = block_sum256(acc, sh);
  if (threadIdx.x == 0) phi[b] = s;
}

// Gradient contraction, diagonal storage of the H_k:
//   g[b, j, k] = sum_p coef_p * 2 Im Tr(H_k X_p L_p)
//   Tr(H X L) = sum_t sum_a H[a, a + o_t] R_t[a],  R_t[a] = sum_c X[a + o_t, c] conj(L[a, c])
// (L Hermitian).  Each wave computes whole row products R_t[a].
template <typename T>
struct PairArgs {
  const cpx<T>* X[MAXP];
  const cpx<T>* L[MAXP];
  double coef[MAXP];
  long x_s, l_s;
  int np;
};

template <typename T>
struct HBand {
  int nH;
  int offH[MAXH];
  const cpx<T>* Hd;  // [K][nH][d]
};

template <typename T>
__global__ __launch_bounds__(256) void band_contract_kernel(PairArgs<T> pa, HBand<T> hb, int K, int d,
                                                            double* __restrict__ g, long g_bs, int jslice,
                                                            int accumulate) {
  __shared__ double sh[4][MAXK];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double acc[MAXK];
#pragma unroll
  for (int k = 0; k < MAXK; ++k) acc[k] = 0.0;
  for (int p = 0; p < pa.np; ++p) {
    const cpx<T>* __restrict__ X = pa.X[p] + (long)b * pa.x_s;
    const cpx<T>* __restrict__ Lm = pa.L[p] + (long)b * pa.l_s;
    const double cf = pa.coef[p];
    for (int w = wave; w < hb.nH * d; w += 4) {
      const int t = w / d, a = w - t * d;
      const int row = a + hb.offH[t];
      if ((unsigned)row >= (unsigned)d) continue;
      double rr = 0.0, ri = 0.0;
      for (int c = lane; c < d; c += 64) {
        const cpx<T> x = X[(long)row * d + c];
        const cpx<T> l = Lm[(long)a * d + c];
        rr += (double)(x.re * l.re + x.im * l.im);
        ri += (double)(x.im * l.re - x.re * l.im);
      }
      rr = wave_sum(rr);
      ri = wave_sum(ri);
      for (int k = 0; k < K; ++k) {
        const cpx<T> h = hb.Hd[((long)k * hb.nH + t) * d + a];
        acc[k] += cf * ((double)h.re * ri + (double)h.im * rr);
      }
    }
  }
  if (lane == 0)
    for (int k = 0; k < K; ++k) sh[wave][k] = acc[k];
  __syncthreads();
  if (tid < K) {
    const double s = ((sh[0][tid] + sh[1][tid]) + sh[2][tid]) + sh[3][tid];
    double* o = g + (long)b * g_bs + (long)jslice * K + tid;
    *o = accumulate ? *o + 2.0 * s : 2.0 * s;
  }
}

// Dense contraction: W_p = X_p L_p already formed; Tr(H_k W) = sum_e HT_k[e] W[e]
// with HT_k the transpose of H_k.  g = sum_p coef_p 2 Im Tr(H_k W_p).
template <typename T>
__global__ __launch_bounds__(256) void dense_contract_kernel(const cpx<T>* __restrict__ W, long w_s_p,
                                                             long w_s_b, int np, double c0, double c1,
                                                             double c2, double c3,
                                                             const cpx<T>* __restrict__ HT, int K, long n,
                                                             double* __restrict__ g, long g_bs, int jslice,
                                                             int accumulate) {
  __shared__ double sh[256];
  const int b = blockIdx.x;
  const double cf[4] = {c0, c1, c2, c3};
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
    for (int p = 0; p < np; ++p) {
      const cpx<T>* __restrict__ Wp = W + (long)b * w_s_b + (long)p * w_s_p;
      double part = 0.0;
      for (long e = threadIdx.x; e < n; e += 256) {
        const cpx<T> h = HT[(long)k * n + e];
        const cpx<T> w = Wp[e];
        part += (double)(h.re * w.im + h.im * w.re);
      }
      acc += cf[p] * part;
    }
    const double s = block_sum256(acc, sh);
    if (threadIdx.x == 0) {
      double* o = g + (long)b * g_bs + (long)jslice * K + k;
      *o = accumulate ? *o + 2.0 * s : 2.0 * s;
    }
  }
}

// ---------------------------------------------------------------------------
// Precision conversions.  hi = fl_T(x), lo = fl_T(x - hi).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void load_state_kernel(const double* __restrict__ src, long src_s, long n,
                                                         cpx<T>* __restrict__ hi, cpx<T>* __restrict__ lo,
                                                         long s_s) {
  const int b = blockIdx.y;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const double xr = src[2 * ((long)b * src_s + e)], xi = src[2 * ((long)b * src_s + e) + 1];
    const T hr = (T)xr, him = (T)xi;
    hi[(long)b * s_s + e] = mkc<T>(hr, him);
    if (lo) lo[(long)b * s_s + e] = mkc<T>((T)(xr - (double)hr), (T)(xi - (double)him));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void store_state_kernel(const cpx<T>* __restrict__ hi,
                                                          const cpx<T>* __restrict__ lo, long s_s, long n,
                                                          double* __restrict__ dst) {
  const int b = blockIdx.y;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const cpx<T> h = hi[(long)b * s_s + e];
    double xr = h.re, xi = h.im;
    if (lo) {
      const cpx<T> l = lo[(long)b * s_s + e];
      xr += (double)l.re;
      xi += (double)l.im;
    }
    dst[2 * ((long)b * n + e)] = xr;
    dst[2 * ((long)b * n + e) + 1] = xi;
  }
}

// max_{b, j} |u[b, j, k]| for every k (one block).
__global__ __launch_bounds__(256) void umax_kernel(const double* __restrict__ u, long n_rows, int K,
                                                   double* __restrict__ out) {
  __shared__ double sh[256];
  for (int k = 0; k < K; ++k) {
    double m = 0.0;
    for (long r = threadIdx.x; r < n_rows; r += 256) {
      const double a = fabs(u[r * K + k]);
      m = (a != a || m != m) ? a + m : fmax(m, a);  // a NaN control propagates
    }
    __syncthreads();
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const double x = sh[threadIdx.x], y = sh[threadIdx.x + s];
        sh[threadIdx.x] = (x != x || y != y) ? x + y : fmax(x, y);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
  }
}

}  // namespace og
