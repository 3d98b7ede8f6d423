// Eigenvalue adjoint as one contraction over the eigenvector pairs.
//
// For unit right eigenvectors v_j = [x_j; y_j] and weights
// gt_j = g_j / (x_j^H x_j - y_j^H y_j) (first-order perturbation with the
// left eigenvector u = S v, Thm 3.2 and eq. 3.5):
//   G_A = sum_j gt_j (x_j x_j^H + conj(y_j) y_j^T)     (Hermitian)
//   G_B = sum_j gt_j (x_j y_j^H + conj(y_j) x_j^T)     (complex symmetric)
// Both outputs share the left factor [gt x_j, gt conj(y_j)], so one kernel
// computes the tile (I, J) of both from one pass over the rows I and J of
// V, and, by the symmetry of both outputs, only tiles with I >= J are
// computed: the tile (J, I) is written from the same registers
// (conjugate transpose for G_A, transpose for G_B).
#include <mutex>

#include "common.h"
#include "vec.h"

// Fixed device memory of the allocation-free adjoint entry point
// (chase_ph_eigval_backward_noalloc): the host weights g (first
// CHASE_PH_NOALLOC_MAX_NEV doubles) and the scaled weights gt (the next
// CHASE_PH_NOALLOC_MAX_NEV).  Each device holds its own copy at its own
// address, resolved once per device with hipGetSymbolAddress; host code
// never passes the array's name itself to a kernel or a copy.
static __device__ __align__(256) double scratch[2 * CHASE_PH_NOALLOC_MAX_NEV];

namespace chase {
namespace {

constexpr int TB = 64;        // output tile (rows and columns)
constexpr int KB = 8;         // eigenpairs per K slab
constexpr int NT = 256;       // 4 waves, each a 32 x 32 quadrant of the tile
constexpr int LDT = TB + 2;   // padded LDS row

__device__ __forceinline__ doublex4 mfma64(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256) void adjoint_weights_kernel(const c128* V, int64_t ldv, int64_t m, const double* g,
                                                              double* gt) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const c128* v = V + (int64_t)j * ldv;
  double s = 0;
  for (int64_t i = threadIdx.x; i < 2 * m; i += 256) {
    const double p = v[i].re * v[i].re + v[i].im * v[i].im;
    s += i < m ? p : -p;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) gt[j] = g[j] / red[0];
}

// Lower tile index t -> (I, J) with I >= J, t = I (I + 1) / 2 + J.
__device__ __forceinline__ void lower_tile(int64_t t, int64_t* I, int64_t* J) {
  int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  *I = i;
  *J = t - i * (i + 1) / 2;
}

__global__ __launch_bounds__(NT) void adjoint_kernel(const c128* __restrict__ V, int64_t ldv, int64_t m, int nev,
                                                     const double* __restrict__ gt, c128* GA, c128* GB, int64_t ldg) {
  // slab layout [buffer][operand][re/im][k][row]: operands 0 = gt x_I,
  // 1 = gt conj(y_I), 2 = x_J, 3 = y_J
  __shared__ double S[2][4][2][KB][LDT];
  int64_t I, J;
  lower_tile(blockIdx.x, &I, &J);
  const int64_t r0 = I * TB, c0 = J * TB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;

  // each thread stages 4 complex values per slab: operand o = tid / 64,
  // rows (tid & 63) ... of each of the KB columns, two columns per pass
  const int o = tid >> 6;          // 0..3
  const int row = tid & 63;
  const int64_t grow = (o < 2 ? r0 : c0) + row;
  const bool row_ok = grow < m;
  const int64_t voff = (o == 1 || o == 3) ? m : 0;   // y half for operands 1, 3
  c128 st[KB];

  const int KT = (nev + KB - 1) / KB;
  auto load = [&](int kt) {
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      const int j = kt * KB + kk;
      const bool ok = row_ok && j < nev;
      st[kk] = ok ? V[(int64_t)j * ldv + voff + grow] : c128{0.0, 0.0};
    }
  };
  auto store = [&](int kt, int buf) {
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      const int j = kt * KB + kk;
      double re = st[kk].re, im = st[kk].im;
      if (o < 2) {
        const double w = j < nev ? gt[j] : 0.0;
        re *= w;
        im *= (o == 1) ? -w : w;     // gt conj(y) for operand 1
      }
      S[buf][o][0][kk][row] = re;
      S[buf][o][1][kk][row] = im;
    }
  };

  doublex4 ar[2][2], ai[2][2], br[2][2], bi[2][2];   // G_A, G_B accumulators
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) ar[i][j][r] = ai[i][j][r] = br[i][j][r] = bi[i][j][r] = 0.0;

  if (KT > 0) {
    load(0);
    store(0, 0);
  }
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < KT; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < KT) load(kt + 1);
#pragma unroll
    for (int ks = 0; ks < KB; ks += 4) {
      double pr[2], pi[2], qr[2], qi[2], xr[2], xi[2], yr[2], yi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        pr[i] = S[buf][0][0][ks + lk][wr + 16 * i + lr];
        pi[i] = S[buf][0][1][ks + lk][wr + 16 * i + lr];
        qr[i] = S[buf][1][0][ks + lk][wr + 16 * i + lr];
        qi[i] = S[buf][1][1][ks + lk][wr + 16 * i + lr];
        xr[i] = S[buf][2][0][ks + lk][wc + 16 * i + lr];
        xi[i] = S[buf][2][1][ks + lk][wc + 16 * i + lr];
        yr[i] = S[buf][3][0][ks + lk][wc + 16 * i + lr];
        yi[i] = S[buf][3][1][ks + lk][wc + 16 * i + lr];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          // G_A += p conj(x_c) + q y_c,   p = gt x_r, q = gt conj(y_r)
          ar[i][j] = mfma64(pr[i], xr[j], ar[i][j]);
          ar[i][j] = mfma64(pi[i], xi[j], ar[i][j]);
          ar[i][j] = mfma64(qr[i], yr[j], ar[i][j]);
          ar[i][j] = mfma64(-qi[i], yi[j], ar[i][j]);
          ai[i][j] = mfma64(pi[i], xr[j], ai[i][j]);
          ai[i][j] = mfma64(-pr[i], xi[j], ai[i][j]);
          ai[i][j] = mfma64(qr[i], yi[j], ai[i][j]);
          ai[i][j] = mfma64(qi[i], yr[j], ai[i][j]);
          // G_B += p conj(y_c) + q x_c
          br[i][j] = mfma64(pr[i], yr[j], br[i][j]);
          br[i][j] = mfma64(pi[i], yi[j], br[i][j]);
          br[i][j] = mfma64(qr[i], xr[j], br[i][j]);
          br[i][j] = mfma64(-qi[i], xi[j], br[i][j]);
          bi[i][j] = mfma64(pi[i], yr[j], bi[i][j]);
          bi[i][j] = mfma64(-pr[i], yi[j], bi[i][j]);
          bi[i][j] = mfma64(qr[i], xi[j], bi[i][j]);
          bi[i][j] = mfma64(qi[i], xr[j], bi[i][j]);
        }
    }
    if (kt + 1 < KT) store(kt + 1, buf ^ 1);
    __syncthreads();
  }

  // D = 16 x 16 block: lane holds rows (lane >> 4) + 4 r, column lane & 15
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = r0 + wr + 16 * i + (lane >> 4) + 4 * r;
        const int64_t gj = c0 + wc + 16 * j + (lane & 15);
        if (gi < m && gj < m) {
          GA[gj * ldg + gi] = c128{ar[i][j][r], ai[i][j][r]};
          GB[gj * ldg + gi] = c128{br[i][j][r], bi[i][j][r]};
          if (I != J) {
            GA[gi * ldg + gj] = c128{ar[i][j][r], -ai[i][j][r]};
            GB[gi * ldg + gj] = c128{br[i][j][r], bi[i][j][r]};
          }
        }
      }
}

}  // namespace

Err adjoint_contract(const c128* V, int64_t ldv, int64_t m, int nev, const double* dg, double* dgt, c128* GA,
                     c128* GB, int64_t ldg, hipStream_t s) {
  if (m <= 0 || nev <= 0) return ok();
  hipLaunchKernelGGL(adjoint_weights_kernel, dim3(nev), dim3(256), 0, s, V, ldv, m, dg, dgt);
  CHASE_LAUNCH_CHECK();
  const int64_t T = ceil_div(m, TB);
  const int64_t tiles = T * (T + 1) / 2;
  if (tiles > 0x7fffffffLL) return fail(CHASE_PH_ERR_ARG, "eigval_backward: m too large");
  hipLaunchKernelGGL(adjoint_kernel, dim3((unsigned)tiles), dim3(NT), 0, s, V, ldv, m, nev, dgt, GA, GB, ldg);
  CHASE_LAUNCH_CHECK();
  return ok();
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_ptr[kMaxDevices] = {};
thread_local std::string noalloc_err;

// Device address of this device's copy of the scratch array (resolved on the
// first call on each device, with that device current).
Err scratch_on_current_device(double** out) {
  int dev = 0;
  CHASE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CHASE_PH_ERR_ARG, "eigval_backward_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    CHASE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(CHASE_PH_ERR_HIP, "eigval_backward_noalloc: no device address for the scratch array");
    scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = scratch_ptr[dev];
  return ok();
}

Err backward_noalloc(int64_t m, int nev, const c128* V, int64_t ldv, const double* hG, c128* GA, c128* GB,
                     int64_t ldg, hipStream_t s) {
  double* ws = nullptr;
  CHASE_TRY(scratch_on_current_device(&ws));
  double* dg = ws;
  double* dgt = ws + CHASE_PH_NOALLOC_MAX_NEV;
  CHASE_HIP(hipMemcpyAsync(dg, hG, (size_t)nev * sizeof(double), hipMemcpyHostToDevice, s));
  CHASE_TRY(adjoint_contract(V, ldv, m, nev, dg, dgt, GA, GB, ldg, s));
  CHASE_HIP(hipStreamSynchronize(s));
  return ok();
}

}  // namespace

const char* noalloc_last_error() { return noalloc_err.c_str(); }

}  // namespace chase

extern "C" chase_ph_status chase_ph_eigval_backward_noalloc(int64_t m, int32_t nev, const void* dV, int64_t ldv,
                                                            const double* hG, void* dGA, void* dGB, int64_t ldg,
                                                            void* hip_stream) {
  using namespace chase;
  Err e;
  if (m <= 0 || nev <= 0 || !dV || !hG || !dGA || !dGB || ldv < 2 * m || ldg < m)
    e = fail(CHASE_PH_ERR_ARG, "eigval_backward_noalloc: bad arguments");
  else if (nev > CHASE_PH_NOALLOC_MAX_NEV)
    e = fail(CHASE_PH_ERR_ARG, "eigval_backward_noalloc: nev = " + std::to_string(nev) +
                                   " exceeds the fixed scratch of " + std::to_string(CHASE_PH_NOALLOC_MAX_NEV) +
                                   " pairs");
  else
    e = backward_noalloc(m, nev, (const c128*)dV, ldv, hG, (c128*)dGA, (c128*)dGB, ldg, (hipStream_t)hip_stream);
  if (e) {
    noalloc_err = e.msg;
    return e.st;
  }
  return CHASE_PH_OK;
}
