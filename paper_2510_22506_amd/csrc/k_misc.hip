// Elementwise and bookkeeping kernels: observed-data setup (Algorithm 1
// initialization), factor casts, the Fourier eigenbasis of L_k (eq. 7),
// the cached pair tensors of the reuse mechanism (Section 3.3), the X update
// of eq. 10 with its norm partials, and the per-sweep scalars.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace fctn {

// ---------------------------------------------------------------------------
// X <- P_Omega(Y); Omega packed to one bit per element; non-finite observed
// values flagged per block.  One wave handles 64 consecutive elements per
// step so that its ballot is exactly two mask words.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) init_observed_k(const T* __restrict__ Y,
                                                       const uint8_t* __restrict__ mask,
                                                       T* __restrict__ X, uint32_t* __restrict__ bits,
                                                       int32_t* __restrict__ bad_part, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  int bad = 0;
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t i = base + lane;
    bool obs = false;
    if (i < n) {
      obs = mask[i] != 0;
      T y = T(0);
      if (obs) {
        y = Y[i];
        if (!isfinite(y)) bad = 1;
      }
      X[i] = y;
    }
    const uint64_t b = __ballot(obs);
    if (lane == 0) bits[base >> 5] = (uint32_t)b;
    if (lane == 1) bits[(base >> 5) + 1] = (uint32_t)(b >> 32);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) bad_part[blockIdx.x] = bad;
}

hipError_t launch_init_observed(int prec, const void* Y, const uint8_t* mask, void* X,
                                uint32_t* bits, int32_t* bad_part, int64_t n, int nblk,
                                hipStream_t st) {
  if (prec == P_F64)
    init_observed_k<double><<<nblk, 256, 0, st>>>((const double*)Y, mask, (double*)X, bits,
                                                   bad_part, n);
  else
    init_observed_k<float><<<nblk, 256, 0, st>>>((const float*)Y, mask, (float*)X, bits,
                                                  bad_part, n);
  return hipGetLastError();
}

__global__ void set_consts_k(double* __restrict__ lam_half, int32_t* __restrict__ ncls,
                             PlanConsts c) {
  const int t = threadIdx.x;
  if (t < c.n) {
    lam_half[t] = c.lam_half[t];
    ncls[t] = c.ncls[t];
  }
}

hipError_t launch_set_consts(double* lam_half, int32_t* ncls, const PlanConsts& c,
                             hipStream_t st) {
  set_consts_k<<<1, 64, 0, st>>>(lam_half, ncls, c);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) any_flag_k(const int32_t* __restrict__ part, int n,
                                                  int32_t* __restrict__ flag) {
  int v = 0;
  for (int i = threadIdx.x; i < n; i += 256) v |= part[i];
  v = __syncthreads_or(v);
  if (threadIdx.x == 0) flag[0] = v ? 1 : 0;
}

hipError_t launch_any_flag(const int32_t* part, int n, int32_t* flag, hipStream_t st) {
  any_flag_k<<<1, 256, 0, st>>>(part, n, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// working-precision copies of a float64 factor (round to nearest even): Aw in
// the factor layout and Au as the row-major mode-k unfolding (I_k x s_k)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void cast_k(const double* __restrict__ a, T* __restrict__ w, T* __restrict__ u,
                       int32_t Ik, int32_t s, int64_t spost) {
  const int64_t n = (int64_t)Ik * s;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    w[e] = (T)a[e];
    const int i = (int)(e / s), j = (int)(e % s);
    u[e] = (T)a[(j / spost) * ((int64_t)Ik * spost) + (int64_t)i * spost + j % spost];
  }
}

hipError_t launch_cast_factor(int prec, const double* A64, void* Aw, void* Au, int32_t Ik,
                              int32_t s, int64_t spost, hipStream_t st) {
  const int64_t n = (int64_t)Ik * s;
  const int nb = (int)(cdiv(n, 256) < 1024 ? cdiv(n, 256) : 1024);
  if (n == 0) return hipSuccess;
  if (prec == P_F64)
    cast_k<double><<<nb, 256, 0, st>>>(A64, (double*)Aw, (double*)Au, Ik, s, spost);
  else
    cast_k<float><<<nb, 256, 0, st>>>(A64, (float*)Aw, (float*)Au, Ik, s, spost);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rank growth: factor k at larger bond ranks.  Entry (m_1 .. m_N) of the new
// factor (last mode fastest) is the old entry when every index is inside the
// old shape; zero when an index along a bond (j, k), j < k (bit j of
// zero_modes) is a new one; otherwise the caller's draw fill[e].  Zero slices
// on the higher-index side of each grown bond keep FCTN(A) unchanged.
// ---------------------------------------------------------------------------
__global__ void regrow_k(const double* __restrict__ old, const double* __restrict__ fill,
                         double* __restrict__ out, RegrowDesc d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = e, off = 0, stride = 1;
    bool inside = true, zero = false;
    for (int j = d.N - 1; j >= 0; --j) {
      const int64_t m = rem % d.shape_new[j];
      rem /= d.shape_new[j];
      if (m >= d.shape_old[j]) {
        inside = false;
        if ((d.zero_modes >> j) & 1) zero = true;
      }
      off += m * stride;
      stride *= d.shape_old[j];
    }
    out[e] = inside ? old[off] : (zero ? 0.0 : fill[e]);
  }
}

hipError_t launch_regrow(const double* old, const double* fill, double* out,
                         const RegrowDesc& d, hipStream_t st) {
  int64_t n = 1;
  for (int j = 0; j < d.N; ++j) n *= d.shape_new[j];
  if (n == 0) return hipSuccess;
  const int nb = (int)(cdiv(n, 256) < 1024 ? cdiv(n, 256) : 1024);
  regrow_k<<<nb, 256, 0, st>>>(old, fill, out, d, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Real orthonormal eigenbasis of the circulant L = (2 + delta) I - S - S^T:
// column 0 is constant; columns 2c-1, 2c are the cosine and sine of frequency
// c (1 <= c < n/2); for even n the last column alternates in sign.  Column
// eigenvalue: delta + 4 sin^2(pi c / n).  Q is n x n row-major (Q[i][col]).
// ---------------------------------------------------------------------------
__global__ void basis_k(double* __restrict__ Q, double* __restrict__ Qt,
                        double* __restrict__ lam_col, int32_t n, double delta) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), col = (int)(e % n);
    double v;
    int c;
    if (col == 0) {
      c = 0;
      v = 1.0 / sqrt((double)n);
    } else if ((n % 2 == 0) && col == n - 1) {
      c = n / 2;
      v = ((i & 1) ? -1.0 : 1.0) / sqrt((double)n);
    } else {
      c = (col + 1) / 2;
      const int64_t m = ((int64_t)i * c) % n;
      const double ang = 2.0 * (double)m / (double)n;   // angle / pi
      v = sqrt(2.0 / n) * ((col & 1) ? cospi(ang) : sinpi(ang));
    }
    Q[e] = v;
    Qt[(int64_t)col * n + i] = v;
    if (i == 0) {
      const double sn = sinpi((double)c / (double)n);
      lam_col[col] = delta + 4.0 * sn * sn;
    }
  }
}

hipError_t launch_build_basis(double* Q, double* Qt, double* lam_col, int32_t n, double delta,
                              hipStream_t st) {
  const int64_t nn = (int64_t)n * n;
  const int nb = (int)(cdiv(nn, 256) < 1024 ? cdiv(nn, 256) : 1024);
  basis_k<<<nb, 256, 0, st>>>(Q, Qt, lam_col, n, delta);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pair tensor of the reuse mechanism (two factors contracted over their
// shared bond), written in the layout the sub-network generator reads.
// ---------------------------------------------------------------------------
// One output per thread, so that a wave's stores are contiguous; the pair
// tensor and the factors stay below 2^31 elements (checked on the host), so
// every index is 32-bit (64-bit division would dominate the kernel).
template <typename T>
__global__ void __launch_bounds__(256) pair_k(PairDesc pd, T* __restrict__ P, int64_t total) {
  const T* Fa = (const T*)pd.Fa;
  const T* Fb = (const T*)pd.Fb;
  const uint32_t n = (uint32_t)total;
  const uint32_t n2b = pd.n2b, n2a = pd.n2a, n1b = pd.n1b, n1a = pd.n1a, Ib = pd.Ib;
  const int a_i = (int)pd.a_i, a_1 = (int)pd.a_1, a_2 = (int)pd.a_2, a_k = (int)pd.a_k;
  const int b_i = (int)pd.b_i, b_1 = (int)pd.b_1, b_2 = (int)pd.b_2, b_k = (int)pd.b_k;
  for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < n; o += gridDim.x * blockDim.x) {
    uint32_t q = o;
    const uint32_t b2 = q % n2b; q /= n2b;
    const uint32_t a2 = q % n2a; q /= n2a;
    const uint32_t b1 = q % n1b; q /= n1b;
    const uint32_t a1 = q % n1a; q /= n1a;
    const uint32_t ib = q % Ib, ia = q / Ib;
    const T* pa = Fa + (int)ia * a_i + (int)a1 * a_1 + (int)a2 * a_2;
    const T* pb = Fb + (int)ib * b_i + (int)b1 * b_1 + (int)b2 * b_2;
    T acc = T(0);
#pragma unroll 4
    for (int k = 0; k < pd.K; ++k) acc += pa[k * a_k] * pb[k * b_k];
    P[o] = acc;
  }
}

hipError_t launch_pair(int prec, const PairDesc& pd, void* P, hipStream_t st) {
  const int64_t total = (int64_t)pd.Ia * pd.Ib * pd.n1a * pd.n1b * pd.n2a * pd.n2b;
  const int nb = (int)(cdiv(total, 256) < 8192 ? cdiv(total, 256) : 8192);
  if (total == 0) return hipSuccess;
  if (prec == P_F64)
    pair_k<double><<<nb, 256, 0, st>>>(pd, (double*)P, total);
  else
    pair_k<float><<<nb, 256, 0, st>>>(pd, (float*)P, total);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Group operand (orders N >= 5): one thread per output entry decodes its
// digits into member offsets, then walks the internal bonds as an odometer,
// accumulating the product of the members' entries.  The group tensors are
// small next to X (I_a I_b times a few hundred bond values), so this plain
// form is HBM- and latency-bound, not a contraction worth MFMA tiles.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) group_k(GroupDesc gd, T* __restrict__ G) {
  // the member offsets of every internal bond value, once per workgroup
  __shared__ int32_t tab[kGroupMaxInner * kGroupMaxMembers];
  for (int t = threadIdx.x; t < gd.inner; t += blockDim.x) {
    int32_t o[kGroupMaxMembers] = {0, 0, 0, 0, 0, 0};
    uint32_t rem = (uint32_t)t;
    for (int i = gd.ni - 1; i >= 0; --i) {
      const uint32_t q = rem % (uint32_t)gd.isize[i];
      rem /= (uint32_t)gd.isize[i];
#pragma unroll
      for (int f = 0; f < kGroupMaxMembers; ++f) {
        o[f] += gd.imem0[i] == f ? (int32_t)q * gd.istr0[i] : 0;
        o[f] += gd.imem1[i] == f ? (int32_t)q * gd.istr1[i] : 0;
      }
    }
#pragma unroll
    for (int f = 0; f < kGroupMaxMembers; ++f) tab[t * kGroupMaxMembers + f] = o[f];
  }
  __syncthreads();
  for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < gd.total;
       e += gridDim.x * blockDim.x) {
    int32_t off[kGroupMaxMembers] = {0, 0, 0, 0, 0, 0};
    uint32_t rem = (uint32_t)e;
    for (int d = gd.nd - 1; d >= 0; --d) {
      const uint32_t sz = (uint32_t)gd.dsize[d];
      const uint32_t q = rem % sz;
      rem /= sz;
      const int32_t add = (int32_t)q * gd.dstr[d];
#pragma unroll
      for (int f = 0; f < kGroupMaxMembers; ++f) off[f] += gd.dmem[d] == f ? add : 0;
    }
    T acc = T(0);
    for (int32_t t = 0; t < gd.inner; ++t) {
      T prod = T(1);
#pragma unroll
      for (int f = 0; f < kGroupMaxMembers; ++f)
        if (f < gd.nm) prod *= ((const T*)gd.F[f])[off[f] + tab[t * kGroupMaxMembers + f]];
      acc += prod;
    }
    G[e] = acc;
  }
}

hipError_t launch_group(int prec, const GroupDesc& gd, void* G, hipStream_t st) {
  if (gd.total == 0) return hipSuccess;
  const int nb = (int)(cdiv(gd.total, 256) < 8192 ? cdiv(gd.total, 256) : 8192);
  if (prec == P_F64)
    group_k<double><<<nb, 256, 0, st>>>(gd, (double*)G);
  else
    group_k<float><<<nb, 256, 0, st>>>(gd, (float*)G);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// eq. 10 as a select: X on Omega already equals Y, so only X, Z and the mask
// bits are read.  Per-block float64 partials: ||X+ - X||^2, ||X||^2,
// ||X+ - Z||^2.  16-byte vector accesses; a fixed grid keeps the partial
// sums (and so the scalars) deterministic.
// ---------------------------------------------------------------------------
template <typename T> struct Vec;
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <> struct Vec<float> { typedef f32x4 t; static constexpr int w = 4; };
template <> struct Vec<double> { typedef f64x2 t; static constexpr int w = 2; };

template <typename T>
__device__ inline void xupd_one(T& x, T z, bool obs, T rho, T opr, double& sdx, double& sxx,
                                double& sdz) {
  const T xn = obs ? x : (z + rho * x) / opr;
  const double d = (double)xn - (double)x;
  const double e = (double)xn - (double)z;
  sdx += d * d;
  sxx += (double)x * (double)x;
  sdz += e * e;
  x = xn;
}

template <typename T, bool NT>
__global__ void __launch_bounds__(256) x_update_k(T* __restrict__ X, const T* __restrict__ Z,
                                                  const uint32_t* __restrict__ bits, double rho_d,
                                                  int64_t n, double* __restrict__ xpart) {
  typedef typename Vec<T>::t V;
  constexpr int W = Vec<T>::w;
  const T rho = (T)rho_d, opr = (T)(1.0 + rho_d);
  double sdx = 0.0, sxx = 0.0, sdz = 0.0;
  // NT (a pass larger than the 256 MB Infinity Cache): one vector per thread
  // over a grid that covers the tensor once, with non-temporal loads and
  // stores (measured on a 1 GiB pass: 6.4-6.6 TB/s against 5.0 for a
  // grid-stride loop of ordinary accesses).  Smaller passes, which the cache
  // serves, run a grid-stride loop over a fixed 1024-block grid (faster there).
  const int64_t nv = n / W;
  const int64_t stride = NT ? nv + 1 : (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
    V xv, zv;
    if constexpr (NT) {
      xv = __builtin_nontemporal_load(&((const V*)X)[v]);
      zv = __builtin_nontemporal_load(&((const V*)Z)[v]);
    } else {
      xv = ((const V*)X)[v];
      zv = ((const V*)Z)[v];
    }
    const int64_t i0 = v * W;
    const uint32_t word = bits[i0 >> 5] >> (i0 & 31);
#pragma unroll
    for (int j = 0; j < W; ++j) {
      T x = xv[j];
      xupd_one<T>(x, zv[j], (word >> j) & 1u, rho, opr, sdx, sxx, sdz);
      xv[j] = x;
    }
    if constexpr (NT)
      __builtin_nontemporal_store(xv, &((V*)X)[v]);
    else
      ((V*)X)[v] = xv;
  }
  {   // the last n mod W elements
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n - nv * W) {
      const int64_t i = nv * W + t;
      T x = X[i];
      xupd_one<T>(x, Z[i], (bits[i >> 5] >> (i & 31)) & 1u, rho, opr, sdx, sxx, sdz);
      X[i] = x;
    }
  }
  __shared__ double red[3][4];
  sdx = wave_sum(sdx);
  sxx = wave_sum(sxx);
  sdz = wave_sum(sdz);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = sdx;
    red[1][w] = sxx;
    red[2][w] = sdz;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int k = 0; k < 4; ++k) s += red[threadIdx.x][k];
    xpart[blockIdx.x * 3 + threadIdx.x] = s;
  }
}

static inline bool x_update_nt(int prec, int64_t n) {
  return (double)n * (prec == P_F64 ? 8 : 4) * 3 > 192.0 * (1 << 20);
}

int x_update_blocks(int prec, int64_t n) {
  if (!x_update_nt(prec, n)) return 1024;
  const int64_t w = prec == P_F64 ? 2 : 4;
  return (int)std::max<int64_t>(1, (n / w + 255) / 256);
}

hipError_t launch_x_update(int prec, void* X, const void* Z, const uint32_t* bits, double rho,
                           int64_t n, int nblk, double* xpart, hipStream_t st) {
  const bool nt = x_update_nt(prec, n);
  if (prec == P_F64) {
    if (nt)
      x_update_k<double, true><<<nblk, 256, 0, st>>>((double*)X, (const double*)Z, bits, rho, n,
                                                     xpart);
    else
      x_update_k<double, false><<<nblk, 256, 0, st>>>((double*)X, (const double*)Z, bits, rho,
                                                      n, xpart);
  } else {
    if (nt)
      x_update_k<float, true><<<nblk, 256, 0, st>>>((float*)X, (const float*)Z, bits, rho, n,
                                                    xpart);
    else
      x_update_k<float, false><<<nblk, 256, 0, st>>>((float*)X, (const float*)Z, bits, rho, n,
                                                     xpart);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-sweep scalars: rel_change, f_data, f_trace, objective (fixed order)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) stats_k(const double* __restrict__ xpart, int nblk,
                                               const double* __restrict__ trace_part,
                                               const double* __restrict__ lam_half,
                                               const int32_t* __restrict__ ncls, int N,
                                               int max_cls, double* __restrict__ slot) {
  // s[0..2]: the X-pass partials; s[3]: sum_k lambda_k/2 sum_c trace_part[k][c]
  // (every sum strided over the threads, then a fixed-order tree)
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += 256)
    for (int q = 0; q < 3; ++q) s[q] += xpart[b * 3 + q];
  for (int f = threadIdx.x; f < N * max_cls; f += 256) {
    const int k = f / max_cls, c = f - k * max_cls;
    if (c < ncls[k]) s[3] += lam_half[k] * trace_part[f];
  }
  __shared__ double red[4][4];
  for (int q = 0; q < 4; ++q) {
    const double v = wave_sum(s[q]);
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[4];
    for (int q = 0; q < 4; ++q) t[q] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
    slot[0] = sqrt(t[0]) / sqrt(t[1]);
    slot[1] = 0.5 * t[2];
    slot[2] = t[3];
    slot[3] = slot[1] + slot[2];
  }
}

hipError_t launch_stats(const double* xpart, int nblk, const double* trace_part,
                        const double* lam_half, const int32_t* ncls, int N, int max_cls,
                        double* hist_slot, hipStream_t st) {
  stats_k<<<1, 256, 0, st>>>(xpart, nblk, trace_part, lam_half, ncls, N, max_cls, hist_slot);
  return hipGetLastError();
}

}  // namespace fctn
