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
// Cached sub-network operands: the pair tensors (N = 4) and the prefix and
// suffix groups (N >= 5), each two members contracted over their shared
// bonds.  For each outer index the entries form a block of sin consecutive
// outputs.  One wave per workgroup, so that the many resident waves of a CU
// work independently: it stages the member-0 rows [i0][t] and member-1 rows
// [i1][t] the block reads (t padded with zeros to a multiple of 4) in LDS,
// loading every member value once per block instead of once per output,
// then forms the outputs from 16-byte LDS reads with contiguous stores.
// `no` outer indices share one pass when the block is short.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) contract2_k(GroupDesc gd, T* __restrict__ G) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const T* F0 = (const T*)gd.F[0];
  const T* F1 = (const T*)gd.F[1];
  const int ip = gd.innerp, nin = gd.sin, n0 = gd.sin0, n1 = gd.sin1, no = gd.no;
  T* A = (T*)smem_raw;                        // [no][n0][ip]
  T* B = A + (size_t)no * n0 * ip;            // [no][n1][ip]
  int32_t* tin = (int32_t*)(B + (size_t)no * n1 * ip);   // i0 | i1 << 16 per inner entry
  int32_t* off0 = tin + nin;                  // member offsets of the inner digits
  int32_t* off1 = off0 + n0;
  int32_t* tt0 = off1 + n1;                   // member offsets of the internal bonds
  int32_t* tt1 = tt0 + ip;
  int32_t* base = tt1 + ip;                   // [no][2] outer offsets of this pass
  const int lane = threadIdx.x;
  // per-workgroup tables: the inner block's member index pairs and offsets
  for (int i = lane; i < nin; i += 64) {
    uint32_t rem = (uint32_t)i;
    int32_t i0 = 0, i1 = 0, s0 = 1, s1 = 1, o0 = 0, o1 = 0;
    for (int d = gd.nd - 1; d >= gd.ds; --d) {
      const uint32_t sz = (uint32_t)gd.dsize[d];
      const uint32_t quo = div_by(rem, gd.m_dsize[d]);
      const int32_t q = (int32_t)(rem - quo * sz);
      rem = quo;
      if (gd.dmem[d] == 0) {
        i0 += q * s0;
        s0 *= (int32_t)sz;
        o0 += q * gd.dstr[d];
      } else {
        i1 += q * s1;
        s1 *= (int32_t)sz;
        o1 += q * gd.dstr[d];
      }
    }
    tin[i] = i0 | (i1 << 16);
    // every member index combination occurs; write its offset once
    if (i1 == 0) off0[i0] = o0;
    if (i0 == 0) off1[i1] = o1;
  }
  for (int t = lane; t < ip; t += 64) {
    int32_t o0 = 0, o1 = 0;
    if (t < gd.inner) {
      uint32_t rem = (uint32_t)t;
      for (int i = gd.ni - 1; i >= 0; --i) {
        const uint32_t sz = (uint32_t)gd.isize[i];
        const int32_t q = (int32_t)(rem % sz);
        rem /= sz;
        o0 += q * gd.istr0[i];
        o1 += q * gd.istr1[i];
      }
    }
    tt0[t] = o0;
    tt1[t] = o1;
  }
  const int inner = gd.inner;
  for (int64_t ob = (int64_t)blockIdx.x * no; ob < gd.nouter; ob += (int64_t)gridDim.x * no) {
    const int nol = (int)(gd.nouter - ob < no ? gd.nouter - ob : no);
    __syncthreads();   // tables written / the previous pass's LDS reads done
    for (int ol = lane; ol < nol; ol += 64) {
      uint32_t rem = (uint32_t)(ob + ol);
      int32_t b0 = 0, b1 = 0;
      for (int d = gd.ds - 1; d >= 0; --d) {
        const uint32_t sz = (uint32_t)gd.dsize[d];
        const int32_t a = (int32_t)(rem % sz) * gd.dstr[d];
        rem /= sz;
        if (gd.dmem[d] == 0) b0 += a; else b1 += a;
      }
      base[2 * ol] = b0;
      base[2 * ol + 1] = b1;
    }
    __syncthreads();
    // stage both members' rows of the nol outer indices (t-padding as zeros)
    const int na = nol * n0 * ip, nb = nol * n1 * ip;
    for (int j = lane; j < na + nb; j += 64) {
      const bool m1 = j >= na;
      const uint32_t jj = (uint32_t)(m1 ? j - na : j);
      const uint32_t r = div_by(jj, gd.m_ip);            // r = ol * n + i
      const int t = (int)(jj - r * ip);
      const int nm = m1 ? n1 : n0;
      const int ol = (int)div_by(r, m1 ? gd.m_n1 : gd.m_n0), i = (int)r - ol * nm;
      T v = T(0);
      if (t < inner)
        v = m1 ? F1[base[2 * ol + 1] + off1[i] + tt1[t]] : F0[base[2 * ol] + off0[i] + tt0[t]];
      (m1 ? B : A)[jj] = v;
    }
    __syncthreads();
    const int ne = nol * nin;
    T* out = G + ob * nin;
    for (int e = lane; e < ne; e += 64) {
      const int ol = (int)div_by((uint32_t)e, gd.m_nin), i = e - ol * nin;
      const int32_t pr = tin[i];
      const T* a = A + ((size_t)ol * n0 + (pr & 0xffff)) * ip;
      const T* b = B + ((size_t)ol * n1 + (pr >> 16)) * ip;
      T acc = T(0);
      for (int t = 0; t < ip; t += 4) {
        if constexpr (sizeof(T) == 4) {
          const f32x4 x = *(const f32x4*)(a + t), y = *(const f32x4*)(b + t);
          acc += x[0] * y[0];
          acc += x[1] * y[1];
          acc += x[2] * y[2];
          acc += x[3] * y[3];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc += a[t + q] * b[t + q];
        }
      }
      out[e] = acc;
    }
  }
}

// The same contraction when the outer index is one digit a of member 0
// followed by one digit b of member 1 (the N = 4 pair tensors, e.g.
// P12[(i1, i2)][..]): a workgroup of 256 threads takes one a and kPairNB
// consecutive b, stages a's member-0 rows once and the member-1 rows of its
// b values, and writes their kPairNB consecutive output blocks with
// contiguous stores.  The same sums, in the same order, as contract2_k.
constexpr int kPairNB = 8;
template <typename T>
__global__ void __launch_bounds__(256) contract2_ab_k(GroupDesc gd, T* __restrict__ G) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const T* F0 = (const T*)gd.F[0];
  const T* F1 = (const T*)gd.F[1];
  const int ip = gd.innerp, nin = gd.sin, n0 = gd.sin0, n1 = gd.sin1;
  const int nbv = gd.dsize[1];
  const int nblk = (nbv + kPairNB - 1) / kPairNB;
  const int a = (int)(blockIdx.x / nblk), b0 = (int)(blockIdx.x - a * nblk) * kPairNB;
  const int nbl = min(kPairNB, nbv - b0);
  T* A = (T*)smem_raw;                            // [n0][ip]
  T* B = A + (size_t)n0 * ip;                     // [nbl][n1][ip]
  int32_t* tin = (int32_t*)(B + (size_t)kPairNB * n1 * ip);
  int32_t* off0 = tin + nin;
  int32_t* off1 = off0 + n0;
  int32_t* tt0 = off1 + n1;
  int32_t* tt1 = tt0 + ip;
  const int tid = threadIdx.x;
  for (int i = tid; i < nin; i += 256) {
    uint32_t rem = (uint32_t)i;
    int32_t i0 = 0, i1 = 0, s0 = 1, s1 = 1, o0 = 0, o1 = 0;
    for (int d = gd.nd - 1; d >= gd.ds; --d) {
      const uint32_t sz = (uint32_t)gd.dsize[d];
      const uint32_t quo = div_by(rem, gd.m_dsize[d]);
      const int32_t q = (int32_t)(rem - quo * sz);
      rem = quo;
      if (gd.dmem[d] == 0) {
        i0 += q * s0;
        s0 *= (int32_t)sz;
        o0 += q * gd.dstr[d];
      } else {
        i1 += q * s1;
        s1 *= (int32_t)sz;
        o1 += q * gd.dstr[d];
      }
    }
    tin[i] = i0 | (i1 << 16);
    if (i1 == 0) off0[i0] = o0;
    if (i0 == 0) off1[i1] = o1;
  }
  for (int t = tid; t < ip; t += 256) {
    int32_t o0 = 0, o1 = 0;
    if (t < gd.inner) {
      uint32_t rem = (uint32_t)t;
      for (int i = gd.ni - 1; i >= 0; --i) {
        const uint32_t sz = (uint32_t)gd.isize[i];
        const int32_t q = (int32_t)(rem % sz);
        rem /= sz;
        o0 += q * gd.istr0[i];
        o1 += q * gd.istr1[i];
      }
    }
    tt0[t] = o0;
    tt1[t] = o1;
  }
  __syncthreads();
  // a's member-0 rows, then the member-1 rows of b0 .. b0 + nbl - 1
  // (t-padding as zeros)
  const int inner = gd.inner;
  const int64_t base0 = (int64_t)a * gd.dstr[0];
  for (int j = tid; j < n0 * ip; j += 256) {
    const int i = (int)div_by((uint32_t)j, gd.m_ip), t = j - i * ip;
    A[j] = t < inner ? F0[base0 + off0[i] + tt0[t]] : T(0);
  }
  for (int j = tid; j < nbl * n1 * ip; j += 256) {
    const int r = (int)div_by((uint32_t)j, gd.m_ip), t = j - r * ip;
    const int bl = (int)div_by((uint32_t)r, gd.m_n1), i = r - bl * n1;
    B[j] = t < inner ? F1[(int64_t)(b0 + bl) * gd.dstr[1] + off1[i] + tt1[t]] : T(0);
  }
  __syncthreads();
  T* out = G + ((int64_t)a * nbv + b0) * nin;
  for (int e = tid; e < nbl * nin; e += 256) {
    const int bl = (int)div_by((uint32_t)e, gd.m_nin), i = e - bl * nin;
    const int32_t pr = tin[i];
    const T* ar = A + (size_t)(pr & 0xffff) * ip;
    const T* br = B + ((size_t)bl * n1 + (pr >> 16)) * ip;
    T acc = T(0);
    for (int t = 0; t < ip; t += 4) {
      if constexpr (sizeof(T) == 4) {
        const f32x4 x = *(const f32x4*)(ar + t), y = *(const f32x4*)(br + t);
        acc += x[0] * y[0];
        acc += x[1] * y[1];
        acc += x[2] * y[2];
        acc += x[3] * y[3];
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += ar[t + q] * br[t + q];
      }
    }
    out[e] = acc;
  }
}

hipError_t launch_group(int prec, const GroupDesc& gd, void* G, hipStream_t st) {
  if (gd.total == 0) return hipSuccess;
  // outer index (a of member 0, b of member 1): one a and kPairNB b values
  // per 256-thread workgroup, when their rows fit 64 KB of LDS and the
  // quotients of the staging and output walks stay below 2^16
  const size_t es = prec == P_F64 ? 8 : 4;
  const int64_t ip = gd.innerp, n0 = gd.sin0, n1 = gd.sin1, nin = gd.sin;
  const size_t lds_ab = (size_t)(n0 + kPairNB * n1) * ip * es + 4 * (nin + n0 + n1 + 2 * ip);
  if (gd.ds == 2 && gd.dmem[0] == 0 && gd.dmem[1] == 1 && lds_ab <= 64 * 1024 &&
      kPairNB * n1 * ip < 65536 && n0 * ip < 65536 && kPairNB * nin < 65536) {
    const int64_t nblk = (gd.dsize[1] + kPairNB - 1) / kPairNB;
    const int64_t nwg = (int64_t)gd.dsize[0] * nblk;
    if (prec == P_F64) {
      hipFuncSetAttribute((const void*)contract2_ab_k<double>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_ab);
      contract2_ab_k<double><<<(unsigned)nwg, 256, lds_ab, st>>>(gd, (double*)G);
    } else {
      hipFuncSetAttribute((const void*)contract2_ab_k<float>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_ab);
      contract2_ab_k<float><<<(unsigned)nwg, 256, lds_ab, st>>>(gd, (float*)G);
    }
    return hipGetLastError();
  }
  // enough single-wave workgroups for 24 per CU, each over several passes
  const int64_t passes = (gd.nouter + gd.no - 1) / gd.no;
  const int nb = (int)(passes < 6144 ? passes : 6144);
  if (prec == P_F64)
    contract2_k<double><<<nb, 64, gd.lds_bytes, st>>>(gd, (double*)G);
  else
    contract2_k<float><<<nb, 64, gd.lds_bytes, st>>>(gd, (float*)G);
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
