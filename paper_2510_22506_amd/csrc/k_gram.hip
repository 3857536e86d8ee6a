// Fused sub-network generation + Gram + right-hand side (Property 1, eq. 5),
// the deterministic float64 split-K reduction, and the reconstruction
// FCTN(A) = A_k(k) M_k used by the X update (Algorithm 2).
//
// gram_rhs: each workgroup owns a range of columns of M_k (split-K) and a
// group of 16x16 output tiles (upper-triangle Gram tiles, then RHS tiles).
// Per 16..32-column tile it regenerates M_k's columns in LDS from the factor
// / pair operands (M_k is never stored in HBM), stages the matching rows of
// X_(k), and accumulates G += M M^T and B += X M^T on MFMA.  Partial tiles go
// to a split-major buffer that reduce_gb sums in float64, in split order.
#include "common.hpp"
#include "kernels.hpp"

namespace fctn {

constexpr int kGramThreads = 256;
constexpr int kTPW = 16;   // output tiles per wave

__device__ inline void upper_tile(int t, int& bi, int& bj) {
  int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (j * (j + 1) / 2 > t) --j;
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  bj = j;
  bi = t - j * (j + 1) / 2;
}

// M[row, col] for row < s, col < C (caller guards), accumulated in T.
template <typename T>
__device__ inline T mgen_entry(const MGen& mg, const T* __restrict__ U, const T* __restrict__ V,
                               int row, int64_t col) {
  const int ru = row / mg.Rv, rv = row - (row / mg.Rv) * mg.Rv;
  const int64_t cu = col / mg.Cv, cv = col - cu * mg.Cv;
  const T* pu = U + ru * mg.u_ru + cu * mg.u_cu;
  const T* pv = V + rv * mg.v_rv + cv * mg.v_cv;
  T acc = T(0);
  for (int k = 0; k < mg.K; ++k) acc += pu[k * mg.u_k] * pv[k * mg.v_k];
  return acc;
}

template <typename T>
__global__ void __launch_bounds__(kGramThreads) gram_rhs_k(MGen mg, const T* __restrict__ X,
                                                           XView xv, GramGeom g,
                                                           T* __restrict__ part) {
  typedef Mfma<T> MM;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Ms = (T*)smem_raw;                    // [tc][ldm]  rows of M fastest
  T* Xs = Ms + (int64_t)g.tc * g.ldm;      // [tc][ldx]  rows of X_(k) fastest
  const T* U = (const T*)mg.U;
  const T* V = (const T*)mg.V;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int split = blockIdx.x, group = blockIdx.y;
  const int t0 = group * g.tilesPerGroup;
  const int t1 = min(t0 + g.tilesPerGroup, g.nTiles);

  int ba_lo = 0, xrows = 0;
  if (t1 > g.nG) {
    const int bfirst = (max(t0, g.nG) - g.nG) / g.nbj;
    const int blast = (t1 - 1 - g.nG) / g.nbj;
    ba_lo = bfirst;
    xrows = (blast - bfirst + 1) * 16;
  }

  int aoff[kTPW], boff[kTPW];
  bool fromX[kTPW], valid[kTPW];
  typename MM::acc_t acc[kTPW];
#pragma unroll
  for (int j = 0; j < kTPW; ++j) {
    const int t = t0 + wave + 4 * j;
    valid[j] = t < t1;
    acc[j] = MM::zero();
    int bi = 0, bj = 0;
    fromX[j] = false;
    if (valid[j]) {
      if (t < g.nG) {
        upper_tile(t, bi, bj);
      } else {
        const int tb = t - g.nG;
        bi = tb / g.nbj - ba_lo;
        bj = tb % g.nbj;
        fromX[j] = true;
      }
    }
    aoff[j] = bi * 16 + (lane & 15);
    boff[j] = bj * 16 + (lane & 15);
  }

  const int64_t C = mg.Cu * mg.Cv;
  const int64_t ct0 = (int64_t)split * g.colTilesPerSplit;
  const int64_t ct1 = min(ct0 + g.colTilesPerSplit, g.nColTiles);
  const int tc = g.tc, sp = g.sp, ldm = g.ldm, ldx = g.ldx;

  for (int64_t ct = ct0; ct < ct1; ++ct) {
    const int64_t col0 = ct * tc;
    for (int e = tid; e < tc * sp; e += kGramThreads) {
      const int c = e / sp, row = e - (e / sp) * sp;
      const int64_t col = col0 + c;
      T v = T(0);
      if (row < g.s && col < C) v = mgen_entry<T>(mg, U, V, row, col);
      Ms[c * ldm + row] = v;
    }
    if (xrows > 0) {
      const int ne = tc * xrows;
      for (int e = tid; e < ne; e += kGramThreads) {
        int c, r;
        if (xv.x_ik == 1) {
          c = e / xrows;
          r = e - c * xrows;
        } else {
          r = e / tc;
          c = e - r * tc;
        }
        const int ik = ba_lo * 16 + r;
        const int64_t col = col0 + c;
        T v = T(0);
        if (ik < xv.Ik && col < C) {
          const int64_t cu = col / mg.Cv, cv = col - cu * mg.Cv;
          v = X[cu * xv.x_cu + cv * xv.x_cv + (int64_t)ik * xv.x_ik];
        }
        Xs[c * ldx + r] = v;
      }
    }
    __syncthreads();
    const int kr = lane >> 4;
#pragma unroll
    for (int j = 0; j < kTPW; ++j) {
      if (valid[j]) {
        const T* Ab = fromX[j] ? Xs : Ms;
        const int lda = fromX[j] ? ldx : ldm;
        for (int kk = 0; kk < tc; kk += MM::kStep) {
          const T a = Ab[(kk + kr) * lda + aoff[j]];
          const T b = Ms[(kk + kr) * ldm + boff[j]];
          acc[j] = MM::mma(a, b, acc[j]);
        }
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int j = 0; j < kTPW; ++j) {
    if (valid[j]) {
      const int t = t0 + wave + 4 * j;
      T* base = part + ((int64_t)split * g.nTiles + t) * 256;
#pragma unroll
      for (int i = 0; i < 4; ++i) base[MM::row(lane, i) * 16 + (lane & 15)] = acc[j][i];
    }
  }
}

int gram_max_lds_bytes() { return 160 * 1024; }

hipError_t launch_gram_rhs(int prec, const MGen& mg, const void* X, const XView& xv,
                           const GramGeom& g, void* part, hipStream_t st) {
  dim3 grid(g.nSplit, g.nGroups);
  if (prec == P_F64) {
    hipFuncSetAttribute((const void*)gram_rhs_k<double>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    gram_rhs_k<double><<<grid, kGramThreads, g.lds_bytes, st>>>(mg, (const double*)X, xv, g,
                                                                (double*)part);
  } else {
    hipFuncSetAttribute((const void*)gram_rhs_k<float>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    gram_rhs_k<float><<<grid, kGramThreads, g.lds_bytes, st>>>(mg, (const float*)X, xv, g,
                                                               (float*)part);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// G = sum_split Gpart (symmetric: element (i, j) is read from the upper tile
// holding (min, max)), B = sum_split Bpart + rho A_k(k); float64, split order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) reduce_gb_k(GramGeom g, const T* __restrict__ part,
                                                   const double* __restrict__ A64, int64_t spost,
                                                   double rho, double* __restrict__ G,
                                                   double* __restrict__ B) {
  const int s = g.s;
  const int64_t nGel = (int64_t)s * s, total = nGel + (int64_t)g.Ik * s;
  const int64_t tstride = (int64_t)g.nTiles * 256;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int t, el;
    double extra = 0.0;
    if (e < nGel) {
      const int i = (int)(e / s), j = (int)(e % s);
      const int lo = min(i, j), hi = max(i, j);
      const int bi = lo >> 4, bj = hi >> 4;
      t = bj * (bj + 1) / 2 + bi;
      el = (lo & 15) * 16 + (hi & 15);
    } else {
      const int64_t e2 = e - nGel;
      const int a = (int)(e2 / s), j = (int)(e2 % s);
      t = g.nG + (a >> 4) * g.nbj + (j >> 4);
      el = (a & 15) * 16 + (j & 15);
      extra = rho * A64[(j / spost) * ((int64_t)g.Ik * spost) + (int64_t)a * spost + j % spost];
    }
    const T* p = part + (int64_t)t * 256 + el;
    double acc = 0.0;
    for (int sp = 0; sp < g.nSplit; ++sp) acc += (double)p[(int64_t)sp * tstride];
    if (e < nGel)
      G[e] = acc;
    else
      B[e - nGel] = acc + extra;
  }
}

hipError_t launch_reduce_gb(int prec, const GramGeom& g, const void* part, const double* A64,
                            int64_t spost, double rho, double* G, double* B, hipStream_t st) {
  const int64_t total = (int64_t)g.s * g.s + (int64_t)g.Ik * g.s;
  const int nb = (int)(cdiv(total, 256) < 2048 ? cdiv(total, 256) : 2048);
  if (prec == P_F64)
    reduce_gb_k<double><<<nb, 256, 0, st>>>(g, (const double*)part, A64, spost, rho, G, B);
  else
    reduce_gb_k<float><<<nb, 256, 0, st>>>(g, (const float*)part, A64, spost, rho, G, B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Z_(k) = A_k(k) M_k with M_k regenerated per column tile in LDS ([row][col],
// columns fastest) and the 16x16 output tiles on MFMA; Z is written through
// the X view (same layout as X).
// ---------------------------------------------------------------------------
constexpr int kRecTC = 64;

template <typename T>
__global__ void __launch_bounds__(256) reconstruct_k(MGen mg, const T* __restrict__ Au,
                                                     T* __restrict__ Z, XView xv, int s, int sp,
                                                     int64_t C, int64_t nColTiles) {
  typedef Mfma<T> MM;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int ldc = kRecTC + 16;   // 80: conflict-free MFMA B-operand reads
  T* Ms = (T*)smem_raw;              // [sp][ldc]
  const T* U = (const T*)mg.U;
  const T* V = (const T*)mg.V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nib = (xv.Ik + 15) / 16;
  const int ntiles = nib * (kRecTC / 16);
  for (int64_t ct = blockIdx.x; ct < nColTiles; ct += gridDim.x) {
    const int64_t col0 = ct * kRecTC;
    for (int e = tid; e < kRecTC * sp; e += 256) {
      const int row = e / kRecTC, c = e - row * kRecTC;
      const int64_t col = col0 + c;
      T v = T(0);
      if (row < s && col < C) v = mgen_entry<T>(mg, U, V, row, col);
      Ms[row * ldc + c] = v;
    }
    __syncthreads();
    for (int t = wave; t < ntiles; t += 4) {
      const int ib = t / (kRecTC / 16), cb = t % (kRecTC / 16);
      typename MM::acc_t acc = MM::zero();
      const int ik_a = ib * 16 + (lane & 15);
      for (int k0 = 0; k0 < sp; k0 += MM::kStep) {
        const int row = k0 + (lane >> 4);
        const T a = (ik_a < xv.Ik && row < s) ? Au[(int64_t)ik_a * s + row] : T(0);
        const T b = Ms[row * ldc + cb * 16 + (lane & 15)];
        acc = MM::mma(a, b, acc);
      }
      const int64_t col = col0 + cb * 16 + (lane & 15);
      if (col < C) {
        const int64_t cu = col / mg.Cv, cv = col - cu * mg.Cv;
        const int64_t base = cu * xv.x_cu + cv * xv.x_cv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int ik = ib * 16 + MM::row(lane, i);
          if (ik < xv.Ik) Z[base + (int64_t)ik * xv.x_ik] = acc[i];
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_reconstruct(int prec, const MGen& mg, const void* Au, void* Z,
                              const XView& xv, int32_t s, int64_t C, hipStream_t st) {
  const int sp = (s + 15) / 16 * 16;
  const int64_t nct = cdiv(C, kRecTC);
  const int nb = (int)(nct < 2048 ? nct : 2048);
  const size_t elt = prec == P_F64 ? 8 : 4;
  const size_t lds = (size_t)sp * (kRecTC + 16) * elt;
  if (prec == P_F64) {
    hipFuncSetAttribute((const void*)reconstruct_k<double>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    reconstruct_k<double><<<nb, 256, lds, st>>>(mg, (const double*)Au, (double*)Z, xv, s, sp,
                                                C, nct);
  } else {
    hipFuncSetAttribute((const void*)reconstruct_k<float>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    reconstruct_k<float><<<nb, 256, lds, st>>>(mg, (const float*)Au, (float*)Z, xv, s, sp, C,
                                               nct);
  }
  return hipGetLastError();
}

}  // namespace fctn
