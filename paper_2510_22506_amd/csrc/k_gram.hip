// Fused sub-network generation + Gram + right-hand side (Property 1, eq. 5),
// the deterministic float64 split-K reduction, and the reconstruction
// FCTN(A) = A_k(k) M_k used by the X update (Algorithm 2).
//
// gram_rhs: each workgroup owns a range of column tiles of M_k (split-K) and
// a group of 16x16 output tiles (upper-triangle Gram tiles, then RHS tiles).
// Per column tile it stages the factor / pair operand slabs in LDS,
// generates the tile's block of M_k on MFMA (M_k is never stored in HBM),
// stages the matching rows of X_(k), and accumulates G += M M^T and
// B += X M^T on MFMA.  Partial tiles go to a split-major buffer that
// reduce_gb sums in float64, in split order (deterministic).
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

// Stage the operand slabs of column tile (cu0, cv0): Us(kap, p) = U[ru, cu, kap]
// with p = cu_l * Ru + ru, Vs(kap, q) = V[rv, cv, kap] with q = cv_l * Rv + rv;
// zero outside the tensor and in the padding.
template <typename T>
__device__ inline void stage_slabs(const MGen& mg, const TileGeom& tg, const T* __restrict__ U,
                                   const T* __restrict__ V, int64_t cu0, int64_t cv0,
                                   T* __restrict__ Us, T* __restrict__ Vs, int tid, int nth) {
  // U slab: iterate kap fastest when the slab is [p][kap] (kap contiguous in HBM)
  const bool u_kfast = tg.us_k == 1;
  const int nu = tg.Kp * tg.Pp;
  for (int e = tid; e < nu; e += nth) {
    int k, p;
    if (u_kfast) { p = e / tg.Kp; k = e - p * tg.Kp; }
    else { k = e / tg.Pp; p = e - k * tg.Pp; }
    T v = T(0);
    if (k < mg.K && p < tg.Pu) {
      const int cul = p / mg.Ru, ru = p - cul * mg.Ru;
      const int64_t cu = cu0 + cul;
      if (cu < mg.Cu) v = U[ru * mg.u_ru + cu * mg.u_cu + (int64_t)k * mg.u_k];
    }
    Us[k * tg.us_k + p * tg.us_p] = v;
  }
  const bool v_kfast = tg.vs_k == 1;
  const int nv = tg.Kp * tg.Qp;
  for (int e = tid; e < nv; e += nth) {
    int k, q;
    if (v_kfast) { q = e / tg.Kp; k = e - q * tg.Kp; }
    else { k = e / tg.Qp; q = e - k * tg.Qp; }
    T v = T(0);
    if (k < mg.K && q < tg.Qv) {
      const int cvl = q / mg.Rv, rv = q - cvl * mg.Rv;
      const int64_t cv = cv0 + cvl;
      if (cv < mg.Cv) v = V[rv * mg.v_rv + cv * mg.v_cv + (int64_t)k * mg.v_k];
    }
    Vs[k * tg.vs_k + q * tg.vs_q] = v;
  }
}

// M block of the tile on MFMA, scattered to Ms[c * ldm + row].
template <typename T>
__device__ inline void mgen_mfma(const MGen& mg, const TileGeom& tg, const T* __restrict__ Us,
                                 const T* __restrict__ Vs, T* __restrict__ Ms, int ldm, int lane,
                                 int wave, int nwaves) {
  typedef Mfma<T> MM;
  const int npt = tg.Pp / 16, nqt = tg.Qp / 16;
  const int kr = lane >> 4, lc = lane & 15;
  for (int t = wave; t < npt * nqt; t += nwaves) {
    const int pt = t / nqt, qt = t - (t / nqt) * nqt;
    typename MM::acc_t acc = MM::zero();
    const T* ua = Us + (pt * 16 + lc) * tg.us_p;
    const T* vb = Vs + (qt * 16 + lc) * tg.vs_q;
    for (int k0 = 0; k0 < tg.Kp; k0 += MM::kStep) {
      const T a = ua[(k0 + kr) * tg.us_k];
      const T b = vb[(k0 + kr) * tg.vs_k];
      acc = MM::mma(a, b, acc);
    }
    const int q = qt * 16 + lc;
    if (q < tg.Qv) {
      const int cvl = q / mg.Rv, rv = q - cvl * mg.Rv;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = pt * 16 + MM::row(lane, i);
        if (p < tg.Pu) {
          const int cul = p / mg.Ru, ru = p - cul * mg.Ru;
          Ms[(cul * tg.TCv + cvl) * ldm + ru * mg.Rv + rv] = acc[i];
        }
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kGramThreads) gram_rhs_k(MGen mg, const T* __restrict__ X,
                                                           XView xv, GramGeom g,
                                                           T* __restrict__ part) {
  typedef Mfma<T> MM;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileGeom& tg = g.tg;
  T* Us = (T*)smem_raw;
  T* Vs = Us + tg.u_len;
  T* Ms = Vs + tg.v_len;                        // [tcolp][ldm]  rows of M fastest
  T* Xs = Ms + (int64_t)tg.tcolp * g.ldm;       // [tcolp][ldx]  rows of X_(k) fastest
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

  // rows of M beyond s and columns beyond the tile (in M and X) stay zero for
  // the whole launch: uninitialized LDS could hold NaN patterns, and NaN * 0
  // would poison the products
  for (int e = tid; e < tg.tcolp * g.ldm; e += kGramThreads) Ms[e] = T(0);
  for (int e = tid; e < tg.tcolp * g.ldx; e += kGramThreads) Xs[e] = T(0);
  __syncthreads();

  const int64_t ct0 = (int64_t)split * g.colTilesPerSplit;
  const int64_t ct1 = min(ct0 + g.colTilesPerSplit, tg.nColTiles);
  const int ldm = g.ldm, ldx = g.ldx;

  for (int64_t ct = ct0; ct < ct1; ++ct) {
    const int64_t tu = ct / tg.nTileV, tv = ct - (ct / tg.nTileV) * tg.nTileV;
    const int64_t cu0 = tu * tg.TCu, cv0 = tv * tg.TCv;
    stage_slabs<T>(mg, tg, U, V, cu0, cv0, Us, Vs, tid, kGramThreads);
    if (xrows > 0) {
      const int ne = tg.tcol * xrows;
      for (int e = tid; e < ne; e += kGramThreads) {
        int cul, cvl, r;
        if (xv.x_ik == 1) {
          r = e % xrows;
          const int c = e / xrows;
          cul = c / tg.TCv;
          cvl = c - cul * tg.TCv;
        } else {
          cvl = e % tg.TCv;
          const int rest = e / tg.TCv;
          cul = rest % tg.TCu;
          r = rest / tg.TCu;
        }
        const int ik = ba_lo * 16 + r;
        const int64_t cu = cu0 + cul, cv = cv0 + cvl;
        T v = T(0);
        if (ik < xv.Ik && cu < mg.Cu && cv < mg.Cv)
          v = X[cu * xv.x_cu + cv * xv.x_cv + (int64_t)ik * xv.x_ik];
        Xs[(cul * tg.TCv + cvl) * ldx + r] = v;
      }
    }
    __syncthreads();
    mgen_mfma<T>(mg, tg, Us, Vs, Ms, ldm, lane, wave, 4);
    __syncthreads();
    const int kr = lane >> 4;
#pragma unroll
    for (int j = 0; j < kTPW; ++j) {
      if (valid[j]) {
        const T* Ab = fromX[j] ? Xs : Ms;
        const int lda = fromX[j] ? ldx : ldm;
        for (int kk = 0; kk < tg.tcolp; kk += MM::kStep) {
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
// Split-K reduction in float64.  One workgroup per (output tile, quarter of
// its 256 elements); wave w sums splits w, w+4, ... with eight independent
// accumulators, and the four wave sums are combined in a fixed order, so the
// result is deterministic.  Gram tiles are written to both triangles from the
// upper element (exact symmetry); RHS tiles get + rho A_k(k).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) reduce_gb_k(GramGeom g, const T* __restrict__ part,
                                                   const double* __restrict__ A64, int64_t spost,
                                                   double rho, double* __restrict__ G,
                                                   double* __restrict__ B) {
  __shared__ double red[4][64];
  const int t = blockIdx.x >> 2, quarter = blockIdx.x & 3;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int el = quarter * 64 + lane;
  const int64_t tstride = (int64_t)g.nTiles * 256;
  const T* p = part + (int64_t)t * 256 + el;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int sp = wave;
  for (; sp + 28 < g.nSplit; sp += 32) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += (double)p[(int64_t)(sp + 4 * u) * tstride];
  }
  for (int u = 0; sp < g.nSplit; sp += 4, ++u) acc[u & 7] += (double)p[(int64_t)sp * tstride];
  red[wave][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (wave != 0) return;
  const double v = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
  const int r = el >> 4, c = el & 15;
  const int s = g.s;
  if (t < g.nG) {
    int bi, bj;
    upper_tile(t, bi, bj);
    const int i = bi * 16 + r, j = bj * 16 + c;
    if (i < s && j < s && (bi != bj || r <= c)) {
      G[(int64_t)i * s + j] = v;
      G[(int64_t)j * s + i] = v;
    }
  } else {
    const int tb = t - g.nG;
    const int a = (tb / g.nbj) * 16 + r, j = (tb % g.nbj) * 16 + c;
    if (a < g.Ik && j < s)
      B[(int64_t)a * s + j] =
          v + rho * A64[(j / spost) * ((int64_t)g.Ik * spost) + (int64_t)a * spost + j % spost];
  }
}

hipError_t launch_reduce_gb(int prec, const GramGeom& g, const void* part, const double* A64,
                            int64_t spost, double rho, double* G, double* B, hipStream_t st) {
  const int nb = g.nTiles * 4;
  if (prec == P_F64)
    reduce_gb_k<double><<<nb, 256, 0, st>>>(g, (const double*)part, A64, spost, rho, G, B);
  else
    reduce_gb_k<float><<<nb, 256, 0, st>>>(g, (const float*)part, A64, spost, rho, G, B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Z_(k) = A_k(k) M_k: per column tile the block of M_k is generated on MFMA
// into LDS (the same generator as above), then Z's 16x16 tiles
// (i_k block x column block) accumulate on MFMA over the s_k rows.  A_k(k) is
// staged in LDS when it fits.  Z is written through the X view.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) reconstruct_k(MGen mg, const T* __restrict__ Au,
                                                     T* __restrict__ Z, XView xv, RecGeom g) {
  typedef Mfma<T> MM;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileGeom& tg = g.tg;
  T* Us = (T*)smem_raw;
  T* Vs = Us + tg.u_len;
  T* Ms = Vs + tg.v_len;                      // [tcolp][ldm]
  T* As = Ms + (int64_t)tg.tcolp * g.ldm;     // [ip][lda] when staged
  const T* U = (const T*)mg.U;
  const T* V = (const T*)mg.V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kr = lane >> 4, lc = lane & 15;

  for (int e = tid; e < tg.tcolp * g.ldm; e += 256) Ms[e] = T(0);
  if (g.lda > 0) {
    for (int e = tid; e < g.ip * g.sp; e += 256) {
      const int i = e / g.sp, r = e - (e / g.sp) * g.sp;
      As[i * g.lda + r] = (i < g.Ik && r < g.s) ? Au[(int64_t)i * g.s + r] : T(0);
    }
  }
  __syncthreads();

  const int nib = g.ip / 16, ncb = tg.tcolp / 16;
  for (int64_t ct = blockIdx.x; ct < tg.nColTiles; ct += gridDim.x) {
    const int64_t tu = ct / tg.nTileV, tv = ct - (ct / tg.nTileV) * tg.nTileV;
    const int64_t cu0 = tu * tg.TCu, cv0 = tv * tg.TCv;
    stage_slabs<T>(mg, tg, U, V, cu0, cv0, Us, Vs, tid, 256);
    __syncthreads();
    mgen_mfma<T>(mg, tg, Us, Vs, Ms, g.ldm, lane, wave, 4);
    __syncthreads();
    for (int t = wave; t < nib * ncb; t += 4) {
      const int ib = t / ncb, cb = t - (t / ncb) * ncb;
      typename MM::acc_t acc = MM::zero();
      const int ik_a = ib * 16 + lc;
      for (int k0 = 0; k0 < g.sp; k0 += MM::kStep) {
        const int row = k0 + kr;
        T a;
        if (g.lda > 0) a = As[ik_a * g.lda + row];
        else a = (ik_a < g.Ik && row < g.s) ? Au[(int64_t)ik_a * g.s + row] : T(0);
        const T b = Ms[(cb * 16 + lc) * g.ldm + row];
        acc = MM::mma(a, b, acc);
      }
      const int c = cb * 16 + lc;
      if (c < tg.tcol) {
        const int cul = c / tg.TCv, cvl = c - (c / tg.TCv) * tg.TCv;
        const int64_t cu = cu0 + cul, cv = cv0 + cvl;
        if (cu < mg.Cu && cv < mg.Cv) {
          const int64_t base = cu * xv.x_cu + cv * xv.x_cv;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int ik = ib * 16 + MM::row(lane, i);
            if (ik < xv.Ik) Z[base + (int64_t)ik * xv.x_ik] = acc[i];
          }
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_reconstruct(int prec, const MGen& mg, const void* Au, void* Z,
                              const XView& xv, const RecGeom& g, hipStream_t st) {
  if (prec == P_F64) {
    hipFuncSetAttribute((const void*)reconstruct_k<double>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    reconstruct_k<double><<<g.nblk, 256, g.lds_bytes, st>>>(mg, (const double*)Au, (double*)Z,
                                                            xv, g);
  } else {
    hipFuncSetAttribute((const void*)reconstruct_k<float>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    reconstruct_k<float><<<g.nblk, 256, g.lds_bytes, st>>>(mg, (const float*)Au, (float*)Z, xv,
                                                           g);
  }
  return hipGetLastError();
}

}  // namespace fctn
