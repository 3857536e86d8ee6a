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

// Phase hooks for timing probes (empty in the library).
#ifndef FCTN_GRAM_MARK
#define FCTN_GRAM_MARK_INIT
#define FCTN_GRAM_MARK(n)
#define FCTN_GRAM_MARK_FLUSH
#endif

constexpr int kGramThreads = 512;   // 8 waves
constexpr int kGramWaves = kGramThreads / 64;
constexpr int kTPW = 16;            // output tiles per wave

__device__ inline void upper_tile(int t, int& bi, int& bj) {
  int j = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (j * (j + 1) / 2 > t) --j;
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  bj = j;
  bi = t - j * (j + 1) / 2;
}

// Index tables of the tile's slabs and columns (once per launch).
//   rows p of the U slab: off = ru u_ru + cu_l u_cu, map = cu_l TCv ldm + ru Rv
//   rows q of the V slab: off = rv v_rv + cv_l v_cv, map = cv_l ldm + rv
//   columns c of the tile: off = cu_l x_cu + cv_l x_cv (X view), cl = cu_l, map = cv_l
// M element (row, c) of the tile sits at row * rs + c * cs in LDS.
__device__ inline void build_tables(const MGen& mg, const TileGeom& tg, const XView* xv, int rs,
                                    int cs, SlabRow* pt, SlabRow* qt, SlabRow* ct, int tid,
                                    int nth) {
  for (int p = tid; p < tg.Pp; p += nth) {
    SlabRow r{0, 1 << 30, -1, 0};
    if (p < tg.Pu) {
      const int cul = p / mg.Ru, ru = p - cul * mg.Ru;
      r.off = (int32_t)(ru * mg.u_ru + cul * mg.u_cu);
      r.cl = cul;
      r.map = cul * tg.TCv * cs + ru * mg.Rv * rs;
    }
    pt[p] = r;
  }
  for (int q = tid; q < tg.Qp; q += nth) {
    SlabRow r{0, 1 << 30, -1, 0};
    if (q < tg.Qv) {
      const int cvl = q / mg.Rv, rv = q - cvl * mg.Rv;
      r.off = (int32_t)(rv * mg.v_rv + cvl * mg.v_cv);
      r.cl = cvl;
      r.map = cvl * cs + rv * rs;
    }
    qt[q] = r;
  }
  if (xv) {
    for (int c = tid; c < tg.tcolp; c += nth) {
      SlabRow r{0, 1 << 30, 1 << 30, 0};
      if (c < tg.tcol) {
        const int cul = c / tg.TCv, cvl = c - cul * tg.TCv;
        r.off = (int32_t)(cul * xv->x_cu + cvl * xv->x_cv);
        r.cl = cul;
        r.map = cvl;
      }
      ct[c] = r;
    }
  }
}

// Batched 2-D gather into LDS.  The calling thread owns the points
// x = x0 + j sx < nx (the fast axis, along which neighbouring lanes read
// neighbouring addresses) and y = y0 + i sy < ny, visited i-fastest; it issues
// kGatherBatch loads before their LDS stores, so that the loads of a batch are
// in flight together instead of one round trip each.  src(x, y) returns the
// value (its own bounds decide whether it reads memory); dst(x, y, v) stores.
constexpr int kGatherBatch = 4;

template <typename T, class Src, class Dst>
__device__ inline void gather2d(int x0, int sx, int nx, int y0, int sy, int ny, Src src,
                                Dst dst) {
  if (x0 >= nx || y0 >= ny) return;
  const int nA = (nx - x0 + sx - 1) / sx, nB = (ny - y0 + sy - 1) / sy, n = nA * nB;
  int j = 0, i = 0;
  for (int n0 = 0; n0 < n; n0 += kGatherBatch) {
    T v[kGatherBatch];
    const int js = j, is = i;
#pragma unroll
    for (int b = 0; b < kGatherBatch; ++b) {
      v[b] = T(0);
      if (n0 + b < n) v[b] = src(x0 + j * sx, y0 + i * sy);
      if (++i == nB) {
        i = 0;
        ++j;
      }
    }
    // the same points again for the stores (fewer live registers than
    // keeping their coordinates)
    j = js;
    i = is;
#pragma unroll
    for (int b = 0; b < kGatherBatch; ++b) {
      if (n0 + b < n) dst(x0 + j * sx, y0 + i * sy, v[b]);
      if (++i == nB) {
        i = 0;
        ++j;
      }
    }
  }
}

typedef __attribute__((address_space(3))) void lds_void_t;
constexpr int kDmaMinRun = 32;   // shortest LDS row the small-tile kernel copies by DMA

// The same slab with global-to-LDS copies (float32): lane l of a copy writes
// the l-th of 64 consecutive LDS values, so a copy moves 64 values without
// holding registers and a wave issues its copies back to back.  [p][kap]:
// one row p per wave at a time, lanes along kap; [kap][p]: lanes along p (the
// lane's table entry read once per 64-row chunk), one kap row per copy.
// Padding (kap >= K) and rows beyond the tensor edge are zeroed with
// ordinary stores.
__device__ inline void stage_slab_dma(const float* __restrict__ F, int64_t base, int64_t f_k,
                                      int K, int Kp, int Pp, int s_k, int s_p,
                                      const SlabRow* __restrict__ tab, int64_t lim,
                                      float* __restrict__ S, int lane, int wave, int nw) {
  const float* Fb = F + base;
  if (s_k == 1) {                       // [p][kap]
    for (int p = wave; p < Pp; p += nw) {
      const SlabRow r = tab[p];
      float* row = S + p * s_p;
      if (r.cl < lim) {
        const float* src = Fb + r.off;
        for (int k0 = 0; k0 < K; k0 += 64)
          if (k0 + lane < K)
            __builtin_amdgcn_global_load_lds((const void*)(src + (int64_t)(k0 + lane) * f_k),
                                             (lds_void_t*)(row + k0), 4, 0, 0);
        for (int k = K + lane; k < Kp; k += 64) row[k] = 0.f;
      } else {
        for (int k = lane; k < Kp; k += 64) row[k] = 0.f;
      }
    }
  } else {                              // [kap][p]
    for (int p0 = 0; p0 < Pp; p0 += 64) {
      const int p = p0 + lane;
      const bool real = p < Pp;
      SlabRow r{0, 0, 0};
      if (real) r = tab[p];
      const bool ok = real && r.cl < lim;
      const float* src = Fb + r.off;
      for (int k = wave; k < Kp; k += nw) {
        float* row = S + k * s_k;
        if (ok && k < K)
          __builtin_amdgcn_global_load_lds((const void*)(src + (int64_t)k * f_k),
                                           (lds_void_t*)(row + p0), 4, 0, 0);
        else if (real)
          row[p] = 0.f;
      }
    }
  }
}

// Stage one operand slab S(kap, p) = F[tab[p].off + base + kap * f_k] (zero
// in the padding and beyond the tensor edge: tab[p].cl >= lim).  Lanes run
// along the slab's contiguous index (2^lw of them).  kBatched: loads issued in
// batches (gather2d); the general float32 Gram kernel, which has no registers
// to spare at two workgroups per CU, stages one element per thread at a time.
// kVec (that kernel's second instance, and the reconstruction): a [kap][p]
// slab whose rows come in aligned runs of four (vec) is staged four at a time
// with 16-byte loads and stores instead.
template <typename T, bool kBatched, bool kVec = false>
__device__ inline void stage_slab(const T* __restrict__ F, int64_t base, int64_t f_k, int K,
                                  int Kp, int Pp, int s_k, int s_p, int lw, bool vec,
                                  const SlabRow* __restrict__ tab, int64_t lim,
                                  T* __restrict__ S, int tid, int nth) {
  const int lanes = 1 << lw, lane = tid & (lanes - 1), grp = tid >> lw, ngrp = nth >> lw;
  const T* Fb = F + base;
  if constexpr (kVec && sizeof(T) == 4) {
    if (vec) {
      // [kap][p] slab in runs of four rows p: one 16-byte load and store
      // each (run structure and alignment checked on the host)
      typedef T v4 __attribute__((ext_vector_type(4)));
      const int n4 = Pp >> 2;
      const int lw4 = 31 - __builtin_clz(n4 < 64 ? n4 : 64);
      const int l4 = tid & ((1 << lw4) - 1), g4 = tid >> lw4, ng4 = nth >> lw4;
      for (int k = g4; k < Kp; k += ng4) {
        const bool okk = k < K;
        for (int p = 4 * l4; p < Pp; p += 4 << lw4) {
          const SlabRow r = tab[p];
          v4 v = {T(0), T(0), T(0), T(0)};
          if (okk && r.cl < lim) v = *(const v4*)(Fb + r.off + (int64_t)k * f_k);
          *(v4*)(S + k * s_k + p) = v;
        }
      }
      return;
    }
  }
  if constexpr (!kBatched) {
    if (s_k == 1) {                     // [p][kap]: lanes along kap
      for (int p = grp; p < Pp; p += ngrp) {
        const SlabRow r = tab[p];
        const bool okp = r.cl < lim;
        const T* src = Fb + r.off;
        for (int k = lane; k < Kp; k += lanes)
          S[p * s_p + k] = (okp && k < K) ? src[(int64_t)k * f_k] : T(0);
      }
    } else {                            // [kap][p]: lanes along p
      for (int k = grp; k < Kp; k += ngrp) {
        const bool okk = k < K;
        for (int p = lane; p < Pp; p += lanes) {
          const SlabRow r = tab[p];
          S[k * s_k + p] = (okk && r.cl < lim) ? Fb[r.off + (int64_t)k * f_k] : T(0);
        }
      }
    }
  } else if (s_k == 1) {                // [p][kap]: lanes along kap
    gather2d<T>(
        lane, lanes, Kp, grp, ngrp, Pp,
        [&](int k, int p) {
          const SlabRow r = tab[p];
          T v = T(0);
          if (r.cl < lim && k < K) v = Fb[r.off + (int64_t)k * f_k];
          return v;
        },
        [&](int k, int p, T v) { S[p * s_p + k] = v; });
  } else {                              // [kap][p]: lanes along p
    gather2d<T>(
        lane, lanes, Pp, grp, ngrp, Kp,
        [&](int p, int k) {
          const SlabRow r = tab[p];
          T v = T(0);
          if (r.cl < lim && k < K) v = Fb[r.off + (int64_t)k * f_k];
          return v;
        },
        [&](int p, int k, T v) { S[k * s_k + p] = v; });
  }
}

// The tile's block of M on MFMA: O[p][q] = sum_kap Us(kap, p) Vs(kap, q),
// scattered to Ms[pt[p].map + qt[q].map].
template <typename T, typename Store>
__device__ inline void mgen_mfma_store(const TileGeom& tg, const T* __restrict__ Us,
                                       const T* __restrict__ Vs, const SlabRow* __restrict__ ptab,
                                       const SlabRow* __restrict__ qtab, Store store, int lane,
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
    const int qm = qtab[qt * 16 + lc].map;
    if (qm >= 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pm = ptab[pt * 16 + MM::row(lane, i)].map;
        if (pm >= 0) store(pm + qm, acc[i]);
      }
    }
  }
}

template <typename T>
__device__ inline void mgen_mfma(const TileGeom& tg, const T* __restrict__ Us,
                                 const T* __restrict__ Vs, const SlabRow* __restrict__ ptab,
                                 const SlabRow* __restrict__ qtab, T* __restrict__ Ms, int lane,
                                 int wave, int nwaves) {
  mgen_mfma_store<T>(tg, Us, Vs, ptab, qtab, [Ms](int idx, T v) { Ms[idx] = v; }, lane, wave,
                     nwaves);
}

template <typename T, bool kBatched, bool kVec = false, bool kDmaStage = false>
__device__ inline void stage_operands(const MGen& mg, const TileGeom& tg, const T* U, const T* V,
                                      int64_t tu, int64_t tv, int64_t& cur_tu, int64_t& cur_tv,
                                      T* Us, T* Vs, const SlabRow* ptab, const SlabRow* qtab,
                                      int tid, int nth) {
  // the float32 Gram kernels stage by global-to-LDS copies: the general
  // one always (its register path holds one load per thread), the
  // small-tile one where the slab's LDS rows are long enough to keep most of
  // a copy's 64 lanes busy (its batched register path is better otherwise)
  constexpr bool kDma = sizeof(T) == 4 && kDmaStage;
  if (tu != cur_tu) {
    const int64_t cu0 = tu * tg.TCu;
    if (kDma && (!kBatched || (tg.us_k == 1 ? mg.K : tg.Pp) >= kDmaMinRun))
      stage_slab_dma((const float*)U, cu0 * mg.u_cu, mg.u_k, mg.K, tg.Kp, tg.Pp, tg.us_k, tg.us_p,
                     ptab, mg.Cu - cu0, (float*)Us, tid & 63, tid >> 6, nth >> 6);
    else
      stage_slab<T, kBatched, kVec>(U, cu0 * mg.u_cu, mg.u_k, mg.K, tg.Kp, tg.Pp, tg.us_k,
                                    tg.us_p, tg.u_lw, tg.u_vec != 0, ptab, mg.Cu - cu0, Us, tid,
                                    nth);
    cur_tu = tu;
  }
  if (tv != cur_tv) {
    const int64_t cv0 = tv * tg.TCv;
    if (kDma && (!kBatched || (tg.vs_k == 1 ? mg.K : tg.Qp) >= kDmaMinRun))
      stage_slab_dma((const float*)V, cv0 * mg.v_cv, mg.v_k, mg.K, tg.Kp, tg.Qp, tg.vs_k, tg.vs_q,
                     qtab, mg.Cv - cv0, (float*)Vs, tid & 63, tid >> 6, nth >> 6);
    else
      stage_slab<T, kBatched, kVec>(V, cv0 * mg.v_cv, mg.v_k, mg.K, tg.Kp, tg.Qp, tg.vs_k,
                                    tg.vs_q, tg.v_lw, tg.v_vec != 0, qtab, mg.Cv - cv0, Vs, tid,
                                    nth);
    cur_tv = tv;
  }
}

// float32: at most 128 VGPRs, so that two workgroups share a CU and one
// stages its next tile while the other runs MFMA (float64 keeps one per CU).
// TPW output tiles per wave: 16 in general; 2 for the modes with at most 16
// output tiles (small s_k), whose freed accumulator registers let the operand
// and X staging keep kGatherBatch loads in flight per thread.  The general
// float32 instance stages the operand slabs and the X block by global-to-LDS
// copies instead: every wave issues its copies back to back with no
// registers held (at 128 VGPRs it can keep only one ordinary load in flight
// per thread), and the barrier after staging waits for all of them.
template <typename T, int TPW, int NW = kGramWaves>
__global__ void __launch_bounds__(64 * NW, sizeof(T) == 4 ? 4 : 1) gram_rhs_k(MGen mg, const T* __restrict__ X,
                                                           XView xv, GramGeom g,
                                                           T* __restrict__ part) {
  constexpr bool kBatch = TPW <= 4;
  typedef Mfma<T> MM;
  constexpr int VW = 16 / (int)sizeof(T);   // columns per 16-byte LDS read
  typedef T vT __attribute__((ext_vector_type(VW)));
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileGeom& tg = g.tg;
  SlabRow* ptab = (SlabRow*)smem_raw;
  SlabRow* qtab = ptab + tg.Pp;
  SlabRow* ctab = qtab + tg.Qp;
  T* Us = (T*)(ctab + tg.tcolp);
  T* Vs = Us + tg.u_len;
  // [row][column] tiles, columns contiguous, row strides ldm = ldx = tcolp +
  // 16 bytes: one 16-byte read per lane covers VW columns, i.e. VW MFMAs
  const int mso = ((int)((unsigned char*)(Vs + tg.v_len) - smem_raw) + 15) & ~15;
  T* Ms = (T*)(smem_raw + mso);                                         // [mrows][ldm]
  T* Xs = Ms + (int64_t)g.mrows * g.ldm;                                // [xalloc][ldx]
  const T* Zr = Xs + (int64_t)g.xalloc * g.ldx;                         // zero row (zrow)
  const T* U = (const T*)mg.U;
  const T* V = (const T*)mg.V;

  // the wave index as a wave-uniform (scalar) value, so that tile-selection
  // branches are scalar branches rather than per-lane masks
  const int tid = threadIdx.x, lane = tid & 63,
            wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // neighbouring splits (adjacent column tiles, sharing X's cache lines) on
  // one XCD: the split count is a multiple of the XCD count (some splits may
  // be empty), so workgroup (x, y) runs on XCD x mod 8 and each XCD takes a
  // contiguous range of splits of every group; groups still dispatch in
  // order, the lighter last group filling the CUs that take two workgroups
  const int split = xcd_order(blockIdx.x, gridDim.x), group = blockIdx.y;
  const int t0 = group * g.tilesPerGroup;
  const int t1 = min(t0 + g.tilesPerGroup, g.nTiles);

  int ba_lo = 0, xrows = 0;
  if (t1 > g.nG) {
    const int bfirst = (max(t0, g.nG) - g.nG) / g.nbj;
    const int blast = (t1 - 1 - g.nG) / g.nbj;
    ba_lo = bfirst;
    xrows = (blast - bfirst + 1) * 16;
  }

  // this wave's output tiles (wave-uniform): bit 0 = A operand from X_(k),
  // bits 1-10 = row block bi, bits 11-20 = column block bj; -1 for no tile
  // (the validity lives in the descriptor's sign: a per-tile flag would take
  // a 64-bit lane mask of scalar registers each, which spill)
  int tdesc[TPW];
  typename MM::acc_t acc[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int t = t0 + wave + NW * j;
    acc[j] = MM::zero();
    int bi = 0, bj = 0;
    bool fx = false;
    if (t < t1) {
      if (t < g.nG) {
        upper_tile(t, bi, bj);
      } else {
        const int tb = t - g.nG;
        bi = tb / g.nbj - ba_lo;
        bj = tb % g.nbj;
        fx = true;
      }
    }
    tdesc[j] = t < t1 ? (fx ? 1 : 0) | (bi << 1) | (bj << 11) : -1;
  }

  build_tables(mg, tg, &xv, g.ldm, 1, ptab, qtab, ctab, tid, (64 * NW));
  // rows of M beyond s and columns beyond the tile (in M and X) stay zero for
  // the whole launch: uninitialized LDS could hold NaN patterns, and NaN * 0
  // would poison the products
  for (int e = tid; e < (g.mrows + g.xalloc + g.zrow) * g.ldm; e += (64 * NW)) Ms[e] = T(0);
  __syncthreads();

  const int64_t ct0 = (int64_t)split * g.colTilesPerSplit;
  const int64_t ct1 = min(ct0 + g.colTilesPerSplit, tg.nColTiles);
  const int ldm = g.ldm, ldx = g.ldx;
  int64_t cur_tu = -1, cur_tv = -1;
  // X staging: lanes along the contiguous index of the X view
  const bool x_rfast = xv.x_ik == 1;
  const int xl = x_rfast ? min(xrows, 16) : 16;   // xrows is a multiple of 16

  // column tile ct = tu nTileV + tv, advanced without a division per tile
  // (32-bit: there are fewer column tiles than tensor elements)
  const int ntv = (int)tg.nTileV;
  int tu32 = (int)(ct0 / ntv), tv32 = (int)ct0 - tu32 * ntv;
  FCTN_GRAM_MARK_INIT
  for (int ct = (int)ct0; ct < (int)ct1; ++ct) {
    const int64_t tu = tu32, tv = tv32;
    if (++tv32 == ntv) {
      tv32 = 0;
      ++tu32;
    }
    stage_operands<T, kBatch, false, true>(mg, tg, U, V, tu, tv, cur_tu, cur_tv, Us, Vs, ptab,
                                           qtab, tid, (64 * NW));
    FCTN_GRAM_MARK(0);
    if (xrows > 0) {
      const int64_t cu0 = tu * tg.TCu, cv0 = tv * tg.TCv;
      const int64_t lim_u = mg.Cu - cu0, lim_v = mg.Cv - cv0;
      const T* xb = X + cu0 * xv.x_cu + cv0 * xv.x_cv + (int64_t)(ba_lo * 16) * xv.x_ik;
      const int xlim = xv.Ik - ba_lo * 16;
      if constexpr (sizeof(T) == 4) {
        // global-to-LDS copies: wave w takes rows w, w + NW, ..; lane l of a
        // copy writes column c0 + l of its row, so one instruction moves 64
        // values with no registers held.  Columns past the tensor edge are
        // skipped: their M columns are zero, so the (finite) values the
        // buffer holds there add nothing; rows past I_k only feed outputs
        // that are discarded.
        // Each lane's column (its table entry) is read once per 64-column
        // chunk, outside the row loop, so the copies issue back to back.
        const int rend = min(xrows, xlim);
        for (int c0 = 0; c0 < tg.tcol; c0 += 64) {
          const int c = c0 + lane;
          bool okc = false;
          int64_t off = 0;
          if (c < tg.tcol) {
            const SlabRow cr = ctab[c];
            okc = cr.cl < lim_u && cr.map < lim_v;
            off = cr.off;
          }
          if (okc) {
            const T* xc = xb + off;
            for (int r = wave; r < rend; r += NW)
              __builtin_amdgcn_global_load_lds((const void*)(xc + (int64_t)r * xv.x_ik),
                                               (lds_void_t*)(Xs + r * ldx + c0), 4, 0, 0);
          }
        }
      } else if constexpr (kBatch) {
        // thread (c, r0): column c, rows r0, r0 + ngrp, ...
        const int ngrp = (64 * NW) / tg.tcol;
        if (tid < ngrp * tg.tcol) {
          gather2d<T>(
              tid % tg.tcol, tg.tcol, tg.tcol, tid / tg.tcol, ngrp, xrows,
              [&](int c, int r) {
                const SlabRow cr = ctab[c];
                T v = T(0);
                if (cr.cl < lim_u && cr.map < lim_v && r < xlim)
                  v = xb[cr.off + (int64_t)r * xv.x_ik];
                return v;
              },
              [&](int c, int r, T v) { Xs[r * ldx + c] = v; });
        }
      } else if (x_rfast) {
        const int l = tid % xl, grp = tid / xl, ngrp = (64 * NW) / xl;
        for (int c = grp; c < tg.tcol; c += ngrp) {
          const SlabRow cr = ctab[c];
          const bool okc = cr.cl < lim_u && cr.map < lim_v;
          for (int r = l; r < xrows; r += xl)
            Xs[r * ldx + c] = (okc && r < xlim) ? xb[cr.off + (int64_t)r * xv.x_ik] : T(0);
        }
      } else {
        // element e = tid + i * (64 * NW) of the row-major (r, c) walk,
        // advanced without a division per element
        const int dr = (64 * NW) / tg.tcol, dc = (64 * NW) - dr * tg.tcol;
        int r = tid / tg.tcol, c = tid - r * tg.tcol;
        while (r < xrows) {
          const SlabRow cr = ctab[c];
          Xs[r * ldx + c] = (cr.cl < lim_u && cr.map < lim_v && r < xlim)
                                ? xb[cr.off + (int64_t)r * xv.x_ik] : T(0);
          c += dc;
          r += dr;
          if (c >= tg.tcol) {
            c -= tg.tcol;
            ++r;
          }
        }
      }
    }
    FCTN_GRAM_MARK(1);
    __syncthreads();
    FCTN_GRAM_MARK(2);
    mgen_mfma<T>(tg, Us, Vs, ptab, qtab, Ms, lane, wave, NW);
    FCTN_GRAM_MARK(3);
    __syncthreads();
    FCTN_GRAM_MARK(4);
    // lane group kr reads columns kk + VW kr .. + VW - 1 of its row in one
    // 16-byte load and feeds them to VW MFMAs; MFMA m therefore sums the
    // columns {kk + VW kr + m}, and the VW MFMAs cover kk .. kk + 4 VW - 1
    // once, in the same order for both operands
    const int kof = (lane >> 4) * VW;
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      if (tdesc[j] >= 0) {
        const int d = tdesc[j];
        // rows past those given LDS (M rows >= s, X rows >= I_k, where the
        // geometry trims them) read the zero row
        const int ra = ((d >> 1) & 1023) * 16 + (lane & 15), rb = (d >> 11) * 16 + (lane & 15);
        const T* Ab = ((d & 1) ? (ra < g.xalloc ? Xs + ra * ldx : Zr)
                               : (ra < g.mrows ? Ms + ra * ldm : Zr)) + kof;
        const T* Bb = (rb < g.mrows ? Ms + rb * ldm : Zr) + kof;
#pragma unroll 1
        for (int kk = 0; kk < tg.tcolp; kk += 4 * VW) {
          const vT a = *(const vT*)(Ab + kk);
          const vT b = *(const vT*)(Bb + kk);
#pragma unroll
          for (int m = 0; m < VW; ++m) acc[j] = MM::mma(a[m], b[m], acc[j]);
        }
      }
    }
    FCTN_GRAM_MARK(5);
    __syncthreads();
    FCTN_GRAM_MARK(6);
  }
  FCTN_GRAM_MARK_FLUSH

#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    if (tdesc[j] >= 0) {
      const int t = t0 + wave + NW * j;
      T* base = part + ((int64_t)split * g.nTiles + t) * 256;
#pragma unroll
      for (int i = 0; i < 4; ++i) base[MM::row(lane, i) * 16 + (lane & 15)] = acc[j][i];
    }
  }
}

int gram_threads() { return kGramThreads; }
int gram_tiles_per_group() { return kGramWaves * kTPW; }

// ---------------------------------------------------------------------------
// Split-bf16 sub-network generation (bf16 forms, contraction length K >= 24).
// The operand slabs are staged as bf16 heads and tails, row p holding kap
// contiguously (row stride ldk, a multiple of 8 plus 8), whatever the slab's
// order in HBM; each product is hi*hi + hi*lo + lo*hi on 16x16x32 bf16 MFMA
// with fp32 accumulation (the dropped lo*lo term is about 2^-16 of the
// product).
// ---------------------------------------------------------------------------
__device__ inline void stage_slab_bf16(const float* __restrict__ F, int64_t base, int64_t f_k,
                                       int K, int Kp, int Pp, bool k_fast, int lw,
                                       const SlabRow* __restrict__ tab, int64_t lim,
                                       uint16_t* __restrict__ Sh, uint16_t* __restrict__ Sl,
                                       int ldk, int tid, int nth) {
  const int lanes = 1 << lw, lane = tid & (lanes - 1), grp = tid >> lw, ngrp = nth >> lw;
  const float* Fb = F + base;
  auto put = [&](int p, int k, float v) {
    const uint16_t h = bf16_bits_rne(v);
    Sh[p * ldk + k] = h;
    Sl[p * ldk + k] = bf16_bits_rne(v - bf16_bits_to_float(h));
  };
  auto src = [&](int k, int p) {
    const SlabRow r = tab[p];
    float v = 0.f;
    if (r.cl < lim && k < K) v = Fb[r.off + (int64_t)k * f_k];
    return v;
  };
  if (k_fast)   // lanes along kap (contiguous in HBM)
    gather2d<float>(lane, lanes, Kp, grp, ngrp, Pp, src, [&](int k, int p, float v) { put(p, k, v); });
  else          // lanes along p
    gather2d<float>(
        lane, lanes, Pp, grp, ngrp, Kp, [&](int p, int k) { return src(k, p); },
        [&](int p, int k, float v) { put(p, k, v); });
}

template <typename Store>
__device__ inline void mgen_bf16x3_store(const TileGeom& tg, const uint16_t* __restrict__ Uh,
                                         const uint16_t* __restrict__ Ul,
                                         const uint16_t* __restrict__ Vh,
                                         const uint16_t* __restrict__ Vl, int ldk, int kend,
                                         const SlabRow* __restrict__ ptab,
                                         const SlabRow* __restrict__ qtab, Store store, int lane,
                                         int wave, int nwaves) {
  const int npt = tg.Pp / 16, nqt = tg.Qp / 16;
  const int lo = (lane & 15) * ldk + 8 * (lane >> 4);
  for (int t = wave; t < npt * nqt; t += nwaves) {
    const int pt = t / nqt, qt = t - (t / nqt) * nqt;
    MfmaBf16::acc_t acc = Mfma<float>::zero();
    const int ao = pt * 16 * ldk + lo, bo = qt * 16 * ldk + lo;
    for (int k0 = 0; k0 < kend; k0 += 32) {
      const bf16x8 a = *(const bf16x8*)(Uh + ao + k0);
      const bf16x8 b = *(const bf16x8*)(Vh + bo + k0);
      const bf16x8 al = *(const bf16x8*)(Ul + ao + k0);
      const bf16x8 bl = *(const bf16x8*)(Vl + bo + k0);
      acc = MfmaBf16::mma(a, b, acc);
      acc = MfmaBf16::mma(a, bl, acc);
      acc = MfmaBf16::mma(al, b, acc);
    }
    const int qm = qtab[qt * 16 + (lane & 15)].map;
    if (qm >= 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pm = ptab[pt * 16 + MfmaBf16::row(lane, i)].map;
        if (pm >= 0) store(pm + qm, acc[i]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// bf16 form of the same pass.  The tile of M_k is generated on fp32 MFMA as
// above and rounded once (nearest even) into bf16 LDS tiles laid out
// [row][column] (columns contiguous), as are the X_(k) rows; the Gram and
// right-hand-side products then run on bf16 MFMA (16x16x32, fp32
// accumulation), each lane reading its 8 consecutive k values with one
// 16-byte load.  With X3 each value is also kept as a bf16 residual
// (x = hi + lo) and every product is hi*hi + hi*lo + lo*hi.
// ---------------------------------------------------------------------------
// bf16: NW waves of TPW tiles.  Eight waves: at most 128 VGPRs (two
// workgroups per CU) except the split form's 16-tile instance, which keeps the
// default budget; sixteen waves (one workgroup per CU): 128 VGPRs.  MG16: the
// sub-network tile is generated in split bf16 (above) instead of float32.
template <int X3, int TPW, int NW = kGramWaves, bool MG16 = false>
__global__ void __launch_bounds__(64 * NW, (X3 && NW == kGramWaves && TPW > 8) ? 1 : 4) gram_rhs_bf16_k(MGen mg, const float* __restrict__ X,
                                                                XView xv, GramGeom g,
                                                                float* __restrict__ part) {
  typedef Mfma<float> MF;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileGeom& tg = g.tg;
  SlabRow* ptab = (SlabRow*)smem_raw;
  SlabRow* qtab = ptab + tg.Pp;
  SlabRow* ctab = qtab + tg.Qp;
  // operand slabs: float32 (u_len, v_len), or with MG16 bf16 heads and
  // tails [p][kap] with row stride g.ldk
  float* Us = (float*)(ctab + tg.tcolp);
  float* Vs = Us + tg.u_len;
  uint16_t* const Ush = (uint16_t*)(ctab + tg.tcolp);
  uint16_t* const Usl = Ush + (size_t)tg.Pp * g.ldk;
  uint16_t* const Vsh = Usl + (size_t)tg.Pp * g.ldk;
  uint16_t* const Vsl = Vsh + (size_t)tg.Qp * g.ldk;
  const int ldb = g.ldm;                         // bf16 row stride (multiple of 8)
  uint16_t* Mh = MG16 ? Vsl + (size_t)tg.Qp * g.ldk
                      : (uint16_t*)(Vs + tg.v_len);   // [sp][ldb]
  uint16_t* Ml = Mh + (X3 ? (size_t)g.sp * ldb : 0);
  uint16_t* Xh = Ml + (size_t)g.sp * ldb;         // [xalloc][ldb]
  uint16_t* Xl = Xh + (X3 ? (size_t)g.xalloc * ldb : 0);
  const uint16_t* Zr = Xl + (size_t)g.xalloc * ldb;   // zero row (zrow)
  const float* U = (const float*)mg.U;
  const float* V = (const float*)mg.V;

  // the wave index as a wave-uniform (scalar) value, so that tile-selection
  // branches are scalar branches rather than per-lane masks
  const int tid = threadIdx.x, lane = tid & 63,
            wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // neighbouring splits (adjacent column tiles, sharing X's cache lines) on
  // one XCD: the split count is a multiple of the XCD count (some splits may
  // be empty), so workgroup (x, y) runs on XCD x mod 8 and each XCD takes a
  // contiguous range of splits of every group; groups still dispatch in
  // order, the lighter last group filling the CUs that take two workgroups
  const int split = xcd_order(blockIdx.x, gridDim.x), group = blockIdx.y;
  const int t0 = group * g.tilesPerGroup;
  const int t1 = min(t0 + g.tilesPerGroup, g.nTiles);
  int ba_lo = 0, xrows = 0;
  if (t1 > g.nG) {
    const int bfirst = (max(t0, g.nG) - g.nG) / g.nbj;
    const int blast = (t1 - 1 - g.nG) / g.nbj;
    ba_lo = bfirst;
    xrows = (blast - bfirst + 1) * 16;
  }
  // this wave's output tiles (wave-uniform): bit 0 = A operand from X_(k),
  // bits 1-10 = row block bi, bits 11-20 = column block bj; -1 for no tile
  // (see gram_rhs_k); the lane's own offset inside a 16-row block is loff
  int tdesc[TPW];
  MF::acc_t acc[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int t = t0 + wave + NW * j;
    acc[j] = MF::zero();
    int bi = 0, bj = 0;
    bool fromX = false;
    if (t < t1) {
      if (t < g.nG) {
        upper_tile(t, bi, bj);
      } else {
        const int tb = t - g.nG;
        bi = tb / g.nbj - ba_lo;
        bj = tb % g.nbj;
        fromX = true;
      }
    }
    tdesc[j] = t < t1 ? (fromX ? 1 : 0) | (bi << 1) | (bj << 11) : -1;
  }
  const int loff = (lane & 15) * ldb + 8 * (lane >> 4);

  build_tables(mg, tg, &xv, ldb, 1, ptab, qtab, ctab, tid, (64 * NW));
  {
    // M tile(s) then X tile(s), hi and (X3) lo copies: every padding column
    // must read as zero; with MG16 also the bf16 slabs (the kap padding up to
    // a multiple of 32 is never staged)
    const int nzero = ((g.sp + g.xalloc) * (1 + X3) + g.zrow) * ldb;
    for (int e = tid; e < nzero; e += (64 * NW)) Mh[e] = 0;
    if (MG16) {
      const int ns = 2 * (tg.Pp + tg.Qp) * g.ldk;
      for (int e = tid; e < ns; e += (64 * NW)) Ush[e] = 0;
    }
  }
  __syncthreads();

  const int64_t ct0 = (int64_t)split * g.colTilesPerSplit;
  const int64_t ct1 = min(ct0 + g.colTilesPerSplit, tg.nColTiles);
  int64_t cur_tu = -1, cur_tv = -1;
  const bool x_rfast = xv.x_ik == 1;
  auto put = [&](uint16_t* hi, uint16_t* lo, int idx, float v) {
    const uint16_t h = bf16_bits_rne(v);
    hi[idx] = h;
    if (X3) lo[idx] = bf16_bits_rne(v - bf16_bits_to_float(h));
  };

  const int ntv = (int)tg.nTileV;
  int tu32 = (int)(ct0 / ntv), tv32 = (int)ct0 - tu32 * ntv;
  for (int ct = (int)ct0; ct < (int)ct1; ++ct) {
    const int64_t tu = tu32, tv = tv32;
    if (++tv32 == ntv) {
      tv32 = 0;
      ++tu32;
    }
    if constexpr (MG16) {
      if (tu != cur_tu) {
        const int64_t cu0 = tu * tg.TCu;
        stage_slab_bf16(U, cu0 * mg.u_cu, mg.u_k, mg.K, tg.Kp, tg.Pp, tg.us_k == 1, tg.u_lw,
                        ptab, mg.Cu - cu0, Ush, Usl, g.ldk, tid, 64 * NW);
        cur_tu = tu;
      }
      if (tv != cur_tv) {
        const int64_t cv0 = tv * tg.TCv;
        stage_slab_bf16(V, cv0 * mg.v_cv, mg.v_k, mg.K, tg.Kp, tg.Qp, tg.vs_k == 1, tg.v_lw,
                        qtab, mg.Cv - cv0, Vsh, Vsl, g.ldk, tid, 64 * NW);
        cur_tv = tv;
      }
    } else {
      stage_operands<float, true>(mg, tg, U, V, tu, tv, cur_tu, cur_tv, Us, Vs, ptab, qtab, tid,
                                  (64 * NW));
    }
    if (xrows > 0) {
      const int64_t cu0 = tu * tg.TCu, cv0 = tv * tg.TCv;
      const int64_t lim_u = mg.Cu - cu0, lim_v = mg.Cv - cv0;
      const float* xb = X + cu0 * xv.x_cu + cv0 * xv.x_cv + (int64_t)(ba_lo * 16) * xv.x_ik;
      const int xlim = xv.Ik - ba_lo * 16;
      auto xsrc = [&](int r, int c) {
        const SlabRow cr = ctab[c];
        float v = 0.f;
        if (cr.cl < lim_u && cr.map < lim_v && r < xlim) v = xb[cr.off + (int64_t)r * xv.x_ik];
        return v;
      };
      // rows below I_k only: the rows past it stay zero from the launch's
      // clearing (or, trimmed, read the zero row)
      const int xr = min(xrows, xlim);
      if (x_rfast) {
        const int xl = min(xrows, 16);
        const int l = tid % xl, grp = tid / xl, ngrp = (64 * NW) / xl;
        gather2d<float>(
            l, xl, xr, grp, ngrp, tg.tcol, xsrc,
            [&](int r, int c, float v) { put(Xh, Xl, r * ldb + c, v); });
      } else {
        gather2d<float>(
            lane, 64, tg.tcol, wave, NW, xr,
            [&](int c, int r) { return xsrc(r, c); },
            [&](int c, int r, float v) { put(Xh, Xl, r * ldb + c, v); });
      }
    }
    __syncthreads();
    if constexpr (MG16)
      mgen_bf16x3_store(tg, Ush, Usl, Vsh, Vsl, g.ldk, tg.Kp,
                        ptab, qtab, [&](int idx, float v) { put(Mh, Ml, idx, v); }, lane, wave,
                        NW);
    else
      mgen_mfma_store<float>(tg, Us, Vs, ptab, qtab,
                             [&](int idx, float v) { put(Mh, Ml, idx, v); }, lane, wave, NW);
    __syncthreads();
    for (int kk = 0; kk < tg.tcolp; kk += 32) {
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        if (tdesc[j] >= 0) {
          const int d = tdesc[j];
          const int ao = ((d >> 1) & 1023) * 16 * ldb + loff + kk;
          const int bo = (d >> 11) * 16 * ldb + loff + kk;
          // X rows past those given LDS read the zero row
          const bool xz = (d & 1) && ((d >> 1) & 1023) * 16 + (lane & 15) >= g.xalloc;
          const int zo = 8 * (lane >> 4) + kk;
          const uint16_t* Ah = (d & 1) ? Xh : Mh;
          const bf16x8 a = *(const bf16x8*)(xz ? Zr + zo : Ah + ao);
          const bf16x8 b = *(const bf16x8*)(Mh + bo);
          acc[j] = MfmaBf16::mma(a, b, acc[j]);
          if (X3) {
            const uint16_t* Al = (d & 1) ? Xl : Ml;
            const bf16x8 al = *(const bf16x8*)(xz ? Zr + zo : Al + ao);
            const bf16x8 bl = *(const bf16x8*)(Ml + bo);
            acc[j] = MfmaBf16::mma(a, bl, acc[j]);
            acc[j] = MfmaBf16::mma(al, b, acc[j]);
          }
        }
        // at most two tiles' fragments in flight (register budget)
        if (j & 1) __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    if (tdesc[j] >= 0) {
      const int t = t0 + wave + NW * j;
      float* base = part + ((int64_t)split * g.nTiles + t) * 256;
#pragma unroll
      for (int i = 0; i < 4; ++i) base[MfmaBf16::row(lane, i) * 16 + (lane & 15)] = acc[j][i];
    }
  }
}

int gram_max_lds_bytes() { return 160 * 1024; }

hipError_t launch_gram_rhs(int prec, const MGen& mg, const void* X, const XView& xv,
                           const GramGeom& g_in, void* part, hipStream_t st) {
  GramGeom g = g_in;
  if ((uintptr_t)mg.U % 16 != 0) g.tg.u_vec = 0;
  if ((uintptr_t)mg.V % 16 != 0) g.tg.v_vec = 0;
  dim3 grid(g.nSplit, g.nGroups);
  // the small-tile variant covers a group's tiles only when all of them fit
  const bool small = g.nGroups == 1 && g.nTiles <= kGramWaves * 2;
  if (prec == P_F64) {
    hipFuncSetAttribute((const void*)gram_rhs_k<double, kTPW>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    gram_rhs_k<double, kTPW><<<grid, kGramThreads, g.lds_bytes, st>>>(mg, (const double*)X, xv,
                                                                      g, (double*)part);
  } else {
    // float32 data: one kernel instance per (precision form, tile variant,
    // workgroup size)
    auto run = [&](auto kern, int threads) {
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)g.lds_bytes);
      hipLaunchKernelGGL(kern, grid, dim3(threads), g.lds_bytes, st, mg, (const float*)X, xv, g,
                         (float*)part);
    };
    const bool wide = g.nw == 2 * kGramWaves;   // 16 waves, 8 tiles each
    constexpr int W2 = 2 * kGramWaves, T2 = kTPW / 2;
    if (prec == P_BF16 || prec == P_BF16X3) {
      const bool x3 = prec == P_BF16X3, mg16 = g.mg16 != 0;
      // instances: form x {small tiles, 16 waves, 8 waves} x generator
      if (small) {
        if (x3) mg16 ? run(gram_rhs_bf16_k<1, 2, kGramWaves, true>, kGramThreads)
                     : run(gram_rhs_bf16_k<1, 2>, kGramThreads);
        else mg16 ? run(gram_rhs_bf16_k<0, 2, kGramWaves, true>, kGramThreads)
                  : run(gram_rhs_bf16_k<0, 2>, kGramThreads);
      } else if (wide) {
        if (x3) mg16 ? run(gram_rhs_bf16_k<1, T2, W2, true>, 2 * kGramThreads)
                     : run(gram_rhs_bf16_k<1, T2, W2>, 2 * kGramThreads);
        else mg16 ? run(gram_rhs_bf16_k<0, T2, W2, true>, 2 * kGramThreads)
                  : run(gram_rhs_bf16_k<0, T2, W2>, 2 * kGramThreads);
      } else {
        if (x3) run(gram_rhs_bf16_k<1, kTPW>, kGramThreads);
        else run(gram_rhs_bf16_k<0, kTPW>, kGramThreads);
      }
    } else if (small) {
      run(gram_rhs_k<float, 2>, kGramThreads);
    } else {
      // the general instance stages its operands and X by global-to-LDS
      // copies, whatever the slab layout
      // (16 waves: 8 tiles each, or 10, 12 or 14 for groups of up to 160,
      // 192 or 224)
      if (wide && g.tilesPerGroup == W2 * 10) run(gram_rhs_k<float, 10, W2>, 2 * kGramThreads);
      else if (wide && g.tilesPerGroup == W2 * 12)
        run(gram_rhs_k<float, 12, W2>, 2 * kGramThreads);
      else if (wide && g.tilesPerGroup == W2 * 14)
        run(gram_rhs_k<float, 14, W2>, 2 * kGramThreads);
      else if (wide) run(gram_rhs_k<float, T2, W2>, 2 * kGramThreads);
      else run(gram_rhs_k<float, kTPW>, kGramThreads);
    }
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
// (i_k block x column block) accumulate on MFMA over the s_k rows; a wave
// takes one i_k block and two column blocks, so that one A fragment feeds two
// independent MFMAs.  A_k(k) is staged in LDS when it is small, else read
// through the cache.  Each workgroup walks a contiguous range of column tiles
// so that operand slabs are reused.  Z is written through the X view.
// ---------------------------------------------------------------------------
constexpr int kRecThreads = 512;
constexpr int kRecWaves = kRecThreads / 64;

template <typename T, bool VEC = false>
__global__ void __launch_bounds__(kRecThreads) reconstruct_k(MGen mg, const T* __restrict__ Au,
                                                             T* __restrict__ Z, XView xv,
                                                             RecGeom g) {
  typedef Mfma<T> MM;
  constexpr int VW = 16 / (int)sizeof(T);   // rows per 16-byte read
  typedef T vT __attribute__((ext_vector_type(VW)));
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TileGeom& tg = g.tg;
  SlabRow* ptab = (SlabRow*)smem_raw;
  SlabRow* qtab = ptab + tg.Pp;
  T* Us = (T*)(qtab + tg.Qp);
  T* Vs = Us + tg.u_len;
  const int mso = ((int)((unsigned char*)(Vs + tg.v_len) - smem_raw) + 15) & ~15;
  T* Ms = (T*)(smem_raw + mso);               // [tcolp][ldm], rows of M contiguous
  T* As = Ms + (int64_t)tg.tcolp * g.ldm;     // [ip][lda] when staged
  const T* U = (const T*)mg.U;
  const T* V = (const T*)mg.V;
  // the wave index as a wave-uniform (scalar) value
  const int tid = threadIdx.x, lane = tid & 63,
            wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kr = lane >> 4, lc = lane & 15;

  build_tables(mg, tg, nullptr, 1, g.ldm, ptab, qtab, nullptr, tid, kRecThreads);
  for (int e = tid; e < tg.tcolp * g.ldm; e += kRecThreads) Ms[e] = T(0);
  if (g.lda > 0) {
    for (int e = tid; e < g.ip * g.sp; e += kRecThreads) {
      const int i = e / g.sp, r = e - (e / g.sp) * g.sp;
      As[i * g.lda + r] = (i < g.Ik && r < g.s) ? Au[(int64_t)i * g.s + r] : T(0);
    }
  }
  __syncthreads();

  const int nib = g.ip / 16, ncb = tg.tcolp / 16, ncg = (ncb + 1) / 2;
  const int64_t per = (tg.nColTiles + gridDim.x - 1) / gridDim.x;
  const int64_t ct0 = (int64_t)xcd_order(blockIdx.x, gridDim.x) * per,
                ct1 = min(ct0 + per, tg.nColTiles);
  int64_t cur_tu = -1, cur_tv = -1;
  const int ntv = (int)tg.nTileV;
  int tu32 = (int)(ct0 / ntv), tv32 = (int)ct0 - tu32 * ntv;
  for (int ct = (int)ct0; ct < (int)ct1; ++ct) {
    const int64_t tu = tu32, tv = tv32;
    if (++tv32 == ntv) {
      tv32 = 0;
      ++tu32;
    }
    const int64_t cu0 = tu * tg.TCu, cv0 = tv * tg.TCv;
    stage_operands<T, true, VEC>(mg, tg, U, V, tu, tv, cur_tu, cur_tv, Us, Vs, ptab, qtab, tid,
                            kRecThreads);
    __syncthreads();
    mgen_mfma<T>(tg, Us, Vs, ptab, qtab, Ms, lane, wave, kRecWaves);
    __syncthreads();
    for (int it = wave; it < nib * ncg; it += kRecWaves) {
      const int ib = it / ncg, cb0 = 2 * (it - (it / ncg) * ncg);
      const bool two = cb0 + 1 < ncb;
      typename MM::acc_t acc0 = MM::zero(), acc1 = MM::zero();
      const int ik_a = ib * 16 + lc;
      const bool oka = ik_a < g.Ik;
      const int ika = oka ? ik_a : 0;
      // lane group kr takes rows k0 + VW kr .. + VW - 1 of its column in one
      // 16-byte read and feeds VW MFMAs (the same row order for A and M)
      const int kof = kr * VW;
      const T* m0 = Ms + (cb0 * 16 + lc) * g.ldm + kof;
      const T* m1 = m0 + 16 * g.ldm;
      const T* ar = g.lda > 0 ? As + ik_a * g.lda + kof : nullptr;
      const T* ag = Au + (int64_t)ika * g.s + kof;
      const bool avec = (g.s % VW) == 0;
      auto load_a = [&](int k0) {
        if (g.lda > 0) return *(const vT*)(ar + k0);
        vT a;
        if (avec) {
          // rows are whole VW-groups here, so row < s covers all VW of them
          a = (oka && k0 + kof < g.s) ? *(const vT*)(ag + k0) : vT{};
        } else {
#pragma unroll
          for (int m = 0; m < VW; ++m) {
            const int row = k0 + kof + m;
            const T av = Au[(int64_t)ika * g.s + min(row, g.s - 1)];
            a[m] = (oka && row < g.s) ? av : T(0);
          }
        }
        return a;
      };
      if (two) {
#pragma unroll 2
        for (int k0 = 0; k0 < g.sp; k0 += 4 * VW) {
          const vT a = load_a(k0);
          const vT b0 = *(const vT*)(m0 + k0);
          const vT b1 = *(const vT*)(m1 + k0);
#pragma unroll
          for (int m = 0; m < VW; ++m) {
            acc0 = MM::mma(a[m], b0[m], acc0);
            acc1 = MM::mma(a[m], b1[m], acc1);
          }
        }
      } else {
#pragma unroll 2
        for (int k0 = 0; k0 < g.sp; k0 += 4 * VW) {
          const vT a = load_a(k0);
          const vT b0 = *(const vT*)(m0 + k0);
#pragma unroll
          for (int m = 0; m < VW; ++m) acc0 = MM::mma(a[m], b0[m], acc0);
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h == 1 && !two) break;
        const int c = (cb0 + h) * 16 + lc;
        if (c < tg.tcol) {
          const int cul = c / tg.TCv, cvl = c - (c / tg.TCv) * tg.TCv;
          const int64_t cu = cu0 + cul, cv = cv0 + cvl;
          if (cu < mg.Cu && cv < mg.Cv) {
            const int64_t base = cu * xv.x_cu + cv * xv.x_cv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int ik = ib * 16 + MM::row(lane, i);
              if (ik < xv.Ik) Z[base + (int64_t)ik * xv.x_ik] = h ? acc1[i] : acc0[i];
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_reconstruct(int prec, const MGen& mg, const void* Au, void* Z,
                              const XView& xv, const RecGeom& g_in, hipStream_t st) {
  RecGeom g = g_in;
  if ((uintptr_t)mg.U % 16 != 0) g.tg.u_vec = 0;
  if ((uintptr_t)mg.V % 16 != 0) g.tg.v_vec = 0;
  if (prec == P_F64) {
    hipFuncSetAttribute((const void*)reconstruct_k<double>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    reconstruct_k<double><<<g.nblk, kRecThreads, g.lds_bytes, st>>>(mg, (const double*)Au,
                                                                    (double*)Z, xv, g);
  } else if (g.tg.u_vec || g.tg.v_vec) {
    // a separate instance, as for the Gram: the 16-byte staging code costs
    // registers that the other modes would pay for
    hipFuncSetAttribute((const void*)reconstruct_k<float, true>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    reconstruct_k<float, true><<<g.nblk, kRecThreads, g.lds_bytes, st>>>(mg, (const float*)Au,
                                                                         (float*)Z, xv, g);
  } else {
    hipFuncSetAttribute((const void*)reconstruct_k<float>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds_bytes);
    reconstruct_k<float><<<g.nblk, kRecThreads, g.lds_bytes, st>>>(mg, (const float*)Au,
                                                                   (float*)Z, xv, g);
  }
  return hipGetLastError();
}

}  // namespace fctn
