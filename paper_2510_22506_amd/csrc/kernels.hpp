// Internal launch interface of the FCTN kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fctn {

// The chip dispatches the workgroups of a grid to its 8 XCDs round-robin by
// linear index, and each XCD has its own L2.  xcd_order maps the linear index
// L of an n-workgroup grid to a logical index so that each XCD receives one
// contiguous range of logical indices (a bijection on [0, n)): workgroups
// whose logical neighbours touch the same cache lines then share an L2.
constexpr int kXcds = 8;
__device__ inline int xcd_order(int L, int n) {
  const int per = n / kXcds, rem = n - per * kXcds;
  const int x = L % kXcds, i = L / kXcds;
  return x * per + (x < rem ? x : rem) + i;
}

// Sub-network generator (Property 1 with the reuse mechanism's operands):
//   M[ru * Rv + rv, cu * Cv + cv] = sum_kap U[ru, cu, kap] * V[rv, cv, kap]
// U, V are strided views of a factor tensor or of a cached pair tensor.
struct MGen {
  const void* U;
  int64_t u_ru, u_cu, u_k;
  const void* V;
  int64_t v_rv, v_cv, v_k;
  int32_t Ru, Rv, K;
  int64_t Cu, Cv;
};

// X_(k)[ik, cu * Cv + cv] = X[cu * x_cu + cv * x_cv + ik * x_ik]
struct XView {
  int64_t x_cu, x_cv, x_ik;
  int32_t Ik;
};

// Column tile: a TCu x TCv block of (cu, cv) pairs; tile column
// c = cu_l * TCv + cv_l.  Its block of M is generated on MFMA as the product
//   O[p][q] = sum_kap Us[kap][p] Vs[kap][q],  p = cu_l * Ru + ru,  q = cv_l * Rv + rv
// of the staged operand slabs, then scattered to M[ru * Rv + rv][c].
// Slab element (kap, p) sits at kap * us_k + p * us_p (either order, chosen so
// that the global reads are contiguous).
struct TileGeom {
  int32_t TCu, TCv, tcol, tcolp;  // tcolp: tcol rounded up to the MFMA k step
  int32_t Pu, Qv, Pp, Qp, Kp;     // GEMM sizes, 16-padded, and K padded to 4
  int32_t us_k, us_p, vs_k, vs_q; // slab strides
  int32_t u_len, v_len;           // slab sizes (elements)
  int32_t u_lw, v_lw;             // log2 of the lanes that run along a slab's
                                  // contiguous index when staging it
  int32_t u_vec, v_vec;           // float32 [kap][p] slab stageable with
                                  // 16-byte loads (rows in aligned runs of 4)
  int64_t nTileU, nTileV, nColTiles;
};

// Per-row / per-column index tables built once per launch in LDS so that the
// staging and scatter loops need no integer division.
struct SlabRow {        // row p = cu_l * Ru + ru of the U slab (or q of V)
  int32_t off;          // ru * u_ru + cu_l * u_cu (element offset in U)
  int32_t cl;           // cu_l (>= 2^30 for padding rows)
  int32_t map;          // cu_l * TCv * ldm + ru * Rv (its part of the M index), -1 if padding
  int32_t pad;
};

// Launch geometry of the fused sub-network / Gram / right-hand-side pass.
struct GramGeom {
  TileGeom tg;
  int32_t s, sp, Ik, ip;     // sizes and 16-padded sizes
  int32_t nG, nB, nTiles;    // upper-triangle Gram tiles, RHS tiles, total
  int32_t nbj;               // 16-blocks along s
  int32_t tilesPerGroup, nGroups;
  int64_t colTilesPerSplit;
  int32_t nSplit;
  int32_t ldm, ldx, xrows;   // LDS leading dims and X rows held per group
  int32_t mrows, xalloc, zrow; // M rows (float32/float64 kernel) and X rows
                             // given LDS; with zrow = 1 the rows past them,
                             // all zero, are read from one shared zero row
  size_t lds_bytes;
  int32_t nw;                // waves per workgroup: 8 (16 tiles each, or 2
                             // for small modes; two workgroups per CU) or 16
                             // (8, 10, 12 or 14 tiles each: tilesPerGroup /
                             // 16; one workgroup per CU with all of its LDS)
  int32_t mg16, ldk;         // bf16 forms: sub-network generated in split
                             // bf16 from bf16 slabs of row stride ldk
};

// Launch geometry of the reconstruction Z_(k) = A_k(k) M_k.
struct RecGeom {
  TileGeom tg;
  int32_t s, sp, Ik, ip;
  int32_t ldm, lda;          // Ms [tcolp][ldm]; staged A [ip][lda] (lda = 0: read from HBM)
  int32_t nblk;
  size_t lds_bytes;
};

// precision codes shared with the C ABI
enum { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3 };

// Cached sub-network operand (the N = 4 pair tensors and the N >= 5 prefix
// and suffix groups): two members contracted over the bonds they share,
//   G[d_0, .., d_{nd-1}] = sum_t F_0[off_0 + t0(t)] F_1[off_1 + t1(t)],
// where output digit d (last fastest) adds d * dstr[d] to member dmem[d]'s
// offset and internal digit i adds i * istr0[i] to member 0's and
// i * istr1[i] to member 1's.  All offsets and the entry count fit 31 bits
// (checked at plan time).
//
// Launch shape (set on the host): the digits from `ds` on are the inner
// block, `sin` consecutive entries made of `sin0` member-0 and `sin1`
// member-1 index combinations; a wave takes `no` outer indices at a time,
// stages their member-0 rows [i0][t] and member-1 rows [i1][t] (t padded to
// `innerp`) in LDS, then writes the no * sin entries.  Every quotient the
// kernel forms inside a block is below 2^16 and uses the multipliers m_*.
constexpr int kGroupMaxDigits = 16;
constexpr int kGroupMaxInner = 1024;   // internal bond values per entry
constexpr int kGroupMaxLds = 32 * 1024;
struct GroupDesc {
  const void* F[2];
  int32_t dsize[kGroupMaxDigits], dmem[kGroupMaxDigits], dstr[kGroupMaxDigits];
  int32_t isize[kGroupMaxDigits], istr0[kGroupMaxDigits], istr1[kGroupMaxDigits];
  uint64_t m_dsize[kGroupMaxDigits];   // for the inner digits
  uint64_t m_ip, m_n0, m_n1, m_nin;
  int32_t nd, ni;
  int32_t total, inner;   // output entries, terms per entry
  int32_t ds, sin, sin0, sin1, innerp, no, nouter;
  int32_t lds_bytes;
};

// x / d exactly for x, d < 2^16 (x * d < 2^32): (x * ceil(2^32 / d)) >> 32
inline uint64_t div_magic(uint32_t d) { return ((1ull << 32) + d - 1) / d; }
__device__ inline uint32_t div_by(uint32_t x, uint64_t m) {
  return (uint32_t)(((uint64_t)x * m) >> 32);
}

// one factor's shapes before and after a rank growth (last mode fastest);
// bit j of zero_modes: new indices along mode j give zero entries
struct RegrowDesc {
  int64_t shape_old[8];
  int64_t shape_new[8];
  int32_t N;
  uint32_t zero_modes;
};

// per-mode constants of a plan, passed by value to the kernel that stores them
struct PlanConsts {
  double lam_half[8];
  int32_t ncls[8];
  int32_t n;
};

hipError_t launch_set_consts(double* lam_half, int32_t* ncls, const PlanConsts& c,
                             hipStream_t st);
// flag[0] = OR of part[0 .. n)
hipError_t launch_any_flag(const int32_t* part, int n, int32_t* flag, hipStream_t st);

hipError_t launch_init_observed(int prec, const void* Y, const uint8_t* mask, void* X,
                                uint32_t* bits, int32_t* bad_part, int64_t n, int nblk,
                                hipStream_t st);
hipError_t launch_regrow(const double* old, const double* fill, double* out,
                         const RegrowDesc& d, hipStream_t st);
hipError_t launch_cast_factor(int prec, const double* A64, void* Aw, void* Au, int32_t Ik,
                              int32_t s, int64_t spost, hipStream_t st);
hipError_t launch_build_basis(double* Q, double* Qt, double* lam_col, int32_t n, double delta,
                              hipStream_t st);
hipError_t launch_group(int prec, const GroupDesc& gd, void* G, hipStream_t st);
hipError_t launch_gram_rhs(int prec, const MGen& mg, const void* X, const XView& xv,
                           const GramGeom& g, void* part, hipStream_t st);
hipError_t launch_reduce_gb(int prec, const GramGeom& g, const void* part, const double* A64,
                            int64_t spost, double rho, double* G, double* B, hipStream_t st);
hipError_t launch_project(const double* Qt, const double* B, int32_t Ik, int32_t s, double* Bt,
                          hipStream_t st);
// err: set to 1 if a class's bounded wait gave up (the result is then invalid)
hipError_t launch_solve_classes(const double* G, int32_t Ik, int32_t s, double lam,
                                double delta, double rho, double* At, double* trace_part,
                                int32_t* err, hipStream_t st);
// A_k = fold(Q a~) into A64 (float64 master), Aw (working precision, factor
// layout) and Au (working precision, mode-k unfolding).  alpha > 0 applies the
// asymmetric extrapolation A <- (1 + alpha) A - alpha beta A64_old elementwise,
// reading the previous factor from A64 before overwriting it.
hipError_t launch_backtransform(int prec, const double* Q, const double* At, int32_t Ik,
                                int32_t s, int64_t spost, double alpha, double beta,
                                double* A64, void* Aw, void* Au, hipStream_t st);
// tr(A_(k)^T L_k A_(k)) of the float64 factor, written to trace_part[0]
// (trace_part[1 .. ncls-1] are cleared), in the slots the class solves use.
hipError_t launch_factor_trace(const double* A64, int32_t Ik, int32_t s, int64_t spost,
                               double delta, int32_t ncls, double* trace_part,
                               hipStream_t st);
hipError_t launch_reconstruct(int prec, const MGen& mg, const void* Au, void* Z,
                              const XView& xv, const RecGeom& g, hipStream_t st);
// blocks of x_update_k for n elements (one 16-byte vector per thread)
int x_update_blocks(int prec, int64_t n);
hipError_t launch_x_update(int prec, void* X, const void* Z, const uint32_t* bits, double rho,
                           int64_t n, int nblk, double* xpart, hipStream_t st);
hipError_t launch_stats(const double* xpart, int nblk, const double* trace_part,
                        const double* lam_half, const int32_t* ncls, int N, int max_cls,
                        double* hist_slot, hipStream_t st);

int gram_max_lds_bytes();
int gram_threads();
int gram_tiles_per_group();
int solve_supported(int32_t s);

}  // namespace fctn
