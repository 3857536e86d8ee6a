// Factor subproblem (eq. 5): A G + lambda L A + rho A = B, float64.
//
// With L = Q diag(Lambda) Q^T in its real orthonormal Fourier basis (eq. 7;
// columns: constant, cos/sin pairs per frequency, alternating for even n),
// A~ = Q^T A turns eq. 5 into one equation per row of A~:
//     a~_v (G + (lambda Lambda_v + rho) I) = b~_v,   b~ = Q^T B.
// Rows that share a frequency share the matrix, so each frequency class is
// one SPD solve.  The two basis changes are float64 MFMA products
// (gemm64_k): b~ = Q^T B for all rows at once before the solves, and
// A = Q A~ after them, stored folded (eq. 9) in float64 and in the working
// precision.  solve_classes_k runs one class per workgroup: a blocked
// right-looking Cholesky of the shifted G with the class's right-hand sides
// appended as extra rows (their rows of the factor are the forward-
// substitution result), then a blocked back substitution, overwriting the
// class's rows of b~ with those of a~.  The same unique solution as eq. 8
// (the shifted matrix is positive definite), reached without an
// eigendecomposition of G.
#include <algorithm>
#include <utility>

#include "common.hpp"
#include "kernels.hpp"

namespace fctn {

int solve_supported(int32_t s) { return s >= 1 && s <= 192; }

// Phase hook for timing probes (empty in the library).
#ifndef FCTN_SOLVE_MARK
#define FCTN_SOLVE_MARK(n)
#endif

// Calls f(integral_constant<int, 0>) .. f(integral_constant<int, N - 1>) in
// order, so that register arrays indexed by the constant stay in registers.
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// LDS of solve_classes_k, in doubles: two transposed panels (32 x 32 SB
// each), the right-hand sides (2 x 32 SB), reciprocal pivots (32 SB), the
// back-substitution partials (64), a wave-sum buffer (16) and the column
// counter of the diagonal block (one word).
static inline size_t solve_lds_doubles(int sb) {
  return (size_t)67 * 32 * sb + 82 + (size_t)32 * (sb - 1) * 33;
}

// Layout: thread (r, cc) = (tid % 32, tid / 32) holds H[r + 32a][cc + 32b]
// for the lower blocks b <= a in registers (32x32 cyclic over 1024 threads).
// Panel p (columns 32p .. 32p + 31) is staged transposed in LDS,
// pan[jj][i] = H[i][32p + jj], so that a half-wave reads 32 consecutive rows.
// Per panel, with a workgroup barrier after (a)+(b) and after (c):
//   (a) wave 0 factors the 32x32 diagonal block column by column; lanes
//       (i, h) hold row i, columns 16h .. 16h + 15; the next pivot's column
//       is updated from registers (readlane), the others from the finished
//       column read back from LDS one step later (no workgroup barrier);
//   (b) meanwhile other waves solve the rows below the block, and the two
//       right-hand-side rows, against the block's factor (TRSM), following
//       the published columns through an LDS counter;
//   (c) every thread keeps its finished part of the column block, applies
//       the rank-32 update to its trailing blocks, updates the right-hand
//       sides and writes the next column block into the other panel buffer.
// Back substitution runs over the panels in reverse: a half-wave reduction
// of the already-solved rows, then a 32-step solve against the diagonal
// block in one wave (register values broadcast by readlane).
template <int SB>
__global__ void __launch_bounds__(1024) solve_classes_k(const double* __restrict__ G, int Ik,
                                                        int s, double lam, double delta,
                                                        double rho, double* __restrict__ At,
                                                        double* __restrict__ trace_part,
                                                        int32_t* __restrict__ err) {
  constexpr int LDP = 32 * SB;
  extern __shared__ double smem[];
  double* const pan0 = smem;
  double* const pan1 = smem + 32 * LDP;
  double* const rhs = smem + 64 * LDP;
  double* const rdiag = rhs + 2 * LDP;
  double* const tpart = rdiag + LDP;
  double* const red = tpart + 64;
  int* const pub = (int*)(red + 16);
  double* const stg = red + 17;     // [32 (SB - 1)][33]: trailing-update tiles
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = tid & 31, cc = tid >> 5;
  FCTN_SOLVE_MARK(0);

  int nv = 2, v0 = 2 * c - 1, v1 = 2 * c;
  if (c == 0) {
    nv = 1; v0 = 0; v1 = 0;
  } else if ((Ik % 2 == 0) && c == Ik / 2) {
    nv = 1; v0 = Ik - 1; v1 = Ik - 1;
  }
  const double sn = sinpi((double)c / (double)Ik);
  const double Lam = delta + 4.0 * sn * sn;
  const double sigma = lam * Lam + rho;

  // every LDS word starts finite: padding rows and columns are read (and
  // multiplied by zero or discarded) but never decide a result
  for (int t = tid; t < 67 * LDP; t += 1024) smem[t] = 0.0;
  __syncthreads();
  FCTN_SOLVE_MARK(1);

  // the class's rows of b~
  for (int t = tid; t < 2 * s; t += 1024) {
    const int v = t >= s ? 1 : 0, m = t - v * s;
    rhs[v * LDP + m] = At[(int64_t)(v ? v1 : v0) * s + m];
  }
  FCTN_SOLVE_MARK(2);

  // H = G + sigma I (G symmetric: G[m][i] is read, consecutive over r), and
  // column block 0 staged
  double H[SB][SB];
#pragma unroll
  for (int a = 0; a < SB; ++a) {
    const int i = r + 32 * a;
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int m = cc + 32 * b;
      H[a][b] = (i < s && m <= i) ? G[(int64_t)m * s + i] + (i == m ? sigma : 0.0) : 0.0;
    }
  }
#pragma unroll
  for (int a = 0; a < SB; ++a) {
    const int i = r + 32 * a;
    if (i < s) pan0[cc * LDP + i] = H[a][0];
  }
  if (tid == 0) *pub = 0;
  __syncthreads();
  FCTN_SOLVE_MARK(3);

  static_for<SB>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = decltype(pc)::value;
    const int p0 = 32 * p;
    if (p0 < s) {
    const int np = min(32, s - p0);
    double* const pan = (p & 1) ? pan1 : pan0;
    double* const pnx = (p & 1) ? pan0 : pan1;

    // (a) diagonal block, wave 0.  Column j is published with zeros at and
    // above the diagonal, so every later product with an entry that must not
    // act (a finished column, a row at or above the pivot) multiplies a stored
    // zero; the pivots live in rdiag only.  After each column the counter
    // *pub is raised (release), so that (b) can follow column by column.
    // (b) rows below the block and the right-hand sides (TRSM), waves 1-3
    // and 5-15 (SIMD 0 is left to wave 0).  Two rows per group of four
    // lanes, eight columns per lane; the finished value of column j reaches
    // the other lanes of the group by a DPP quad broadcast.  Step j waits
    // (acquire) for column j.
    const int nbelow = max(s - p0 - 32, 0);
    if (wave == 0) {
      // wave 0 parks its register blocks of H in the (idle) staging area for
      // the duration of the column loop, which needs the registers
      if constexpr (SB >= 3) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < SB; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) stg[64 * t++ + lane] = H[a][b];
      }
      const int i = lane & 31, h = lane >> 5;
      double d[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) d[q] = pan[(16 * h + q) * LDP + p0 + i];
      // Column j in three parts, software-pipelined so that the LDS round
      // trip of one column overlaps the pivot chain of the next:
      //   pivot: readlane of the diagonal entry, L[i][j] = d * rsqrt(pivot),
      //          stored to the panel;
      //   fast path: column j + 1 (the next pivot's column) updated from
      //          registers in unscaled form, d[i][j+1] -= d[i][j] d[j+1][j] /
      //          pivot, so that the serial chain from one pivot to the next
      //          holds a readlane, a reciprocal and one multiply-add;
      //   rest: the other columns' multipliers L[16h + q][j] read back from
      //          the panel (one address per half: broadcast reads) and
      //          applied at the start of step j + 1.
      // No branch inside the loop: rows and columns past np (last panel) are
      // zero padding with a unit diagonal, so all they produce is zero.
#pragma unroll
      for (int q = 0; q < 16; ++q) d[q] = (i >= np && 16 * h + q == i) ? 1.0 : d[q];
      double dn = d[0];     // column j of this lane's row, all updates applied
      double pl[16], pli = 0.0;
      double rsl = 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) pl[q] = 0.0;
      static_for<32>([&](auto jc) __attribute__((always_inline)) {
        constexpr int j = decltype(jc)::value;
        constexpr int hj = j >> 4, jn = j + 1, hn = jn >> 4, cn = jn & 15;
        // columns still open after column j - 1 (for j > 16 only those of
        // the upper half above j - 1)
        if constexpr (j > 0) {
#pragma unroll
          for (int q = 0; q < 16; ++q)
            if (j <= 16 || q >= j - 16) d[q] -= pli * pl[q];
        }
        if constexpr (j == 16) dn = d[0];   // first column of the upper half
        const double piv = bcast_lane(dn, j + 32 * hj);
        const double rs = rsqrt_f64(piv);
        rsl = i == j ? rs : rsl;
        // L[i][j], valid in the half that holds column j (h == hj)
        const double own = i > j ? dn * rs : 0.0;
        *(h == hj ? pan + j * LDP + p0 + i : tpart + i) = own;
        if constexpr (jn < 32 && hn == hj) {
          const double lq = bcast_lane(own, jn + 32 * hj);
          dn = d[cn] - (h == hn ? own : 0.0) * lq;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        pli = pan[j * LDP + p0 + i];
        const double2* colj = (const double2*)(pan + j * LDP + p0 + 16 * h);
#pragma unroll
        for (int q2 = 0; q2 < 8; ++q2) {
          if (j < 16 || 2 * q2 + 1 >= j - 15) {
            const double2 v = colj[q2];
            pl[2 * q2] = v.x;
            pl[2 * q2 + 1] = v.y;
          }
        }
        // the fast-path column is already done in its half
        if constexpr (jn < 32 && hn == hj) pl[cn] = h == hn ? 0.0 : pl[cn];
        // publish every fourth column: reciprocal pivots, then the counter
        // (release: the columns and pivots are visible before it)
        if constexpr ((j & 3) == 3) {
          rdiag[p0 + i] = rsl;
          __hip_atomic_store(pub, j + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        // the previous column's update is complete here (bounds the loads'
        // live range)
#pragma unroll
        for (int q = 0; q < 16; ++q) asm volatile("" ::"v"(d[q]));
        __builtin_amdgcn_sched_barrier(0);
      });
      if constexpr (SB >= 3) {
        int t = 0;
#pragma unroll
        for (int a = 0; a < SB; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) H[a][b] = stg[64 * t++ + lane];
      }
    } else if (wave != 4 && (wave - 1 - (wave > 4)) * 32 < nbelow + 2) {
      // rows 2 rp and 2 rp + 1 of the row list (rows below, then the two
      // right-hand sides) go to the four lanes of quad rp; lane g of the quad
      // holds their columns 8g .. 8g + 7
      const int g = lane & 3;
      const int rp = (wave - 1 - (wave > 4)) * 16 + (lane >> 2);
      const int nrow = nbelow + 2;
      const int ra = 2 * rp, rb = 2 * rp + 1;
      const bool va = ra < nrow, vb = rb < nrow;
      // row pointers (an absent row reads the first right-hand side)
      const int ia = va ? ra - nbelow : 0, ib = vb ? rb - nbelow : 0;
      double* const pa = ia < 0 ? pan + p0 + 32 + ra : rhs + ia * LDP + p0;
      double* const pb = ib < 0 ? pan + p0 + 32 + rb : rhs + ib * LDP + p0;
      const int sa = ia < 0 ? LDP : 1, sb = ib < 0 ? LDP : 1;
      double xa[8], xb[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        xa[q] = pa[(8 * g + q) * sa];
        xb[q] = pb[(8 * g + q) * sb];
      }
      int avail = 0;
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        if (j < np) {
          // bounded wait: column j is always published (j < np), the bound
          // only guards against a logic error turning into a hang
          for (int spin = 0; avail <= j && spin < (1 << 16); ++spin) {
            avail = __hip_atomic_load(pub, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (avail <= j) __builtin_amdgcn_s_sleep(1);
          }
          // bound reached: the result is invalid; flag it for the host, which
          // reports FCTN_E_DEVICE at its next read of results
          if (avail <= j) *err = 1;
          const int gj = j >> 3, cj = j & 7;
          const double sc = g == gj ? rdiag[p0 + j] : 1.0;
          xa[cj] *= sc;
          xb[cj] *= sc;
          const double ya = quad_bcast(xa[cj], gj), yb = quad_bcast(xb[cj], gj);
          // entries at and above the diagonal of column j are stored zeros
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double l = pan[j * LDP + p0 + 8 * g + q];
            xa[q] -= ya * l;
            xb[q] -= yb * l;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (8 * g + q < np) {
          if (va) pa[(8 * g + q) * sa] = xa[q];
          if (vb) pb[(8 * g + q) * sb] = xb[q];
        }
      }
    }
    __syncthreads();
    FCTN_SOLVE_MARK(5 + 3 * p);

    // (c) keep the finished column block, trailing update, next panel out
    // strictly lower part of the diagonal block (the stored diagonal is zero)
    H[p][p] = pan[cc * LDP + p0 + r];
#pragma unroll
    for (int a = p + 1; a < SB; ++a) H[a][p] = pan[cc * LDP + r + 32 * a];
    if (nbelow > 0) {
      // rank-32 update of the trailing blocks on FP64 MFMA, one column block
      // b at a time: the product (rows 32b ..) x (columns 32b .. 32b + 31) of
      // the finished panel with itself is formed in 16 x 16 tiles, staged in
      // LDS, and subtracted from the cyclic register blocks H[a][b], a >= b
      static_for<SB>([&](auto bc) __attribute__((always_inline)) {
        constexpr int b = decltype(bc)::value;
        if constexpr (b > p) {
          if (32 * b < s) {
            typedef Mfma<double> MD;
            const int kr = lane >> 4, lc = lane & 15;
            const int nrt = 2 * (SB - b);
            for (int t = wave; t < 2 * nrt; t += 16) {
              const int rt = t >> 1, ct = t & 1;
              const int row0 = 32 * b + 16 * rt, col0 = 32 * b + 16 * ct;
              typename MD::acc_t acc = MD::zero();
              if (row0 < s) {
#pragma unroll
                for (int k0 = 0; k0 < 32; k0 += 4) {
                  const double av = pan[(k0 + kr) * LDP + row0 + lc];
                  const double bv = pan[(k0 + kr) * LDP + col0 + lc];
                  acc = MD::mma(av, bv, acc);
                }
              }
#pragma unroll
              for (int i = 0; i < 4; ++i)
                stg[(16 * rt + MD::row(lane, i)) * 33 + 16 * ct + lc] = acc[i];
            }
            __syncthreads();
#pragma unroll
            for (int a = b; a < SB; ++a) H[a][b] -= stg[(r + 32 * (a - b)) * 33 + cc];
            __syncthreads();
          }
        }
      });
      for (int t = tid; t < 2 * nbelow; t += 1024) {
        const int v = t >= nbelow ? 1 : 0;
        const int m = p0 + 32 + t - v * nbelow;
        double acc = rhs[v * LDP + m];
        for (int jj = 0; jj < 32; ++jj) acc -= rhs[v * LDP + p0 + jj] * pan[jj * LDP + m];
        rhs[v * LDP + m] = acc;
      }
      if constexpr (p + 1 < SB) {
#pragma unroll
        for (int a = p + 1; a < SB; ++a) {
          const int i = r + 32 * a;
          if (i < s) pnx[cc * LDP + i] = H[a][p + 1];
        }
      }
    }
    if (tid == 0) *pub = 0;
    __syncthreads();
    FCTN_SOLVE_MARK(6 + 3 * p);
    }
  });

  // back substitution L^T x = y, panels in reverse
  static_for<SB>([&](auto pc) __attribute__((always_inline)) {
    constexpr int p = SB - 1 - decltype(pc)::value;
    const int p0 = 32 * p;
    if (p0 < s) {
    const int np = min(32, s - p0);
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int a = p + 1; a < SB; ++a) {
      const int i = r + 32 * a;
      if (i < s) {
        t0 += H[a][p] * rhs[i];
        t1 += H[a][p] * rhs[LDP + i];
      }
    }
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) {
      t0 += __shfl_xor(t0, off, 32);
      t1 += __shfl_xor(t1, off, 32);
    }
    if (r == 0) {
      tpart[cc] = t0;
      tpart[32 + cc] = t1;
    }
    smem[r * 33 + cc] = H[p][p];
    __syncthreads();
    FCTN_SOLVE_MARK(24 + 2 * p);
    if (wave == 0) {
      // lane q (and q + 32 for the second right-hand side) carries z_q; step j
      // takes x_j = z_j / L_jj from lane j and removes L[j][q] x_j.  The
      // multipliers L[j][q] are read from LDS eight steps ahead, and each lane
      // scales its own z by its own 1 / L_qq, so the serial chain holds only
      // the two readlanes and a multiply-add.
      const int q = lane & 31, v = lane >> 5;
      double z = q < np ? rhs[v * LDP + p0 + q] - tpart[v * 32 + q] : 0.0;
      const double rd = rdiag[p0 + q];
#pragma unroll
      for (int j8 = 3; j8 >= 0; --j8) {
        double l8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) l8[u] = smem[(8 * j8 + u) * 33 + q];
#pragma unroll
        for (int u = 7; u >= 0; --u) {
          const int j = 8 * j8 + u;
          if (j < np) {
            const double w = z * rd;
            const double xa = bcast_lane(w, j), xb = bcast_lane(w, 32 + j);
            const double xj = v ? xb : xa;
            const double l = q < j ? l8[u] : 0.0;
            z = q == j ? xj : z - l * xj;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (q < np) rhs[v * LDP + p0 + q] = z;
    }
    __syncthreads();
    FCTN_SOLVE_MARK(25 + 2 * p);
    }
  });

  double tr = 0.0;
  for (int m = tid; m < s; m += 1024) {
    const double x0 = rhs[m];
    At[(int64_t)v0 * s + m] = x0;
    tr += x0 * x0;
    if (nv == 2) {
      const double x1 = rhs[LDP + m];
      At[(int64_t)v1 * s + m] = x1;
      tr += x1 * x1;
    }
  }
  tr = wave_sum(tr);
  if (lane == 0) red[wave] = tr;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    trace_part[c] = Lam * t;
  }
  FCTN_SOLVE_MARK(40);
}

hipError_t launch_solve_classes(const double* G, int32_t Ik, int32_t s, double lam,
                                double delta, double rho, double* At, double* trace_part,
                                int32_t* err, hipStream_t st) {
  const int ncls = Ik / 2 + 1;
  const int sb = (s + 31) / 32;
  const size_t lds = solve_lds_doubles(sb) * sizeof(double);
  switch (sb) {
#define FCTN_SOLVE_CASE(N)                                                                 \
  case N:                                                                                  \
    hipFuncSetAttribute((const void*)solve_classes_k<N>,                                   \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);             \
    solve_classes_k<N><<<ncls, 1024, lds, st>>>(G, Ik, s, lam, delta, rho, At,           \
                                                trace_part, err);                          \
    break;
    FCTN_SOLVE_CASE(1)
    FCTN_SOLVE_CASE(2)
    FCTN_SOLVE_CASE(3)
    FCTN_SOLVE_CASE(4)
    FCTN_SOLVE_CASE(5)
    FCTN_SOLVE_CASE(6)
#undef FCTN_SOLVE_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// C = A X for row-major float64 A (M x K) and X (K x N) on float64 MFMA.
// One 16x16 output tile per workgroup; its four waves take interleaved
// 4-wide k slices (wave w: k = 4w + 16t .. + 3) with eight slices of loads in
// flight, and the four partial tiles are summed in a fixed order through LDS.
// EPI 0 stores C row-major; EPI 1 stores the factor update: folded (eq. 9)
// into A64 (float64) and Aw (working precision), and row-major into Au.
template <int EPI, typename W>
__global__ void __launch_bounds__(256) gemm64_k(const double* __restrict__ A,
                                                const double* __restrict__ X, int M, int K,
                                                int N, double* __restrict__ C, int64_t spost,
                                                double alpha, double beta,
                                                double* __restrict__ A64, W* __restrict__ Aw,
                                                W* __restrict__ Au) {
  typedef Mfma<double> MM;
  __shared__ double part[3][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbn = (N + 15) >> 4;
  const int i0 = (blockIdx.x / nbn) * 16, j0 = (blockIdx.x % nbn) * 16;
  const int kr = lane >> 4, lc = lane & 15;
  const bool oka = i0 + lc < M, okb = j0 + lc < N;
  const int ia = min(i0 + lc, M - 1), jb = min(j0 + lc, N - 1);
  typename MM::acc_t acc = MM::zero();
  for (int kb = 4 * wave; kb < K; kb += 128) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kb + 16 * u + kr;
      const int kc = min(k, K - 1);
      const double av = A[(int64_t)ia * K + kc], bv = X[(int64_t)kc * N + jb];
      a[u] = (oka && k < K) ? av : 0.0;
      b[u] = (okb && k < K) ? bv : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = MM::mma(a[u], b[u], acc);
  }
  if (wave > 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wave - 1][r][lane] = acc[r];
  }
  __syncthreads();
  if (wave == 0 && okb) {
    const int j = j0 + lc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + MM::row(lane, r);
      if (i < M) {
        const double vs = ((acc[r] + part[0][r][lane]) + part[1][r][lane]) + part[2][r][lane];
        if constexpr (EPI == 0) {
          C[(int64_t)i * N + j] = vs;
        } else {
          const int64_t f = (j / spost) * ((int64_t)M * spost) + (int64_t)i * spost + j % spost;
          double v = vs;
          // asymmetric extrapolation (Section 4.2) against the factor this
          // subproblem started from, still held in A64
          if (alpha > 0.0) v = vs + alpha * (vs - beta * A64[f]);
          A64[f] = v;
          Aw[f] = (W)v;
          Au[(int64_t)i * N + j] = (W)v;
        }
      }
    }
  }
}

static inline int gemm_blocks(int32_t M, int32_t N) { return ((M + 15) / 16) * ((N + 15) / 16); }

hipError_t launch_project(const double* Qt, const double* B, int32_t Ik, int32_t s, double* Bt,
                          hipStream_t st) {
  gemm64_k<0, double><<<gemm_blocks(Ik, s), 256, 0, st>>>(Qt, B, Ik, Ik, s, Bt, 1, 0.0, 0.0,
                                                          nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_backtransform(int prec, const double* Q, const double* At, int32_t Ik,
                                int32_t s, int64_t spost, double alpha, double beta,
                                double* A64, void* Aw, void* Au, hipStream_t st) {
  const int nb = gemm_blocks(Ik, s);
  if (prec == P_F64)
    gemm64_k<1, double><<<nb, 256, 0, st>>>(Q, At, Ik, Ik, s, nullptr, spost, alpha, beta, A64,
                                            (double*)Aw, (double*)Au);
  else
    gemm64_k<1, float><<<nb, 256, 0, st>>>(Q, At, Ik, Ik, s, nullptr, spost, alpha, beta, A64,
                                           (float*)Aw, (float*)Au);
  return hipGetLastError();
}

// tr(A^T L A) = sum over the entries a_ij of delta a_ij^2 + (a_ij -
// a_{i+1 mod I, j})^2, the quadratic form of L = (2 + delta) I - S - S^T
// (Section 3.1) written with periodic first differences.  One workgroup: the
// factor holds at most a few hundred thousand entries.  Each thread takes the
// entries e = tid, tid + 1024, .. of the row-major (i, j) walk (neighbouring
// threads read neighbouring entries of a row), so every load is independent
// and the sum order is fixed.
__global__ void __launch_bounds__(1024) factor_trace_k(const double* __restrict__ A64, int Ik,
                                                      int s, int64_t spost, double delta,
                                                      int ncls, double* __restrict__ trace_part) {
  __shared__ double red[16];
  double t = 0.0;
  const int64_t n = (int64_t)Ik * s;
  for (int64_t e = threadIdx.x; e < n; e += 1024) {
    const int i = (int)(e / s), j = (int)(e - (int64_t)i * s);
    const double* col = A64 + (j / spost) * ((int64_t)Ik * spost) + j % spost;
    const double a = col[(int64_t)i * spost];
    const double an = col[(int64_t)(i + 1 == Ik ? 0 : i + 1) * spost];
    t += delta * a * a + (a - an) * (a - an);
  }
  t = wave_sum(t);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < 16; ++w) tot += red[w];
    trace_part[0] = tot;
  }
  for (int c = 1 + threadIdx.x; c < ncls; c += 1024) trace_part[c] = 0.0;
}

hipError_t launch_factor_trace(const double* A64, int32_t Ik, int32_t s, int64_t spost,
                               double delta, int32_t ncls, double* trace_part, hipStream_t st) {
  factor_trace_k<<<1, 1024, 0, st>>>(A64, Ik, s, spost, delta, ncls, trace_part);
  return hipGetLastError();
}

}  // namespace fctn
