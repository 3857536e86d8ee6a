// Factor subproblem (eq. 5): A G + lambda L A + rho A = B, float64.
//
// With L = Q diag(Lambda) Q^T in its real orthonormal Fourier basis (eq. 7;
// columns: constant, cos/sin pairs per frequency, alternating for even n),
// A~ = Q^T A turns eq. 5 into one equation per row of A~:
//     a~_v (G + (lambda Lambda_v + rho) I) = b~_v,   b~ = Q^T B.
// Rows that share a frequency share the matrix, so each frequency class is
// one SPD solve.  solve_classes_k runs one class per workgroup: b~ by
// wavefront-level reductions over i_k, then a register-resident Cholesky of
// the shifted G (1024 threads, 32x32 cyclic distribution) with the class's
// right-hand sides appended as extra rows (their rows of the factor are the
// forward-substitution result), then back substitution.  The same unique
// solution as eq. 8 (the shifted matrix is positive definite), reached
// without an eigendecomposition of G.  backtransform_k forms A = Q A~ and
// stores it folded (eq. 9) in float64 and in the working precision.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace fctn {

int solve_supported(int32_t s) { return s >= 1 && s <= 192; }

template <int SB>
__global__ void __launch_bounds__(1024) solve_classes_k(const double* __restrict__ G,
                                                        const double* __restrict__ B,
                                                        const double* __restrict__ Qt, int Ik,
                                                        int s, double lam, double delta,
                                                        double rho, double* __restrict__ At,
                                                        double* __restrict__ trace_part) {
  __shared__ double colbuf[2][32 * SB];
  __shared__ double rhs[2][32 * SB];
  __shared__ double diag[32 * SB];
  __shared__ double rdiag[32 * SB];
  __shared__ double red[16];
  extern __shared__ double Lp[];   // s (s + 1) / 2 packed lower factor
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  int nv = 2, v0 = 2 * c - 1, v1 = 2 * c;
  if (c == 0) {
    nv = 1; v0 = 0; v1 = 0;
  } else if ((Ik % 2 == 0) && c == Ik / 2) {
    nv = 1; v0 = Ik - 1; v1 = Ik - 1;
  }
  const double sn = sinpi((double)c / (double)Ik);
  const double Lam = delta + 4.0 * sn * sn;
  const double sigma = lam * Lam + rho;

  // b~_v[m] = sum_i Q[i][v] B[i][m]: output o = (v, m) gets nsub threads that
  // each sum an interleaved slice of i (reads coalesced over m); the slices
  // are combined in a fixed order through LDS (the L buffer, unused yet)
  {
    const int nout = 2 * s;
    const int nsub = 1024 / nout;
    const int o = tid % nout, sub = tid / nout;
    if (sub < nsub) {
      const int v = o >= s ? 1 : 0, m = o - v * s;
      const double* q = Qt + (int64_t)(v ? v1 : v0) * Ik;
      double p = 0.0;
      for (int i = sub; i < Ik; i += nsub) p += q[i] * B[(int64_t)i * s + m];
      Lp[sub * nout + o] = p;
    }
    __syncthreads();
    if (tid < nout) {
      double p = 0.0;
      for (int k = 0; k < nsub; ++k) p += Lp[k * nout + tid];
      rhs[tid >= s ? 1 : 0][tid >= s ? tid - s : tid] = p;
    }
  }

  // H = G + sigma I, 32x32 cyclic: thread (r, c) = (tid % 32, tid / 32) holds
  // rows r + 32a and columns c + 32b (lower blocks b <= a only).  The 32
  // holders of a column are one half-wave.  G is symmetric, so G[m][i] is read
  // (consecutive lanes, consecutive addresses).
  const int r = tid & 31, cc = tid >> 5;
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
  __syncthreads();

  // right-looking Cholesky.  Per column j the half-wave holding it publishes
  // the raw column to LDS and the pivot's holder publishes sqrt(d_j) and its
  // reciprocal; after the barrier every thread forms its row and column
  // multipliers (zero outside the trailing range, so the rank-1 update needs
  // no per-element tests: strictly upper entries of diagonal blocks receive
  // values that are never read) and updates its trailing blocks.  Finished
  // blocks are skipped with wave-uniform tests.
  for (int j = 0; j < s; ++j) {
    const int jb = j >> 5, jt = j & 31;
    double* cb = colbuf[j & 1];
    if (cc == jt) {
      double pv = 1.0;
#pragma unroll
      for (int a = 0; a < SB; ++a) {
        if (a < jb) continue;
        double v = 0.0;
#pragma unroll
        for (int b = 0; b <= a; ++b)
          if (b == jb) v = H[a][b];
        const int i = r + 32 * a;
        if (i >= j && i < s) cb[i] = v;
        if (i == j) pv = v;
      }
      if (r == jt) {
        const double sq = sqrt(pv);
        diag[j] = sq;
        rdiag[j] = 1.0 / sq;
      }
    }
    __syncthreads();
    const double rs = rdiag[j];
    double lm[SB], li[SB];
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      const int m = cc + 32 * b, i = r + 32 * b;
      const bool act = 32 * b + 31 > j;
      lm[b] = (act && m > j && m < s) ? cb[m] * rs : 0.0;
      li[b] = (act && i > j && i < s) ? cb[i] * rs : 0.0;
    }
#pragma unroll
    for (int a = 0; a < SB; ++a) {
      if (32 * a + 31 <= j) continue;
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        if (32 * b + 31 <= j) continue;
        H[a][b] -= li[a] * lm[b];
      }
    }
    if (cc == jt) {
      const double sd = diag[j];
#pragma unroll
      for (int a = 0; a < SB; ++a) {
        if (a < jb) continue;
        const int i = r + 32 * a;
#pragma unroll
        for (int b = 0; b <= a; ++b)
          if (b == jb) H[a][b] = (i == j) ? sd : ((i > j && i < s) ? li[a] : H[a][b]);
      }
    }
  }
  // L to LDS (packed lower: row i starts at i (i + 1) / 2)
#pragma unroll
  for (int a = 0; a < SB; ++a) {
    const int i = r + 32 * a;
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const int m = cc + 32 * b;
      if (i < s && m <= i) Lp[i * (i + 1) / 2 + m] = H[a][b];
    }
  }
  __syncthreads();

  // forward (L y = b~) and back (L^T x = y) substitution in one wave,
  // column-oriented: lane l keeps entries i = l + 64 q in registers; the
  // pivot entry is broadcast from its owner lane with readlane
  if (wave == 0) {
    constexpr int NQ = (32 * SB + 63) / 64;
    double y0[NQ], y1[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      y0[q] = i < s ? rhs[0][i] : 0.0;
      y1[q] = i < s ? rhs[1][i] : 0.0;
    }
    for (int m = 0; m < s; ++m) {
      const int owner = m & 63, qm = m >> 6;
      double ym0 = 0.0, ym1 = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (q == qm) {
          ym0 = y0[q];
          ym1 = y1[q];
        }
      const double rd = rdiag[m];
      const double x0 = bcast_lane(ym0, owner) * rd;
      const double x1 = bcast_lane(ym1, owner) * rd;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        if (i > m && i < s) {
          const double l = Lp[i * (i + 1) / 2 + m];
          y0[q] -= l * x0;
          y1[q] -= l * x1;
        } else if (i == m) {
          y0[q] = x0;
          y1[q] = x1;
        }
      }
    }
    for (int m = s - 1; m >= 0; --m) {
      const int owner = m & 63, qm = m >> 6;
      double ym0 = 0.0, ym1 = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (q == qm) {
          ym0 = y0[q];
          ym1 = y1[q];
        }
      const double rd = rdiag[m];
      const double x0 = bcast_lane(ym0, owner) * rd;
      const double x1 = bcast_lane(ym1, owner) * rd;
      const double* Lrow = Lp + m * (m + 1) / 2;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        if (i < m) {
          const double l = Lrow[i];
          y0[q] -= l * x0;
          y1[q] -= l * x1;
        } else if (i == m) {
          y0[q] = x0;
          y1[q] = x1;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      if (i < s) {
        rhs[0][i] = y0[q];
        rhs[1][i] = y1[q];
      }
    }
  }
  __syncthreads();

  double tr = 0.0;
  for (int m = tid; m < s; m += 1024) {
    const double x0 = rhs[0][m];
    At[(int64_t)v0 * s + m] = x0;
    tr += x0 * x0;
    if (nv == 2) {
      const double x1 = rhs[1][m];
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
}

hipError_t launch_solve_classes(const double* G, const double* B, const double* Qt,
                                int32_t Ik, int32_t s, double lam, double delta, double rho,
                                double* At, double* trace_part, hipStream_t st) {
  const int ncls = Ik / 2 + 1;
  const int sb = (s + 31) / 32;
  // packed factor, or the projection partials before it exists
  const size_t lds = (size_t)std::max(s * (s + 1) / 2, 1024) * sizeof(double);
  switch (sb) {
#define FCTN_SOLVE_CASE(N)                                                                 \
  case N:                                                                                  \
    hipFuncSetAttribute((const void*)solve_classes_k<N>,                                   \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);             \
    solve_classes_k<N><<<ncls, 1024, lds, st>>>(G, B, Qt, Ik, s, lam, delta, rho, At,    \
                                                trace_part);                               \
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

// A = Q A~ on float64 MFMA: one 16x16 output tile per wave, k = i_k.
template <typename W>
__global__ void __launch_bounds__(256) backtransform_k(const double* __restrict__ Q,
                                                       const double* __restrict__ At, int Ik,
                                                       int s, int64_t spost,
                                                       double* __restrict__ A64,
                                                       W* __restrict__ Aw, W* __restrict__ Au) {
  typedef Mfma<double> MM;
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nbj = (s + 15) / 16, nbi = (Ik + 15) / 16;
  if (t >= nbi * nbj) return;
  const int i0 = (t / nbj) * 16, j0 = (t % nbj) * 16;
  const int kr = lane >> 4, lc = lane & 15;
  const int ia = i0 + lc, jb = j0 + lc;
  typename MM::acc_t acc = MM::zero();
  for (int k0 = 0; k0 < Ik; k0 += 4) {
    const int k = k0 + kr;
    const double a = (ia < Ik && k < Ik) ? Q[(int64_t)ia * Ik + k] : 0.0;
    const double b = (k < Ik && jb < s) ? At[(int64_t)k * s + jb] : 0.0;
    acc = MM::mma(a, b, acc);
  }
  if (jb < s) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + MM::row(lane, r);
      if (i < Ik) {
        const double v = acc[r];
        const int64_t f = (jb / spost) * ((int64_t)Ik * spost) + (int64_t)i * spost + jb % spost;
        A64[f] = v;
        Aw[f] = (W)v;
        Au[(int64_t)i * s + jb] = (W)v;
      }
    }
  }
}

hipError_t launch_backtransform(int prec, const double* Q, const double* At, int32_t Ik,
                                int32_t s, int64_t spost, double* A64, void* Aw, void* Au,
                                hipStream_t st) {
  const int tiles = ((Ik + 15) / 16) * ((s + 15) / 16);
  const int nb = (tiles + 3) / 4;
  if (prec == P_F64)
    backtransform_k<double><<<nb, 256, 0, st>>>(Q, At, Ik, s, spost, A64, (double*)Aw,
                                                (double*)Au);
  else
    backtransform_k<float><<<nb, 256, 0, st>>>(Q, At, Ik, s, spost, A64, (float*)Aw, (float*)Au);
  return hipGetLastError();
}

}  // namespace fctn
