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
  __shared__ double colbuf[2][2][32 * SB];
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

  // Right-looking Cholesky, two columns per barrier.  Columns j (even) and
  // j + 1 are held by the two halves of one wave (lanes 0-31: column j, rows
  // r + 32a; lanes 32-63: column j + 1).  That wave factors both without a
  // workgroup barrier: pivot j by readlane, column j scaled and published to
  // LDS, column j + 1 updated from it (same wave, in-order LDS), pivot j + 1,
  // column j + 1 published.  After the barrier every thread applies the
  // rank-2 update to its trailing blocks.  Multipliers outside the trailing
  // range are zero, so the update needs no per-element tests (strictly upper
  // entries of diagonal blocks receive values that are never read).
  for (int j = 0; j < s; j += 2) {
    const int jb = j >> 5, jt = j & 31;
    const bool two = j + 1 < s;
    const int jlast = two ? j + 1 : j;
    double* cb0 = colbuf[(j >> 1) & 1][0];
    double* cb1 = colbuf[(j >> 1) & 1][1];
    if (wave == (jt >> 1)) {
      const int half = lane >> 5;
      // this lane's column (j or j + 1), raw
      double v[SB];
#pragma unroll
      for (int a = 0; a < SB; ++a) {
        v[a] = 0.0;
#pragma unroll
        for (int b = 0; b <= a; ++b)
          if (b == jb) v[a] = H[a][b];
      }
      double vj = 0.0;
#pragma unroll
      for (int a = 0; a < SB; ++a)
        if (a == jb) vj = v[a];
      const double d0 = bcast_lane(vj, jt);
      const double rs0 = rsqrt_f64(d0);
      const double sd0 = d0 * rs0;
#pragma unroll
      for (int a = 0; a < SB; ++a) {
        const int i = r + 32 * a;
        if (half == 0 && i > j && i < s) cb0[i] = v[a] * rs0;
      }
      double rs1 = 0.0, sd1 = 0.0;
      if (two) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const double l10 = cb0[j + 1];
#pragma unroll
        for (int a = 0; a < SB; ++a) {
          const int i = r + 32 * a;
          if (half == 1 && i > j && i < s) v[a] -= cb0[i] * l10;
        }
        double vj1 = 0.0;
#pragma unroll
        for (int a = 0; a < SB; ++a)
          if (a == jb) vj1 = v[a];
        const double d1 = bcast_lane(vj1, 32 + jt + 1);
        rs1 = rsqrt_f64(d1);
        sd1 = d1 * rs1;
#pragma unroll
        for (int a = 0; a < SB; ++a) {
          const int i = r + 32 * a;
          if (half == 1 && i > j + 1 && i < s) cb1[i] = v[a] * rs1;
        }
      }
      // the owning lanes keep their finished column of L
      const int jc = j + half;
      const double rsc = half ? rs1 : rs0, sdc = half ? sd1 : sd0;
#pragma unroll
      for (int a = 0; a < SB; ++a) {
        const int i = r + 32 * a;
#pragma unroll
        for (int b = 0; b <= a; ++b)
          if (b == jb && jc < s) H[a][b] = (i == jc) ? sdc : ((i > jc && i < s) ? v[a] * rsc : H[a][b]);
      }
      if (lane == 0) {
        diag[j] = sd0;
        rdiag[j] = rs0;
        if (two) {
          diag[j + 1] = sd1;
          rdiag[j + 1] = rs1;
        }
      }
    }
    __syncthreads();
    double lm0[SB], lm1[SB], li0[SB], li1[SB];
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      const int m = cc + 32 * b, i = r + 32 * b;
      const bool act = 32 * b + 31 > jlast;
      const bool okm = act && m > jlast && m < s, oki = act && i > jlast && i < s;
      lm0[b] = okm ? cb0[m] : 0.0;
      li0[b] = oki ? cb0[i] : 0.0;
      lm1[b] = (two && okm) ? cb1[m] : 0.0;
      li1[b] = (two && oki) ? cb1[i] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < SB; ++a) {
      if (32 * a + 31 <= jlast) continue;
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        if (32 * b + 31 <= jlast) continue;
        H[a][b] -= li0[a] * lm0[b] + li1[a] * lm1[b];
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
  // pivot entry is broadcast from its owner lane with readlane.  The next
  // step's column (row) of L and its reciprocal pivot are loaded while the
  // current step's updates run.
  if (wave == 0) {
    constexpr int NQ = (32 * SB + 63) / 64;
    double y0[NQ], y1[NQ];
    int rowbase[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      y0[q] = i < s ? rhs[0][i] : 0.0;
      y1[q] = i < s ? rhs[1][i] : 0.0;
      rowbase[q] = i * (i + 1) / 2;
    }
    // forward: column m of L is Lp[rowbase(i) + m] for i > m
    double lc[NQ], ln[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      lc[q] = (i > 0 && i < s) ? Lp[rowbase[q]] : 0.0;
    }
    double rdc = rdiag[0];
    for (int m = 0; m < s; ++m) {
      const int mn = m + 1;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        ln[q] = (mn < s && i > mn && i < s) ? Lp[rowbase[q] + mn] : 0.0;
      }
      const double rdn = mn < s ? rdiag[mn] : 0.0;
      const int owner = m & 63, qm = m >> 6;
      double ym0 = 0.0, ym1 = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (q == qm) {
          ym0 = y0[q];
          ym1 = y1[q];
        }
      const double x0 = bcast_lane(ym0, owner) * rdc;
      const double x1 = bcast_lane(ym1, owner) * rdc;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        if (i == m) {
          y0[q] = x0;
          y1[q] = x1;
        } else {
          y0[q] -= lc[q] * x0;
          y1[q] -= lc[q] * x1;
        }
        lc[q] = ln[q];
      }
      rdc = rdn;
    }
    // back: row m of L is Lp[m (m + 1) / 2 + i] for i < m
    const int ms = s - 1;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = lane + 64 * q;
      lc[q] = (i < ms) ? Lp[ms * (ms + 1) / 2 + i] : 0.0;
    }
    rdc = rdiag[ms];
    for (int m = ms; m >= 0; --m) {
      const int mn = m - 1;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        ln[q] = (mn >= 0 && i < mn) ? Lp[mn * (mn + 1) / 2 + i] : 0.0;
      }
      const double rdn = mn >= 0 ? rdiag[mn] : 0.0;
      const int owner = m & 63, qm = m >> 6;
      double ym0 = 0.0, ym1 = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        if (q == qm) {
          ym0 = y0[q];
          ym1 = y1[q];
        }
      const double x0 = bcast_lane(ym0, owner) * rdc;
      const double x1 = bcast_lane(ym1, owner) * rdc;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        if (i == m) {
          y0[q] = x0;
          y1[q] = x1;
        } else {
          y0[q] -= lc[q] * x0;
          y1[q] -= lc[q] * x1;
        }
        lc[q] = ln[q];
      }
      rdc = rdn;
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
