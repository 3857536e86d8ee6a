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
#include "common.hpp"
#include "kernels.hpp"

namespace fctn {

int solve_supported(int32_t s) { return s >= 1 && s <= 192; }

template <int SB>
__global__ void __launch_bounds__(1024) solve_classes_k(const double* __restrict__ G,
                                                        const double* __restrict__ B,
                                                        const double* __restrict__ Q, int Ik,
                                                        int s, double lam, double delta,
                                                        double rho, double* __restrict__ At,
                                                        double* __restrict__ trace_part) {
  constexpr int RA = SB + 1;
  __shared__ double colbuf[2][32 * RA];
  __shared__ double rhs[2][32 * SB];
  __shared__ double diag[32 * SB];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5, lane = tid & 63, wave = tid >> 6;

  int nv = 2, v0 = 2 * c - 1, v1 = 2 * c;
  if (c == 0) {
    nv = 1; v0 = 0; v1 = 0;
  } else if ((Ik % 2 == 0) && c == Ik / 2) {
    nv = 1; v0 = Ik - 1; v1 = Ik - 1;
  }
  const double sn = sinpi((double)c / (double)Ik);
  const double Lam = delta + 4.0 * sn * sn;
  const double sigma = lam * Lam + rho;

  // b~_v[m] = sum_i Q[i][v] B[i][m]
  for (int m = wave; m < s; m += 16) {
    double p0 = 0.0, p1 = 0.0;
    for (int i = lane; i < Ik; i += 64) {
      const double b = B[(int64_t)i * s + m];
      p0 += Q[(int64_t)i * Ik + v0] * b;
      p1 += Q[(int64_t)i * Ik + v1] * b;
    }
    p0 = wave_sum(p0);
    p1 = wave_sum(p1);
    if (lane == 0) {
      rhs[0][m] = p0;
      rhs[1][m] = p1;
    }
  }
  __syncthreads();

  double H[RA][SB];
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int i = ty + 32 * a;
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      const int m = tx + 32 * b;
      double v = 0.0;
      if (i < s && m <= i) v = G[(int64_t)i * s + m] + (i == m ? sigma : 0.0);
      else if (i >= s && i < s + nv && m < s) v = rhs[i - s][m];
      H[a][b] = v;
    }
  }

  for (int j = 0; j < s; ++j) {
    const int jb = j >> 5, jt = j & 31;
    double* cb = colbuf[j & 1];
    if (tx == jt) {
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        const int i = ty + 32 * a;
        if (i >= j && i < s + nv) {
#pragma unroll
          for (int b = 0; b < SB; ++b)
            if (b == jb) cb[i] = H[a][b];
        }
      }
    }
    __syncthreads();
    const double d = cb[j];
    const double sd = sqrt(d);
    const double rs = 1.0 / sd;
    double lm[SB];
#pragma unroll
    for (int b = 0; b < SB; ++b) {
      const int m = tx + 32 * b;
      lm[b] = (m > j && m < s) ? cb[m] * rs : 0.0;
    }
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int i = ty + 32 * a;
      if (i > j && i < s + nv) {
        const double li = cb[i] * rs;
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          const int m = tx + 32 * b;
          if (m > j && m <= i && m < s) H[a][b] -= li * lm[b];
        }
      }
    }
    if (tx == jt) {
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        const int i = ty + 32 * a;
#pragma unroll
        for (int b = 0; b < SB; ++b) {
          if (b == jb) {
            if (i == j) H[a][b] = sd;
            else if (i > j && i < s + nv) H[a][b] = cb[i] * rs;
          }
        }
      }
    }
    if (tid == 0) diag[j] = sd;
  }
  __syncthreads();

  // forward-substitution results live in the appended rows: move them to rhs[]
#pragma unroll
  for (int a = 0; a < RA; ++a) {
    const int i = ty + 32 * a;
    if (i >= s && i < s + nv) {
#pragma unroll
      for (int b = 0; b < SB; ++b) {
        const int m = tx + 32 * b;
        if (m < s) rhs[i - s][m] = H[a][b];
      }
    }
  }
  __syncthreads();

  // back substitution L^T x = y: rhs[v][i] -= L[m][i] x_m for i < m
  for (int m = s - 1; m >= 0; --m) {
    if (ty == (m & 31)) {
      const int am = m >> 5;
      const double x0 = rhs[0][m] / diag[m];
      const double x1 = rhs[1][m] / diag[m];
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        if (a == am) {
#pragma unroll
          for (int b = 0; b < SB; ++b) {
            const int i = tx + 32 * b;
            if (i < m) {
              rhs[0][i] -= H[a][b] * x0;
              if (nv == 2) rhs[1][i] -= H[a][b] * x1;
            }
          }
        }
      }
    }
    __syncthreads();
  }

  double tr = 0.0;
  for (int m = tid; m < s; m += 1024) {
    const double x0 = rhs[0][m] / diag[m];
    At[(int64_t)v0 * s + m] = x0;
    tr += x0 * x0;
    if (nv == 2) {
      const double x1 = rhs[1][m] / diag[m];
      At[(int64_t)v1 * s + m] = x1;
      tr += x1 * x1;
    }
  }
  // deterministic block sum of the class's trace contribution
  __shared__ double red[16];
  tr = wave_sum(tr);
  if (lane == 0) red[wave] = tr;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    trace_part[c] = Lam * t;
  }
}

hipError_t launch_solve_classes(const double* G, const double* B, const double* Q,
                                int32_t Ik, int32_t s, double lam, double delta, double rho,
                                double* At, double* trace_part, hipStream_t st) {
  const int ncls = Ik / 2 + 1;
  const int sb = (s + 31) / 32;
  switch (sb) {
#define FCTN_SOLVE_CASE(N)                                                                 \
  case N:                                                                                  \
    solve_classes_k<N><<<ncls, 1024, 0, st>>>(G, B, Q, Ik, s, lam, delta, rho, At, trace_part); \
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

template <typename W>
__global__ void __launch_bounds__(256) backtransform_k(const double* __restrict__ Q,
                                                       const double* __restrict__ At, int Ik,
                                                       int s, int64_t spost,
                                                       double* __restrict__ A64,
                                                       W* __restrict__ Aw, W* __restrict__ Au) {
  const int64_t total = (int64_t)Ik * s;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / s), j = (int)(e % s);
    const double* q = Q + (int64_t)i * Ik;
    double acc = 0.0;
    for (int v = 0; v < Ik; ++v) acc += q[v] * At[(int64_t)v * s + j];
    const int64_t f = (j / spost) * ((int64_t)Ik * spost) + (int64_t)i * spost + j % spost;
    A64[f] = acc;
    Aw[f] = (W)acc;
    Au[e] = (W)acc;
  }
}

hipError_t launch_backtransform(int prec, const double* Q, const double* At, int32_t Ik,
                                int32_t s, int64_t spost, double* A64, void* Aw, void* Au,
                                hipStream_t st) {
  const int64_t total = (int64_t)Ik * s;
  const int nb = (int)(cdiv(total, 256) < 2048 ? cdiv(total, 256) : 2048);
  if (prec == P_F64)
    backtransform_k<double><<<nb, 256, 0, st>>>(Q, At, Ik, s, spost, A64, (double*)Aw,
                                                (double*)Au);
  else
    backtransform_k<float><<<nb, 256, 0, st>>>(Q, At, Ik, s, spost, A64, (float*)Aw, (float*)Au);
  return hipGetLastError();
}

}  // namespace fctn
