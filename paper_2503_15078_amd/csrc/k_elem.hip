// Per-node and per-tet kernels: predicted state (Sec. 3.1), pin targets, the local
// step with its right-hand-side contributions (Eq. PD local / PD global), the
// deterministic node gather of those contributions, and integration (Algorithm 4).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "lanes.hpp"

namespace lg {

// ---------------------------------------------------------------- predicted state
__global__ void k_predict(Dev d) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= d.N) return;
  const float h = (float)d.h, h2 = (float)(d.h * d.h);
  for (int c = 0; c < 3; ++c) {
    float x = d.qt[c * d.N4 + v] + h * d.vt[c * d.N4 + v] + h2 * (float)d.g[c];
    d.qp[c * d.N4 + v] = x;
    d.q[c * d.N4 + v] = x;  // q^0 = q~
  }
}

void launch_predict(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_predict, dim3((d.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

// ---------------------------------------------------------------- pin targets at t+h
// target = pivot + lin (t+h) + R(ang (t+h)) (x0 - pivot), Rodrigues' formula in float64.
__global__ void k_pins(Dev d) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.P) return;
  const double t = d.t[0] + d.h;
  const double* G = d.grp + 9 * d.pin_group[p];
  double th[3] = {G[3] * t, G[4] * t, G[5] * t};
  double a = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
  double r[3] = {d.pin_x0[p] - G[6], d.pin_x0[d.P + p] - G[7], d.pin_x0[2 * d.P + p] - G[8]};
  double out[3] = {r[0], r[1], r[2]};
  if (a > 0.0) {
    double k[3] = {th[0] / a, th[1] / a, th[2] / a};
    double sa = sin(a), ca = 1.0 - cos(a);
    double kx[3] = {k[1] * r[2] - k[2] * r[1], k[2] * r[0] - k[0] * r[2], k[0] * r[1] - k[1] * r[0]};
    double kkx[3] = {k[1] * kx[2] - k[2] * kx[1], k[2] * kx[0] - k[0] * kx[2], k[0] * kx[1] - k[1] * kx[0]};
    for (int c = 0; c < 3; ++c) out[c] = r[c] + sa * kx[c] + ca * kkx[c];
  }
  int v = d.pin_node[p];
  for (int c = 0; c < 3; ++c) d.tgt[c * d.N4 + v] = (float)(G[6 + c] + G[c] * t + out[c]);
}

void launch_pins(const Dev& d, hipStream_t st) {
  if (d.P == 0) return;
  hipLaunchKernelGGL(k_pins, dim3((d.P + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

// ---------------------------------------------------------------- 3x3 SVD (float32)
// Rotation-variant SVD F = U diag(s) V^T with det U = det V = +1: cyclic Jacobi on
// F^T F for V, columns of B = F V sorted by norm, then a Givens QR of B for U and s
// (the smallest singular value carries the sign of det F).
// Reciprocal, reciprocal square root and square root by the hardware's approximations
// (about 1 ulp) instead of the correctly rounded sequences: the local step is a long
// dependent chain per tet, and float32 rounding of these steps is far inside the
// tolerance of the method.
__device__ inline float rcp1(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline float rsq1(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline float sqrt1(float x) { return __builtin_amdgcn_sqrtf(x); }

__device__ inline void jacobi_rot(float S[3][3], float V[3][3], int p, int q) {
  float apq = S[p][q];
  if (fabsf(apq) <= 1e-30f) return;
  float theta = (S[q][q] - S[p][p]) * (0.5f * rcp1(apq));
  float t = copysignf(rcp1(fabsf(theta) + sqrt1(theta * theta + 1.0f)), theta);
  float c = rsq1(t * t + 1.0f), s = t * c;
  int r = 3 - p - q;
  float srp = S[r][p], srq = S[r][q];
  S[p][p] -= t * apq;
  S[q][q] += t * apq;
  S[p][q] = S[q][p] = 0.0f;
  S[r][p] = S[p][r] = c * srp - s * srq;
  S[r][q] = S[q][r] = s * srp + c * srq;
  for (int k = 0; k < 3; ++k) {
    float a = V[k][p], b = V[k][q];
    V[k][p] = c * a - s * b;
    V[k][q] = s * a + c * b;
  }
}

__device__ inline void givens_rows(float B[3][3], float U[3][3], int i, int k, int col) {
  float a = B[i][col], b = B[k][col];
  float r2 = a * a + b * b;
  float c = 1.0f, s = 0.0f;
  if (r2 > 1e-35f) {  // a pair below ~3e-18 is left as it is
    float ir = rsq1(r2);
    c = a * ir;
    s = b * ir;
  }
  for (int j = 0; j < 3; ++j) {
    float bi = B[i][j], bk = B[k][j];
    B[i][j] = c * bi + s * bk;
    B[k][j] = -s * bi + c * bk;
    float ui = U[j][i], uk = U[j][k];
    U[j][i] = c * ui + s * uk;
    U[j][k] = -s * ui + c * uk;
  }
}

__device__ inline void swap_cols(float A[3][3], int i, int j) {
  for (int k = 0; k < 3; ++k) {
    float t = A[k][i];
    A[k][i] = A[k][j];
    A[k][j] = -t;  // negate one column: keeps the determinant
  }
}

__device__ void svd3(const float F[3][3], float U[3][3], float s[3], float V[3][3]) {
  float S[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
      V[i][j] = (i == j) ? 1.0f : 0.0f;
    }
  // four cyclic sweeps: on float32 3x3 matrices the eigenvalues are then within float32
  // rounding (~3e-7 relative) of an exact SVD, as with more sweeps
  for (int sweep = 0; sweep < 4; ++sweep) {
    jacobi_rot(S, V, 0, 1);
    jacobi_rot(S, V, 0, 2);
    jacobi_rot(S, V, 1, 2);
  }
  float B[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[i][j] = F[i][0] * V[0][j] + F[i][1] * V[1][j] + F[i][2] * V[2][j];
  float n0 = B[0][0] * B[0][0] + B[1][0] * B[1][0] + B[2][0] * B[2][0];
  float n1 = B[0][1] * B[0][1] + B[1][1] * B[1][1] + B[2][1] * B[2][1];
  float n2 = B[0][2] * B[0][2] + B[1][2] * B[1][2] + B[2][2] * B[2][2];
  if (n0 < n1) {
    swap_cols(B, 0, 1);
    swap_cols(V, 0, 1);
    float t = n0; n0 = n1; n1 = t;
  }
  if (n0 < n2) {
    swap_cols(B, 0, 2);
    swap_cols(V, 0, 2);
    float t = n0; n0 = n2; n2 = t;
  }
  if (n1 < n2) {
    swap_cols(B, 1, 2);
    swap_cols(V, 1, 2);
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) U[i][j] = (i == j) ? 1.0f : 0.0f;
  givens_rows(B, U, 0, 1, 0);
  givens_rows(B, U, 0, 2, 0);
  givens_rows(B, U, 1, 2, 1);
  s[0] = B[0][0];
  s[1] = B[1][1];
  s[2] = B[2][2];
}

// ---------------------------------------------------------------- energies on s
// COROT  psi = mu sum (s-1)^2 + lam/2 (J-1)^2
// SNH    psi = mu/2 (Ic-3) + lam/2 (J-alpha)^2 - mu/2 log(Ic+1), alpha = 1 + 3mu/(4lam)
// MR     psi = c (J^-2/3 I1 - 3) + c (J^-4/3 I2 - 3) + kap/2 (J-1)^2, c = mu/4,
//        kap = lam + 2mu/3, J clamped below at 1e-4 in the isochoric factors
// psi, and in mag the sum of the magnitudes of its terms: the scale of its float32
// rounding error, which cancellation between the terms can leave far above |psi|
__device__ float psi_m(int model, const float s[3], float mu, float lam, float& mag) {
  float J = s[0] * s[1] * s[2];
  float I1 = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
  if (model == 1) {
    float a = s[0] - 1.0f, b = s[1] - 1.0f, c = s[2] - 1.0f;
    float v = mu * (a * a + b * b + c * c) + 0.5f * lam * (J - 1.0f) * (J - 1.0f);
    mag = v;
    return v;
  }
  if (model == 2) {
    float alpha = 1.0f + 0.75f * mu * rcp1(lam);
    float vol = 0.5f * lam * (J - alpha) * (J - alpha), lg = 0.5f * mu * __logf(I1 + 1.0f);
    mag = 0.5f * mu * (I1 + 3.0f) + vol + fabsf(lg);
    return 0.5f * mu * (I1 - 3.0f) + vol - lg;
  }
  float q0 = s[0] * s[0], q1 = s[1] * s[1], q2 = s[2] * s[2];
  float I2 = q0 * q1 + q0 * q2 + q1 * q2;
  float Jh = fmaxf(J, 1e-4f);
  float jm23 = 1.0f / (cbrtf(Jh) * cbrtf(Jh));
  float c10 = 0.25f * mu, kap = lam + 2.0f * mu / 3.0f;
  float vol = 0.5f * kap * (J - 1.0f) * (J - 1.0f);
  mag = c10 * (jm23 * I1 + 3.0f) + c10 * (jm23 * jm23 * I2 + 3.0f) + vol;
  return c10 * (jm23 * I1 - 3.0f) + c10 * (jm23 * jm23 * I2 - 3.0f) + vol;
}
__device__ inline float psi(int model, const float s[3], float mu, float lam) {
  float mag;
  return psi_m(model, s, mu, lam, mag);
}

__device__ void psi_grad_hess(int model, const float s[3], float mu, float lam, float g[3], float H[3][3]) {
  float J = s[0] * s[1] * s[2];
  float Ji[3] = {s[1] * s[2], s[0] * s[2], s[0] * s[1]};
  float Jij[3][3] = {{0.0f, s[2], s[1]}, {s[2], 0.0f, s[0]}, {s[1], s[0], 0.0f}};
  if (model == 1) {
    for (int i = 0; i < 3; ++i) {
      g[i] = 2.0f * mu * (s[i] - 1.0f) + lam * (J - 1.0f) * Ji[i];
      for (int j = 0; j < 3; ++j)
        H[i][j] = (i == j ? 2.0f * mu : 0.0f) + lam * Ji[i] * Ji[j] + lam * (J - 1.0f) * Jij[i][j];
    }
    return;
  }
  if (model == 2) {
    float alpha = 1.0f + 0.75f * mu * rcp1(lam);
    float I1 = s[0] * s[0] + s[1] * s[1] + s[2] * s[2];
    float qi = rcp1(I1 + 1.0f);
    for (int i = 0; i < 3; ++i) {
      g[i] = mu * s[i] + lam * (J - alpha) * Ji[i] - mu * qi * s[i];
      for (int j = 0; j < 3; ++j)
        H[i][j] = (i == j ? mu - mu * qi : 0.0f) + lam * Ji[i] * Ji[j] + lam * (J - alpha) * Jij[i][j] +
                  2.0f * mu * qi * qi * s[i] * s[j];
    }
    return;
  }
  // Mooney-Rivlin
  float c10 = 0.25f * mu, kap = lam + 2.0f * mu / 3.0f;
  float q[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
  float I1 = q[0] + q[1] + q[2];
  float I2 = q[0] * q[1] + q[0] * q[2] + q[1] * q[2];
  bool active = J > 1e-4f;
  float Jh = fmaxf(J, 1e-4f);
  float jm13 = 1.0f / cbrtf(Jh);
  for (int i = 0; i < 3; ++i) {
    g[i] = kap * (J - 1.0f) * Ji[i];
    for (int j = 0; j < 3; ++j) H[i][j] = kap * Ji[i] * Ji[j] + kap * (J - 1.0f) * Jij[i][j];
  }
  for (int term = 0; term < 2; ++term) {
    float a = term == 0 ? -2.0f / 3.0f : -4.0f / 3.0f;
    float Ja = term == 0 ? jm13 * jm13 : jm13 * jm13 * jm13 * jm13;
    float X = term == 0 ? I1 : I2;
    float Xi[3], Xij[3][3];
    for (int i = 0; i < 3; ++i) {
      Xi[i] = term == 0 ? 2.0f * s[i] : 2.0f * s[i] * (I1 - q[i]);
      for (int j = 0; j < 3; ++j)
        Xij[i][j] = term == 0 ? (i == j ? 2.0f : 0.0f) : (i == j ? 2.0f * (I1 - q[i]) : 4.0f * s[i] * s[j]);
    }
    float A1 = active ? a * Ja / Jh : 0.0f;                 // a J^(a-1)
    float A2 = active ? a * (a - 1.0f) * Ja / (Jh * Jh) : 0.0f;
    for (int i = 0; i < 3; ++i) {
      g[i] += c10 * (Ja * Xi[i] + A1 * X * Ji[i]);
      for (int j = 0; j < 3; ++j)
        H[i][j] += c10 * (Ja * Xij[i][j] + A2 * X * Ji[i] * Ji[j] + A1 * X * Jij[i][j] +
                          A1 * (Ji[i] * Xi[j] + Xi[i] * Ji[j]));
    }
  }
}

__device__ inline bool chol3_solve(const float K[3][3], float tau, const float rhs[3], float x[3]) {
  // pivots below 1e-30 count as failures (the caller then shifts the diagonal)
  float a00 = K[0][0] + tau, a11 = K[1][1] + tau, a22 = K[2][2] + tau;
  if (!(a00 > 1e-30f)) return false;
  float i00 = rsq1(a00);
  float l10 = K[1][0] * i00, l20 = K[2][0] * i00;
  float d1 = a11 - l10 * l10;
  if (!(d1 > 1e-30f)) return false;
  float i11 = rsq1(d1);
  float l21 = (K[2][1] - l20 * l10) * i11;
  float d2 = a22 - l20 * l20 - l21 * l21;
  if (!(d2 > 1e-30f)) return false;
  float i22 = rsq1(d2);
  float z0 = rhs[0] * i00, z1 = (rhs[1] - l10 * z0) * i11, z2 = (rhs[2] - l20 * z0 - l21 * z1) * i22;
  x[2] = z2 * i22;
  x[1] = (z1 - l21 * x[2]) * i11;
  x[0] = (z0 - l10 * x[1] - l20 * x[2]) * i00;
  return true;
}

// s* = argmin k/2 |s - sigma|^2 + psi(s): Newton from sigma with the shifted-Hessian
// rule (tau = 0, 1e-2 k, 1e-1 k, ...) and Armijo halving, at most 8 iterations.  The
// objective is evaluated in float32, so a decrease below its rounding error cannot be
// tested: the Armijo test allows 8 ulp of the magnitude of the objective's terms.
// Without that allowance, steps near the minimiser are rejected on rounding noise: the
// line search halves the step to nothing and Newton stops early or runs to its cap
// farther from the minimiser, while every lane of the wavefront waits.
__device__ void prox3(int model, const float sig[3], float mu, float lam, float k, float s[3]) {
  s[0] = sig[0];
  s[1] = sig[1];
  s[2] = sig[2];
  if (model == 0) {
    s[0] = s[1] = s[2] = 1.0f;
    return;
  }
  constexpr float kRound = 8.0f * 1.1920929e-7f;  // 8 ulp (float32 epsilon 2^-23)
  float scale = fmaxf(1.0f, fmaxf(fabsf(sig[0]), fmaxf(fabsf(sig[1]), fabsf(sig[2]))));
  float f0 = 0.0f, m0 = 0.0f;  // objective at s and the magnitude of its terms
  bool have_f0 = false;
  for (int it = 0; it < 8; ++it) {
    float g[3], H[3][3];
    psi_grad_hess(model, s, mu, lam, g, H);
    for (int i = 0; i < 3; ++i) {
      g[i] += k * (s[i] - sig[i]);
      H[i][i] += k;
    }
    float gn = fmaxf(fabsf(g[0]), fmaxf(fabsf(g[1]), fabsf(g[2])));
    if (gn <= 2e-6f * k * scale) break;
    float dx[3];
    float ng[3] = {-g[0], -g[1], -g[2]};
    float tau = 0.0f;
    bool ok = false;
    for (int tries = 0; tries < 12 && !ok; ++tries) {
      ok = chol3_solve(H, tau, ng, dx);
      if (!ok) tau = (tau == 0.0f) ? 1e-2f * k : 10.0f * tau;
    }
    if (!ok) break;
    float slope = g[0] * dx[0] + g[1] * dx[1] + g[2] * dx[2];
    if (!have_f0) {  // later iterations start from the accepted line-search value
      float a = s[0] - sig[0], b = s[1] - sig[1], c = s[2] - sig[2];
      const float prox = 0.5f * k * (a * a + b * b + c * c);
      f0 = psi_m(model, s, mu, lam, m0) + prox;
      m0 += prox;
      have_f0 = true;
    }
    float t = 1.0f;
    bool acc = false;
    for (int ls = 0; ls < 10; ++ls) {
      float tr[3] = {s[0] + t * dx[0], s[1] + t * dx[1], s[2] + t * dx[2]};
      float a = tr[0] - sig[0], b = tr[1] - sig[1], c = tr[2] - sig[2];
      const float prox = 0.5f * k * (a * a + b * b + c * c);
      float m1;
      float f1 = psi_m(model, tr, mu, lam, m1) + prox;
      if (f1 <= f0 + 1e-4f * t * slope + kRound * m0) {
        s[0] = tr[0];
        s[1] = tr[1];
        s[2] = tr[2];
        f0 = f1;
        m0 = m1 + prox;
        acc = true;
        break;
      }
      t *= 0.5f;
    }
    if (!acc) break;
  }
}

// ---------------------------------------------------------------- local step + RHS
// Per tet: F = sum_{a=1..3} (x_a - x_0) d_a^T at q^k and at q~, p = prox(F), and the
// delta-form contribution P = h^2 w (p - F(q~)) scattered as corner forces P d_a
// (so that the global step solves for q - q~).
// FORM: 0 projective dynamics, 1 ADMM-PD (one instantiation each, so that the PD form
// carries no dual registers)
template <int FORM>
__global__ void __launch_bounds__(kBlock) k_element(Dev d) {
  if (frame_done(d)) return;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.M) return;
  int vi[4];
  for (int a = 0; a < 4; ++a) vi[a] = d.tidx[a * d.M + t];
  float D[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) D[a][c] = d.dinv[(3 * a + c) * d.M + t];
  float F[3][3], Fp[3][3];
  float e[3][3], ep[3][3];
  for (int c = 0; c < 3; ++c) {
    float x0 = d.q[c * d.N4 + vi[0]], p0 = d.qp[c * d.N4 + vi[0]];
    for (int a = 0; a < 3; ++a) {
      e[a][c] = d.q[c * d.N4 + vi[a + 1]] - x0;
      ep[a][c] = d.qp[c * d.N4 + vi[a + 1]] - p0;
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      F[i][j] = e[0][i] * D[0][j] + e[1][i] * D[1][j] + e[2][i] * D[2][j];
      Fp[i][j] = ep[0][i] * D[0][j] + ep[1][i] * D[1][j] + ep[2][i] * D[2][j];
    }
  // ADMM-PD: project F + u (u the tet's dual), then u += F - p and the global step takes
  // p - u; PD projects F itself
  constexpr bool admm = FORM == 1;
  float Fz[3][3], du[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      du[i][j] = admm ? d.dual[(3 * i + j) * d.M + t] : 0.0f;
      Fz[i][j] = F[i][j] + du[i][j];
    }
  float U[3][3], V[3][3], sig[3], s[3];
  svd3(Fz, U, sig, V);
  int model = d.tmodel[t];
  if (admm && model == 0) {  // ARAP's energy mu |F - R|^2 (weight w = 2 mu V): s* = (sigma + 1) / 2
    for (int i = 0; i < 3; ++i) s[i] = 0.5f * (sig[i] + 1.0f);
  } else {
    prox3(model, sig, d.tmu[t], d.tlam[t], d.tk[t], s);
  }
  float hw = d.hw[t];
  float P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      float pij = U[i][0] * s[0] * V[j][0] + U[i][1] * s[1] * V[j][1] + U[i][2] * s[2] * V[j][2];
      if (admm) {
        const float un = du[i][j] + F[i][j] - pij;
        d.dual[(3 * i + j) * d.M + t] = un;
        pij -= un;
      }
      P[i][j] = hw * (pij - Fp[i][j]);
    }
  float f0[3] = {0.0f, 0.0f, 0.0f};
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      float fa = P[c][0] * D[a][0] + P[c][1] * D[a][1] + P[c][2] * D[a][2];
      d.fc[((a + 1) * 3 + c) * d.M + t] = fa;
      f0[c] -= fa;
    }
  for (int c = 0; c < 3; ++c) d.fc[c * d.M + t] = f0[c];
}

__global__ void k_zero_dual(Dev d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.M) return;
  for (int q = 0; q < 9; ++q) d.dual[q * d.M + t] = 0.0f;
}

// ADMM-PD duals start every frame at zero (a kernel, so that captured frames clear them)
void launch_zero_dual(const Dev& d, hipStream_t st) {
  if (d.lg_form != 1) return;
  hipLaunchKernelGGL(k_zero_dual, dim3((d.M + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

void launch_element(const Dev& d, hipStream_t st) {
  const int bs = d.elem_block > 0 ? d.elem_block : kBlock;
  if (d.lg_form == 1) hipLaunchKernelGGL(k_element<1>, dim3((d.M + bs - 1) / bs), dim3(bs), 0, st, d);
  else hipLaunchKernelGGL(k_element<0>, dim3((d.M + bs - 1) / bs), dim3(bs), 0, st, d);
}

// ---------------------------------------------------------------- L-G objective
// The objective the local-global iteration minimises at the current iterate q, at its
// optimal local variables (Eq. PD local and PD global):
//   1/2 (q - q~)^T M (q - q~) + h^2 sum_t [w_t/2 |F_t - p_t|^2 + V_t psi(p_t)]
//   + 1/2 sum_pins h^2 w_pin |q_v - target|^2,
// with p_t the prox of F_t (same singular vectors, so |F_t - p_t|^2 = |sigma - s*|^2;
// ARAP: psi is the indicator of SO(3), zero at s* = 1).  Blocks [0, nbt) sum tets,
// the rest nodes; each block writes one float64 partial (fixed-order tree sum).
__global__ void __launch_bounds__(kBlock) k_lg_energy(Dev d, int nbt, double* part) {
  __shared__ double red[kBlock];
  double e = 0.0;
  if ((int)blockIdx.x < nbt) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < d.M) {
      float D[3][3], F[3][3], e3[3][3];
      int vi[4];
      for (int a = 0; a < 4; ++a) vi[a] = d.tidx[a * d.M + t];
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) D[a][c] = d.dinv[(3 * a + c) * d.M + t];
      for (int c = 0; c < 3; ++c) {
        const float x0 = d.q[c * d.N4 + vi[0]];
        for (int a = 0; a < 3; ++a) e3[a][c] = d.q[c * d.N4 + vi[a + 1]] - x0;
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) F[i][j] = e3[0][i] * D[0][j] + e3[1][i] * D[1][j] + e3[2][i] * D[2][j];
      float U[3][3], V[3][3], sig[3], s[3];
      svd3(F, U, sig, V);
      const int model = d.tmodel[t];
      prox3(model, sig, d.tmu[t], d.tlam[t], d.tk[t], s);
      const double hw = d.hw[t];
      double dist = 0.0;
      for (int i = 0; i < 3; ++i) dist += (double)(sig[i] - s[i]) * (double)(sig[i] - s[i]);
      e = 0.5 * hw * dist;
      if (model != 0) e += hw / (double)d.tk[t] * (double)psi(model, s, d.tmu[t], d.tlam[t]);
    }
  } else {
    const int v = (blockIdx.x - nbt) * kBlock + threadIdx.x;
    if (v < d.N) {
      const double m = 1.0 / (double)d.inv_mass[v], w = d.pin_w[v];
      for (int c = 0; c < 3; ++c) {
        const double dq = (double)d.q[c * d.N4 + v] - (double)d.qp[c * d.N4 + v];
        e += 0.5 * m * dq * dq;
        if (w > 0.0) {
          const double r = (double)d.q[c * d.N4 + v] - (double)d.tgt[c * d.N4 + v];
          e += 0.5 * w * r * r;
        }
      }
    }
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

int lg_energy_blocks(const Dev& d) { return (d.M + kBlock - 1) / kBlock + (d.N + kBlock - 1) / kBlock; }

void launch_lg_energy(const Dev& d, hipStream_t st, double* part) {
  const int nbt = (d.M + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_lg_energy, dim3(lg_energy_blocks(d)), dim3(kBlock), 0, st, d, nbt, part);
}

// ---------------------------------------------------------------- node gather
// b'_v = sum of the corner forces of v + h^2 w_pin (target - q~_v).  Eight lanes per
// node: lane l adds slots l, l+8, ... in order, then the eight partial sums are combined
// by a fixed butterfly, so the result does not depend on timing.
constexpr int kGatherLanes = 8;
__global__ void k_gather(Dev d) {
  if (frame_done(d)) return;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = gid / kGatherLanes, l = gid % kGatherLanes;
  const bool ok = v < d.N;  // whole groups of 8 lanes share v, so the butterfly stays in range
  float acc[3] = {0.0f, 0.0f, 0.0f};
  if (ok) {
    // the node's corner forces, three per lane in flight, added in list order per lane
    const int e = d.g_ptr[v + 1];
    constexpr int U = 3;
    for (int p0 = d.g_ptr[v] + l; p0 < e; p0 += U * kGatherLanes) {
      int base[U];
#pragma unroll
      for (int u = 0; u < U; ++u) base[u] = p0 + u * kGatherLanes < e ? d.g_slot[p0 + u * kGatherLanes] : -1;
      float f[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < 3; ++c) f[u][c] = base[u] >= 0 ? d.fc[base[u] + c * d.M] : 0.0f;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (base[u] >= 0)
          for (int c = 0; c < 3; ++c) acc[c] += f[u][c];
    }
  }
  static_assert(kGatherLanes == 8, "one node per half row of 8 lanes");
  for (int c = 0; c < 3; ++c) acc[c] = sum8(acc[c]);
  if (!ok || l != 0) return;
  float w = d.pin_w[v];
  if (w != 0.0f)
    for (int c = 0; c < 3; ++c) acc[c] += w * (d.tgt[c * d.N4 + v] - d.qp[c * d.N4 + v]);
  for (int c = 0; c < 3; ++c) d.b[c * d.N4 + v] = acc[c];
}

void launch_gather(const Dev& d, hipStream_t st) {
  const int64_t threads = (int64_t)d.N * kGatherLanes;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, d);
}

// ---------------------------------------------------------------- finiteness check
__global__ void k_check_finite(Dev d) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (v < d.N)
    for (int c = 0; c < 3; ++c) bad |= !isfinite(d.q[c * d.N4 + v]);
  if (bad) atomicOr(d.bad, 1);
}

void launch_check_finite(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_check_finite, dim3((d.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

// ---------------------------------------------------------------- integration
// v = (q - q_t)/h, q_t = q (Algorithm 4, last two lines); skipped if the frame
// produced a non-finite state.  Also advances the simulation time.
__global__ void k_integrate(Dev d) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (d.bad[0] || d.overflow[0]) return;
  if (v == 0) d.t[0] += d.h;  // no thread of this kernel reads the time
  if (v < d.N) {
    const float ih = (float)(1.0 / d.h);
    for (int c = 0; c < 3; ++c) {
      float x = d.q[c * d.N4 + v];
      d.vt[c * d.N4 + v] = (x - d.qt[c * d.N4 + v]) * ih;
      d.qt[c * d.N4 + v] = x;
    }
  }
}

// Save the frame's contacts (key and world-space impulse) for the next warm start.
__global__ void k_save_contacts(Dev d) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (d.bad[0] || d.overflow[0]) return;
  int c = min(d.n_contacts[0], d.CMAX);
  if (j == 0) {
    d.pc_count[0] = c;
    d.pc_count[1] = d.self_on ? min(d.n_obst_c[0], c) : c;  // the sorted single-node part
  }
  if (j >= c) return;
  d.pc_node[j] = d.c_node[j];
  d.pc_obst[j] = d.c_obst[j];
  float l[3] = {d.lam[j], d.lam[d.CMAX + j], d.lam[2 * d.CMAX + j]};
  for (int i = 0; i < 3; ++i)
    d.pc_world[i * d.CMAX + j] = d.cC[(0 * 3 + i) * d.CMAX + j] * l[0] + d.cC[(1 * 3 + i) * d.CMAX + j] * l[1] +
                                 d.cC[(2 * 3 + i) * d.CMAX + j] * l[2];
}

void launch_integrate(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_save_contacts, dim3((d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_integrate, dim3((d.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

// positions (q_t) in caller order, float32 [3][N]
__global__ void k_export_positions(Dev d, float* out) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= d.N) return;
  int ci = d.iperm_caller[v];
  for (int c = 0; c < 3; ++c) out[c * d.N + ci] = d.qt[c * d.N4 + v];
}

void launch_export_positions(const Dev& d, hipStream_t st, float* out) {
  hipLaunchKernelGGL(k_export_positions, dim3((d.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d, out);
}

}  // namespace lg
