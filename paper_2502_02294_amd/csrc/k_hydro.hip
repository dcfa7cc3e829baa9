// Relaxing-TVD hydro sweeps and their adjoints (Sec. 2.3.1-2.3.2, eq. TVD_halfstep,
// eq. TVD_fullstep).
//
// One sweep along axis d over a full dt:
//   stage 1: F1_{j+1/2} = F^R_j - F^L_{j+1}  (first-order upwind, freezing speed at a1)
//            Uh_j = U_j - dt/2 (F1_{j+1/2} - F1_{j-1/2})
//   stage 2: F^R, F^L of Uh at a2; per wave and component
//            FRf_{j+1/2} = F^R_j + phi((F^R_j - F^R_{j-1})/2, (F^R_{j+1} - F^R_j)/2)
//            FLf_{j+1/2} = F^L_{j+1} - phi((F^L_{j+1} - F^L_j)/2, (F^L_{j+2} - F^L_{j+1})/2)
//            U'_j = U_j - dt (F2_{j+1/2} - F2_{j-1/2}),  F2 = FRf - FLf.
// Stencil: U' at j depends on U at j-3..j+3 (periodic).
//
// Kernels
//   sweep_x      x is contiguous: a block stages whole rows (512 cells) in LDS, two cells
//                per thread, so the periodic wrap stays inside the block.
//   sweep_walk   y and z: each thread owns one (x, other) column and walks a segment of S
//                cells along the pencil with a register pipeline (loads coalesced across x,
//                3-cell halos re-read from cache).
//   sweep_x_vjp  adjoint along x in LDS.
//   vjp_walk_h + vjp_finish   adjoint along y/z in two passes: the first walks the pencil
//                and writes lambda_h = dL/dUh, the second applies the stage-1 transpose
//                with a +-1 stencil.
#include "dh_kernels.h"

namespace dh {

namespace {

constexpr int kRowCells = 512;   // cells per x-sweep block (whole rows)
constexpr int kRowThreads = 256;

__device__ __forceinline__ int wrap(int j, int n) { return j & (n - 1); }

// out = in over the cells [base, base + count) of all five components (inactive samples)
__device__ __forceinline__ void copy_block(const float* __restrict__ in, float* __restrict__ out,
                                           long long nc, long long base, int count, int tid,
                                           int threads) {
  for (int i = tid; i < count; i += threads)
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c * nc + base + i] = in[c * nc + base + i];
}

// coefficients of the limited right-moving face flux FRf_m with respect to F^R at m-1, m, m+1
__device__ __forceinline__ void face_r_coef(float fm1, float f0, float fp1, float& cm1, float& c0,
                                            float& cp1) {
  float da, db;
  van_leer_d(0.5f * (f0 - fm1), 0.5f * (fp1 - f0), da, db);
  cm1 = -0.5f * da;
  c0 = 1.0f + 0.5f * da - 0.5f * db;
  cp1 = 0.5f * db;
}
// coefficients of the limited left-moving face flux FLf_m with respect to F^L at m, m+1, m+2
__device__ __forceinline__ void face_l_coef(float f0, float fp1, float fp2, float& c0, float& cp1,
                                            float& cp2) {
  float da, db;
  van_leer_d(0.5f * (fp1 - f0), 0.5f * (fp2 - fp1), da, db);
  c0 = 0.5f * da;
  cp1 = 1.0f - 0.5f * da + 0.5f * db;
  cp2 = -0.5f * db;
}

template <int D>
__device__ __forceinline__ void call_split(int d, const float* q, const HydroK& h, float* fr,
                                           float* fl) {
  split_flux<D>(q, h, fr, fl);
}

// ------------------------------------------------------------------------------- forward x
__global__ void __launch_bounds__(kRowThreads) sweep_x_kernel(const float* __restrict__ qin,
                                                              float* __restrict__ qout, int n,
                                                              long long nc,
                                                              const StepScal* __restrict__ tab) {
  __shared__ float U[5][kRowCells];
  __shared__ float FR[5][kRowCells];
  __shared__ float FL[5][kRowCells];
  const long long base = static_cast<long long>(blockIdx.x) * kRowCells;
  const int tid = threadIdx.x;
  const StepScal& sc = tab[blockIdx.y];
  qin += blockIdx.y * 5 * nc;
  qout += blockIdx.y * 5 * nc;
  if (!sc.active) {
    copy_block(qin, qout, nc, base, kRowCells, tid, kRowThreads);
    return;
  }
  const float dt = sc.dt;
  const HydroK h1 = sc.h1, h2 = sc.h2;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    U[c][tid] = qin[c * nc + base + tid];
    U[c][tid + kRowThreads] = qin[c * nc + base + tid + kRowThreads];
  }
  __syncthreads();
  const float hdt = 0.5f * dt;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
    float q[5], fr[5], fl[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) q[c] = U[c][j];
    split_flux<0>(q, h1, fr, fl);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      FR[c][j] = fr[c];
      FL[c][j] = fl[c];
    }
  }
  __syncthreads();
  float r2[2][5], l2[2][5];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
    const int row0 = j - (j & (n - 1));
    const int col = j & (n - 1);
    const int jp = row0 + wrap(col + 1, n), jm = row0 + wrap(col - 1, n);
    float qh[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const float fp = FR[c][j] - FL[c][jp];
      const float fm = FR[c][jm] - FL[c][j];
      qh[c] = U[c][j] - hdt * (fp - fm);
    }
    split_flux<0>(qh, h2, r2[r], l2[r]);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      FR[c][j] = r2[r][c];
      FL[c][j] = l2[r][c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
    const int row0 = j - (j & (n - 1));
    const int col = j & (n - 1);
    const int jm2 = row0 + wrap(col - 2, n), jm1 = row0 + wrap(col - 1, n);
    const int jp1 = row0 + wrap(col + 1, n), jp2 = row0 + wrap(col + 2, n);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const float rm2 = FR[c][jm2], rm1 = FR[c][jm1], r0 = FR[c][j], rp1 = FR[c][jp1];
      const float lm1 = FL[c][jm1], l0 = FL[c][j], lp1 = FL[c][jp1], lp2 = FL[c][jp2];
      // face j+1/2
      const float frp = r0 + van_leer(0.5f * (r0 - rm1), 0.5f * (rp1 - r0));
      const float flp = lp1 - van_leer(0.5f * (lp1 - l0), 0.5f * (lp2 - lp1));
      // face j-1/2
      const float frm = rm1 + van_leer(0.5f * (rm1 - rm2), 0.5f * (r0 - rm1));
      const float flm = l0 - van_leer(0.5f * (l0 - lm1), 0.5f * (lp1 - l0));
      qout[c * nc + base + j] = U[c][j] - dt * ((frp - flp) - (frm - flm));
    }
  }
}

// ---------------------------------------------------------------------- forward y / z walk
// Thread t: x = t % n, other = (t / n) % n, segment = t / n^2.  Column base and stride:
//   D = 1 (y): base = other*n*n + x, stride n;   D = 2 (z): base = other*n + x, stride n*n.
template <int D>
__global__ void __launch_bounds__(256) sweep_walk_kernel(const float* __restrict__ qin,
                                                         float* __restrict__ qout, int n,
                                                         long long nc, int seg_len, int nseg,
                                                         const StepScal* __restrict__ tab) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<long long>(n) * n * nseg) return;
  const int x = static_cast<int>(t % n);
  const int other = static_cast<int>((t / n) % n);
  const int seg = static_cast<int>(t / (static_cast<long long>(n) * n));
  const long long base = D == 1 ? static_cast<long long>(other) * n * n + x
                                : static_cast<long long>(other) * n + x;
  const long long stride = D == 1 ? n : static_cast<long long>(n) * n;
  const int s = seg * seg_len;
  const StepScal& sc = tab[blockIdx.y];
  qin += blockIdx.y * 5 * nc;
  qout += blockIdx.y * 5 * nc;
  if (!sc.active) {
    for (int i = 0; i < seg_len; ++i) {
      const long long off = base + static_cast<long long>(s + i) * stride;
#pragma unroll
      for (int c = 0; c < 5; ++c) qout[c * nc + off] = qin[c * nc + off];
    }
    return;
  }
  const float dt = sc.dt;
  const HydroK h1 = sc.h1, h2 = sc.h2;
  const float hdt = 0.5f * dt;

  float ut[4][5];          // U at k-3 .. k
  float r1[2][5], l1[2][5];  // stage-1 split fluxes at k-1, k
  float f1prev[5];         // F1 at (k-1)-1/2
  float r2[4][5], l2[4][5];  // stage-2 split fluxes at k-4 .. k-1
  float f2prev[5];         // F2 at (k-3)-1/2
  float nxt[5];
  {
    const long long off = base + static_cast<long long>(wrap(s - 3, n)) * stride;
#pragma unroll
    for (int c = 0; c < 5; ++c) nxt[c] = qin[c * nc + off];
  }
  const int iters = seg_len + 6;
  for (int i = 0; i < iters; ++i) {
    const int k = s - 3 + i;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int c = 0; c < 5; ++c) ut[w][c] = ut[w + 1][c];
#pragma unroll
    for (int c = 0; c < 5; ++c) ut[3][c] = nxt[c];
    if (i + 1 < iters) {
      const long long off = base + static_cast<long long>(wrap(k + 1, n)) * stride;
#pragma unroll
      for (int c = 0; c < 5; ++c) nxt[c] = qin[c * nc + off];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      r1[0][c] = r1[1][c];
      l1[0][c] = l1[1][c];
    }
    split_flux<D>(ut[3], h1, r1[1], l1[1]);
    if (i >= 1) {
      float f1[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) f1[c] = r1[0][c] - l1[1][c];   // face k-1/2
      if (i >= 2) {
        float qh[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) qh[c] = ut[2][c] - hdt * (f1[c] - f1prev[c]);  // cell k-1
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            r2[w][c] = r2[w + 1][c];
            l2[w][c] = l2[w + 1][c];
          }
        split_flux<D>(qh, h2, r2[3], l2[3]);
        if (i >= 5) {
          float f2[5];   // face (k-3)+1/2
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            const float fr = r2[1][c] + van_leer(0.5f * (r2[1][c] - r2[0][c]),
                                                 0.5f * (r2[2][c] - r2[1][c]));
            const float fl = l2[2][c] - van_leer(0.5f * (l2[2][c] - l2[1][c]),
                                                 0.5f * (l2[3][c] - l2[2][c]));
            f2[c] = fr - fl;
          }
          if (i >= 6) {
            const long long off = base + static_cast<long long>(wrap(k - 3, n)) * stride;
#pragma unroll
            for (int c = 0; c < 5; ++c) qout[c * nc + off] = ut[0][c] - dt * (f2[c] - f2prev[c]);
          }
#pragma unroll
          for (int c = 0; c < 5; ++c) f2prev[c] = f2[c];
        }
      }
#pragma unroll
      for (int c = 0; c < 5; ++c) f1prev[c] = f1[c];
    }
  }
}

// --------------------------------------------------------------------------- adjoint x
__global__ void __launch_bounds__(kRowThreads) sweep_x_vjp_kernel(
    const float* __restrict__ qin, const float* __restrict__ lam_out, float* __restrict__ lam_in,
    int n, long long nc, const StepScal* __restrict__ tab) {
  __shared__ float U[5][kRowCells];
  __shared__ float L[5][kRowCells];
  __shared__ float FR[5][kRowCells];
  __shared__ float FL[5][kRowCells];
  __shared__ float LH[5][kRowCells];
  const long long base = static_cast<long long>(blockIdx.x) * kRowCells;
  const int tid = threadIdx.x;
  const StepScal& sc = tab[blockIdx.y];
  qin += blockIdx.y * 5 * nc;
  lam_out += blockIdx.y * 5 * nc;
  lam_in += blockIdx.y * 5 * nc;
  if (!sc.active) {
    copy_block(lam_out, lam_in, nc, base, kRowCells, tid, kRowThreads);
    return;
  }
  const float dt = sc.dt;
  const HydroK h1 = sc.h1, h2 = sc.h2;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    U[c][tid] = qin[c * nc + base + tid];
    U[c][tid + kRowThreads] = qin[c * nc + base + tid + kRowThreads];
    L[c][tid] = lam_out[c * nc + base + tid];
    L[c][tid + kRowThreads] = lam_out[c * nc + base + tid + kRowThreads];
  }
  __syncthreads();
  const float hdt = 0.5f * dt;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
    float q[5], fr[5], fl[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) q[c] = U[c][j];
    split_flux<0>(q, h1, fr, fl);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      FR[c][j] = fr[c];
      FL[c][j] = fl[c];
    }
  }
  __syncthreads();
  float qh[2][5], r2[2][5], l2[2][5];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
    const int row0 = j - (j & (n - 1));
    const int col = j & (n - 1);
    const int jp = row0 + wrap(col + 1, n), jm = row0 + wrap(col - 1, n);
#pragma unroll
    for (int c = 0; c < 5; ++c)
      qh[r][c] = U[c][j] - hdt * ((FR[c][j] - FL[c][jp]) - (FR[c][jm] - FL[c][j]));
    split_flux<0>(qh[r], h2, r2[r], l2[r]);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      FR[c][j] = r2[r][c];
      FL[c][j] = l2[r][c];
    }
  }
  __syncthreads();
  // lambda_h_j = VJP of the split at Uh_j with gR_j, gL_j gathered from the faces around j.
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
    const int row0 = j - (j & (n - 1));
    const int col = j & (n - 1);
    int idx[7];
#pragma unroll
    for (int o = -3; o <= 3; ++o) idx[o + 3] = row0 + wrap(col + o, n);
    float gR[5], gL[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      float fr[5], fl[5], lm[5];
#pragma unroll
      for (int o = -2; o <= 2; ++o) {
        fr[o + 2] = FR[c][idx[o + 3]];
        fl[o + 2] = FL[c][idx[o + 3]];
      }
#pragma unroll
      for (int o = -2; o <= 2; ++o) lm[o + 2] = L[c][idx[o + 3]];
      // G2_m = dL/dF2_{m+1/2} = -dt (lambda_m - lambda_{m+1}); fr/fl/lm index o+2 <-> j+o
      float acc = 0.0f;
      {  // R faces m = j-1, j, j+1
        float a0, a1, a2;
        face_r_coef(fr[0], fr[1], fr[2], a0, a1, a2);   // m = j-1: coefficient of j is a2
        acc += -dt * (lm[1] - lm[2]) * a2;
        face_r_coef(fr[1], fr[2], fr[3], a0, a1, a2);   // m = j: coefficient of j is a1
        acc += -dt * (lm[2] - lm[3]) * a1;
        face_r_coef(fr[2], fr[3], fr[4], a0, a1, a2);   // m = j+1: coefficient of j is a0
        acc += -dt * (lm[3] - lm[4]) * a0;
      }
      gR[c] = acc;
      acc = 0.0f;
      {  // L faces m = j-2, j-1, j; dL/dFLf = -G2
        float b0, b1, b2;
        face_l_coef(fl[0], fl[1], fl[2], b0, b1, b2);   // m = j-2: coefficient of j is b2
        acc += dt * (lm[0] - lm[1]) * b2;
        face_l_coef(fl[1], fl[2], fl[3], b0, b1, b2);   // m = j-1: coefficient of j is b1
        acc += dt * (lm[1] - lm[2]) * b1;
        face_l_coef(fl[2], fl[3], fl[4], b0, b1, b2);   // m = j: coefficient of j is b0
        acc += dt * (lm[2] - lm[3]) * b0;
      }
      gL[c] = acc;
    }
    float sv[5], dv[5], out[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sv[c] = gR[c] + gL[c];
      dv[c] = gR[c] - gL[c];
    }
    split_flux_vjp<0>(qh[r], h2, sv, dv, out);
#pragma unroll
    for (int c = 0; c < 5; ++c) LH[c][j] = out[c];
  }
  __syncthreads();
  // stage-1 transpose: gR1_j = G1_{j+1/2}, gL1_j = -G1_{j-1/2}, G1_m = -dt/2 (lh_m - lh_{m+1})
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int j = tid + r * kRowThreads;
    const int row0 = j - (j & (n - 1));
    const int col = j & (n - 1);
    const int jp = row0 + wrap(col + 1, n), jm = row0 + wrap(col - 1, n);
    float q[5], sv[5], dv[5], out[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      q[c] = U[c][j];
      const float gp = -hdt * (LH[c][j] - LH[c][jp]);
      const float gm = -hdt * (LH[c][jm] - LH[c][j]);
      sv[c] = gp - gm;
      dv[c] = gp + gm;
    }
    split_flux_vjp<0>(q, h1, sv, dv, out);
#pragma unroll
    for (int c = 0; c < 5; ++c) lam_in[c * nc + base + j] = L[c][j] + LH[c][j] + out[c];
  }
}

// ----------------------------------------------------------------- adjoint y / z, pass 1
template <int D>
__global__ void __launch_bounds__(256) vjp_walk_h_kernel(const float* __restrict__ qin,
                                                         const float* __restrict__ lam_out,
                                                         float* __restrict__ lam_h, int n,
                                                         long long nc, int seg_len, int nseg,
                                                         const StepScal* __restrict__ tab) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<long long>(n) * n * nseg) return;
  const StepScal& sc = tab[blockIdx.y];
  if (!sc.active) return;
  qin += blockIdx.y * 5 * nc;
  lam_out += blockIdx.y * 5 * nc;
  lam_h += blockIdx.y * 5 * nc;
  const float dt = sc.dt;
  const HydroK h1 = sc.h1, h2 = sc.h2;
  const int x = static_cast<int>(t % n);
  const int other = static_cast<int>((t / n) % n);
  const int seg = static_cast<int>(t / (static_cast<long long>(n) * n));
  const long long base = D == 1 ? static_cast<long long>(other) * n * n + x
                                : static_cast<long long>(other) * n + x;
  const long long stride = D == 1 ? n : static_cast<long long>(n) * n;
  const int s = seg * seg_len;
  const float hdt = 0.5f * dt;

  float ut[2][5];              // U at k-1, k
  float r1[2][5], l1[2][5];    // stage-1 split at k-1, k
  float f1prev[5];
  float uh[3][5];              // Uh at k-3 .. k-1
  float r2[3][5], l2[3][5];    // stage-2 split at k-3 .. k-1
  float lm[4][5];              // lambda at k-3 .. k
  float gR[3][5], gL[3][5];    // accumulators for cells k-3 .. k-1
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      gR[w][c] = 0.0f;
      gL[w][c] = 0.0f;
    }
  const int iters = seg_len + 6;
  for (int i = 0; i < iters; ++i) {
    const int k = s - 3 + i;
    const long long off = base + static_cast<long long>(wrap(k, n)) * stride;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      ut[0][c] = ut[1][c];
      ut[1][c] = qin[c * nc + off];
      lm[0][c] = lm[1][c];
      lm[1][c] = lm[2][c];
      lm[2][c] = lm[3][c];
      lm[3][c] = lam_out[c * nc + off];
      r1[0][c] = r1[1][c];
      l1[0][c] = l1[1][c];
    }
    split_flux<D>(ut[1], h1, r1[1], l1[1]);
    if (i >= 1) {
      float f1[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) f1[c] = r1[0][c] - l1[1][c];
      if (i >= 2) {
#pragma unroll
        for (int w = 0; w < 2; ++w)
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            uh[w][c] = uh[w + 1][c];
            r2[w][c] = r2[w + 1][c];
            l2[w][c] = l2[w + 1][c];
          }
#pragma unroll
        for (int c = 0; c < 5; ++c) uh[2][c] = ut[0][c] - hdt * (f1[c] - f1prev[c]);
        split_flux<D>(uh[2], h2, r2[2], l2[2]);
        if (i >= 4) {
          // R face m = k-2 (F^R at k-3, k-2, k-1 = r2[0..2]); G2_m = -dt (lam[k-2] - lam[k-1])
          // L face m = k-3 (F^L at k-3, k-2, k-1 = l2[0..2]); dL/dFLf = dt (lam[k-3] - lam[k-2])
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            float a0, a1, a2;
            face_r_coef(r2[0][c], r2[1][c], r2[2][c], a0, a1, a2);
            const float gr = -dt * (lm[1][c] - lm[2][c]);
            gR[0][c] += gr * a0;
            gR[1][c] += gr * a1;
            gR[2][c] += gr * a2;
            face_l_coef(l2[0][c], l2[1][c], l2[2][c], a0, a1, a2);
            const float gl = dt * (lm[0][c] - lm[1][c]);
            gL[0][c] += gl * a0;
            gL[1][c] += gl * a1;
            gL[2][c] += gl * a2;
          }
          if (i >= 6) {   // cell k-3 is complete
            float sv[5], dv[5], out[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) {
              sv[c] = gR[0][c] + gL[0][c];
              dv[c] = gR[0][c] - gL[0][c];
            }
            split_flux_vjp<D>(uh[0], h2, sv, dv, out);
            const long long o3 = base + static_cast<long long>(wrap(k - 3, n)) * stride;
#pragma unroll
            for (int c = 0; c < 5; ++c) lam_h[c * nc + o3] = out[c];
          }
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            gR[0][c] = gR[1][c];
            gR[1][c] = gR[2][c];
            gR[2][c] = 0.0f;
            gL[0][c] = gL[1][c];
            gL[1][c] = gL[2][c];
            gL[2][c] = 0.0f;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 5; ++c) f1prev[c] = f1[c];
    }
  }
}

// ----------------------------------------------------------------- adjoint, pass 2 (any D)
template <int D>
__global__ void __launch_bounds__(256) vjp_finish_kernel(const float* __restrict__ qin,
                                                         const float* __restrict__ lam_out,
                                                         const float* __restrict__ lam_h,
                                                         float* __restrict__ lam_in, int n,
                                                         long long nc,
                                                         const StepScal* __restrict__ tab) {
  const long long cell = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= nc) return;
  const StepScal& sc = tab[blockIdx.y];
  qin += blockIdx.y * 5 * nc;
  lam_out += blockIdx.y * 5 * nc;
  lam_h += blockIdx.y * 5 * nc;
  lam_in += blockIdx.y * 5 * nc;
  if (!sc.active) {
#pragma unroll
    for (int c = 0; c < 5; ++c) lam_in[c * nc + cell] = lam_out[c * nc + cell];
    return;
  }
  const float dt = sc.dt;
  const HydroK h1 = sc.h1;
  const int x = static_cast<int>(cell % n);
  const int y = static_cast<int>((cell / n) % n);
  const int z = static_cast<int>(cell / (static_cast<long long>(n) * n));
  long long cp, cm;
  if (D == 0) {
    cp = cell - x + wrap(x + 1, n);
    cm = cell - x + wrap(x - 1, n);
  } else if (D == 1) {
    cp = cell + static_cast<long long>(wrap(y + 1, n) - y) * n;
    cm = cell + static_cast<long long>(wrap(y - 1, n) - y) * n;
  } else {
    cp = cell + static_cast<long long>(wrap(z + 1, n) - z) * n * n;
    cm = cell + static_cast<long long>(wrap(z - 1, n) - z) * n * n;
  }
  const float hdt = 0.5f * dt;
  float q[5], sv[5], dv[5], out[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    q[c] = qin[c * nc + cell];
    const float h0 = lam_h[c * nc + cell];
    const float gp = -hdt * (h0 - lam_h[c * nc + cp]);
    const float gm = -hdt * (lam_h[c * nc + cm] - h0);
    sv[c] = gp - gm;
    dv[c] = gp + gm;
  }
  split_flux_vjp<D>(q, h1, sv, dv, out);
#pragma unroll
  for (int c = 0; c < 5; ++c)
    lam_in[c * nc + cell] = lam_out[c * nc + cell] + lam_h[c * nc + cell] + out[c];
}

int pick_segment(int n) { return n >= 64 ? 64 : n; }

}  // namespace

void launch_sweep(hipStream_t st, const float* qin, float* qout, const Batch& b, int axis) {
  const int n = b.n;
  const long long nc = b.nc();
  if (!b.tab) throw ArgError("sweep: step table required");
  if (axis == 0) {
    if (qin == qout) throw ArgError("sweep_x: in-place not supported");
    hipLaunchKernelGGL(sweep_x_kernel, dim3(static_cast<unsigned>(nc / kRowCells), b.S),
                       dim3(kRowThreads), 0, st, qin, qout, n, nc, b.tab);
  } else {
    const int seg = pick_segment(n);
    const int nseg = n / seg;
    const long long threads = static_cast<long long>(n) * n * nseg;
    const dim3 grid(blocks_for(threads, 256), b.S);
    if (axis == 1)
      hipLaunchKernelGGL(sweep_walk_kernel<1>, grid, dim3(256), 0, st, qin, qout, n, nc, seg,
                         nseg, b.tab);
    else
      hipLaunchKernelGGL(sweep_walk_kernel<2>, grid, dim3(256), 0, st, qin, qout, n, nc, seg,
                         nseg, b.tab);
  }
  DH_LAUNCH_CHECK();
}

void launch_sweep_vjp(hipStream_t st, const float* qin, const float* lam_out, float* lam_in,
                      float* lam_h_scratch, const Batch& b, int axis) {
  const int n = b.n;
  const long long nc = b.nc();
  if (!b.tab) throw ArgError("sweep adjoint: step table required");
  if (axis == 0) {
    hipLaunchKernelGGL(sweep_x_vjp_kernel, dim3(static_cast<unsigned>(nc / kRowCells), b.S),
                       dim3(kRowThreads), 0, st, qin, lam_out, lam_in, n, nc, b.tab);
  } else {
    const int seg = pick_segment(n);
    const int nseg = n / seg;
    const long long threads = static_cast<long long>(n) * n * nseg;
    const dim3 grid(blocks_for(threads, 256), b.S), grid2(blocks_for(nc, 256), b.S);
    if (axis == 1) {
      hipLaunchKernelGGL(vjp_walk_h_kernel<1>, grid, dim3(256), 0, st, qin, lam_out,
                         lam_h_scratch, n, nc, seg, nseg, b.tab);
      DH_LAUNCH_CHECK();
      hipLaunchKernelGGL(vjp_finish_kernel<1>, grid2, dim3(256), 0, st, qin, lam_out,
                         lam_h_scratch, lam_in, n, nc, b.tab);
    } else {
      hipLaunchKernelGGL(vjp_walk_h_kernel<2>, grid, dim3(256), 0, st, qin, lam_out,
                         lam_h_scratch, n, nc, seg, nseg, b.tab);
      DH_LAUNCH_CHECK();
      hipLaunchKernelGGL(vjp_finish_kernel<2>, grid2, dim3(256), 0, st, qin, lam_out,
                         lam_h_scratch, lam_in, n, nc, b.tab);
    }
  }
  DH_LAUNCH_CHECK();
}

}  // namespace dh
