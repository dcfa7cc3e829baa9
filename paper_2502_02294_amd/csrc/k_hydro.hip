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
//   sweep_x      x is contiguous: a block stages whole rows (512 cells) in LDS, one cell
//                per thread, so the periodic wrap stays inside the block.
//   sweep_walk   y and z: each thread owns one (x, other) column and walks a segment of S
//                cells along the pencil with a register pipeline (loads coalesced across x,
//                two cells prefetched, 3-cell halos re-read from cache).
//   sweep_x_vjp  adjoint along x in LDS.
//   vjp_walk_h + vjp_finish   adjoint along y/z in two passes: the first walks the pencil
//                and writes lambda_h = dL/dUh, the second applies the stage-1 transpose
//                with a +-1 stencil.
#include "dh_kernels.h"

namespace dh {

namespace {

constexpr int kRowCells = 512;   // cells per x-sweep block (whole rows), one per thread
constexpr int kRowThreads = kRowCells;

__device__ __forceinline__ int wrap(int j, int n) { return j & (n - 1); }

// out = in over the cells [base, base + count) of all five components (inactive samples)
template <int NQ>
__device__ __forceinline__ void copy_block(const float* __restrict__ in, float* __restrict__ out,
                                           long long nc, long long base, int count, int tid,
                                           int threads) {
  for (int i = tid; i < count; i += threads)
#pragma unroll
    for (int c = 0; c < NQ; ++c) out[c * nc + base + i] = in[c * nc + base + i];
}

// coefficients of the limited right-moving face flux FRf_m = F_m + phi((F_m - F_{m-1})/2,
// (F_{m+1} - F_m)/2) with respect to F^R at m-1, m, m+1
__device__ __forceinline__ void face_r_coef(float fm1, float f0, float fp1, float& cm1, float& c0,
                                            float& cp1) {
  float da, db;
  van_leer_half_d(f0 - fm1, fp1 - f0, da, db);
  cm1 = -da;
  c0 = 1.0f + da - db;
  cp1 = db;
}
// coefficients of the limited left-moving face flux FLf_m = F_{m+1} - phi((F_{m+1} - F_m)/2,
// (F_{m+2} - F_{m+1})/2) with respect to F^L at m, m+1, m+2
__device__ __forceinline__ void face_l_coef(float f0, float fp1, float fp2, float& c0, float& cp1,
                                            float& cp2) {
  float da, db;
  van_leer_half_d(fp1 - f0, fp2 - fp1, da, db);
  c0 = da;
  cp1 = 1.0f - da + db;
  cp2 = -db;
}

// ------------------------------------------------------------------------------- forward x
// Whole rows in LDS, one cell per thread; the limited stage-2 flux is formed once per face.
// KICK (the first sweep of a step): the opening gas half kick with g4 and the table's h is
// applied to each cell as it is loaded (the reverse pass applies it again, so the kicked state
// is not stored).
template <bool KICK, int NQ>
__global__ void __launch_bounds__(kRowThreads) sweep_x_kernel(const float* __restrict__ qin,
                                                              float* __restrict__ qout, int n,
                                                              long long nc,
                                                              const StepScal* __restrict__ tab,
                                                              const float4* __restrict__ g4) {
  __shared__ float FR[NQ][kRowCells];
  __shared__ float FL[NQ][kRowCells];
  const long long base = static_cast<long long>(blockIdx.x) * kRowCells;
  const int j = threadIdx.x;
  const StepScal& sc = tab[blockIdx.y];
  qin += blockIdx.y * NQ * nc;
  qout += blockIdx.y * NQ * nc;
  if (!sc.active) {
    copy_block<NQ>(qin, qout, nc, base, kRowCells, j, kRowThreads);
    return;
  }
  const float dt = sc.dt;
  const HydroK h1 = sc.h1, h2 = sc.h2;
  const float hdt = 0.5f * dt;
  const int row0 = j - (j & (n - 1)), col = j & (n - 1);
  const int jm = row0 + wrap(col - 1, n), jp = row0 + wrap(col + 1, n);
  const int jpp = row0 + wrap(col + 2, n);
  float u[NQ], fr[NQ], fl[NQ];
#pragma unroll
  for (int c = 0; c < NQ; ++c) u[c] = qin[c * nc + base + j];
  if (KICK) {
    float m[3] = {u[1], u[2], u[3]};
    kick_cell(u[0], g4[blockIdx.y * nc + base + j], sc.h, m, u[4]);
    u[1] = m[0];
    u[2] = m[1];
    u[3] = m[2];
  }
  split_flux<0, NQ>(u, h1, fr, fl);
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    FR[c][j] = fr[c];
    FL[c][j] = fl[c];
  }
  __syncthreads();
  float qh[NQ];
#pragma unroll
  for (int c = 0; c < NQ; ++c)
    qh[c] = u[c] - hdt * ((fr[c] - FL[c][jp]) - (FR[c][jm] - fl[c]));
  split_flux<0, NQ>(qh, h2, fr, fl);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    FR[c][j] = fr[c];
    FL[c][j] = fl[c];
  }
  __syncthreads();
  float f2[NQ];   // limited stage-2 flux of face j+1/2
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const float rm1 = FR[c][jm], r0 = fr[c], rp1 = FR[c][jp];
    const float l0 = fl[c], lp1 = FL[c][jp], lp2 = FL[c][jpp];
    f2[c] = (r0 + van_leer_half(r0 - rm1, rp1 - r0)) - (lp1 - van_leer_half(lp1 - l0, lp2 - lp1));
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NQ; ++c) FR[c][j] = f2[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NQ; ++c) qout[c * nc + base + j] = u[c] - dt * (f2[c] - FR[c][jm]);
}

// ---------------------------------------------------------------------- forward y / z walk
// Thread t: x = t % n, other = (t / n) % n, segment = t / n^2.  Column base and stride:
//   D = 1 (y): base = other*n*n + x, stride n;   D = 2 (z): base = other*n + x, stride n*n.
// The thread visits cells k = s-3 .. s+seg+2; at visit i (cell k = s-3+i) it loads cell
// k+kAhead, splits U_k, forms the stage-1 face k-1/2, the half step and stage-2 split of cell
// k-1, the limited stage-2 face (k-3)+1/2 and the update of cell k-3.  Every carried quantity
// sits in a ring indexed by the visit number, so with the visits unrolled eight at a time all
// ring slots are compile-time registers and nothing is shifted.  Offsets within one component
// of a sample are 32-bit (at most 256^3 floats).
constexpr int kAhead = 4;   // cells loaded ahead of the one being split

// The opening gas kick applied to a loaded state in place (the first sweep of a step).  The
// walks load g two (forward) or one (adjoint) visits before a cell is first used and kick it
// then: kicking on load would make a visit wait for the loads of the cells ahead.
template <int NQ>
__device__ __forceinline__ void kick_loaded(float (&u)[NQ], const float (&g)[3], float h) {
  float m[3] = {u[1], u[2], u[3]};
  kick_cell(u[0], make_float4(g[0], g[1], g[2], 0.0f), h, m, u[4]);
  u[1] = m[0];
  u[2] = m[1];
  u[3] = m[2];
}

template <int D, int NQ>
struct WalkFwd {
  float u[8][NQ];             // U of cell k - j in slot (i - j) & 7 (j = -kAhead .. 3)
  float r1[2][NQ];            // stage-1 F^R of cell k - j in slot (i - j) & 1
  float f1[2][NQ];            // stage-1 face flux (k - j) - 1/2 in slot (i - j) & 1
  float r2[4][NQ], l2[4][NQ];  // stage-2 split of cell k - 1 - j in slot (i - j) & 3
  float f2[2][NQ];            // limited stage-2 face (k - 3 - j) + 1/2 in slot (i - j) & 1
  float dr[2][NQ], dl[2][NQ];  // upper slopes of face (k - 3 - j) + 1/2 in slot (i - j) & 1: the
                             // lower slopes of the next face
  float g[4][3];              // first sweep: g of cell k + 2 - j in slot (i + 2 - j) & 3
};

template <int NQ>
struct WalkPtr {
  const float* __restrict__ q[NQ];
  float* __restrict__ o[NQ];
  unsigned base, stride;   // in bytes
  int n;
  // opening gas kick on load (first sweep of a step): g of the sample's cells, the half kick
  const char* g4;
  float h;
  // byte offset of cell k of the column (periodic)
  __device__ __forceinline__ unsigned at(int k) const {
    return base + static_cast<unsigned>(k & (n - 1)) * stride;
  }
  __device__ __forceinline__ float ld(int c, unsigned off) const {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(q[c]) + off);
  }
  __device__ __forceinline__ void st(int c, unsigned off, float v) const {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(o[c]) + off) = v;
  }
};

// U of cell kk of the column into u
template <int NQ>
__device__ __forceinline__ void walk_load(const WalkPtr<NQ>& p, int kk, float (&u)[NQ]) {
  const unsigned off = p.at(kk);
#pragma unroll
  for (int c = 0; c < NQ; ++c) u[c] = p.ld(c, off);
}

// g of cell kk of the column (the float4 of cell i is at byte 16 i, i.e. 4 times the byte
// offset of its float)
template <int NQ>
__device__ __forceinline__ void walk_load_g(const WalkPtr<NQ>& p, int kk, float (&g)[3]) {
  const float4 v = *reinterpret_cast<const float4*>(p.g4 + 4ull * p.at(kk));
  g[0] = v.x;
  g[1] = v.y;
  g[2] = v.z;
}

template <int D, int I, int STAGE, bool KICK, int NQ>
__device__ __forceinline__ void walk_fwd_visit(WalkFwd<D, NQ>& w, const WalkPtr<NQ>& p, int k,
                                               const HydroK& h1, const HydroK& h2, float dt,
                                               float hdt) {
  constexpr int s0 = I & 7, s1 = (I + 7) & 7, s3 = (I + 5) & 7, sa = (I + kAhead) & 7;
  constexpr int t0 = I & 3, t1 = (I + 3) & 3, t2 = (I + 2) & 3, t3 = (I + 1) & 3;
  constexpr int p0 = I & 1, p1 = (I + 1) & 1;
  walk_load<NQ>(p, k + kAhead, w.u[sa]);
  if (KICK) {
    // g two visits ahead; cell k, first used now, takes the opening kick
    walk_load_g<NQ>(p, k + 2, w.g[(I + 2) & 3]);
    kick_loaded(w.u[s0], w.g[I & 3], p.h);
  }
  float l1[NQ];
  split_flux<D, NQ>(w.u[s0], h1, w.r1[p0], l1);
  if (STAGE < 1) return;
#pragma unroll
  for (int c = 0; c < NQ; ++c) w.f1[p0][c] = w.r1[p1][c] - l1[c];   // face k-1/2
  if (STAGE < 2) return;
  float qh[NQ];   // half step of cell k-1 from faces (k-1) -+ 1/2
#pragma unroll
  for (int c = 0; c < NQ; ++c) qh[c] = w.u[s1][c] - hdt * (w.f1[p0][c] - w.f1[p1][c]);
  split_flux<D, NQ>(qh, h2, w.r2[t0], w.l2[t0]);
  if (STAGE < 3) return;
  // face (k-3)+1/2: F^R at cells k-4, k-3, k-2 (slots t3, t2, t1), F^L at k-3, k-2, k-1; the
  // lower slopes are the previous face's upper ones
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const float r0 = w.r2[t2][c], lp = w.l2[t1][c];
    const float sr = STAGE == 3 ? r0 - w.r2[t3][c] : w.dr[p1][c];
    const float sl = STAGE == 3 ? lp - w.l2[t2][c] : w.dl[p1][c];
    w.dr[p0][c] = w.r2[t1][c] - r0;
    w.dl[p0][c] = w.l2[t0][c] - lp;
    const float fr = r0 + van_leer_half(sr, w.dr[p0][c]);
    const float fl = lp - van_leer_half(sl, w.dl[p0][c]);
    w.f2[p0][c] = fr - fl;
  }
  if (STAGE < 4) return;
  const unsigned off = p.at(k - 3);
#pragma unroll
  for (int c = 0; c < NQ; ++c) p.st(c, off, w.u[s3][c] - dt * (w.f2[p0][c] - w.f2[p1][c]));
}

template <int D, bool KICK, int NQ>
__global__ void __launch_bounds__(256) sweep_walk_kernel(const float* __restrict__ qin,
                                                         float* __restrict__ qout, int n,
                                                         long long nc, int seg_len, int nseg,
                                                         const StepScal* __restrict__ tab,
                                                         const float4* __restrict__ g4) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<long long>(n) * n * nseg) return;
  const int x = static_cast<int>(t % n);
  const int other = static_cast<int>((t / n) % n);
  const int seg = static_cast<int>(t / (static_cast<long long>(n) * n));
  WalkPtr<NQ> p;
  p.n = n;
  p.base = 4u * (D == 1 ? static_cast<unsigned>(other) * n * n + x
                        : static_cast<unsigned>(other) * n + x);
  p.stride = 4u * (D == 1 ? n : static_cast<unsigned>(n) * n);
  const int s = seg * seg_len;
  const StepScal& sc = tab[blockIdx.y];
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    p.q[c] = qin + (blockIdx.y * NQ + c) * nc;
    p.o[c] = qout + (blockIdx.y * NQ + c) * nc;
  }
  p.g4 = KICK ? reinterpret_cast<const char*>(g4 + blockIdx.y * nc) : nullptr;
  p.h = sc.h;
  if (!sc.active) {
    for (int i = 0; i < seg_len; ++i) {
      const unsigned off = p.at(s + i);
#pragma unroll
      for (int c = 0; c < NQ; ++c) p.st(c, off, p.ld(c, off));
    }
    return;
  }
  const float dt = sc.dt;
  const HydroK h1 = sc.h1, h2 = sc.h2;
  const float hdt = 0.5f * dt;
  WalkFwd<D, NQ> w;
#pragma unroll
  for (int j = 0; j < kAhead; ++j) walk_load<NQ>(p, s - 3 + j, w.u[j]);
  if (KICK) {
    walk_load_g<NQ>(p, s - 3, w.g[0]);
    walk_load_g<NQ>(p, s - 2, w.g[1]);
  }
  // visits 0..5 fill the pipeline; from visit 6 on every visit writes a cell
  walk_fwd_visit<D, 0, 0, KICK, NQ>(w, p, s - 3, h1, h2, dt, hdt);
  walk_fwd_visit<D, 1, 1, KICK, NQ>(w, p, s - 2, h1, h2, dt, hdt);
  walk_fwd_visit<D, 2, 2, KICK, NQ>(w, p, s - 1, h1, h2, dt, hdt);
  walk_fwd_visit<D, 3, 2, KICK, NQ>(w, p, s, h1, h2, dt, hdt);
  walk_fwd_visit<D, 4, 2, KICK, NQ>(w, p, s + 1, h1, h2, dt, hdt);
  walk_fwd_visit<D, 5, 3, KICK, NQ>(w, p, s + 2, h1, h2, dt, hdt);
  // seg_len is a multiple of 8: visits 6 + 8m .. 13 + 8m have ring phases 6, 7, 0, .., 5
  for (int k = s + 3; k < s + 3 + seg_len; k += 8) {
    walk_fwd_visit<D, 6, 4, KICK, NQ>(w, p, k, h1, h2, dt, hdt);
    walk_fwd_visit<D, 7, 4, KICK, NQ>(w, p, k + 1, h1, h2, dt, hdt);
    walk_fwd_visit<D, 0, 4, KICK, NQ>(w, p, k + 2, h1, h2, dt, hdt);
    walk_fwd_visit<D, 1, 4, KICK, NQ>(w, p, k + 3, h1, h2, dt, hdt);
    walk_fwd_visit<D, 2, 4, KICK, NQ>(w, p, k + 4, h1, h2, dt, hdt);
    walk_fwd_visit<D, 3, 4, KICK, NQ>(w, p, k + 5, h1, h2, dt, hdt);
    walk_fwd_visit<D, 4, 4, KICK, NQ>(w, p, k + 6, h1, h2, dt, hdt);
    walk_fwd_visit<D, 5, 4, KICK, NQ>(w, p, k + 7, h1, h2, dt, hdt);
  }
}

// --------------------------------------------------------------------------- adjoint x
// Whole rows in LDS, one cell per thread, each face handled once:
//   1. U, lambda' from memory; stage-1 split of the own cell into LDS.
//   2. half step Uh and its stage-2 split into LDS.
//   3. per face m: G2_m = -dt (lambda'_m - lambda'_{m+1}) times the limiter coefficients gives
//      the adjoints of F^R at m-1, m, m+1 and of F^L at m, m+1, m+2; the own-cell terms stay in
//      registers, the four that belong to neighbours go through LDS.
//   4. lambda_h = split VJP at Uh of the gathered adjoints.
//   5. stage-1 transpose: lambda = lambda' + lambda_h + split VJP at U of (G1_j, -G1_{j-1}),
//      G1_m = -dt/2 (lambda_h_m - lambda_h_{m+1}).
// KICK: the adjoint of the first sweep of a step; qin is the state before the opening gas
// kick, which the load applies again (as the forward sweep did).
template <bool KICK, int NQ>
__global__ void __launch_bounds__(kRowThreads) sweep_x_vjp_kernel(
    const float* __restrict__ qin, const float* __restrict__ lam_out, float* __restrict__ lam_in,
    int n, long long nc, const StepScal* __restrict__ tab, const float4* __restrict__ g4) {
  __shared__ float S[5][NQ][kRowCells];
  const long long base = static_cast<long long>(blockIdx.x) * kRowCells;
  const int j = threadIdx.x;
  const StepScal& sc = tab[blockIdx.y];
  qin += blockIdx.y * NQ * nc;
  lam_out += blockIdx.y * NQ * nc;
  lam_in += blockIdx.y * NQ * nc;
  if (!sc.active) {
    copy_block<NQ>(lam_out, lam_in, nc, base, kRowCells, j, kRowThreads);
    return;
  }
  const float dt = sc.dt;
  const HydroK h1 = sc.h1, h2 = sc.h2;
  const float hdt = 0.5f * dt;
  const int row0 = j - (j & (n - 1)), col = j & (n - 1);
  const int jm = row0 + wrap(col - 1, n), jmm = row0 + wrap(col - 2, n);
  const int jp = row0 + wrap(col + 1, n), jpp = row0 + wrap(col + 2, n);
  float u[NQ], lm[NQ];
  {  // 1. S[0] = lambda', S[1] = F^R(U), S[2] = F^L(U)
    float fr[NQ], fl[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      u[c] = qin[c * nc + base + j];
      lm[c] = lam_out[c * nc + base + j];
    }
    if (KICK) {
      float m[3] = {u[1], u[2], u[3]};
      kick_cell(u[0], g4[blockIdx.y * nc + base + j], sc.h, m, u[4]);
      u[1] = m[0];
      u[2] = m[1];
      u[3] = m[2];
    }
    split_flux<0, NQ>(u, h1, fr, fl);
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      S[0][c][j] = lm[c];
      S[1][c][j] = fr[c];
      S[2][c][j] = fl[c];
    }
  }
  __syncthreads();
  float qh[NQ];
  {  // 2. S[3] = F^R(Uh), S[4] = F^L(Uh)
    float fr[NQ], fl[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c)
      qh[c] = u[c] - hdt * ((S[1][c][j] - S[2][c][jp]) - (S[1][c][jm] - S[2][c][j]));
    split_flux<0, NQ>(qh, h2, fr, fl);
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      S[3][c][j] = fr[c];
      S[4][c][j] = fl[c];
    }
  }
  __syncthreads();
  // 3. face m = j; S[1], S[2] are free since step 2
  float gr[NQ], gl[NQ], xl1[NQ], xl2[NQ];
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    const float g = -dt * (S[0][c][j] - S[0][c][jp]);
    float a0, a1, a2, b0, b1, b2;
    face_r_coef(S[3][c][jm], S[3][c][j], S[3][c][jp], a0, a1, a2);
    face_l_coef(S[4][c][j], S[4][c][jp], S[4][c][jpp], b0, b1, b2);
    S[1][c][j] = g * a0;   // F^R at m-1
    gr[c] = g * a1;        // F^R at m
    S[2][c][j] = g * a2;   // F^R at m+1
    gl[c] = -g * b0;       // F^L at m
    xl1[c] = -g * b1;      // F^L at m+1
    xl2[c] = -g * b2;      // F^L at m+2
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    S[3][c][j] = xl1[c];
    S[4][c][j] = xl2[c];
  }
  __syncthreads();
  {  // 4. lambda_h into S[0]
    float sv[NQ], dv[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      const float gR = gr[c] + S[2][c][jm] + S[1][c][jp];
      const float gL = gl[c] + S[3][c][jm] + S[4][c][jmm];
      sv[c] = gR + gL;
      dv[c] = gR - gL;
    }
    split_flux_vjp<0, NQ>(qh, h2, sv, dv, gr);
#pragma unroll
    for (int c = 0; c < NQ; ++c) S[0][c][j] = gr[c];
  }
  __syncthreads();
  {  // 5. stage-1 transpose
    float sv[NQ], dv[NQ], out[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      const float gp = -hdt * (gr[c] - S[0][c][jp]);
      const float gm = -hdt * (S[0][c][jm] - gr[c]);
      sv[c] = gp - gm;
      dv[c] = gp + gm;
    }
    split_flux_vjp<0, NQ>(u, h1, sv, dv, out);
#pragma unroll
    for (int c = 0; c < NQ; ++c) lam_in[c * nc + base + j] = lm[c] + gr[c] + out[c];
  }
}

// ------------------------------------------------------------------------ adjoint y / z walk
// One pass per column segment.  At visit i the thread holds cell k = s-4+i as the newest U and
// lambda' and, with the rings of the forward walk:
//   splits U_k at a1, forms F1_{k-1/2}, the half step Uh_{k-1} and its split at a2;
//   pushes G2 of R face k-2 and L face k-3 (G2_m = -dt (lambda'_m - lambda'_{m+1})) through the
//   limiter coefficients into the adjoints gR, gL of cells k-3 .. k-1 (cell k-3 is then
//   complete);
//   lambda_h_{k-3} = split VJP at Uh_{k-3}; G1_{k-4} = -dt/2 (lambda_h_{k-4} - lambda_h_{k-3});
//   lambda_{k-4} = lambda'_{k-4} + lambda_h_{k-4} + split VJP at U_{k-4} of (G1_{k-4}, -G1_{k-5}).
// Output cell c needs U at c-4 .. c+4 and lambda' at c-3 .. c+3, so a segment of seg cells
// takes seg + 8 visits.
constexpr int kAheadU = 2;   // U loaded this many cells ahead of the newest one
constexpr int kAheadL = 1;   // lambda' likewise

template <int NQ>
struct WalkVjp {
  float u[8][NQ];             // U of cell k - j in slot (i - j) & 7
  float lm[8][NQ];            // lambda' of cell k - j in slot (i - j) & 7
  float r1[2][NQ];            // stage-1 F^R of cell k - j in slot (i - j) & 1
  float f1[2][NQ];            // F1 of face (k - j) - 1/2 in slot (i - j) & 1
  float uh[4][NQ];            // Uh of cell k - 1 - j in slot (i - j) & 3
  float r2[4][NQ], l2[4][NQ];  // stage-2 split of cell k - 1 - j in slot (i - j) & 3
  float gr[4][NQ], gl[4][NQ];  // adjoints of F^R, F^L of cell k - 1 - j in slot (i - j) & 3
  float lh[2][NQ];            // lambda_h of cell k - 3 - j in slot (i - j) & 1
  float g1[2][NQ];            // G1 of face (k - 4 - j) + 1/2 in slot (i - j) & 1
  float g[2][3];              // first sweep: g of cell k + 1 - j in slot (i + 1 - j) & 1
};

// Returns x unchanged through an empty asm statement, so that the compiler cannot reuse
// values it derived from x visits earlier (it would keep them in registers that long).
__device__ __forceinline__ float opaque(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int NQ>
struct WalkVjpPtr {
  const float* __restrict__ q[NQ];
  const float* __restrict__ l[NQ];
  float* __restrict__ o[NQ];
  unsigned base, stride;   // in bytes
  int n;
  // adjoint of the first sweep of a step: q is the state before the opening gas kick, which
  // every load applies again (g of the sample's cells, the half kick)
  const char* g4;
  float h;
  __device__ __forceinline__ unsigned at(int k) const {
    return base + static_cast<unsigned>(k & (n - 1)) * stride;
  }
  __device__ __forceinline__ static float ld(const float* p, unsigned off) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(p) + off);
  }
  __device__ __forceinline__ void st(int c, unsigned off, float v) const {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(o[c]) + off) = v;
  }
  // g of the cell at byte offset off (its float4 is at byte 16 off / 4)
  __device__ __forceinline__ void load_g(unsigned off, float (&g)[3]) const {
    const float4 v = *reinterpret_cast<const float4*>(g4 + 4ull * off);
    g[0] = v.x;
    g[1] = v.y;
    g[2] = v.z;
  }
};


// STAGE: 0 split only, 1 + F1, 2 + half step and stage-2 split, 3 + first faces (every
// adjoint assigned), 4 + faces, 5 + lambda_h, 6 + G1, 7 + output
template <int D, int I, int STAGE, bool KICK, int NQ>
__device__ __forceinline__ void walk_vjp_visit(WalkVjp<NQ>& w, const WalkVjpPtr<NQ>& p, int k,
                                               const HydroK& h1, const HydroK& h2, float dt,
                                               float hdt) {
  constexpr int u0 = I & 7, u1 = (I + 7) & 7, u4 = (I + 4) & 7;
  constexpr int ua = (I + kAheadU) & 7, la = (I + kAheadL) & 7;
  constexpr int l1s = (I + 7) & 7, l2s = (I + 6) & 7, l3s = (I + 5) & 7;
  constexpr int t0 = I & 3, t1 = (I + 3) & 3, t2 = (I + 2) & 3;
  constexpr int p0 = I & 1, p1 = (I + 1) & 1;
  // keep the scheduler from hoisting the loads of later visits (and their registers) up here
  __builtin_amdgcn_sched_barrier(0);
  {
    const unsigned offu = p.at(k + kAheadU), offl = p.at(k + kAheadL);
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      w.u[ua][c] = WalkVjpPtr<NQ>::ld(p.q[c], offu);
      w.lm[la][c] = WalkVjpPtr<NQ>::ld(p.l[c], offl);
    }
    if (KICK) p.load_g(p.at(k + 1), w.g[(I + 1) & 1]);
  }
  if (KICK) kick_loaded(w.u[u0], w.g[I & 1], p.h);
  float l1[NQ];
  split_flux<D, NQ>(w.u[u0], h1, w.r1[p0], l1);
  if (STAGE < 1) return;
#pragma unroll
  for (int c = 0; c < NQ; ++c) w.f1[p0][c] = w.r1[p1][c] - l1[c];
  if (STAGE < 2) return;
#pragma unroll
  for (int c = 0; c < NQ; ++c) w.uh[t0][c] = w.u[u1][c] - hdt * (w.f1[p0][c] - w.f1[p1][c]);
  split_flux<D, NQ>(w.uh[t0], h2, w.r2[t0], w.l2[t0]);
  if (STAGE < 3) return;
  // R face k-2 (F^R at k-3, k-2, k-1), L face k-3 (F^L at k-3, k-2, k-1)
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    float a0, a1, a2;
    face_r_coef(w.r2[t2][c], w.r2[t1][c], w.r2[t0][c], a0, a1, a2);
    const float gR = -dt * (w.lm[l2s][c] - w.lm[l1s][c]);
    float b0, b1, b2;
    face_l_coef(w.l2[t2][c], w.l2[t1][c], w.l2[t0][c], b0, b1, b2);
    const float gL = dt * (w.lm[l3s][c] - w.lm[l2s][c]);
    if (STAGE == 3) {
      w.gr[t2][c] = gR * a0;
      w.gr[t1][c] = gR * a1;
      w.gl[t2][c] = gL * b0;
      w.gl[t1][c] = gL * b1;
    } else {
      w.gr[t2][c] += gR * a0;
      w.gr[t1][c] += gR * a1;
      w.gl[t2][c] += gL * b0;
      w.gl[t1][c] += gL * b1;
    }
    w.gr[t0][c] = gR * a2;
    w.gl[t0][c] = gL * b2;
  }
  if (STAGE < 5) return;
  {  // lambda_h of cell k-3
    float sv[NQ], dv[NQ], q[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      sv[c] = w.gr[t2][c] + w.gl[t2][c];
      dv[c] = w.gr[t2][c] - w.gl[t2][c];
      q[c] = opaque(w.uh[t2][c]);
    }
    split_flux_vjp<D, NQ>(q, h2, sv, dv, w.lh[p0]);
  }
  if (STAGE < 6) return;
#pragma unroll
  for (int c = 0; c < NQ; ++c) w.g1[p0][c] = -hdt * (w.lh[p1][c] - w.lh[p0][c]);   // face k-4+1/2
  if (STAGE < 7) return;
  {  // lambda of cell k-4
    float sv[NQ], dv[NQ], out[NQ], q[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      sv[c] = w.g1[p0][c] - w.g1[p1][c];
      dv[c] = w.g1[p0][c] + w.g1[p1][c];
      q[c] = opaque(w.u[u4][c]);
    }
    split_flux_vjp<D, NQ>(q, h1, sv, dv, out);
    const unsigned off = p.at(k - 4);
#pragma unroll
    for (int c = 0; c < NQ; ++c) p.st(c, off, w.lm[u4][c] + w.lh[p1][c] + out[c]);
  }
}

template <int D, bool KICK, int NQ>
__global__ void __launch_bounds__(256) sweep_walk_vjp_kernel(const float* __restrict__ qin,
                                                             const float* __restrict__ lam_out,
                                                             float* __restrict__ lam_in, int n,
                                                             long long nc, int seg_len, int nseg,
                                                             const StepScal* __restrict__ tab,
                                                             const float4* __restrict__ g4) {
  const long long t = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<long long>(n) * n * nseg) return;
  const int x = static_cast<int>(t % n);
  const int other = static_cast<int>((t / n) % n);
  const int seg = static_cast<int>(t / (static_cast<long long>(n) * n));
  WalkVjpPtr<NQ> p;
  p.n = n;
  p.base = 4u * (D == 1 ? static_cast<unsigned>(other) * n * n + x
                        : static_cast<unsigned>(other) * n + x);
  p.stride = 4u * (D == 1 ? n : static_cast<unsigned>(n) * n);
  const int s = seg * seg_len;
  const StepScal& sc = tab[blockIdx.y];
#pragma unroll
  for (int c = 0; c < NQ; ++c) {
    p.q[c] = qin + (blockIdx.y * NQ + c) * nc;
    p.l[c] = lam_out + (blockIdx.y * NQ + c) * nc;
    p.o[c] = lam_in + (blockIdx.y * NQ + c) * nc;
  }
  p.g4 = KICK ? reinterpret_cast<const char*>(g4 + blockIdx.y * nc) : nullptr;
  p.h = sc.h;
  if (!sc.active) {
    for (int i = 0; i < seg_len; ++i) {
      const unsigned off = p.at(s + i);
#pragma unroll
      for (int c = 0; c < NQ; ++c) p.st(c, off, WalkVjpPtr<NQ>::ld(p.l[c], off));
    }
    return;
  }
  const float dt = sc.dt;
  const HydroK h1 = sc.h1, h2 = sc.h2;
  const float hdt = 0.5f * dt;
  WalkVjp<NQ> w;
#pragma unroll
  for (int j = 0; j < kAheadU; ++j) {
    const unsigned off = p.at(s - 4 + j);
#pragma unroll
    for (int c = 0; c < NQ; ++c) w.u[j][c] = WalkVjpPtr<NQ>::ld(p.q[c], off);
  }
  if (KICK) p.load_g(p.at(s - 4), w.g[0]);
#pragma unroll
  for (int j = 0; j < kAheadL; ++j) {
    const unsigned off = p.at(s - 4 + j);
#pragma unroll
    for (int c = 0; c < NQ; ++c) w.lm[j][c] = WalkVjpPtr<NQ>::ld(p.l[c], off);
  }
  walk_vjp_visit<D, 0, 0, KICK, NQ>(w, p, s - 4, h1, h2, dt, hdt);
  walk_vjp_visit<D, 1, 1, KICK, NQ>(w, p, s - 3, h1, h2, dt, hdt);
  walk_vjp_visit<D, 2, 2, KICK, NQ>(w, p, s - 2, h1, h2, dt, hdt);
  walk_vjp_visit<D, 3, 2, KICK, NQ>(w, p, s - 1, h1, h2, dt, hdt);
  walk_vjp_visit<D, 4, 3, KICK, NQ>(w, p, s, h1, h2, dt, hdt);
  walk_vjp_visit<D, 5, 4, KICK, NQ>(w, p, s + 1, h1, h2, dt, hdt);
  walk_vjp_visit<D, 6, 5, KICK, NQ>(w, p, s + 2, h1, h2, dt, hdt);
  walk_vjp_visit<D, 7, 6, KICK, NQ>(w, p, s + 3, h1, h2, dt, hdt);
  // seg_len is a multiple of 8: visits 8 + 8m .. 15 + 8m have ring phases 0 .. 7
  for (int k = s + 4; k < s + 4 + seg_len; k += 8) {
    walk_vjp_visit<D, 0, 7, KICK, NQ>(w, p, k, h1, h2, dt, hdt);
    walk_vjp_visit<D, 1, 7, KICK, NQ>(w, p, k + 1, h1, h2, dt, hdt);
    walk_vjp_visit<D, 2, 7, KICK, NQ>(w, p, k + 2, h1, h2, dt, hdt);
    walk_vjp_visit<D, 3, 7, KICK, NQ>(w, p, k + 3, h1, h2, dt, hdt);
    walk_vjp_visit<D, 4, 7, KICK, NQ>(w, p, k + 4, h1, h2, dt, hdt);
    walk_vjp_visit<D, 5, 7, KICK, NQ>(w, p, k + 5, h1, h2, dt, hdt);
    walk_vjp_visit<D, 6, 7, KICK, NQ>(w, p, k + 6, h1, h2, dt, hdt);
    walk_vjp_visit<D, 7, 7, KICK, NQ>(w, p, k + 7, h1, h2, dt, hdt);
  }
}

int pick_segment(int n) { return n >= 64 ? 64 : n; }

}  // namespace

namespace {

template <int NQ>
void sweep_nq(hipStream_t st, const float* qin, float* qout, const Batch& b, int axis,
              const float4* g4) {
  const int n = b.n;
  const long long nc = b.nc();
  if (axis == 0) {
    const dim3 grid(static_cast<unsigned>(nc / kRowCells), b.S);
    if (g4)
      hipLaunchKernelGGL((sweep_x_kernel<true, NQ>), grid, dim3(kRowThreads), 0, st, qin, qout, n,
                         nc, b.tab, g4);
    else
      hipLaunchKernelGGL((sweep_x_kernel<false, NQ>), grid, dim3(kRowThreads), 0, st, qin, qout,
                         n, nc, b.tab, nullptr);
  } else {
    const int seg = pick_segment(n);
    const int nseg = n / seg;
    const long long threads = static_cast<long long>(n) * n * nseg;
    const dim3 grid(blocks_for(threads, 256), b.S);
#define DH_WALK(D, KICK)                                                                     \
  hipLaunchKernelGGL((sweep_walk_kernel<D, KICK, NQ>), grid, dim3(256), 0, st, qin, qout, n, nc, \
                     seg, nseg, b.tab, g4)
    if (axis == 1) {
      if (g4) DH_WALK(1, true);
      else DH_WALK(1, false);
    } else {
      if (g4) DH_WALK(2, true);
      else DH_WALK(2, false);
    }
#undef DH_WALK
  }
}

template <int NQ>
void sweep_vjp_nq(hipStream_t st, const float* qin, const float* lam_out, float* lam_in,
                  const Batch& b, int axis, const float4* g4) {
  const int n = b.n;
  const long long nc = b.nc();
  if (axis == 0) {
    const dim3 grid(static_cast<unsigned>(nc / kRowCells), b.S);
    if (g4)
      hipLaunchKernelGGL((sweep_x_vjp_kernel<true, NQ>), grid, dim3(kRowThreads), 0, st, qin,
                         lam_out, lam_in, n, nc, b.tab, g4);
    else
      hipLaunchKernelGGL((sweep_x_vjp_kernel<false, NQ>), grid, dim3(kRowThreads), 0, st, qin,
                         lam_out, lam_in, n, nc, b.tab, nullptr);
  } else {
    const int seg = pick_segment(n);
    const int nseg = n / seg;
    const long long threads = static_cast<long long>(n) * n * nseg;
    const dim3 grid(blocks_for(threads, 256), b.S);
#define DH_WALK_VJP(D, KICK)                                                                  \
  hipLaunchKernelGGL((sweep_walk_vjp_kernel<D, KICK, NQ>), grid, dim3(256), 0, st, qin, lam_out, \
                     lam_in, n, nc, seg, nseg, b.tab, g4)
    if (axis == 1) {
      if (g4) DH_WALK_VJP(1, true);
      else DH_WALK_VJP(1, false);
    } else {
      if (g4) DH_WALK_VJP(2, true);
      else DH_WALK_VJP(2, false);
    }
#undef DH_WALK_VJP
  }
}

}  // namespace

void launch_sweep(hipStream_t st, const float* qin, float* qout, const Batch& b, int axis,
                  const float4* g4) {
  if (!b.tab) throw ArgError("sweep: step table required");
  if (axis == 0 && qin == qout) throw ArgError("sweep_x: in-place not supported");
  if (b.nq == 6)
    sweep_nq<6>(st, qin, qout, b, axis, g4);
  else
    sweep_nq<5>(st, qin, qout, b, axis, g4);
  DH_LAUNCH_CHECK();
}

void launch_sweep_vjp(hipStream_t st, const float* qin, const float* lam_out, float* lam_in,
                      const Batch& b, int axis, const float4* g4) {
  if (!b.tab) throw ArgError("sweep adjoint: step table required");
  if (qin == lam_in || lam_out == lam_in) throw ArgError("sweep adjoint: in-place not supported");
  if (b.nq == 6)
    sweep_vjp_nq<6>(st, qin, lam_out, lam_in, b, axis, g4);
  else
    sweep_vjp_nq<5>(st, qin, lam_out, lam_in, b, axis, g4);
  DH_LAUNCH_CHECK();
}

}  // namespace dh
