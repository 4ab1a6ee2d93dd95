// Blocked right-looking FP64 Cholesky W = L L^T (Algorithm 1 step 2), in place on a row-major
// n x n matrix, lower triangle. Block size 64; per block column k:
//   1. potf2   four waves factor the 64 x 64 diagonal block (right-looking: lane i keeps row i
//              in registers, wave w columns 16 w .. 16 w + 15; wave w factors its 16 columns
//              alone, then the later waves subtract them through LDS) and invert its four
//              16 x 16 diagonal sub-blocks, each wave its own while the later waves subtract.
//   2. trsm    rows below the block: A_ik <- A_ik L_kk^-T by blocked forward substitution over
//              the four 16-column panels with those inverses, on the FP64 matrix cores, 64 rows
//              per workgroup.
//   3. update  trailing lower triangle A_IJ -= A_Ik A_Jk^T in 64 x 64 tiles on the FP64 matrix
//              cores (v_mfma_f64_16x16x4), panels staged in LDS. Its first tile is the next
//              diagonal block, which needs no later update: that workgroup runs step 1 of the
//              next block column on it straight away, so only block column 0 has a potf2 launch
//              of its own and a step costs two launches.
// A pivot d with !(d > 0) (NaN included) stores the 1-based global index in *info and raises
// *flag; every later kernel sees the flag and returns at once, so the device work drains
// without touching the matrix further.
// Batched form: grid dimension y indexes independent matrices (A + b sA, info[b], flag[b], Dkk
// block b), which then share every launch; a breakdown stops only its own matrix.
#include "dfisher_internal.h"

namespace dfi {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int NB = 64;
constexpr int LDP = NB + 1;  // padded LDS row (doubles)

constexpr int PW = 4;          // waves of the diagonal-block kernel
constexpr int PC = NB / PW;    // 16 columns per wave (factor), rows and columns of a sub-block inverse

// Diagonal block: L_kk = chol(A_kk) and the inverses of its 16 x 16 diagonal sub-blocks, with 4 waves.
// Lane i holds row i of the block, wave w its columns 16 w .. 16 w + 15, in registers. The four
// 16-column panels are taken in order; wave p factors its panel alone, right-looking, with no
// barrier: at step j the pivot (lane j's entry, read across lanes) gives 1 / l_jj by the hardware
// reciprocal square root and two Newton steps, column j is scaled, and the panel's later columns
// c lose l_ij l_cj (l_cj read from lane c). The finished panel is published in LDS
// (column-major), and after a barrier the waves of later panels subtract it from their columns
// (l_ij from LDS per lane, l_cj as broadcasts). Every a_ic thus loses its products in the order
// l = 0, 1, ..., c - 1, as in the column-by-column algorithm. The first pivot that is not > 0
// (NaN included) is reported as its 1-based global index; the block is then not stored (later
// steps run on garbage but index nothing out of range). Only 4 barriers per block, against one
// per column before.
// The panel solve needs only D_p = L_pp^-1 for the four 16 x 16 diagonal sub-blocks, not the
// whole L_kk^-1 (whose cross-panel rows, formed in the same loop, were a third of the kernel's
// time on the serial chain): wave p forms D_p by forward substitution inside its panel after the
// panel's barrier, in the time the later waves spend subtracting the panel.
constexpr int LDT = NB + 1;   // padded column stride of the LDS copy of L_kk (doubles)

// Lane j's value of a double (j wave-uniform): two v_readlane, no LDS round trip.
__device__ __forceinline__ double lane_read(double v, int j) {
  const uint64_t b = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), j);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// 1 / sqrt(d) for a normal d > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1 - d y^2) / 2 (each roughly doubles the correct bits; the result is within a few
// units in the last place, the pivot then being l_jj = d y).
__device__ __forceinline__ double rsqrt_f64(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// The diagonal block's factor for block column k (the body of potf2_kernel, also run by the
// trailing update's first tile, which produces that block), and the inverses of its four 16 x 16
// diagonal sub-blocks for the panel solve. blk(i, c) reads entry (i, c) of the block, c <= i < nb;
// lt is NB x LDT doubles of LDS, rp NB doubles, failed an int in LDS. The caller has checked the
// breakdown flag.
template <class Blk>
__device__ __forceinline__ void potf2_block(double* __restrict__ A, int64_t n, int64_t k, int64_t* __restrict__ info,
                                            int32_t* __restrict__ flag, double* __restrict__ Dkk, Blk blk, double* lt,
                                            double* rp, int* failed_p) {
  int& failed = *failed_p;
  const int i = threadIdx.x & 63;      // row of the block
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar branches
  const int c0 = w * PC;               // this wave's first column
  const int64_t nb = min<int64_t>(NB, n - k);
  const bool below = k + NB < n;       // rows below: the panel solve needs the sub-block inverses
  if (threadIdx.x == 0) failed = 0;
  double r[PC];
#pragma unroll
  for (int u = 0; u < PC; ++u) {
    const int c = c0 + u;
    double val = (c == i) ? 1.0 : 0.0;   // identity padding past nb
    if (i < nb && c < nb && c <= i) val = blk(i, c);
    r[u] = val;
  }
  __syncthreads();
  // D_w = L_ww^-1 (this wave's 16 x 16 diagonal sub-block) by forward substitution, lane c0 + c
  // forming column c (x_t *= 1 / l_tt, then x_u -= l_ut x_t for the later rows u, l_ut and 1 / l_tt
  // read from LDS as broadcasts); stored as D_w[u][c] at Dkk[(w PC + u) PC + c]. Run by the four
  // waves together once every panel is published.
  auto diag_inverse = [&]() {
    double x[PC];
#pragma unroll
    for (int u = 0; u < PC; ++u) x[u] = (c0 + u == i) ? 1.0 : 0.0;
#pragma unroll
    for (int tt = 0; tt < PC; ++tt) {
      x[tt] *= rp[c0 + tt];
#pragma unroll
      for (int u = tt + 1; u < PC; ++u) x[u] -= lt[(c0 + tt) * LDT + c0 + u] * x[tt];
    }
    if (i >= c0 && i < c0 + PC) {
#pragma unroll
      for (int u = 0; u < PC; ++u) Dkk[(c0 + u) * PC + (i - c0)] = x[u];
    }
  };
#pragma unroll 1
  for (int p = 0; p < PW; ++p) {
    if (w == p) {
      int bad = 0;   // uniform
#pragma unroll
      for (int jj = 0; jj < PC; ++jj) {
        const int j = c0 + jj;
        const double d = lane_read(r[jj], j);
        if (!(d > 0.0) && bad == 0) bad = j + 1;
        const double rinv = rsqrt_f64(d);
        const double ljj = d * rinv;
        const double lij = (i > j) ? r[jj] * rinv : ((i == j) ? ljj : 0.0);
        r[jj] = lij;
        if (i == j) rp[j] = rinv;
#pragma unroll
        for (int u = jj + 1; u < PC; ++u) r[u] -= lij * lane_read(lij, c0 + u);
      }
#pragma unroll
      for (int u = 0; u < PC; ++u) lt[(c0 + u) * LDT + i] = r[u];
      // the first breakdown is reported; panels after it run on garbage and are ignored
      if (bad && i == 0 && failed == 0) failed = bad;
    }
    __syncthreads();
    if (w > p) {   // subtract panel p from this wave's columns, in panel order
      const int p0 = p * PC;
#pragma unroll
      for (int jj = 0; jj < PC; ++jj) {
        const double* col = lt + (p0 + jj) * LDT;
        const double lij = col[i];
#pragma unroll
        for (int u = 0; u < PC; ++u) r[u] -= lij * col[c0 + u];
      }
    }
  }
  if (below) diag_inverse();   // every wave its own sub-block, all four at once
  // every panel has been published before the last barrier; failed was set before a barrier too
  if (failed) {
    if (threadIdx.x == 0) {
      *info = k + failed;
      *flag = 1;
    }
    return;
  }
  // the factor's lower triangle: wave w stores rows w, w + 4, ..., lane c column c
  for (int rr = w; rr < nb; rr += PW)
    if (i <= rr) A[(k + rr) * n + k + i] = lt[i * LDT + rr];
}

__global__ void __launch_bounds__(64 * PW)
potf2_kernel(double* __restrict__ A, int64_t n, int64_t k, int64_t* __restrict__ info, int32_t* __restrict__ flag,
             double* __restrict__ Dkk, int64_t sA, const FactorJob* __restrict__ jobs) {
  __shared__ double lt[NB * LDT];   // l_ij at lt[j * LDT + i], published panel by panel
  __shared__ double rp[NB];         // 1 / l_jj
  __shared__ int failed;            // 1-based local index of the first bad pivot, 0 if none
  const int64_t bb = blockIdx.y;
  if (jobs) {
    const FactorJob& jb = jobs[bb];
    A = jb.A;
    n = jb.n;
    info = jb.info;
    flag = jb.flag;
    Dkk = jb.dkk;
    if (k >= n) return;
  } else {
    A += bb * sA;
    info += bb;
    flag += bb;
    Dkk += bb * NB * NB;
  }
  if (*(volatile int32_t*)flag) return;
  potf2_block(A, n, k, info, flag, Dkk, [&](int i, int c) { return A[(k + i) * n + k + c]; }, lt, rp, &failed);
}

// Rows i in [k + NB, n): A[i][k .. k+NB) <- A[i][k .. k+NB) L_kk^-T, by blocked forward substitution
// over the block's four 16-column panels: X_p = (A_p - sum_{q<p} X_q L_pq^T) D_p^T, with L_pq the
// 16 x 16 sub-blocks of L_kk and D_p = L_pp^-1 from the diagonal-block factor. 64 rows per
// workgroup; wave w owns rows 16 w .. 16 w + 15 through all four panels (a row of X depends only
// on the same row of A), so after the staging of L_kk and D nothing crosses waves. Both products
// of a panel run on the FP64 matrix cores (v_mfma_f64_16x16x4f64, K = 16 p and 16); the panel's
// T goes through the wave's LDS to become an A operand, X_p likewise for the later panels.
constexpr int LDD = PC + 1;   // padded row of a 16 x 16 LDS tile (doubles)

__global__ void __launch_bounds__(256)
trsm_kernel(double* __restrict__ A, int64_t n, int64_t k, const int32_t* __restrict__ flag,
            const double* __restrict__ Dkk, int64_t sA, const FactorJob* __restrict__ jobs) {
  __shared__ double Lb[NB * LDP];          // L_kk row-major (lower triangle, zeros above)
  __shared__ double Db[PW * PC * LDD];     // D_p[u][c] at Db[(p PC + u) LDD + c]
  __shared__ double Xw[PW][PC * LDP];      // per wave: its 16 rows of X, panel by panel
  __shared__ double Tw[PW][PC * LDD];      // per wave: the current panel's T
  const int64_t bb = blockIdx.y;
  if (jobs) {
    const FactorJob& j = jobs[bb];
    A = j.A;
    n = j.n;
    flag = j.flag;
    Dkk = j.dkk;
  } else {
    A += bb * sA;
    flag += bb;
    Dkk += bb * NB * NB;
  }
  const int tid = threadIdx.x;
  const int64_t row0 = k + NB + (int64_t)blockIdx.x * NB;
  if (row0 >= n) return;   // grouped launches size the grid for the largest matrix
  if (*(volatile const int32_t*)flag) return;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, kq = lane >> 4;
  // every load in flight before the first LDS store: L_kk's lower triangle (the diagonal block is
  // whole: rows below exist), the four D_p, and this wave's A tiles in the MFMA's D layout (lane l
  // register r = row l/16 + 4 r, column l%16; a row past n loads row n - 1 and is not stored)
  constexpr int PER = NB * NB / 256;
  double lg[PER], dg[PW];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int r = (tid + 256 * u) / NB, c = (tid + 256 * u) % NB;
    lg[u] = (c <= r) ? A[(k + r) * n + k + c] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < PW; ++u) dg[u] = Dkk[u * PC * PC + tid];
  f64x4 cacc[PW];
#pragma unroll
  for (int p = 0; p < PW; ++p)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + wv * PC + kq + 4 * r;
      cacc[p][r] = A[min<int64_t>(row, n - 1) * n + k + p * PC + l16];
    }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int r = (tid + 256 * u) / NB, c = (tid + 256 * u) % NB;
    Lb[r * LDP + c] = lg[u];
  }
#pragma unroll
  for (int u = 0; u < PW; ++u) Db[(u * PC + tid / PC) * LDD + tid % PC] = dg[u];
  __syncthreads();
  double* X = Xw[wv];
  double* T = Tw[wv];
#pragma unroll
  for (int p = 0; p < PW; ++p) {
    // T = A_p - X_{<p} L_{p,<p}^T: A operand lane l = (row l%16, k l/16), B operand lane l =
    // (k l/16, column l%16) with B[k][c] = L_kk[16 p + c][k]
    f64x4 t = cacc[p];
#pragma unroll
    for (int kk = 0; kk < p * PC; kk += 4) {
      const double a = -X[l16 * LDP + kk + kq];
      const double b = Lb[(p * PC + l16) * LDP + kk + kq];
      t = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, t, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(kq + 4 * r) * LDD + l16] = t[r];
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): this wave's LDS writes are readable
    __builtin_amdgcn_wave_barrier();
    // X_p = T D_p^T: B[k][c] = D_p[c][k]
    f64x4 xa = (f64x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < PC; kk += 4) {
      const double a = T[l16 * LDD + kk + kq];
      const double b = Db[(p * PC + l16) * LDD + kk + kq];
      xa = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, xa, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) X[(kq + 4 * r) * LDP + p * PC + l16] = xa[r];
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + wv * PC + kq + 4 * r;
      if (row < n) A[row * n + k + p * PC + l16] = xa[r];
    }
  }
}

// Trailing update of the lower triangle below/right of block column k: for tiles (I >= J) of the
// trailing matrix, A_IJ -= P_I P_J^T with P = A[:, k .. k+NB). Four waves, each a 32 x 32 quarter
// of the tile as 2 x 2 blocks of 16 x 16 FP64 MFMA accumulators; K = 64 in 16 steps of 4.
// MFMA lane layout (16x16x4 f64): A lane l = (row l%16, k l/16), B lane l = (k l/16, col l%16),
// D lane l register r = (row l/16 + 4r, col l%16).
// Tile 0 is the next diagonal block, A_{k+1,k+1}, final after this update: its workgroup keeps the
// result in LDS instead of storing it and factors it at once (potf2_block for block column
// k + NB: L_{k+1,k+1} and its sub-block inverses into Dkk, or the breakdown), so the diagonal factor of the
// next step runs alongside the rest of this update instead of in a launch of its own. The factor
// is the same bits as a separate potf2 launch on the stored tile would give.
__global__ void __launch_bounds__(256)
update_kernel(double* __restrict__ A, int64_t n, int64_t k, int64_t* __restrict__ info, int32_t* __restrict__ flag,
              double* __restrict__ Dkk, int64_t sA, const FactorJob* __restrict__ jobs) {
  static_assert(LDP == LDT, "the staged tile is the diagonal factor's LDS layout");
  __shared__ double PI[NB * LDP];
  __shared__ double PJ[NB * LDP];
  __shared__ double rp[NB];
  __shared__ int failed;
  if (jobs) {
    const FactorJob& j = jobs[blockIdx.y];
    A = j.A;
    n = j.n;
    info = j.info;
    flag = j.flag;
    Dkk = j.dkk;
  } else {
    A += (int64_t)blockIdx.y * sA;
    info += blockIdx.y;
    flag += blockIdx.y;
    Dkk += (int64_t)blockIdx.y * NB * NB;
  }
  if (k + NB >= n) return;
  {
    // tiles of this matrix's trailing triangle: rb (rb + 1) / 2 of the grid's
    const int64_t rb = (n - k - NB + NB - 1) / NB;
    if ((int64_t)blockIdx.x >= rb * (rb + 1) / 2) return;
  }
  if (*(volatile const int32_t*)flag) return;
  const int64_t t = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int64_t J = t - I * (I + 1) / 2;
  const int64_t base = k + NB;
  const int64_t ri = base + I * NB, rj = base + J * NB;
  const int tid = threadIdx.x;
  // All 32 loads in flight before the first LDS store; a row past n loads row n - 1 of the same
  // block instead and is zeroed.
  constexpr int PER = NB * NB / 256;
  double pi[PER], pj[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int r = (tid + 256 * u) / NB, c = (tid + 256 * u) % NB;
    pi[u] = A[min<int64_t>(ri + r, n - 1) * n + k + c];
    pj[u] = A[min<int64_t>(rj + r, n - 1) * n + k + c];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int r = (tid + 256 * u) / NB, c = (tid + 256 * u) % NB;
    PI[r * LDP + c] = (ri + r < n) ? pi[u] : 0.0;
    PJ[r * LDP + c] = (rj + r < n) ? pj[u] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int l16 = lane & 15, kq = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < NB; k0 += 4) {
    double av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = PI[(wy * 32 + a * 16 + l16) * LDP + k0 + kq];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = PJ[(wx * 32 + b * 16 + l16) * LDP + k0 + kq];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
  // The 16 old values are read together (indices clamped into the tile's own rows and columns,
  // so every read is in bounds), then written back through a buffer resource based at the tile's
  // origin: an entry that must not be written (past n, or above the diagonal of a diagonal tile)
  // gets an offset past the record count and the hardware drops that store, so the stores need
  // no branch and no wait between them. Offsets stay below 64 n * 8 bytes, far under 2^31 for
  // any n whose n x n FP64 matrix fits in device memory.
  double old[2][2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = ri + wy * 32 + a * 16 + kq + 4 * r;
        const int64_t gj = rj + wx * 32 + b * 16 + l16;
        old[a][b][r] = A[min<int64_t>(gi, n - 1) * n + min<int64_t>(gj, n - 1)];
      }
  if (t == 0) {
    // the next diagonal block: the updated tile to LDS (PI, free once every wave's products are
    // done), then its factor; rows and columns past n are the factor's identity padding
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int li = wy * 32 + a * 16 + kq + 4 * r, lj = wx * 32 + b * 16 + l16;
          PI[li * LDP + lj] = old[a][b][r] - acc[a][b][r];
        }
    __syncthreads();
    potf2_block(A, n, k + NB, info, flag, Dkk, [&](int i, int c) { return PI[i * LDP + c]; }, PI, rp, &failed);
    return;
  }
  constexpr int OOB = 0x7FFFFFF0;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(A + ri * n + rj, 0, OOB, 0x00020000);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li = wy * 32 + a * 16 + kq + 4 * r, lj = wx * 32 + b * 16 + l16;
        const bool keep = ri + li < n && rj + lj <= ri + li;
        const int off = keep ? (int)((li * n + lj) * 8) : OOB;
        const double v = old[a][b][r] - acc[a][b][r];
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, off, 0, 0);
      }
}

__global__ void zero_upper_kernel(double* __restrict__ A, int64_t n) {
  const int64_t nb = (n + 255) / 256;
  const int64_t i = (int64_t)blockIdx.x / nb;
  const int64_t j = ((int64_t)blockIdx.x - i * nb) * 256 + threadIdx.x;
  if (i < n && j < n && j > i) A[i * n + j] = 0.0;
}

// dst = src + (scale * dmax[0] + lam) I
__global__ void shift_copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n, double scale,
                                  const double* __restrict__ dmax, double lam) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx - i * n;
  double add = 0.0;
  if (i == j) add = lam + ((scale != 0.0) ? scale * dmax[0] : 0.0);
  dst[idx] = src[idx] + add;
}

__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += d[i];
}

__global__ void fill_zero_kernel(double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0;
}

__global__ void diag_max_kernel(const double* __restrict__ W, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double d = W[i * n + i];
    mx = (d > mx) ? d : mx;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// *out = sum_i x_i^2 (FP64, one workgroup, fixed order: strided per-thread sums, then a tree).
__global__ void sumsq_kernel(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc = fma(x[i], x[i], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ void clear_status_kernel(int64_t* info, int32_t* flag, int64_t nbatch) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nbatch) {
    info[b] = 0;
    flag[b] = 0;
  }
}

}  // namespace

hipError_t potrf_launch_batched(double* A, int64_t n, int64_t nbatch, int64_t sA, int64_t* info_dev, int32_t* flag_dev,
                                double* dkk, hipStream_t st) {
  if (nbatch < 1 || nbatch > 65535) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)nbatch;
  hipLaunchKernelGGL(clear_status_kernel, dim3((unsigned)((nbatch + 255) / 256)), dim3(256), 0, st, info_dev, flag_dev,
                     nbatch);
  const FactorJob* nj = nullptr;
  // the first diagonal block alone; every later one inside the update that finishes it
  hipLaunchKernelGGL(potf2_kernel, dim3(1, nb), dim3(64 * PW), 0, st, A, n, (int64_t)0, info_dev, flag_dev, dkk, sA, nj);
  for (int64_t k = 0; k + NB < n; k += NB) {
    const int64_t rb = (n - k - NB + 63) / 64;
    hipLaunchKernelGGL(trsm_kernel, dim3((unsigned)rb, nb), dim3(256), 0, st, A, n, k, flag_dev, (const double*)dkk, sA,
                       nj);
    hipLaunchKernelGGL(update_kernel, dim3((unsigned)(rb * (rb + 1) / 2), nb), dim3(256), 0, st, A, n, k, info_dev,
                       flag_dev, dkk, sA, nj);
  }
  return hipGetLastError();
}

__global__ void clear_jobs_kernel(const FactorJob* __restrict__ jobs, int64_t njobs) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < njobs) {
    *jobs[b].info = 0;
    *jobs[b].flag = 0;
  }
}

hipError_t potrf_launch_grouped(const FactorJob* jobs_dev, int64_t njobs, int64_t nmax, hipStream_t st) {
  if (njobs < 1 || njobs > 65535) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)njobs;
  hipLaunchKernelGGL(clear_jobs_kernel, dim3((unsigned)((njobs + 255) / 256)), dim3(256), 0, st, jobs_dev, njobs);
  // the first diagonal blocks alone; every later one inside the update that finishes it (a job
  // whose matrix ends at block column k has no update there and no block k + NB to factor)
  hipLaunchKernelGGL(potf2_kernel, dim3(1, nb), dim3(64 * PW), 0, st, (double*)nullptr, (int64_t)0, (int64_t)0,
                     (int64_t*)nullptr, (int32_t*)nullptr, (double*)nullptr, (int64_t)0, jobs_dev);
  for (int64_t k = 0; k + NB < nmax; k += NB) {
    const int64_t rb = (nmax - k - NB + 63) / 64;
    hipLaunchKernelGGL(trsm_kernel, dim3((unsigned)rb, nb), dim3(256), 0, st, (double*)nullptr, (int64_t)0, k,
                       (const int32_t*)nullptr, (const double*)nullptr, (int64_t)0, jobs_dev);
    hipLaunchKernelGGL(update_kernel, dim3((unsigned)(rb * (rb + 1) / 2), nb), dim3(256), 0, st, (double*)nullptr,
                       (int64_t)0, k, (int64_t*)nullptr, (int32_t*)nullptr, (double*)nullptr, (int64_t)0, jobs_dev);
  }
  return hipGetLastError();
}

hipError_t potrf_launch(double* A, int64_t n, int64_t* info_dev, int32_t* flag_dev, double* dkk, hipStream_t st) {
  return potrf_launch_batched(A, n, 1, n * n, info_dev, flag_dev, dkk, st);
}

hipError_t zero_upper(double* A, int64_t n, hipStream_t st) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)(nb * n)), dim3(256), 0, st, A, n);
  return hipGetLastError();
}

hipError_t shift_copy(const double* src, double* dst, int64_t n, double scale, const double* dmax, hipStream_t st) {
  const int64_t tot = n * n;
  hipLaunchKernelGGL(shift_copy_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, src, dst, n, scale, dmax,
                     0.0);
  return hipGetLastError();
}

hipError_t add_diag_copy(const double* src, double* dst, int64_t n, double lam, hipStream_t st) {
  const int64_t tot = n * n;
  hipLaunchKernelGGL(shift_copy_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, src, dst, n, 0.0,
                     (const double*)nullptr, lam);
  return hipGetLastError();
}

hipError_t shift_add_copy(const double* src, double* dst, int64_t n, double scale, const double* dmax, double lam,
                          hipStream_t st) {
  const int64_t tot = n * n;
  hipLaunchKernelGGL(shift_copy_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, src, dst, n, scale, dmax,
                     lam);
  return hipGetLastError();
}

hipError_t axpy_inplace(double* y, const double* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, d, n);
  return hipGetLastError();
}

hipError_t fill_zero(double* y, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, y, n);
  return hipGetLastError();
}

hipError_t diag_max(const double* W, int64_t n, double* out_dev, hipStream_t st) {
  hipLaunchKernelGGL(diag_max_kernel, dim3(1), dim3(256), 0, st, W, n, out_dev);
  return hipGetLastError();
}

hipError_t sumsq(const double* x, int64_t n, double* out_dev, hipStream_t st) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(256), 0, st, x, n, out_dev);
  return hipGetLastError();
}

}  // namespace dfi
