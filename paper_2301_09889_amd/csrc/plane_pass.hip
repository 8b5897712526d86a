// Plane pass of one RK3 stage: the six velocity/vorticity fields at every Chebyshev node
// go to the 3/2-padded (x, z) grid, H = u x omega is formed pointwise, and the three
// products come back to the stored Fourier modes (§3.1; 3/2-rule dealiasing in x and z).
//
// Every FFT has a compile-time length L = A B and runs as two register passes with one
// LDS exchange (Cooley--Tukey, n = B n1 + n2, k = k1 + A k2):
//   pass 1, task n2:  DFT_A over n1 of x[B n1 + n2], then the twiddle w_L^(n2 k1);
//   pass 2, task k1:  DFT_B over n2, giving X[k1 + A k2].
// Three kernels per stage:
//   k_zinv<M_z>  inverse FFT along z of every (field, node, p) pencil, zero padding;
//   k_xrow<M_x>  per pair of padded z rows: six inverse real FFTs along x (the two rows
//                packed as real and imaginary part), the products, three forward FFTs,
//                all on one block's LDS with one task per thread in every phase;
//   k_zfwd<M_z>  forward FFT along z, truncation to |q| < N_z/2, 1/(M_x M_z), Hermitian fix.
// For padded lengths 48 and 96 the first two may run as one launch (k_zxrow, the padded rows
// kept in LDS), and for 24 x 24 all three (k_plane_small); the tuner picks per batch.
//
// Layouts (complex):  F6[f][j][p][q], Z6[f][j][zz][p], W3[g][j][zz][p], H3[g][j][p][q].
// A launch covers nch channels of one shape: blockIdx.z = channel * N_y + node.
//
// The z inverse exists in two kernels (k_zinv2, and k_zxrow, which redoes its first pass and
// keeps two outputs) that must give bitwise the same values.  Which multiplies the compiler
// fuses into adds depends on how a transform's outputs are used next, so both take their DFTs
// and twiddles from chanenv::strict, a copy compiled without multiply-add contraction (every
// operation rounds on its own); the other transforms, each in one code path, contract.
#include "device_common.h"

namespace chanenv {
namespace strict {
#pragma clang fp contract(off)
#include "small_dft.inc"
#pragma clang fp contract(fast)
}  // namespace strict

#include "small_dft.inc"

template <int L>
struct FftPlan;
template <> struct FftPlan<6> { static constexpr int A = 3, B = 2; };
template <> struct FftPlan<12> { static constexpr int A = 4, B = 3; };
template <> struct FftPlan<24> { static constexpr int A = 6, B = 4; };
template <> struct FftPlan<48> { static constexpr int A = 8, B = 6; };
template <> struct FftPlan<96> { static constexpr int A = 12, B = 8; };
template <> struct FftPlan<192> { static constexpr int A = 16, B = 12; };

// LDS layout of a transform: pass 1 writes each task's A outputs at stride AP (odd, so that
// the tasks of a wavefront land in different banks) and sequences lie LS apart (odd, at least
// L + 1 and B AP).  Pass 2 reads back at the same strides; the data stay bitwise the same.
template <int L>
struct FftLds {
  static constexpr int A = FftPlan<L>::A, B = FftPlan<L>::B;
  static constexpr int AP = A | 1;
  static constexpr int LS = ((L + 1 > B * AP) ? L + 1 : B * AP) | 1;
};



// Threads of a z-kernel block: PB pencils (at most 32) times the first pass's length A.  The
// launch bound states that maximum, so that the compiler may give the long transforms more than
// the 128 registers a 1024-thread bound allows (k_zinv2<192> spilled 52 of them under it).
template <int L>
constexpr int zkernel_threads() { return ((32 * FftPlan<L>::A + 63) / 64) * 64; }

// ---------------------------------------------------------------------------
// z inverse: block (p chunk, field, node); F6 -> Z6.
// ---------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(zkernel_threads<L>()) void k_zinv2(const PlaneChan* __restrict__ chans, int ny, int PB) {
  constexpr int FA = FftPlan<L>::A, FB = FftPlan<L>::B;
  constexpr int LP = FftLds<L>::LS, AP = FftLds<L>::AP;
  extern __shared__ double dyn_lds[];
  cplx* tw = reinterpret_cast<cplx*>(dyn_lds);
  cplx* Y = tw + L;
  const PlaneChan A = chans[blockIdx.z / ny];
  // a rejected action leaves every buffer untouched (tested at the stores, so that the
  // status load overlaps the data loads)
  const bool skip = (*A.status & STATUS_BAD_ACTION) != 0;
  const int p0 = blockIdx.x * PB, f = blockIdx.y, j = blockIdx.z % ny;
  const int np = min(PB, A.nkx - p0);
  constexpr int nz = 2 * L / 3, h = nz / 2;  // N_z (M_z = 3 N_z/2; checked at launch)
  for (int t = threadIdx.x; t < L; t += blockDim.x) tw[t] = A.twz[t];
  __syncthreads();
  const size_t fj = (size_t)f * A.ny + j;
  const cplx* src = A.F6 + (fj * A.nkx + p0) * nz;
  for (int task = threadIdx.x; task < np * FB; task += blockDim.x) {
    // unsigned, so that n2 < B is known and the padding test of each term n1 folds where all
    // of its B rows lie on one side
    const int p = (int)((unsigned)task / FB), n2 = (int)((unsigned)task % FB);
    cplx t[FA];
#pragma unroll
    for (int n1 = 0; n1 < FA; ++n1) {
      const int zz = FB * n1 + n2;
      const int q = (zz < h) ? zz : ((zz > L - h) ? zz - L + nz : -1);
      t[n1] = (q >= 0) ? src[(size_t)p * nz + q] : cz();
    }
    strict::Dft<FA, 1>::run(t);
    cplx* y = Y + p * LP + n2 * AP;
#pragma unroll
    for (int k1 = 0; k1 < FA; ++k1) y[k1] = strict::twiddle<L, 1>(t[k1], tw, n2 * k1);
  }
  __syncthreads();
  cplx* dst = A.Z6 + fj * L * A.nkx + p0;
  for (int task = threadIdx.x; task < FA * np; task += blockDim.x) {
    const int k1 = task / np, p = task - k1 * np;
    cplx u[FB];
#pragma unroll
    for (int n2 = 0; n2 < FB; ++n2) u[n2] = Y[p * LP + n2 * AP + k1];
    strict::Dft<FB, 1>::run(u);
    if (skip) continue;
#pragma unroll
    for (int k2 = 0; k2 < FB; ++k2) dst[(size_t)(k1 + FA * k2) * A.nkx + p] = u[k2];
  }
}

// ---------------------------------------------------------------------------
// z forward: block (p chunk, product, node); W3 -> H3.
// ---------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(zkernel_threads<L>()) void k_zfwd2(const PlaneChan* __restrict__ chans, int ny, int PB) {
  constexpr int FA = FftPlan<L>::A, FB = FftPlan<L>::B;
  constexpr int LP = FftLds<L>::LS, AP = FftLds<L>::AP;
  extern __shared__ double dyn_lds[];
  cplx* tw = reinterpret_cast<cplx*>(dyn_lds);
  cplx* X0 = tw + L;       // the p = 0 pencil, for the Hermitian fix
  cplx* Y = X0 + L;
  const PlaneChan A = chans[blockIdx.z / ny];
  const bool skip = (*A.status & STATUS_BAD_ACTION) != 0;  // tested at the stores
  const int p0 = blockIdx.x * PB, g = blockIdx.y, j = blockIdx.z % ny;
  const int np = min(PB, A.nkx - p0);
  constexpr int nz = 2 * L / 3, h = nz / 2;  // N_z (checked at launch)
  for (int t = threadIdx.x; t < L; t += blockDim.x) tw[t] = A.twz[t];
  __syncthreads();
  const size_t gj = (size_t)g * A.ny + j;
  const cplx* src = A.W3 + gj * L * A.nkx + p0;
  for (int task = threadIdx.x; task < FB * np; task += blockDim.x) {
    const int n2 = task / np, p = task - n2 * np;
    cplx t[FA];
#pragma unroll
    for (int n1 = 0; n1 < FA; ++n1) t[n1] = src[(size_t)(FB * n1 + n2) * A.nkx + p];
    Dft<FA, -1>::run(t);
    cplx* y = Y + p * LP + n2 * AP;
#pragma unroll
    for (int k1 = 0; k1 < FA; ++k1) y[k1] = twiddle<L, -1>(t[k1], tw, n2 * k1);
  }
  __syncthreads();
  cplx* dst = A.H3 + (gj * A.nkx + p0) * nz;
  const double sc = A.scale;
  for (int task = threadIdx.x; task < np * FA; task += blockDim.x) {
    const int p = (int)((unsigned)task / FA), k1 = (int)((unsigned)task % FA);  // k1 < A known
    cplx u[FB];
#pragma unroll
    for (int n2 = 0; n2 < FB; ++n2) u[n2] = Y[p * LP + n2 * AP + k1];
    Dft<FB, -1>::run(u);
#pragma unroll
    for (int k2 = 0; k2 < FB; ++k2) {
      const int zz = k1 + FA * k2;
      const int q = (zz < h) ? zz : ((zz > L - h) ? zz - L + nz : -1);
      if (q < 0) continue;
      const cplx v = cscale(u[k2], sc);
      if (p0 + p == 0) {
        X0[q] = v;
      } else if (!skip) {
        dst[(size_t)p * nz + q] = v;
      }
    }
  }
  if (p0 == 0 && !skip) {
    __syncthreads();
    for (int q = threadIdx.x; q < nz; q += blockDim.x) {
      cplx v = cz();
      if (q == 0) {
        v = make_double2(X0[0].x, 0.0);
      } else if (q < h) {
        v = X0[q];
      } else if (q > h) {
        v = cconj(X0[nz - q]);
      }
      dst[q] = v;
    }
  }
  // Nyquist row q = N_z/2 stays zero (written once when the buffers are cleared).
}

// ---------------------------------------------------------------------------
// x rows on a block's staged sequences S[field * P + pair][LS] (the packed spectra of P pairs
// of padded z rows of node j, see k_xrow2, and a zero at S[.][2 N_x/2]): six inverse real FFTs, the products, three
// forward FFTs and the unpacking, one task per thread in every phase (the block has 6 P A
// threads).  Pair pr holds rows z = row0 + rstep pr and z + 1; the products go to W3 unless
// skip.  Pass 1 writes each task's A outputs at stride AP, sequences lie LS apart.
// ---------------------------------------------------------------------------
template <int L, int LS, int AP>
__device__ __forceinline__ void xrow_body(const PlaneChan& A, cplx* S, const cplx* tw, int P, int j, int row0,
                                          int rstep, bool skip) {
  constexpr int FA = FftPlan<L>::A, FB = FftPlan<L>::B;
  static_assert(FA >= FB, "pass 1 has at most one task per thread");
  static_assert(LS > L && LS >= (FB - 1) * AP + FA, "LDS sequence stride too small");
  static_assert(2 * (L / 3) < LS, "room for the zero slot after the packed spectrum");
  constexpr int nkx = L / 3;  // stored x modes N_x/2 (M_x = 3 N_x/2; checked at launch)
  const int ny = A.ny;
  const int mz = 3 * A.nz / 2;
  const int tid = threadIdx.x, nthr = blockDim.x;
  // 1. inverse pass 1, one task (f, pair, n2) per thread: the packed spectrum k = B n1 + n2 is
  // read into registers (the unstored modes from the sequence's zero slot S[seq][2 nkx], so that
  // every read is unconditional), then (after every task has read its inputs) transformed and
  // written back over the staged rows
  {
    const int task = tid;
    const bool have = task < 6 * P * FB;
    const int seq = task / FB, n2 = task - seq * FB;
    cplx t[FA];
    if (have) {
      const cplx* z = S + seq * LS;
#pragma unroll
      for (int n1 = 0; n1 < FA; ++n1) {
        const int k = FB * n1 + n2;
        t[n1] = z[(k < nkx) ? k : ((k > L - nkx) ? nkx + (L - k) : 2 * nkx)];
      }
    }
    __syncthreads();
    if (have) {
      Dft<FA, 1>::run(t);
      cplx* y = S + seq * LS + n2 * AP;
#pragma unroll
      for (int k1 = 0; k1 < FA; ++k1) y[k1] = twiddle<L, 1>(t[k1], tw, n2 * k1);
    }
  }
  __syncthreads();
  // 2. inverse pass 2, tasks (f, pair, k1): values at x = k1 + A k2, back into S in order
  {
    const int ntask = 6 * P * FA;
    cplx X[FB];
    int base = 0, k1 = 0;
    const bool have = tid < ntask;
    if (have) {
      const int seq = tid / FA;
      k1 = tid - seq * FA;
      base = seq * LS;
#pragma unroll
      for (int n2 = 0; n2 < FB; ++n2) X[n2] = S[base + n2 * AP + k1];
      Dft<FB, 1>::run(X);
    }
    __syncthreads();
    if (have) {
#pragma unroll
      for (int k2 = 0; k2 < FB; ++k2) S[base + k1 + FA * k2] = X[k2];
    }
  }
  __syncthreads();
  // 3. products at every (pair, x); re = the pair's first row, im = its second
  for (int task = tid; task < P * L; task += nthr) {
    const int pr = task / L, x = task - pr * L;
    const cplx U = S[(0 * P + pr) * LS + x], V = S[(1 * P + pr) * LS + x], W = S[(2 * P + pr) * LS + x];
    const cplx OX = S[(3 * P + pr) * LS + x], OY = S[(4 * P + pr) * LS + x], OZ = S[(5 * P + pr) * LS + x];
    S[(0 * P + pr) * LS + x] = make_double2(V.x * OZ.x - W.x * OY.x, V.y * OZ.y - W.y * OY.y);
    S[(1 * P + pr) * LS + x] = make_double2(W.x * OX.x - U.x * OZ.x, W.y * OX.y - U.y * OZ.y);
    S[(2 * P + pr) * LS + x] = make_double2(U.x * OY.x - V.x * OX.x, U.y * OY.y - V.y * OX.y);
  }
  __syncthreads();
  // 4. forward pass 1, tasks (g, pair, n2)
  {
    const int ntask = 3 * P * FB;
    cplx t[FA];
    int base = 0, n2 = 0;
    const bool have = tid < ntask;
    if (have) {
      const int seq = tid / FB;
      n2 = tid - seq * FB;
      base = seq * LS;
#pragma unroll
      for (int n1 = 0; n1 < FA; ++n1) t[n1] = S[base + FB * n1 + n2];
      Dft<FA, -1>::run(t);
    }
    __syncthreads();
    if (have) {
#pragma unroll
      for (int k1 = 0; k1 < FA; ++k1) S[base + n2 * AP + k1] = twiddle<L, -1>(t[k1], tw, n2 * k1);
    }
  }
  __syncthreads();
  // 5. forward pass 2, tasks (g, pair, k1): spectrum k = k1 + A k2 back into S in order
  {
    const int ntask = 3 * P * FA;
    cplx X[FB];
    int base = 0, k1 = 0;
    const bool have = tid < ntask;
    if (have) {
      const int seq = tid / FA;
      k1 = tid - seq * FA;
      base = seq * LS;
#pragma unroll
      for (int n2 = 0; n2 < FB; ++n2) X[n2] = S[base + n2 * AP + k1];
      Dft<FB, -1>::run(X);
    }
    __syncthreads();
    if (have) {
#pragma unroll
      for (int k2 = 0; k2 < FB; ++k2) S[base + k1 + FA * k2] = X[k2];
    }
  }
  __syncthreads();
  // 6. unpack the two rows of each pair: a = (Y_k + conj Y_{L-k})/2, b = (Y_k - conj Y_{L-k})/(2i)
  for (int task = tid; task < 3 * P * nkx && !skip; task += nthr) {
    const int seq = task / nkx, k = task - seq * nkx;
    const int g = seq / P, pr = seq - g * P;
    const cplx Yk = S[seq * LS + k];
    const cplx Ym = cconj(S[seq * LS + ((L - k) % L)]);
    const cplx Xa = make_double2(0.5 * (Yk.x + Ym.x), 0.5 * (Yk.y + Ym.y));
    const cplx Xb = make_double2(0.5 * (Yk.y - Ym.y), -0.5 * (Yk.x - Ym.x));
    const int za = row0 + rstep * pr;
    cplx* wa = A.W3 + (((size_t)g * ny + j) * mz + za) * nkx;
    wa[k] = Xa;
    wa[nkx + k] = Xb;
  }
}

// Threads of an x-row block of P pairs of rows: one per task of the second pass, 6 P A.
template <int L>
constexpr int xrow_threads_c(int P) { return ((6 * P * FftPlan<L>::A + 63) / 64) * 64; }

// ---------------------------------------------------------------------------
// x rows: block (pair chunk, node); Z6 -> W3.  Each phase gives one task per thread so
// that the six inverse transforms, the products and the three forward transforms of a
// block are all in flight together; S holds 6 sequences per pair, transformed in place.
// PC: the pairs per block as a compile-time constant (the tuner's usual picks, so that the
// index arithmetic has no division by a run-time P), or 0 for P taken from the argument.
// ---------------------------------------------------------------------------
template <int L, int PC>
__global__ __launch_bounds__(PC > 0 ? xrow_threads_c<L>(PC) : 1024) void k_xrow2(const PlaneChan* __restrict__ chans,
                                                                                  int nyc, int Parg) {
  constexpr int LP = FftLds<L>::LS;
  const int P = PC > 0 ? PC : Parg;
  extern __shared__ double dyn_lds[];
  cplx* tw = reinterpret_cast<cplx*>(dyn_lds);
  cplx* S = tw + L;         // [field][pair][LP]
  const PlaneChan A = chans[blockIdx.y / nyc];
  const bool skip = (*A.status & STATUS_BAD_ACTION) != 0;  // tested at the stores
  const int pair0 = blockIdx.x * P, j = blockIdx.y % nyc;
  constexpr int nkx = L / 3;  // stored x modes N_x/2 (checked at launch)
  const int ny = A.ny;
  const int mz = 3 * A.nz / 2;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int t = tid; t < L; t += nthr) tw[t] = A.twx[t];
  // 0. stage the rows: for every (field, pair) sequence and stored mode m < N_x/2, the packed
  // spectrum P_m = a_m + i b_m of the two rows (a_0, b_0 real) at S[seq][m] and the packed
  // conjugates Q_m = conj(a_m) + i conj(b_m), which give modes L - m, at S[seq][nkx + m]
  // (2 nkx <= L + 1 slots), and a zero at S[seq][2 nkx].  Each stored mode is loaded once,
  // coalesced; a thread issues the loads of all its items (at most IT: the block has 6 P A
  // threads and N_x/2 = L/3 modes per sequence) before it waits for any.
  constexpr int IT = (nkx + FftPlan<L>::A - 1) / FftPlan<L>::A;
  cplx xa[IT], xb[IT];
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const int it = tid + r * nthr;
    if (it < 6 * P * nkx) {
      const int seq = it / nkx, m = it - seq * nkx;
      const int f = seq / P, pr = seq - f * P;
      const int za = 2 * (pair0 + pr);
      const cplx* ra = A.Z6 + (((size_t)f * ny + j) * mz + za) * nkx;
      xa[r] = ra[m];
      xb[r] = ra[nkx + m];
    }
  }
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const int it = tid + r * nthr;
    if (it < 6 * P * nkx) {
      const int seq = it / nkx, m = it - seq * nkx;
      cplx a = xa[r], b = xb[r];
      if (m == 0) {
        a.y = 0.0;
        b.y = 0.0;
        S[seq * LP + 2 * nkx] = cz();
      }
      S[seq * LP + m] = make_double2(a.x - b.y, a.y + b.x);
      S[seq * LP + nkx + m] = make_double2(a.x + b.y, b.x - a.y);
    }
  }
  __syncthreads();
  xrow_body<L, LP, FftLds<L>::AP>(A, S, tw, P, j, 2 * pair0, 2, skip);
}

// ---------------------------------------------------------------------------
// z inverse and x rows in one launch (M_z, M_x in {48, 96}): the padded z rows never leave
// the block.  Block (node, k1 pair): the rows z = k1 + A_z k2 and z + 1 (k1 even, every k2)
// of one node, which are the outputs k1, k1 + 1 of the z inverse's second pass for every
// (field, p) pencil.  The first pass (the DFT over n1 of each task n2) is done in full and
// its outputs k1, k1 + 1 kept, so every value is the one k_zinv2 writes to Z6, and the rows
// are paired as in k_xrow2 (two rows 2m, 2m + 1 per complex sequence): W3 is bitwise that of
// k_zinv2 + k_xrow2.  Each node's blocks run on one XCD (the hardware deals workgroup b to
// XCD b mod 8), so that its input plane, read by A_z / 2 blocks, is fetched into one L2.
// ---------------------------------------------------------------------------
template <int MZ, int MX>
constexpr bool zx_fusable() { return (MZ == 48 || MZ == 96) && (MX == 48 || MX == 96); }

template <int MZ, int MX>
struct ZxPlan {
  static constexpr int ZA = FftPlan<MZ>::A, ZB = FftPlan<MZ>::B, XA = FftPlan<MX>::A, XB = FftPlan<MX>::B;
  static constexpr int NKX = MX / 3;             // stored x modes: N_x / 2 with M_x = 3 N_x / 2
  static constexpr int P = ZB;                   // pairs of rows per block, one per k2
  static constexpr int NG = ZA / 2;              // blocks per node
  static constexpr int AP = XA | 1;
  static constexpr int LS = ((MX + 1 > (XB - 1) * AP + XA) ? MX + 1 : (XB - 1) * AP + XA) | 1;
  static constexpr int YS = 2 * ZB + 1;          // first-pass outputs kept per pencil, padded odd
  static constexpr int THREADS = ((6 * P * XA + 63) / 64) * 64;
  static constexpr int TW = MZ + (MX == MZ ? 0 : MX);
  static constexpr int LDS_CPLX = TW + 6 * P * LS;
  static_assert(ZA % 2 == 0, "k1 pairs");
  static_assert(NKX * YS <= P * LS, "first-pass outputs fit in the row buffer");
  static_assert(12 * NKX <= THREADS, "one second-pass task per thread");
};

template <int MZ, int MX>
__global__ __launch_bounds__((ZxPlan<MZ, MX>::THREADS)) void k_zxrow(const PlaneChan* __restrict__ chans, int ny,
                                                                   int nnodes) {
  using ZP = ZxPlan<MZ, MX>;
  constexpr int ZA = ZP::ZA, ZB = ZP::ZB, P = ZP::P, LS = ZP::LS, YS = ZP::YS, NKX = ZP::NKX;
  extern __shared__ double dyn_lds[];
  cplx* twz = reinterpret_cast<cplx*>(dyn_lds);
  cplx* twx = (MX == MZ) ? twz : twz + MZ;       // the same table when the lengths agree
  cplx* S = twz + ZP::TW;                        // [field][pair][LS]
  cplx* Y = S;                                   // first-pass outputs [field][p][YS], read before S is written
  const int b = blockIdx.x, xcd = b & 7, sl = b >> 3;
  const int grp = sl % ZP::NG, node = (sl / ZP::NG) * 8 + xcd;
  if (node >= nnodes) return;                    // the whole block: before any barrier
  const PlaneChan A = chans[node / ny];
  const int j = node % ny;
  const bool skip = (*A.status & STATUS_BAD_ACTION) != 0;  // tested at the stores
  const int kb = 2 * grp;                        // this block's k1 pair: kb, kb + 1
  constexpr int nz = 2 * MZ / 3, h = nz / 2;  // N_z (checked at launch)
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int t = tid; t < MZ; t += nthr) twz[t] = A.twz[t];
  if (MX != MZ)
    for (int t = tid; t < MX; t += nthr) twx[t] = A.twx[t];
  __syncthreads();
  // z pass 1, tasks (f, p, n2): the full DFT over n1 of x[B n1 + n2] (zero padding as in
  // k_zinv2), outputs kb and kb + 1 twiddled and kept
  for (int task = tid; task < 6 * NKX * ZB; task += nthr) {
    const int fp = (int)((unsigned)task / ZB), n2 = (int)((unsigned)task % ZB);  // n2 < B known
    const int f = fp / NKX, p = fp - f * NKX;
    const cplx* src = A.F6 + (((size_t)f * A.ny + j) * NKX + p) * nz;
    cplx t[ZA];
#pragma unroll
    for (int n1 = 0; n1 < ZA; ++n1) {
      const int zz = ZB * n1 + n2;
      const int q = (zz < h) ? zz : ((zz > MZ - h) ? zz - MZ + nz : -1);
      t[n1] = (q >= 0) ? src[q] : cz();
    }
    strict::Dft<ZA, 1>::run(t);
    cplx y0 = t[0], y1 = t[1];
#pragma unroll
    for (int k1 = 2; k1 < ZA; k1 += 2) {
      if (k1 == kb) {
        y0 = t[k1];
        y1 = t[k1 + 1];
      }
    }
    Y[fp * YS + 2 * n2] = strict::twiddle<MZ, 1>(y0, twz, n2 * kb);
    Y[fp * YS + 2 * n2 + 1] = strict::twiddle<MZ, 1>(y1, twz, n2 * (kb + 1));
  }
  __syncthreads();
  // z pass 2, tasks (f, p, s): the DFT over n2 gives rows kb + s + A_z k2 of pencil (f, p);
  // lane pairs (s = 0, 1) exchange their values and write the packed sequences of k_xrow2's
  // staging: the s = 0 lane P_p = a_p + i b_p at S[f P + k2][p], the s = 1 lane
  // Q_p = conj(a_p) + i conj(b_p) at S[f P + k2][N_x/2 + p] (a, b: rows kb, kb + 1).  Every
  // lane takes part in the exchange (out-of-range tasks on a clamped pencil, not stored).
  {
    const int task = tid;
    const bool have = task < 12 * NKX;
    const int fp = have ? (task >> 1) : 0, sidx = task & 1;
    cplx u[ZB];
#pragma unroll
    for (int n2 = 0; n2 < ZB; ++n2) u[n2] = Y[fp * YS + 2 * n2 + sidx];
    strict::Dft<ZB, 1>::run(u);
    __syncthreads();                             // every Y read before S is written
    const int f = fp / NKX, p = fp - f * NKX;
#pragma unroll
    for (int k2 = 0; k2 < ZB; ++k2) {
      const cplx o = cmov<DPP_QUAD_XOR1>(u[k2]);  // the partner row's value
      cplx xa = sidx ? o : u[k2], xb = sidx ? u[k2] : o;
      if (p == 0) {
        xa.y = 0.0;
        xb.y = 0.0;
      }
      if (have) {
        cplx* seq = S + (f * P + k2) * LS;
        if (sidx == 0) {
          seq[p] = make_double2(xa.x - xb.y, xa.y + xb.x);
        } else {
          seq[NKX + p] = make_double2(xa.x + xb.y, xb.x - xa.y);
          if (p == 0) seq[2 * NKX] = cz();       // the zero slot the x rows' first pass reads
        }
      }
    }
  }
  __syncthreads();
  xrow_body<MX, LS, ZP::AP>(A, S, twx, P, j, kb, ZA, skip);
}

// ---------------------------------------------------------------------------
// Small grids (M_z = M_x = 24): the whole plane pass of one node in one block, the z-inverse
// output and the x-row products kept in LDS instead of Z6 / W3.  Every phase is the
// corresponding phase of k_zinv2, k_xrow2 (all M_z/2 pairs of rows) and k_zfwd2 with the same
// operations in the same order, so the results are bitwise those of the three launches; what
// goes is two kernel boundaries and the Z6 / W3 round trips, which dominate these small planes.
// Block: channel * N_y + node.
// ---------------------------------------------------------------------------
template <int MZ, int MX>
struct SmallPlane {
  static constexpr int NKX = MX / 3;
  static constexpr int P = MZ / 2;                 // pairs of z rows
  static constexpr int LPZ = FftLds<MZ>::LS, APZ = FftLds<MZ>::AP;
  static constexpr int LPX = FftLds<MX>::LS;
  static constexpr int SCR_A = 6 * NKX * LPZ, SCR_B = 6 * P * LPX, SCR_C = 3 * NKX * LPZ;
  static constexpr int SCR = (SCR_A > SCR_B ? (SCR_A > SCR_C ? SCR_A : SCR_C) : (SCR_B > SCR_C ? SCR_B : SCR_C));
  static constexpr int LDS_CPLX = MZ + MX + 6 * MZ * NKX + SCR + 3 * MZ;
  static constexpr int THREADS = ((6 * P * FftPlan<MX>::A + 63) / 64) * 64;
};

template <int MZ, int MX>
__global__ __launch_bounds__((SmallPlane<MZ, MX>::THREADS)) void k_plane_small(const PlaneChan* __restrict__ chans,
                                                                             int ny) {
  using SP = SmallPlane<MZ, MX>;
  constexpr int NKX = SP::NKX, P = SP::P, LPZ = SP::LPZ, APZ = SP::APZ;
  constexpr int ZA = FftPlan<MZ>::A, ZB = FftPlan<MZ>::B;
  constexpr int XA = FftPlan<MX>::A, XB = FftPlan<MX>::B;
  constexpr int LPX = FftLds<MX>::LS, APX = FftLds<MX>::AP;
  static_assert(XA >= XB, "x pass 1 has at most one task per thread");
  extern __shared__ double dyn_lds[];
  cplx* twz = reinterpret_cast<cplx*>(dyn_lds);
  cplx* twx = twz + MZ;
  cplx* ZW = twx + MX;             // Z [f][zz][p] (z inverse), later W [g][zz][p] (x-row output)
  cplx* SCR = ZW + 6 * MZ * NKX;   // pass scratch of each phase
  cplx* X0 = SCR + SP::SCR;        // [g][q]: the p = 0 pencils, for the Hermitian fix
  const PlaneChan A = chans[blockIdx.x / ny];
  const bool skip = (*A.status & STATUS_BAD_ACTION) != 0;  // tested at the stores
  const int j = blockIdx.x % ny;
  constexpr int nz = 2 * MZ / 3, h = nz / 2;  // N_z (checked at launch)
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int t = tid; t < MZ; t += nthr) twz[t] = A.twz[t];
  for (int t = tid; t < MX; t += nthr) twx[t] = A.twx[t];
  __syncthreads();

  // A. z inverse of every (field, p) pencil (k_zinv2)
  for (int task = tid; task < 6 * NKX * ZB; task += nthr) {
    const int f = task / (NKX * ZB), rem = task - f * NKX * ZB;
    const int p = (int)((unsigned)rem / ZB), n2 = (int)((unsigned)rem % ZB);  // n2 < B known
    const cplx* src = A.F6 + (((size_t)f * A.ny + j) * NKX + p) * nz;
    cplx t[ZA];
#pragma unroll
    for (int n1 = 0; n1 < ZA; ++n1) {
      const int zz = ZB * n1 + n2;
      const int q = (zz < h) ? zz : ((zz > MZ - h) ? zz - MZ + nz : -1);
      t[n1] = (q >= 0) ? src[q] : cz();
    }
    Dft<ZA, 1>::run(t);
    cplx* y = SCR + (f * NKX + p) * LPZ + n2 * APZ;
#pragma unroll
    for (int k1 = 0; k1 < ZA; ++k1) y[k1] = twiddle<MZ, 1>(t[k1], twz, n2 * k1);
  }
  __syncthreads();
  for (int task = tid; task < 6 * ZA * NKX; task += nthr) {
    const int f = task / (ZA * NKX), rem = task - f * ZA * NKX;
    const int k1 = rem / NKX, p = rem - k1 * NKX;
    cplx u[ZB];
#pragma unroll
    for (int n2 = 0; n2 < ZB; ++n2) u[n2] = SCR[(f * NKX + p) * LPZ + n2 * APZ + k1];
    Dft<ZB, 1>::run(u);
#pragma unroll
    for (int k2 = 0; k2 < ZB; ++k2) ZW[(f * MZ + k1 + ZA * k2) * NKX + p] = u[k2];
  }
  __syncthreads();

  // B. x rows, all pairs (k_xrow2 with pair0 = 0); S = SCR [field][pair][LPX]
  cplx* S = SCR;
  for (int it = tid; it < 6 * P * NKX; it += nthr) {
    const int seq = it / NKX, m = it - seq * NKX;
    const int f = seq / P, pr = seq - f * P;
    const cplx* ra = ZW + (f * MZ + 2 * pr) * NKX;
    cplx xa = ra[m], xb = ra[NKX + m];
    if (m == 0) {
      xa.y = 0.0;
      xb.y = 0.0;
    }
    S[seq * LPX + m] = make_double2(xa.x - xb.y, xa.y + xb.x);
    S[seq * LPX + NKX + m] = make_double2(xa.x + xb.y, xb.x - xa.y);
  }
  __syncthreads();
  {
    const int task = tid;
    const bool have = task < 6 * P * XB;
    const int seq = task / XB, n2 = task - seq * XB;
    cplx t[XA];
    if (have) {
      const cplx* z = S + seq * LPX;
#pragma unroll
      for (int n1 = 0; n1 < XA; ++n1) {
        const int k = XB * n1 + n2;
        t[n1] = (k < NKX) ? z[k] : ((k > MX - NKX) ? z[NKX + (MX - k)] : cz());
      }
    }
    __syncthreads();
    if (have) {
      Dft<XA, 1>::run(t);
      cplx* y = S + seq * LPX + n2 * APX;
#pragma unroll
      for (int k1 = 0; k1 < XA; ++k1) y[k1] = twiddle<MX, 1>(t[k1], twx, n2 * k1);
    }
  }
  __syncthreads();
  {
    const int ntask = 6 * P * XA;
    cplx X[XB];
    int base = 0, k1 = 0;
    const bool have = tid < ntask;
    if (have) {
      const int seq = tid / XA;
      k1 = tid - seq * XA;
      base = seq * LPX;
#pragma unroll
      for (int n2 = 0; n2 < XB; ++n2) X[n2] = S[base + n2 * APX + k1];
      Dft<XB, 1>::run(X);
    }
    __syncthreads();
    if (have) {
#pragma unroll
      for (int k2 = 0; k2 < XB; ++k2) S[base + k1 + XA * k2] = X[k2];
    }
  }
  __syncthreads();
  for (int task = tid; task < P * MX; task += nthr) {
    const int pr = task / MX, x = task - pr * MX;
    const cplx U = S[(0 * P + pr) * LPX + x], V = S[(1 * P + pr) * LPX + x], W = S[(2 * P + pr) * LPX + x];
    const cplx OX = S[(3 * P + pr) * LPX + x], OY = S[(4 * P + pr) * LPX + x], OZ = S[(5 * P + pr) * LPX + x];
    S[(0 * P + pr) * LPX + x] = make_double2(V.x * OZ.x - W.x * OY.x, V.y * OZ.y - W.y * OY.y);
    S[(1 * P + pr) * LPX + x] = make_double2(W.x * OX.x - U.x * OZ.x, W.y * OX.y - U.y * OZ.y);
    S[(2 * P + pr) * LPX + x] = make_double2(U.x * OY.x - V.x * OX.x, U.y * OY.y - V.y * OX.y);
  }
  __syncthreads();
  {
    const int ntask = 3 * P * XB;
    cplx t[XA];
    int base = 0, n2 = 0;
    const bool have = tid < ntask;
    if (have) {
      const int seq = tid / XB;
      n2 = tid - seq * XB;
      base = seq * LPX;
#pragma unroll
      for (int n1 = 0; n1 < XA; ++n1) t[n1] = S[base + XB * n1 + n2];
      Dft<XA, -1>::run(t);
    }
    __syncthreads();
    if (have) {
#pragma unroll
      for (int k1 = 0; k1 < XA; ++k1) S[base + n2 * APX + k1] = twiddle<MX, -1>(t[k1], twx, n2 * k1);
    }
  }
  __syncthreads();
  {
    const int ntask = 3 * P * XA;
    cplx X[XB];
    int base = 0, k1 = 0;
    const bool have = tid < ntask;
    if (have) {
      const int seq = tid / XA;
      k1 = tid - seq * XA;
      base = seq * LPX;
#pragma unroll
      for (int n2 = 0; n2 < XB; ++n2) X[n2] = S[base + n2 * APX + k1];
      Dft<XB, -1>::run(X);
    }
    __syncthreads();
    if (have) {
#pragma unroll
      for (int k2 = 0; k2 < XB; ++k2) S[base + k1 + XA * k2] = X[k2];
    }
  }
  __syncthreads();
  for (int task = tid; task < 3 * P * NKX; task += nthr) {
    const int seq = task / NKX, k = task - seq * NKX;
    const int g = seq / P, pr = seq - g * P;
    const cplx Yk = S[seq * LPX + k];
    const cplx Ym = cconj(S[seq * LPX + ((MX - k) % MX)]);
    const cplx Xa = make_double2(0.5 * (Yk.x + Ym.x), 0.5 * (Yk.y + Ym.y));
    const cplx Xb = make_double2(0.5 * (Yk.y - Ym.y), -0.5 * (Yk.x - Ym.x));
    cplx* wa = ZW + (g * MZ + 2 * pr) * NKX;
    wa[k] = Xa;
    wa[NKX + k] = Xb;
  }
  __syncthreads();

  // C. z forward of every (product, p) pencil, truncation, 1/(M_x M_z), Hermitian fix (k_zfwd2)
  for (int task = tid; task < 3 * ZB * NKX; task += nthr) {
    const int g = task / (ZB * NKX), rem = task - g * ZB * NKX;
    const int n2 = rem / NKX, p = rem - n2 * NKX;
    cplx t[ZA];
#pragma unroll
    for (int n1 = 0; n1 < ZA; ++n1) t[n1] = ZW[(g * MZ + ZB * n1 + n2) * NKX + p];
    Dft<ZA, -1>::run(t);
    cplx* y = SCR + (g * NKX + p) * LPZ + n2 * APZ;
#pragma unroll
    for (int k1 = 0; k1 < ZA; ++k1) y[k1] = twiddle<MZ, -1>(t[k1], twz, n2 * k1);
  }
  __syncthreads();
  const double sc = A.scale;
  for (int task = tid; task < 3 * NKX * ZA; task += nthr) {
    const int g = task / (NKX * ZA), rem = task - g * NKX * ZA;
    const int p = rem / ZA, k1 = rem - p * ZA;
    cplx u[ZB];
#pragma unroll
    for (int n2 = 0; n2 < ZB; ++n2) u[n2] = SCR[(g * NKX + p) * LPZ + n2 * APZ + k1];
    Dft<ZB, -1>::run(u);
    cplx* dst = A.H3 + (((size_t)g * A.ny + j) * NKX + p) * nz;
#pragma unroll
    for (int k2 = 0; k2 < ZB; ++k2) {
      const int zz = k1 + ZA * k2;
      const int q = (zz < h) ? zz : ((zz > MZ - h) ? zz - MZ + nz : -1);
      if (q < 0) continue;
      const cplx v = cscale(u[k2], sc);
      if (p == 0) {
        X0[g * MZ + q] = v;
      } else if (!skip) {
        dst[q] = v;
      }
    }
  }
  __syncthreads();
  if (!skip) {
    for (int task = tid; task < 3 * nz; task += nthr) {
      const int g = task / nz, q = task - g * nz;
      const cplx* x0 = X0 + g * MZ;
      cplx v = cz();
      if (q == 0) {
        v = make_double2(x0[0].x, 0.0);
      } else if (q < h) {
        v = x0[q];
      } else if (q > h) {
        v = cconj(x0[nz - q]);
      }
      A.H3[(((size_t)g * A.ny + j) * NKX) * nz + q] = v;
    }
  }
  // Nyquist row q = N_z/2 stays zero (written once when the buffers are cleared).
}

// LDS of the x-row kernel with P pairs of rows per block, and its thread count.
template <int MX>
static size_t xrow_lds(int P) { return (size_t)(MX + (size_t)6 * P * FftLds<MX>::LS) * sizeof(cplx); }
template <int MX>
static int xrow_threads(int P) { return xrow_threads_c<MX>(P); }

// k_xrow2 with P pairs per block: the compile-time instance for the usual P, else the generic one.
template <int MX, int PC>
static void launch_xrow_pc(KernelTimer* tm, dim3 grid, int P, hipStream_t st, const PlaneChan* chans, int ny) {
  if constexpr (PC > 0 && xrow_threads_c<MX>(PC) <= 1024) {
    timed_launch(tm, KC_XROW, k_xrow2<MX, PC>, grid, dim3(xrow_threads<MX>(P)), xrow_lds<MX>(P), st, chans, ny, P);
  } else {
    timed_launch(tm, KC_XROW, k_xrow2<MX, 0>, grid, dim3(xrow_threads<MX>(P)), xrow_lds<MX>(P), st, chans, ny, P);
  }
}
template <int MX>
static void launch_xrow(KernelTimer* tm, dim3 grid, int P, hipStream_t st, const PlaneChan* chans, int ny) {
  switch (P) {
    case 1: launch_xrow_pc<MX, 1>(tm, grid, P, st, chans, ny); break;
    case 2: launch_xrow_pc<MX, 2>(tm, grid, P, st, chans, ny); break;
    case 3: launch_xrow_pc<MX, 3>(tm, grid, P, st, chans, ny); break;
    case 4: launch_xrow_pc<MX, 4>(tm, grid, P, st, chans, ny); break;
    case 6: launch_xrow_pc<MX, 6>(tm, grid, P, st, chans, ny); break;
    case 8: launch_xrow_pc<MX, 8>(tm, grid, P, st, chans, ny); break;
    case 12: launch_xrow_pc<MX, 12>(tm, grid, P, st, chans, ny); break;
    default: launch_xrow_pc<MX, 0>(tm, grid, P, st, chans, ny); break;
  }
}

template <int MZ, int MX>
static int launch_plane2(const Dims& d, const PlaneChan* chans, int nch, const PlaneTiles& t, hipStream_t st,
                         KernelTimer* tm) {
  if (d.nz != 2 * MZ / 3) return -1;       // the kernels take N_z from M_z
  if constexpr (MZ == 24 && MX == 24) {  // one launch per stage for the small planes
    using SP = SmallPlane<MZ, MX>;
    if (d.nkx != SP::NKX) return -1;
    const size_t shm = (size_t)SP::LDS_CPLX * sizeof(cplx);
    timed_launch(tm, KC_XROW, k_plane_small<MZ, MX>, dim3((unsigned)(d.ny * nch)), dim3(SP::THREADS), shm, st,
                 chans, d.ny);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  const int PB = t.PB, P = t.P;
  const int pairs = MZ / 2;
  if (PB < 1 || PB > d.nkx || d.nkx != MX / 3) return -1;
  if (((PB * FftPlan<MZ>::A + 63) / 64) * 64 > zkernel_threads<MZ>()) return -1;  // the z kernels' bound
  const int nblk = (d.nkx + PB - 1) / PB;
  const size_t shz = (size_t)(MZ + (size_t)PB * FftLds<MZ>::LS) * sizeof(cplx);
  const size_t shf = (size_t)(2 * MZ + (size_t)PB * FftLds<MZ>::LS) * sizeof(cplx);
  constexpr int ZA = FftPlan<MZ>::A;
  const int zthr = ((PB * ZA + 63) / 64) * 64;
  const unsigned nyz = (unsigned)(d.ny * nch);
  if (t.fused) {
    if constexpr (zx_fusable<MZ, MX>()) {
      using ZP = ZxPlan<MZ, MX>;
      if (d.nkx != ZP::NKX || P != ZP::P) return -1;
      const long nodes = (long)d.ny * nch;
      const long nblocks = (nodes + 7) / 8 * 8 * ZP::NG;
      if (nblocks > 0x7fffffffL) return -1;
      timed_launch(tm, KC_XROW, k_zxrow<MZ, MX>, dim3((unsigned)nblocks), dim3(ZP::THREADS),
                   (size_t)ZP::LDS_CPLX * sizeof(cplx), st, chans, d.ny, (int)nodes);
    } else {
      return -1;
    }
  } else {
    if (P < 1 || pairs % P != 0 || xrow_threads<MX>(P) > 1024) return -1;
    timed_launch(tm, KC_ZINV, k_zinv2<MZ>, dim3(nblk, 6, nyz), dim3(zthr), shz, st, chans, d.ny, PB);
    launch_xrow<MX>(tm, dim3(pairs / P, nyz), P, st, chans, d.ny);
  }
  timed_launch(tm, KC_ZFWD, k_zfwd2<MZ>, dim3(nblk, 3, nyz), dim3(zthr), shf, st, chans, d.ny, PB);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Valid tilings: z-kernel blocks of 8, 16 or 32 pencils (at most N_x/2); x-row blocks of P
// pairs of rows with P dividing M_z/2, at most 1024 threads and 80 KiB of LDS; where M_z and
// M_x are 48 or 96, also the fused z inverse and x rows with each of those z-forward blocks.
// form: 0 every tiling, 1 only the three-launch ones, 2 only the fused ones.
template <int MZ, int MX>
static void tiles2(const Dims& d, std::vector<PlaneTiles>* out, int form) {
  const int pairs = MZ / 2;
  std::vector<int> pbs;
  for (int pb : {8, 16, 32})
    if (pb <= d.nkx) pbs.push_back(pb);
  if (pbs.empty()) pbs.push_back(d.nkx);
  if (form != 2) {
    for (int P = 1; P <= pairs; ++P) {
      if (pairs % P != 0 || xrow_threads<MX>(P) > 1024 || xrow_lds<MX>(P) > 80 * 1024) continue;
      for (int pb : pbs) out->push_back(PlaneTiles{pb, P, 0});
    }
  }
  if constexpr (zx_fusable<MZ, MX>()) {
    if (form != 1 && d.nkx == ZxPlan<MZ, MX>::NKX)
      for (int pb : pbs) out->push_back(PlaneTiles{pb, ZxPlan<MZ, MX>::P, 1});
  }
}

template <int MZ>
static int dispatch_mx(const Dims& d, const PlaneChan* chans, int nch, const PlaneTiles& t, hipStream_t st,
                       KernelTimer* tm, std::vector<PlaneTiles>* tiles, int form) {
  switch (d.mx) {
#define CHANENV_MX(M)                                              \
    case M:                                                       \
      if (tiles) {                                                \
        tiles2<MZ, M>(d, tiles, form);                            \
        return 0;                                                 \
      }                                                           \
      return launch_plane2<MZ, M>(d, chans, nch, t, st, tm);
    CHANENV_MX(6)
    CHANENV_MX(12)
    CHANENV_MX(24)
    CHANENV_MX(48)
    CHANENV_MX(96)
    CHANENV_MX(192)
#undef CHANENV_MX
    default: return -1;
  }
}

static int dispatch_mz(const Dims& d, const PlaneChan* chans, int nch, const PlaneTiles& t, hipStream_t st,
                       KernelTimer* tm, std::vector<PlaneTiles>* tiles, int form) {
  switch (d.mz) {
    case 6: return dispatch_mx<6>(d, chans, nch, t, st, tm, tiles, form);
    case 12: return dispatch_mx<12>(d, chans, nch, t, st, tm, tiles, form);
    case 24: return dispatch_mx<24>(d, chans, nch, t, st, tm, tiles, form);
    case 48: return dispatch_mx<48>(d, chans, nch, t, st, tm, tiles, form);
    case 96: return dispatch_mx<96>(d, chans, nch, t, st, tm, tiles, form);
    case 192: return dispatch_mx<192>(d, chans, nch, t, st, tm, tiles, form);
    default: return -1;
  }
}

int launch_plane_pass(const Dims& d, const PlaneChan* chans, int nch, const PlaneTiles& t, hipStream_t st,
                      KernelTimer* tm) {
  if (nch < 1) return 0;
  if ((size_t)d.ny * nch > 65535) return -1;   // grid z limit
  return dispatch_mz(d, chans, nch, t, st, tm, nullptr, 0);
}

int plane_tile_candidates(const Dims& d, std::vector<PlaneTiles>* out, int form) {
  out->clear();
  const int rc = dispatch_mz(d, nullptr, 0, PlaneTiles{0, 0, 0}, nullptr, nullptr, out, form);
  return (rc == 0 && !out->empty()) ? 0 : -1;
}

}  // namespace chanenv
