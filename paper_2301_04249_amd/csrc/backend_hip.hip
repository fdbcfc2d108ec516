// gfx950 (MI355X) kernels of the RT-EOM-CCSD engine and the HIP backend.
//
//  gemm_mfma  complex/real GEMM on the matrix cores in float64
//             (v_mfma_f64_16x16x4f64) or float32 (v_mfma_f32_16x16x4f32),
//             64x64, 64x128, 128x64 or 128x128 output tile per work-group of four
//             or eight waves, operands staged through LDS.  Complex operands are
//             planar; a complex x complex product is three real MFMA products per
//             fragment pair (Gauss form), complex x real two.  Split-K and an
//             XCD-aware tile order fill the 256 CUs.
//  gemm_bf16x3  the same product with bf16 hi/lo operands, three bf16 products
//             (hi hi, hi lo, lo hi) per real product with float32 accumulation.
//  gemm_smallk  sums of K <= 16 on the vector ALUs.
//  permute    strided tensor copy / accumulate / scale (HBM bound).
//  ss_*       same-spin doubles between pair storage and blocks of full storage.
//  update     fused trapezoid update of all amplitudes with the per-spin masks,
//             the optional diagonal map and a max-|change| reduction.
//  energy     <Phi|(H_N e^T)_C|Phi> as a two-pass deterministic reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "backend.h"

namespace rteom {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int kThreads = 256;

struct GemmArgs {
  int64_t M, N, K, batch;
  const double* ar; const double* ai; int64_t asm_, ask, asb;
  const double* br; const double* bi; int64_t bsk, bsn, bsb;
  double* cr; double* ci; int64_t csm, csn, csb;
  double alpha;
  int beta;
  int64_t tiles_m, tiles_n;
  int splitk;
  int64_t kchunk;             // K elements per split (multiple of BK)
  double* pr; double* pi;     // partials [splitk][M][N]
  int m_fast;                 // logical tile order: row tiles fastest (B is the larger operand)
  int prio;                   // float64: raise the wave priority around the MFMA block
  // pre-split bf16 planes (gemm_bf16x3_split): A planes [batch][M][sld], B planes
  // [batch][N][sld] in the order re hi, re lo, im hi, im lo
  const unsigned short* sa[4];
  const unsigned short* sb[4];
  int64_t sld, sab, sbb;      // row length and batch strides (0: one matrix for all batch entries)
  // fp16x3 planes: per-row inverse scale factors (powers of two) of A [batch][M] and B [batch][N]
  const float* sca; const float* scb;
  int64_t aext, bext;         // elements spanned by A and B from ar / br (all batch entries)
};

// Output tile of work-group `bid`.  Work-groups are dispatched round-robin over
// the 8 XCDs; each XCD gets a contiguous range of logical tiles, so the ~64
// work-groups resident on one XCD hold consecutive logical tiles.  Logical
// tiles run in bands of kGroup tiles along one dimension (M when m_fast), the
// other dimension outermost within a band: the resident work-groups then cover
// about kGroup x kGroup tiles and read kGroup panels of each operand, each
// panel shared through that XCD's L2 by kGroup work-groups.
constexpr int64_t kGroup = 8;
__device__ inline void tile_coords(const GemmArgs& g, int64_t bid, int64_t& tm, int64_t& tn) {
  const int64_t nt = g.tiles_m * g.tiles_n;
  const int64_t q = nt / 8, r = nt % 8, xcd = bid % 8, slot = bid / 8;
  const int64_t logical = xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
  const int64_t tf = g.m_fast ? g.tiles_m : g.tiles_n;     // banded dimension
  const int64_t ts = g.m_fast ? g.tiles_n : g.tiles_m;
  const int64_t band = logical / (kGroup * ts), within = logical % (kGroup * ts);
  const int64_t width = min(kGroup, tf - band * kGroup);
  const int64_t f = band * kGroup + within % width, o = within / width;
  if (g.m_fast) { tm = f; tn = o; }
  else          { tn = f; tm = o; }
}

// Buffer resource over [p, p + n) elements (n clamped to the 31-bit byte range);
// loads outside it return zero.  Raw (unswizzled, stride 0) resource whose last
// descriptor word selects the 32-bit data format of gfx9 buffer loads.
template <typename S>
__device__ inline __amdgpu_buffer_rsrc_t window(const S* p, int64_t n) {
  const int64_t bytes = n <= 0 ? 0 : (n * (int64_t)sizeof(S) > 0x7fffffffLL ? 0x7fffffffLL : n * (int64_t)sizeof(S));
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename S>
__device__ inline S ldbuf(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ inline double ldbuf<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ inline float ldbuf<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Operand tiles are staged k-major in LDS ([BK][BM] for A, [BK][BN] for B) so
// that the MFMA fragment reads (row = lane % 16, k = lane / 16) are unit stride
// across lanes.  The next K tile is loaded into registers while the current one
// is multiplied, into the other of two LDS buffers: one barrier per K tile.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register r of a lane holds row 4*r + lane/16 of the 16x16 block
  static __device__ inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register r of a lane holds row 4*(lane/16) + r of the 16x16 block
  static __device__ inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Work-group tile (16*WM*GM) x (16*WN*GN): GM x GN waves, each holding WM x WN
// accumulator blocks of 16 x 16.  Wider tiles stage fewer
// operand bytes per MFMA; the complex x complex product already has four MFMAs
// per staged fragment pair and keeps 64 x 64.
// S is the operand storage type: double, or float for operands converted to
// float planes before the product (their pointers travel in the double fields of
// GemmArgs and their strides count floats).
// GM x GN waves (4 or 8) per work-group; with 8 waves each holds 2 x 2 blocks and
// uses at most 128 registers, so four waves share a SIMD and hide each other's
// LDS and barrier waits.
template <typename T, typename S, bool AC, bool BC, bool AKC, bool BKC, int WM, int WN, int GM = 2, int GN = 2>
__global__ __launch_bounds__(64 * GM * GN)
    __attribute__((amdgpu_waves_per_eu(GM * GN == 8 ? 4 : 2, 8))) void gemm_mfma(GemmArgs g) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NT = 64 * GM * GN;
  constexpr int TM = 16 * WM * GM, TN = 16 * WN * GN;
  constexpr int NA = TM * BK / NT, NB = TN * BK / NT;   // staged elements per thread and plane
  // LDS tiles: a k-contiguous operand is kept [row][BK + 1] (odd stride: the
  // coalesced writes and the fragment reads are both free of bank conflicts),
  // otherwise [k][row + 16] (the two 16-lane halves of a read hit disjoint banks).
  constexpr int AR = AKC ? TM : BK, AC_ = AKC ? BK + 1 : TM + 16;
  constexpr int BR = BKC ? TN : BK, BC_ = BKC ? BK + 1 : TN + 16;
  __shared__ T sa_r[2][AR][AC_];
  __shared__ T sa_i[AC ? 2 : 1][AC ? AR : 1][AC_];
  __shared__ T sb_r[2][BR][BC_];
  __shared__ T sb_i[BC ? 2 : 1][BC ? BR : 1][BC_];
  auto A_at = [&](int kk, int mm) -> int { return AKC ? mm * AC_ + kk : kk * AC_ + mm; };
  auto B_at = [&](int kk, int nn) -> int { return BKC ? nn * BC_ + kk : kk * BC_ + nn; };

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / GN, wn = wave % GN;
  int64_t tm, tn;
  tile_coords(g, blockIdx.x, tm, tn);
  const int64_t m0 = tm * TM, n0 = tn * TN;
  // Staging: element r of this thread sits at (row, k) = (am0 + r * AMS, ak0 + r * AKS)
  // of the A tile (likewise for B), so one base offset per operand and strides
  // that are the same for every thread address all of them.
  constexpr int AMS = AKC ? NT / 16 : 0, AKS = AKC ? 0 : NT / TM;
  constexpr int BNS = BKC ? NT / 16 : 0, BKS = BKC ? 0 : NT / TN;
  const int am0 = AKC ? (tid >> 4) : (tid % TM), ak0 = AKC ? (tid & 15) : (tid / TM);
  const int bn0 = BKC ? (tid >> 4) : (tid % TN), bk0 = BKC ? (tid & 15) : (tid / TN);
  const int lda0 = A_at(ak0, am0), ldb0 = B_at(bk0, bn0);
  const int ldas = A_at(AKS, AMS) - A_at(0, 0), ldbs = B_at(BKS, BNS) - B_at(0, 0);

  int64_t kbeg = 0, kend = g.K, b0 = blockIdx.y, bstep = gridDim.y;
  if (g.splitk > 1) {
    kbeg = (int64_t)blockIdx.y * g.kchunk;
    kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
    b0 = 0;
    bstep = 1;
  }
  // Operands are read through buffer resources whose base is the tile's origin at
  // the current k (scalar registers); a thread adds its own 32-bit byte offset and
  // a uniform offset per staged element.  Reads past the operand's extent return
  // zero; rows and columns past M and N hold values that only reach output
  // elements that are never stored, and the k positions past the end of the sum
  // are zeroed explicitly in the last K tile.
  const int a_rs = (int)((AMS * g.asm_ + AKS * g.ask) * (int64_t)sizeof(S));
  const int b_rs = (int)((BKS * g.bsk + BNS * g.bsn) * (int64_t)sizeof(S));
  const int a_thr = (int)((am0 * g.asm_ + ak0 * g.ask) * (int64_t)sizeof(S));
  const int b_thr = (int)((bn0 * g.bsn + bk0 * g.bsk) * (int64_t)sizeof(S));
  for (int64_t b = b0; b < g.batch; b += bstep) {
    // complex x complex in three real products (Gauss): accr = sum Ar Br,
    // acci = sum Ai Bi, accs = sum (Ar + Ai)(Br + Bi); re = accr - acci,
    // im = accs - accr - acci.  Otherwise accr, acci are the real and imaginary sums.
    constexpr bool G3 = AC && BC;
    acc_t accr[WM][WN], acci[WM][WN], accs[G3 ? WM : 1][G3 ? WN : 1];
#pragma unroll
    for (int x = 0; x < WM; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y) {
        accr[x][y] = acc_t{0, 0, 0, 0};
        acci[x][y] = acc_t{0, 0, 0, 0};
        if constexpr (G3) accs[x][y] = acc_t{0, 0, 0, 0};
      }
    S pa_r[NA], pa_i[NA], pb_r[NB], pb_i[NB];
    const int64_t a_org = b * g.asb + m0 * g.asm_, b_org = b * g.bsb + n0 * g.bsn;
    auto fetch = [&](int64_t k0) {
      const int64_t ao = a_org + k0 * g.ask, bo = b_org + k0 * g.bsk;
      const auto rar = window<S>(reinterpret_cast<const S*>(g.ar) + ao, g.aext - ao);
      const auto rai = window<S>(AC ? reinterpret_cast<const S*>(g.ai) + ao : nullptr, g.aext - ao);
      const auto rbr = window<S>(reinterpret_cast<const S*>(g.br) + bo, g.bext - bo);
      const auto rbi = window<S>(BC ? reinterpret_cast<const S*>(g.bi) + bo : nullptr, g.bext - bo);
#pragma unroll
      for (int r = 0; r < NA; ++r) {
        pa_r[r] = ldbuf<S>(rar, a_thr, r * a_rs);
        pa_i[r] = AC ? ldbuf<S>(rai, a_thr, r * a_rs) : (S)0;
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        pb_r[r] = ldbuf<S>(rbr, b_thr, r * b_rs);
        pb_i[r] = BC ? ldbuf<S>(rbi, b_thr, r * b_rs) : (S)0;
      }
      if (k0 + BK > kend) {   // last, partial K tile
        const int64_t ka = kend - k0 - ak0, kb = kend - k0 - bk0;
#pragma unroll
        for (int r = 0; r < NA; ++r)
          if (!(r * AKS < ka)) { pa_r[r] = 0; pa_i[r] = 0; }
#pragma unroll
        for (int r = 0; r < NB; ++r)
          if (!(r * BKS < kb)) { pb_r[r] = 0; pb_i[r] = 0; }
      }
    };
    auto stage = [&](int buf) {
#pragma unroll
      for (int r = 0; r < NA; ++r) {
        (&sa_r[buf][0][0])[lda0 + r * ldas] = (T)pa_r[r];
        if (AC) (&sa_i[buf][0][0])[lda0 + r * ldas] = (T)pa_i[r];
      }
#pragma unroll
      for (int r = 0; r < NB; ++r) {
        (&sb_r[buf][0][0])[ldb0 + r * ldbs] = (T)pb_r[r];
        if (BC) (&sb_i[buf][0][0])[ldb0 + r * ldbs] = (T)pb_i[r];
      }
    };
    if (kbeg < kend) {
      fetch(kbeg);
      stage(0);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) fetch(k0 + BK);
      // float64 (g.prio): the wave multiplying runs at raised priority, so that its
      // MFMA chain is not held up by another wave on the SIMD staging its next tile
      constexpr bool kPrio = sizeof(T) == 8;
      if (kPrio && g.prio) __builtin_amdgcn_s_setprio(1);
      // Four-wave work-groups unroll the whole K tile; eight-wave ones (at most 128
      // registers per wave) keep fragments of one (float64) or two (float32) k-steps
      // in flight.
#pragma unroll (GM * GN == 4 ? BK / 4 : (sizeof(T) == 8 ? 1 : 2))
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        T a_r[WM], a_i[WM], b_r[WN], b_i[WN];
#pragma unroll
        for (int x = 0; x < WM; ++x) {
          const int ia = A_at(kr, wm * 16 * WM + x * 16 + (lane & 15));
          a_r[x] = (&sa_r[buf][0][0])[ia];
          a_i[x] = AC ? (&sa_i[buf][0][0])[ia] : (T)0;
        }
#pragma unroll
        for (int y = 0; y < WN; ++y) {
          const int ib = B_at(kr, wn * 16 * WN + y * 16 + (lane & 15));
          b_r[y] = (&sb_r[buf][0][0])[ib];
          b_i[y] = BC ? (&sb_i[buf][0][0])[ib] : (T)0;
        }
        T a_s[G3 ? WM : 1], b_s[G3 ? WN : 1];
        if constexpr (G3) {
#pragma unroll
          for (int x = 0; x < WM; ++x) a_s[x] = a_r[x] + a_i[x];
#pragma unroll
          for (int y = 0; y < WN; ++y) b_s[y] = b_r[y] + b_i[y];
        }
#pragma unroll
        for (int x = 0; x < WM; ++x)
#pragma unroll
          for (int y = 0; y < WN; ++y) {
            accr[x][y] = Mfma<T>::mma(a_r[x], b_r[y], accr[x][y]);
            if constexpr (G3) {
              acci[x][y] = Mfma<T>::mma(a_i[x], b_i[y], acci[x][y]);
              accs[x][y] = Mfma<T>::mma(a_s[x], b_s[y], accs[x][y]);
            } else if (AC) {
              acci[x][y] = Mfma<T>::mma(a_i[x], b_r[y], acci[x][y]);
            } else if (BC) {
              acci[x][y] = Mfma<T>::mma(a_r[x], b_i[y], acci[x][y]);
            }
          }
      }
      if (kPrio && g.prio) __builtin_amdgcn_s_setprio(0);
      if (more) stage(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
    // ---- epilogue (row of accumulator register r: Mfma<T>::row)
    const bool split = g.splitk > 1;
    double* Cr = split ? g.pr + (int64_t)blockIdx.y * g.M * g.N : g.cr + b * g.csb;
    double* Ci = (AC || BC) ? (split ? g.pi + (int64_t)blockIdx.y * g.M * g.N : g.ci + b * g.csb) : nullptr;
    const int64_t sm = split ? g.N : g.csm, sn = split ? 1 : g.csn;
#pragma unroll
    for (int x = 0; x < WM; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gm = m0 + wm * 16 * WM + x * 16 + Mfma<T>::row(lane, r);
          const int64_t gn = n0 + wn * 16 * WN + y * 16 + (lane & 15);
          if (gm < g.M && gn < g.N) {
            const int64_t o = gm * sm + gn * sn;
            double pr = (double)accr[x][y][r], pi = (double)acci[x][y][r];
            if constexpr (G3) {
              const double p1 = pr, p2 = pi;
              pr = p1 - p2;
              pi = (double)accs[x][y][r] - p1 - p2;
            }
            if (split) {
              Cr[o] = pr;
              if (AC || BC) Ci[o] = pi;
            } else {
              double vr = g.alpha * pr;
              if (g.beta) vr += Cr[o];
              Cr[o] = vr;
              if (AC || BC) {
                double vi = g.alpha * pi;
                if (g.beta) vi += Ci[o];
                Ci[o] = vi;
              }
            }
          }
        }
  }
}

// ---------------------------------------------------------------------------
// bf16 x 3 split precision: every float64 operand x is split into
// hi = bf16(x) and lo = bf16(x - hi); a*b ~ ah*bh + ah*bl + al*bh (the lo*lo
// term, ~2^-16 relative, is dropped), accumulated in float32 on the
// v_mfma_f32_16x16x32_bf16 matrix cores.  Tile 64x64x32, one LDS buffer.
constexpr int BKH = 32, PADH = 8;

__device__ inline unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline void split_bf16(double x, unsigned short& hi, unsigned short& lo) {
  hi = bf16_rne((float)x);
  const float fh = __uint_as_float(((unsigned)hi) << 16);
  lo = bf16_rne((float)(x - (double)fh));
}

__device__ inline bf8 ld8(const unsigned short* p) { return *reinterpret_cast<const bf8*>(p); }

__device__ inline bf8 neg8(bf8 v) {
  typedef unsigned short u8v __attribute__((ext_vector_type(8)));
  u8v u = __builtin_bit_cast(u8v, v);
  u ^= (unsigned short)0x8000;
  return __builtin_bit_cast(bf8, u);
}

__device__ inline f4 mma3(bf8 ah, bf8 al, bf8 bh, bf8 bl, f4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  return c;
}

template <bool AC, bool BC, bool AKC, bool BKC>
__global__ __launch_bounds__(kThreads) void gemm_bf16x3(GemmArgs g) {
  // [row][k] with k contiguous: each lane reads 8 consecutive k values
  __shared__ __attribute__((aligned(16))) unsigned short arh[BM][BKH + PADH], arl[BM][BKH + PADH];
  __shared__ __attribute__((aligned(16))) unsigned short aih[AC ? BM : 1][BKH + PADH], ail[AC ? BM : 1][BKH + PADH];
  __shared__ __attribute__((aligned(16))) unsigned short brh[BN][BKH + PADH], brl[BN][BKH + PADH];
  __shared__ __attribute__((aligned(16))) unsigned short bih[BC ? BN : 1][BKH + PADH], bil[BC ? BN : 1][BKH + PADH];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t tm, tn;
  tile_coords(g, blockIdx.x, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  int a_k[8], a_m[8], b_k[8], b_n[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (AKC) { a_k[r] = tid & 31; a_m[r] = (tid >> 5) + 8 * r; }
    else     { a_m[r] = tid & 63; a_k[r] = (tid >> 6) + 4 * r; }
    if (BKC) { b_k[r] = tid & 31; b_n[r] = (tid >> 5) + 8 * r; }
    else     { b_n[r] = tid & 63; b_k[r] = (tid >> 6) + 4 * r; }
  }
  int64_t kbeg = 0, kend = g.K, b0 = blockIdx.y, bstep = gridDim.y;
  if (g.splitk > 1) {
    kbeg = (int64_t)blockIdx.y * g.kchunk;
    kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
    b0 = 0;
    bstep = 1;
  }
  for (int64_t b = b0; b < g.batch; b += bstep) {
    const double* Ar = g.ar + b * g.asb;
    const double* Ai = AC ? g.ai + b * g.asb : nullptr;
    const double* Br = g.br + b * g.bsb;
    const double* Bi = BC ? g.bi + b * g.bsb : nullptr;
    f4 accr[2][2], acci[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        accr[x][y] = f4{0.f, 0.f, 0.f, 0.f};
        acci[x][y] = f4{0.f, 0.f, 0.f, 0.f};
      }
    double pa_r[8], pa_i[8], pb_r[8], pb_i[8];
    auto fetch = [&](int64_t k0) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t gm = m0 + a_m[r], gk = k0 + a_k[r];
        pa_r[r] = 0.0;
        pa_i[r] = 0.0;
        if (gm < g.M && gk < kend) {
          const int64_t o = gm * g.asm_ + gk * g.ask;
          pa_r[r] = Ar[o];
          if (AC) pa_i[r] = Ai[o];
        }
        const int64_t gn = n0 + b_n[r], gk2 = k0 + b_k[r];
        pb_r[r] = 0.0;
        pb_i[r] = 0.0;
        if (gn < g.N && gk2 < kend) {
          const int64_t o = gk2 * g.bsk + gn * g.bsn;
          pb_r[r] = Br[o];
          if (BC) pb_i[r] = Bi[o];
        }
      }
    };
    auto stage = [&]() {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        split_bf16(pa_r[r], arh[a_m[r]][a_k[r]], arl[a_m[r]][a_k[r]]);
        if (AC) split_bf16(pa_i[r], aih[a_m[r]][a_k[r]], ail[a_m[r]][a_k[r]]);
        split_bf16(pb_r[r], brh[b_n[r]][b_k[r]], brl[b_n[r]][b_k[r]]);
        if (BC) split_bf16(pb_i[r], bih[b_n[r]][b_k[r]], bil[b_n[r]][b_k[r]]);
      }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += BKH) {
      stage();
      __syncthreads();
      if (k0 + BKH < kend) fetch(k0 + BKH);
      const int kk = (lane >> 4) * 8;
      bf8 xrh[2], xrl[2], xih[2], xil[2], yrh[2], yrl[2], yih[2], yil[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int row = wm * 32 + x * 16 + (lane & 15);
        xrh[x] = ld8(&arh[row][kk]);
        xrl[x] = ld8(&arl[row][kk]);
        if (AC) { xih[x] = ld8(&aih[row][kk]); xil[x] = ld8(&ail[row][kk]); }
        const int col = wn * 32 + x * 16 + (lane & 15);
        yrh[x] = ld8(&brh[col][kk]);
        yrl[x] = ld8(&brl[col][kk]);
        if (BC) { yih[x] = ld8(&bih[col][kk]); yil[x] = ld8(&bil[col][kk]); }
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          accr[x][y] = mma3(xrh[x], xrl[x], yrh[y], yrl[y], accr[x][y]);
          if (AC && BC) {
            accr[x][y] = mma3(neg8(xih[x]), neg8(xil[x]), yih[y], yil[y], accr[x][y]);
            acci[x][y] = mma3(xrh[x], xrl[x], yih[y], yil[y], acci[x][y]);
            acci[x][y] = mma3(xih[x], xil[x], yrh[y], yrl[y], acci[x][y]);
          } else if (AC) {
            acci[x][y] = mma3(xih[x], xil[x], yrh[y], yrl[y], acci[x][y]);
          } else if (BC) {
            acci[x][y] = mma3(xrh[x], xrl[x], yih[y], yil[y], acci[x][y]);
          }
        }
      __syncthreads();
    }
    const bool split = g.splitk > 1;
    double* Cr = split ? g.pr + (int64_t)blockIdx.y * g.M * g.N : g.cr + b * g.csb;
    double* Ci = (AC || BC) ? (split ? g.pi + (int64_t)blockIdx.y * g.M * g.N : g.ci + b * g.csb) : nullptr;
    const int64_t sm = split ? g.N : g.csm, sn = split ? 1 : g.csn;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gm = m0 + wm * 32 + x * 16 + 4 * (lane >> 4) + r;
          const int64_t gn = n0 + wn * 32 + y * 16 + (lane & 15);
          if (gm < g.M && gn < g.N) {
            const int64_t o = gm * sm + gn * sn;
            if (split) {
              Cr[o] = (double)accr[x][y][r];
              if (AC || BC) Ci[o] = (double)acci[x][y][r];
            } else {
              double vr = g.alpha * (double)accr[x][y][r];
              if (g.beta) vr += Cr[o];
              Cr[o] = vr;
              if (AC || BC) {
                double vi = g.alpha * (double)acci[x][y][r];
                if (g.beta) vi += Ci[o];
                Ci[o] = vi;
              }
            }
          }
        }
  }
}

// Short sums (K <= 16): one output element per thread on the vector units,
// threads ordered along the output's unit-stride dimension.
template <bool AC, bool BC>
__global__ __launch_bounds__(256) void gemm_smallk(GemmArgs g, int n_inner) {
  const int64_t total = g.batch * g.M * g.N;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    int64_t m, n, b;
    if (n_inner) { n = t % g.N; int64_t r = t / g.N; m = r % g.M; b = r / g.M; }
    else         { m = t % g.M; int64_t r = t / g.M; n = r % g.N; b = r / g.N; }
    const double* A = g.ar + b * g.asb + m * g.asm_;
    const double* Ai = AC ? g.ai + b * g.asb + m * g.asm_ : nullptr;
    const double* B = g.br + b * g.bsb + n * g.bsn;
    const double* Bi = BC ? g.bi + b * g.bsb + n * g.bsn : nullptr;
    double sr = 0.0, si = 0.0;
    for (int64_t k = 0; k < g.K; ++k) {
      const double ar = A[k * g.ask], br = B[k * g.bsk];
      const double ai = AC ? Ai[k * g.ask] : 0.0, bi = BC ? Bi[k * g.bsk] : 0.0;
      sr += ar * br;
      if (AC && BC) sr -= ai * bi;
      if (AC || BC) si += (AC ? ai * br : 0.0) + (BC ? ar * bi : 0.0);
    }
    const int64_t o = b * g.csb + m * g.csm + n * g.csn;
    double vr = g.alpha * sr;
    if (g.beta) vr += g.cr[o];
    g.cr[o] = vr;
    if (AC || BC) {
      double vi = g.alpha * si;
      if (g.beta) vi += g.ci[o];
      g.ci[o] = vi;
    }
  }
}

// C = alpha * sum_s P[s] + beta * C, summed in split order (deterministic).
// ---------------------------------------------------------------------------
// bf16 x 3 with operands split once before the product: split_kernel writes a
// strided float64 plane as hi/lo bf16 planes [batch][rows][ld] (k contiguous,
// zero padded from K to ld, ld a multiple of 32); gemm_bf16x3_split then stages
// 16-byte chunks of those planes into LDS with no conversion work.  The split of
// each element and the MFMA sequence per output element are those of
// gemm_bf16x3, so both kernels give the same result.
__global__ __launch_bounds__(256) void split_kernel(const double* src, int64_t rows, int64_t K, int64_t s_row,
                                                    int64_t s_k, int64_t s_b, int64_t ld, unsigned short* hi,
                                                    unsigned short* lo) {
  __shared__ double tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64, b = blockIdx.z;
  const double* S = src + b * s_b;
  const int t = threadIdx.x;
  const bool kfast = s_k == 1;    // read along the unit-stride index
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int a = t & 63, c = (t >> 6) + 4 * i;
    const int rr = kfast ? c : a, kk = kfast ? a : c;
    const int64_t r = r0 + rr, k = k0 + kk;
    tile[rr][kk] = (r < rows && k < K) ? S[r * s_row + k * s_k] : 0.0;
  }
  __syncthreads();
  unsigned short* H = hi + b * rows * ld;
  unsigned short* L = lo + b * rows * ld;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int kk = t & 63, rr = (t >> 6) + 4 * i;
    const int64_t r = r0 + rr, k = k0 + kk;
    if (r < rows && k < ld) {
      unsigned short h, l;
      split_bf16(tile[rr][kk], h, l);
      H[r * ld + k] = h;
      L[r * ld + k] = l;
    }
  }
}

// The float counterpart: a strided float64 plane as float [batch][rows][ld].
__global__ __launch_bounds__(256) void f32_kernel(const double* src, int64_t rows, int64_t K, int64_t s_row,
                                                  int64_t s_k, int64_t s_b, int64_t ld, float* dst) {
  __shared__ double tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64, b = blockIdx.z;
  const double* S = src + b * s_b;
  const int t = threadIdx.x;
  const bool kfast = s_k == 1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int a = t & 63, c = (t >> 6) + 4 * i;
    const int rr = kfast ? c : a, kk = kfast ? a : c;
    const int64_t r = r0 + rr, k = k0 + kk;
    tile[rr][kk] = (r < rows && k < K) ? S[r * s_row + k * s_k] : 0.0;
  }
  __syncthreads();
  float* D = dst + b * rows * ld;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int kk = t & 63, rr = (t >> 6) + 4 * i;
    const int64_t r = r0 + rr, k = k0 + kk;
    if (r < rows && k < ld) D[r * ld + k] = (float)tile[rr][kk];
  }
}

// fp16x3 operands: the largest |x| of every row (both planes of a complex operand), as
// the bit pattern of a non-negative float (which orders like the value), over 64 x 64
// tiles of (rows, k) read along the unit-stride index.
__global__ __launch_bounds__(256) void rowmax_kernel(const double* src, int64_t rows, int64_t K, int64_t s_row,
                                                     int64_t s_k, int64_t s_b, unsigned int* rmax) {
  __shared__ float tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64, b = blockIdx.z;
  const double* S = src + b * s_b;
  const int t = threadIdx.x;
  const bool kfast = s_k == 1;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int a = t & 63, c = (t >> 6) + 4 * i;
    const int rr = kfast ? c : a, kk = kfast ? a : c;
    const int64_t r = r0 + rr, k = k0 + kk;
    tile[rr][kk] = (r < rows && k < K) ? (float)fabs(S[r * s_row + k * s_k]) : 0.f;
  }
  __syncthreads();
  if (t < 64 && r0 + t < rows) {
    float m = 0.f;
    for (int kk = 0; kk < 64; ++kk) m = fmaxf(m, tile[t][kk]);
    atomicMax(rmax + b * rows + r0 + t, __float_as_uint(m));
  }
}

// x scaled by 2^e per row into fp16's range (the row maximum to [2^13, 2^14)), split into
// hi = fp16(x 2^e) and lo = fp16(x 2^e - hi); inv [batch][rows] receives 2^-e.
__global__ __launch_bounds__(256) void split_f16_kernel(const double* src, int64_t rows, int64_t K, int64_t s_row,
                                                        int64_t s_k, int64_t s_b, int64_t ld, const unsigned int* rmax,
                                                        unsigned short* hi, unsigned short* lo, float* inv) {
  __shared__ double tile[64][65];
  __shared__ double scale[64];
  const int64_t r0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64, b = blockIdx.z;
  const double* S = src + b * s_b;
  const int t = threadIdx.x;
  const bool kfast = s_k == 1;
  if (t < 64) {
    const int64_t r = r0 + t;
    const float m = r < rows ? __uint_as_float(rmax[b * rows + r]) : 0.f;
    int e = 0;
    if (m > 0.f) {
      frexpf(m, &e);          // m = f 2^e with f in [0.5, 1)
      e = 14 - e;             // m 2^e in [2^13, 2^14)
    }
    scale[t] = ldexp(1.0, e);
    if (r < rows && k0 == 0) inv[b * rows + r] = ldexpf(1.f, -e);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int a = t & 63, c = (t >> 6) + 4 * i;
    const int rr = kfast ? c : a, kk = kfast ? a : c;
    const int64_t r = r0 + rr, k = k0 + kk;
    tile[rr][kk] = (r < rows && k < K) ? S[r * s_row + k * s_k] : 0.0;
  }
  __syncthreads();
  unsigned short* H = hi + b * rows * ld;
  unsigned short* L = lo + b * rows * ld;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int kk = t & 63, rr = (t >> 6) + 4 * i;
    const int64_t r = r0 + rr, k = k0 + kk;
    if (r < rows && k < ld) {
      const double x = tile[rr][kk] * scale[rr];
      const _Float16 h = (_Float16)x;
      const _Float16 l = (_Float16)(x - (double)h);
      H[r * ld + k] = __builtin_bit_cast(unsigned short, h);
      L[r * ld + k] = __builtin_bit_cast(unsigned short, l);
    }
  }
}

typedef float f16v __attribute__((ext_vector_type(16)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

// The two 16-bit split formats: bf16 (8-bit significand, float32's range) and fp16
// (11-bit significand, planes scaled per row into its range).  Both keep the sign in
// bit 15, so negating a fragment flips that bit in either.
struct SplitBf16 {
  typedef bf8 vec;
  static constexpr bool scaled = false;
  static __device__ inline f16v mma(vec a, vec b, f16v c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};
struct SplitF16 {
  typedef h8 vec;
  static constexpr bool scaled = true;
  static __device__ inline f16v mma(vec a, vec b, f16v c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};

template <typename E>
__device__ inline typename E::vec ldv(const unsigned short* p) { return *reinterpret_cast<const typename E::vec*>(p); }
template <typename V>
__device__ inline V negv(V v) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 u = __builtin_bit_cast(u4, v);
  u ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(V, u);
}

template <typename E>
__device__ inline f16v mma3_32(typename E::vec ah, typename E::vec al, typename E::vec bh, typename E::vec bl, f16v c) {
  c = E::mma(ah, bh, c);
  c = E::mma(ah, bl, c);
  c = E::mma(al, bh, c);
  return c;
}

// bf16x3 product of pre-split operands on the 32 x 32 x 16 bf16 matrix cores:
// twice the products of the 16 x 16 x 32 form per fragment read from LDS, which
// bounds these short bf16 k-steps.  Work-group tile (64 WM) x (64 WN), 2 x 2 waves
// of WM x WN blocks of 32 x 32; a fragment lane holds row (lane % 32) and k
// (lane / 32) * 8 .. + 7 of its block; accumulator register r of a lane holds row
// 8 (r / 4) + 4 (lane / 32) + r % 4 and column lane % 32.
// NB: LDS stages (the next k tile is always fetched into registers while the current
// one is read; 2: staged into the other stage, one barrier per tile; 1: staged after
// every wave has read the current one, two barriers per tile).
// OCC: waves per SIMD the registers are sized for (1 lets the 128 x 128 tiles keep
// their accumulators, operands and prefetch in registers: 512 per lane, no spills).
// BK: k per LDS stage (32 in every launched shape: with 16 the mixed 128 x 128 tile spills
// less but runs 2.8x slower).
template <typename E, bool AC, bool BC, int WM, int WN, int NB, int OCC, int BK>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(OCC, 8))) void gemm_bf16x3_split(GemmArgs g) {
  typedef typename E::vec V;
  constexpr int TM = 64 * WM, TN = 64 * WN, LDK = BK + PADH;
  constexpr int PA = AC ? 4 : 2, PB = BC ? 4 : 2;      // hi, lo of each real plane
  constexpr int CPR = BK / 8, RPP = kThreads / CPR;     // 16-byte chunks per row, rows per pass
  static_assert(TM % RPP == 0 && TN % RPP == 0, "tile rows must fill whole passes");
  constexpr int CA = TM / RPP, CB = TN / RPP;           // 16-byte chunks per thread and plane
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) unsigned short sa[NB][PA][TM][LDK];
  __shared__ __attribute__((aligned(16))) unsigned short sb[NB][PB][TN][LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t tm, tn;
  tile_coords(g, blockIdx.x, tm, tn);
  const int64_t m0 = tm * TM, n0 = tn * TN;
  const int crow = tid / CPR, cofs = (tid % CPR) * 8;  // RPP rows x CPR chunks of 8 k per pass
  int64_t kbeg = 0, kend = g.sld, b0 = blockIdx.y, bstep = gridDim.y;
  if (g.splitk > 1) {
    kbeg = (int64_t)blockIdx.y * g.kchunk;
    kend = kbeg + g.kchunk < g.sld ? kbeg + g.kchunk : g.sld;
    b0 = 0;
    bstep = 1;
  }
  for (int64_t b = b0; b < g.batch; b += bstep) {
    const int64_t ao = b * g.sab, bo = b * g.sbb;
    f16v accr[WM][WN], acci[WM][WN];
#pragma unroll
    for (int x = 0; x < WM; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          accr[x][y][r] = 0.f;
          acci[x][y][r] = 0.f;
        }
      }
    u4 ra[PA][CA], rb[PB][CB];
    auto fetch = [&](int64_t k0) {
#pragma unroll
      for (int c = 0; c < CA; ++c) {
        const int64_t gm = m0 + crow + RPP * c;
#pragma unroll
        for (int p = 0; p < PA; ++p)
          ra[p][c] = gm < g.M ? *reinterpret_cast<const u4*>(g.sa[p] + ao + gm * g.sld + k0 + cofs) : u4{0, 0, 0, 0};
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int64_t gn = n0 + crow + RPP * c;
#pragma unroll
        for (int p = 0; p < PB; ++p)
          rb[p][c] = gn < g.N ? *reinterpret_cast<const u4*>(g.sb[p] + bo + gn * g.sld + k0 + cofs) : u4{0, 0, 0, 0};
      }
    };
    auto stage = [&](int buf) {
#pragma unroll
      for (int c = 0; c < CA; ++c)
#pragma unroll
        for (int p = 0; p < PA; ++p) *reinterpret_cast<u4*>(&sa[buf][p][crow + RPP * c][cofs]) = ra[p][c];
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int p = 0; p < PB; ++p) *reinterpret_cast<u4*>(&sb[buf][p][crow + RPP * c][cofs]) = rb[p][c];
    };
    if (kbeg < kend) {
      fetch(kbeg);
      stage(0);
    }
    __syncthreads();
    int buf = 0;
    const int l32 = lane & 31, kh = (lane >> 5) * 8;
    for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) fetch(k0 + BK);
#pragma unroll
      for (int ks = 0; ks < BK / 16; ++ks) {
        const int kk = ks * 16 + kh;
        V xrh[WM], xrl[WM], xih[WM], xil[WM], yrh[WN], yrl[WN], yih[WN], yil[WN];
#pragma unroll
        for (int x = 0; x < WM; ++x) {
          const int row = wm * 32 * WM + x * 32 + l32;
          xrh[x] = ldv<E>(&sa[buf][0][row][kk]);
          xrl[x] = ldv<E>(&sa[buf][1][row][kk]);
          if (AC) { xih[x] = ldv<E>(&sa[buf][2 % PA][row][kk]); xil[x] = ldv<E>(&sa[buf][3 % PA][row][kk]); }
        }
#pragma unroll
        for (int y = 0; y < WN; ++y) {
          const int col = wn * 32 * WN + y * 32 + l32;
          yrh[y] = ldv<E>(&sb[buf][0][col][kk]);
          yrl[y] = ldv<E>(&sb[buf][1][col][kk]);
          if (BC) { yih[y] = ldv<E>(&sb[buf][2 % PB][col][kk]); yil[y] = ldv<E>(&sb[buf][3 % PB][col][kk]); }
        }
#pragma unroll
        for (int x = 0; x < WM; ++x)
#pragma unroll
          for (int y = 0; y < WN; ++y) {
            accr[x][y] = mma3_32<E>(xrh[x], xrl[x], yrh[y], yrl[y], accr[x][y]);
            if (AC && BC) {
              accr[x][y] = mma3_32<E>(negv(xih[x]), negv(xil[x]), yih[y], yil[y], accr[x][y]);
              acci[x][y] = mma3_32<E>(xrh[x], xrl[x], yih[y], yil[y], acci[x][y]);
              acci[x][y] = mma3_32<E>(xih[x], xil[x], yrh[y], yrl[y], acci[x][y]);
            } else if (AC) {
              acci[x][y] = mma3_32<E>(xih[x], xil[x], yrh[y], yrl[y], acci[x][y]);
            } else if (BC) {
              acci[x][y] = mma3_32<E>(xrh[x], xrl[x], yih[y], yil[y], acci[x][y]);
            }
          }
      }
      if constexpr (NB == 2) {
        if (more) stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      } else {
        __syncthreads();   // every wave has read the tile
        if (more) {
          stage(0);
          __syncthreads();
        }
      }
    }
    const bool split = g.splitk > 1;
    double* Cr = split ? g.pr + (int64_t)blockIdx.y * g.M * g.N : g.cr + b * g.csb;
    double* Ci = (AC || BC) ? (split ? g.pi + (int64_t)blockIdx.y * g.M * g.N : g.ci + b * g.csb) : nullptr;
    const int64_t sm = split ? g.N : g.csm, sn = split ? 1 : g.csn;
#pragma unroll
    for (int x = 0; x < WM; ++x)
#pragma unroll
      for (int y = 0; y < WN; ++y)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t gm = m0 + wm * 32 * WM + x * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int64_t gn = n0 + wn * 32 * WN + y * 32 + l32;
          if (gm < g.M && gn < g.N) {
            const int64_t o = gm * sm + gn * sn;
            // fp16 planes: undo the rows' power-of-two scales (exact)
            const double us = E::scaled ? (double)g.sca[b * (g.sab ? g.M : 0) + gm] * (double)g.scb[b * (g.sbb ? g.N : 0) + gn]
                                        : 1.0;
            if (split) {
              Cr[o] = us * (double)accr[x][y][r];
              if (AC || BC) Ci[o] = us * (double)acci[x][y][r];
            } else {
              double vr = g.alpha * us * (double)accr[x][y][r];
              if (g.beta) vr += Cr[o];
              Cr[o] = vr;
              if (AC || BC) {
                double vi = g.alpha * us * (double)acci[x][y][r];
                if (g.beta) vi += Ci[o];
                Ci[o] = vi;
              }
            }
          }
        }
  }
}

__global__ __launch_bounds__(256) void splitk_reduce(GemmArgs g, int cplx) {
  const int64_t total = g.M * g.N;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < g.splitk; ++s) {
      sr += g.pr[s * total + t];
      if (cplx) si += g.pi[s * total + t];
    }
    const int64_t m = t / g.N, n = t - m * g.N;
    const int64_t o = m * g.csm + n * g.csn;
    double vr = g.alpha * sr;
    if (g.beta) vr += g.cr[o];
    g.cr[o] = vr;
    if (cplx) {
      double vi = g.alpha * si;
      if (g.beta) vi += g.ci[o];
      g.ci[o] = vi;
    }
  }
}

struct PermArgs {
  int nd;
  int64_t dim[kMaxDims];
  int64_t istr[kMaxDims], ostr[kMaxDims];
  const double* ir; const double* ii;
  double* orr; double* oi;
  const double* sc[kMaxDims];
  double ar, ai;
  int beta;
  int64_t total;
};

__global__ __launch_bounds__(256) void permute_kernel(PermArgs p) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < p.total; t += stride) {
    int64_t r = t, io = 0, oo = 0;
    double s = 1.0;
    for (int d = p.nd - 1; d >= 0; --d) {
      const int64_t dd = p.dim[d];
      const int64_t x = r % dd;
      r /= dd;
      io += x * p.istr[d];
      oo += x * p.ostr[d];
      if (p.sc[d]) s *= p.sc[d][x];
    }
    const double xr = p.ir[io];
    const double xi = p.ii ? p.ii[io] : 0.0;
    double vr = s * (p.ar * xr - p.ai * xi);
    double vi = s * (p.ar * xi + p.ai * xr);
    if (p.ar == 0.0 && p.ai == 0.0) vr = vi = 0.0;   // a zero fill whatever the input holds
    if (p.beta) {
      vr += p.orr[oo];
      if (p.oi) vi += p.oi[oo];
    }
    p.orr[oo] = vr;
    if (p.oi) p.oi[oo] = vi;
  }
}

// Same-spin pair storage (SsOp): pairs p = (i < j) of n in lexicographic order
// start at pstart(i, n) = i (2n - i - 1) / 2.
struct SsArgs {
  int64_t n1, n2, np2, i0, ci, j0, cj, rows;
  int pair2, anti1, anti2, beta;
  double alpha;
  double* xr; double* xi;
  double* yr; double* yi;
  const double* ur; const double* ui;
  const double* m1; const double* m2;
  const int32_t* oi; const int32_t* oj; const int32_t* va; const int32_t* vb;
};

__device__ inline int64_t pstart(int64_t i, int64_t n) { return i * (2 * n - i - 1) / 2; }
__device__ inline int64_t pidx(int64_t i, int64_t j, int64_t n) { return pstart(i, n) + j - i - 1; }

// kExpand: one row (ii, jj, a) of the full block per iteration, b across the threads.
__global__ __launch_bounds__(256) void ss_expand(SsArgs g) {
  for (int64_t row = blockIdx.x; row < g.rows; row += gridDim.x) {
    const int64_t a = row % g.n2, r = row / g.n2, jj = r % g.cj, ii = r / g.cj;
    const int64_t i = g.i0 + ii, j = g.j0 + jj;
    const int64_t xo = row * g.n2;
    const bool diag = i == j;
    const int64_t p = diag ? 0 : pidx(i < j ? i : j, i < j ? j : i, g.n1);
    const double si = i < j ? g.alpha : -g.alpha;
    for (int64_t b = threadIdx.x; b < g.n2; b += blockDim.x) {
      double vr = 0.0, vi = 0.0;
      if (!diag && a != b) {
        const int64_t q = p * g.np2 + (a < b ? pidx(a, b, g.n2) : pidx(b, a, g.n2));
        const double sg = a < b ? si : -si;
        vr = sg * g.yr[q];
        if (g.yi) vi = sg * g.yi[q];
      }
      if (g.beta) {
        vr += g.xr[xo + b];
        if (g.xi) vi += g.xi[xo + b];
      }
      g.xr[xo + b] = vr;
      if (g.xi) g.xi[xo + b] = vi;
    }
  }
}

// kAccum: one row (ii, jj, a) of the block per iteration, b > a across the threads.
// A row with i < j owns pair (i, j) and adds the partner row (j, i) when the block
// holds it (anti1); a row with i > j writes pair (j, i) with a minus sign only when
// the block does not hold (j, i).  Every pair element has one writer.
__global__ __launch_bounds__(256) void ss_accum(SsArgs g) {
  for (int64_t row = blockIdx.x; row < g.rows; row += gridDim.x) {
    const int64_t a = row % g.n2, r = row / g.n2, jj = r % g.cj, ii = r / g.cj;
    const int64_t i = g.i0 + ii, j = g.j0 + jj;
    if (i == j) continue;
    const bool partner_in = j >= g.i0 && j < g.i0 + g.ci && i >= g.j0 && i < g.j0 + g.cj;
    if (i > j && (!g.anti1 || partner_in)) continue;
    const bool lo = i < j;
    const int64_t p = lo ? pidx(i, j, g.n1) : pidx(j, i, g.n1);
    const double sgn = lo ? g.alpha : -g.alpha;
    const bool partner = lo && g.anti1 && partner_in;
    const int64_t xo = ((ii * g.cj + jj) * g.n2 + a) * g.n2;
    const int64_t xq = partner ? (((j - g.i0) * g.cj + (i - g.j0)) * g.n2 + a) * g.n2 : 0;
    const int64_t xo2 = ((ii * g.cj + jj) * g.n2) * g.n2 + a;    // x[ii][jj][.][a]
    const int64_t xq2 = partner ? (((j - g.i0) * g.cj + (i - g.j0)) * g.n2) * g.n2 + a : 0;
    const int64_t yo = p * g.np2 + pidx(a, a + 1, g.n2) - (a + 1);   // + b gives pair (a, b)
    for (int64_t b = a + 1 + threadIdx.x; b < g.n2; b += blockDim.x) {
      double vr = g.xr[xo + b], vi = g.xi ? g.xi[xo + b] : 0.0;
      if (g.anti2) {
        vr -= g.xr[xo2 + b * g.n2];
        if (g.xi) vi -= g.xi[xo2 + b * g.n2];
      }
      if (partner) {
        vr -= g.xr[xq + b];
        if (g.xi) vi -= g.xi[xq + b];
        if (g.anti2) {
          vr += g.xr[xq2 + b * g.n2];
          if (g.xi) vi += g.xi[xq2 + b * g.n2];
        }
      }
      g.yr[yo + b] += sgn * vr;
      if (g.yi) g.yi[yo + b] += sgn * vi;
    }
  }
}

// kAccumRows: rows (pp, a), b > a across the threads.
__global__ __launch_bounds__(256) void ss_accum_rows(SsArgs g) {
  for (int64_t row = blockIdx.x; row < g.rows; row += gridDim.x) {
    const int64_t a = row % g.n2, pp = row / g.n2;
    const int64_t xo = (pp * g.n2 + a) * g.n2, xo2 = pp * g.n2 * g.n2 + a;
    const int64_t yo = (g.i0 + pp) * g.np2 + pidx(a, a + 1, g.n2) - (a + 1);
    for (int64_t b = a + 1 + threadIdx.x; b < g.n2; b += blockDim.x) {
      double vr = g.xr[xo + b], vi = g.xi ? g.xi[xo + b] : 0.0;
      if (g.anti2) {
        vr -= g.xr[xo2 + b * g.n2];
        if (g.xi) vi -= g.xi[xo2 + b * g.n2];
      }
      g.yr[yo + b] += g.alpha * vr;
      if (g.yi) g.yi[yo + b] += g.alpha * vi;
    }
  }
}

// kT1T1 and kMask: rows (p, a) of the pair block, b > a across the threads.
__global__ __launch_bounds__(256) void ss_pairwise(SsArgs g, int mask) {
  for (int64_t row = blockIdx.x; row < g.rows; row += gridDim.x) {
    const int64_t a = row % g.n2, p = row / g.n2;
    const int64_t i = g.oi[p], j = g.oj[p];
    const int64_t yo = p * g.np2 + pidx(a, a + 1, g.n2) - (a + 1);
    if (mask) {
      const double ma = g.m1[i] * g.m1[j] * g.m2[a];
      for (int64_t b = a + 1 + threadIdx.x; b < g.n2; b += blockDim.x) {
        const double m = ma * g.m2[b];
        g.yr[yo + b] *= m;
        if (g.yi) g.yi[yo + b] *= m;
      }
      continue;
    }
    const double iar = g.ur[i * g.n2 + a], iai = g.ui[i * g.n2 + a];
    const double jar = g.ur[j * g.n2 + a], jai = g.ui[j * g.n2 + a];
    for (int64_t b = a + 1 + threadIdx.x; b < g.n2; b += blockDim.x) {
      const double jbr = g.ur[j * g.n2 + b], jbi = g.ui[j * g.n2 + b];
      const double ibr = g.ur[i * g.n2 + b], ibi = g.ui[i * g.n2 + b];
      const double vr = (iar * jbr - iai * jbi) - (ibr * jar - ibi * jai);
      const double vi = (iar * jbi + iai * jbr) - (ibr * jai + ibi * jar);
      double yr = g.alpha * vr, yi = g.alpha * vi;
      if (g.beta) {
        yr += g.yr[yo + b];
        yi += g.yi[yo + b];
      }
      g.yr[yo + b] = yr;
      g.yi[yo + b] = yi;
    }
  }
}

// kPackSlab: rows (ee, f) (and a with pair2) of the slab; pairs (e < f) only.
__global__ __launch_bounds__(256) void ss_pack_slab(SsArgs g) {
  const int64_t rest = g.pair2 ? g.n2 * g.n2 : g.n2, nq = g.pair2 ? g.np2 : g.n2;
  const int64_t base = pstart(g.i0, g.n1);
  for (int64_t row = blockIdx.x; row < g.rows; row += gridDim.x) {
    int64_t r = row, a = 0;
    if (g.pair2) { a = r % g.n2; r /= g.n2; }
    const int64_t f = r % g.n1, ee = r / g.n1, e = g.i0 + ee;
    if (f <= e) continue;
    const int64_t p = pidx(e, f, g.n1) - base;
    const int64_t xo = (ee * g.n1 + f) * rest;
    if (g.pair2) {
      const int64_t yo = p * nq + pidx(a, a + 1, g.n2) - (a + 1);
      for (int64_t b = a + 1 + threadIdx.x; b < g.n2; b += blockDim.x) {
        g.yr[yo + b] = g.alpha * (g.xr[xo + a * g.n2 + b] - g.xr[xo + b * g.n2 + a]);
        if (g.yi) g.yi[yo + b] = g.alpha * (g.xi[xo + a * g.n2 + b] - g.xi[xo + b * g.n2 + a]);
      }
    } else {
      for (int64_t c = threadIdx.x; c < g.n2; c += blockDim.x) {
        g.yr[p * nq + c] = g.alpha * g.xr[xo + c];
        if (g.yi) g.yi[p * nq + c] = g.alpha * g.xi[xo + c];
      }
    }
  }
}

// The same operation when the input's and the output's unit-stride dimensions
// differ (a transpose): 32 x 32 tiles of (din, dout) pass through LDS so that both
// the reads (along din) and the writes (along dout) are coalesced.  The value of
// every element is computed exactly as in permute_kernel (same scale order).
__global__ __launch_bounds__(256) void permute_tiled(PermArgs p, int din, int dout, int64_t tiles_i,
                                                     int64_t tiles_o, int64_t nblocks) {
  __shared__ double tr[32][33], ti[32][33];
  const int64_t ni = p.dim[din], no = p.dim[dout], ntile = tiles_i * tiles_o;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int64_t w = blockIdx.x; w < nblocks; w += gridDim.x) {
    const int64_t tile = w % ntile;
    int64_t rest = w / ntile;
    const int64_t a0 = (tile % tiles_i) * 32, b0 = (tile / tiles_i) * 32;
    int64_t x[kMaxDims];
    int64_t io = 0, oo = 0;
    for (int d = p.nd - 1; d >= 0; --d) {
      if (d == din || d == dout) { x[d] = 0; continue; }
      x[d] = rest % p.dim[d];
      rest /= p.dim[d];
      io += x[d] * p.istr[d];
      oo += x[d] * p.ostr[d];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t a = a0 + tx, c = b0 + ty + 8 * j;
      double vr = 0.0, vi = 0.0;
      if (a < ni && c < no) {
        double sv = 1.0;
        for (int d = p.nd - 1; d >= 0; --d)
          if (p.sc[d]) sv *= p.sc[d][d == din ? a : (d == dout ? c : x[d])];
        const int64_t o = io + a * p.istr[din] + c * p.istr[dout];
        const double xr = p.ir[o], xi = p.ii ? p.ii[o] : 0.0;
        vr = sv * (p.ar * xr - p.ai * xi);
        vi = sv * (p.ar * xi + p.ai * xr);
        if (p.ar == 0.0 && p.ai == 0.0) vr = vi = 0.0;
      }
      tr[ty + 8 * j][tx] = vr;
      ti[ty + 8 * j][tx] = vi;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t c = b0 + tx, a = a0 + ty + 8 * j;
      if (a < ni && c < no) {
        const int64_t o = oo + a * p.ostr[din] + c * p.ostr[dout];
        double vr = tr[tx][ty + 8 * j], vi = ti[tx][ty + 8 * j];
        if (p.beta) {
          vr += p.orr[o];
          if (p.oi) vi += p.oi[o];
        }
        p.orr[o] = vr;
        if (p.oi) p.oi[o] = vi;
      }
    }
    __syncthreads();
  }
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) p[t] = v;
}

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

struct UpdArgs {
  int64_t no, nv, n1, nss, npv, off_ab, total;
  const int32_t* oi; const int32_t* oj; const int32_t* va; const int32_t* vb;
  double* xr; double* xi;
  const double* rr; const double* ri;
  double* hr_; double* hi_;
  double h;
  int mode, start;
  const double* mo[2]; const double* mv[2]; const double* fo[2]; const double* fv[2];
  unsigned long long* delta;
};

__global__ __launch_bounds__(256) void update_kernel(UpdArgs u) {
  __shared__ double red[4];
  double dmax = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < u.total; k += stride) {
    double mask, dd;
    if (k < 2 * u.n1) {
      const int s = k >= u.n1;
      const int64_t r = k - s * u.n1, i = r / u.nv, a = r - i * u.nv;
      mask = u.mo[s][i] * u.mv[s][a];
      dd = u.fo[s][i] - u.fv[s][a];
    } else if (k < u.off_ab) {
      // same-spin pair element (i < j, a < b) of block s
      const int64_t k2 = k - 2 * u.n1;
      const int s = k2 >= u.nss;
      const int64_t r = k2 - s * u.nss, p = r / u.npv, q = r - p * u.npv;
      const int64_t i = u.oi[p], j = u.oj[p], a = u.va[q], b = u.vb[q];
      mask = u.mo[s][i] * u.mo[s][j] * u.mv[s][a] * u.mv[s][b];
      dd = u.fo[s][i] + u.fo[s][j] - u.fv[s][a] - u.fv[s][b];
    } else {
      int64_t r = k - u.off_ab;
      const int64_t b = r % u.nv; r /= u.nv;
      const int64_t a = r % u.nv; r /= u.nv;
      const int64_t j = r % u.no, i = r / u.no;
      mask = u.mo[0][i] * u.mo[1][j] * u.mv[0][a] * u.mv[1][b];
      dd = u.fo[0][i] + u.fo[1][j] - u.fv[0][a] - u.fv[1][b];
    }
    const double xr = u.xr[k], xi = u.xi[k], rr = u.rr[k], ri = u.ri[k];
    double nr, ni;
    if (u.mode == 2) {
      // Jacobi step towards R(T) = 0 (ground state): x + r / D
      nr = dd != 0.0 ? xr + rr / dd : 0.0;
      ni = dd != 0.0 ? xi + ri / dd : 0.0;
    } else {
      double hr, hi;
      if (u.start) {
        hr = xr - u.h * ri;
        hi = xi + u.h * rr;
        if (u.hr_) {   // kept for later passes
          u.hr_[k] = hr;
          u.hi_[k] = hi;
        }
      } else {
        hr = u.hr_[k];
        hi = u.hi_[k];
      }
      if (u.mode == 0) {
        nr = hr - u.h * ri;
        ni = hi + u.h * rr;
      } else {
        const double pr = rr + dd * xr, pi = ri + dd * xi;
        const double numr = hr - u.h * pi, numi = hi + u.h * pr;
        const double di = u.h * dd, den = 1.0 + di * di;
        nr = (numr + numi * di) / den;
        ni = (numi - numr * di) / den;
      }
    }
    if (mask == 0.0) { nr = 0.0; ni = 0.0; }
    const double dr = nr - xr, dq = ni - xi;
    const double dv = sqrt(dr * dr + dq * dq);
    dmax = (dv != dv) ? dv : fmax(dmax, dv);   // keep NaN
    u.xr[k] = nr;
    u.xi[k] = ni;
  }
  // NaN-propagating max over the block; doubles >= 0 order like their bit patterns
  unsigned long long bits = __double_as_longlong(dmax);
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long other = __shfl_xor(bits, o);
    bits = other > bits ? other : bits;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = __longlong_as_double(bits);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      unsigned long long v = __double_as_longlong(red[w]);
      m = v > m ? v : m;
    }
    atomicMax(u.delta, m);
  }
}

struct EnArgs {
  int64_t no, nv, n1, npv, off_aa, off_bb, off_ab;
  const double* xr; const double* xi;
  const double* jov;
  const double* fov0; const double* fov1; int64_t ld;
  int ft1;
  double* part;
  double* out;
};

constexpr int kEnergyBlocks = 1024;

__global__ __launch_bounds__(256) void energy_pass1(EnArgs e) {
  __shared__ double sr[4], si[4];
  const int64_t total = e.no * e.nv * e.no * e.nv;
  const double* T1r = e.xr;
  const double* T1i = e.xi;
  const double* Tr = e.xr + e.off_ab;
  const double* Ti = e.xi + e.off_ab;
  double accr = 0.0, acci = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    int64_t r = t;
    const int64_t b = r % e.nv; r /= e.nv;
    const int64_t j = r % e.no; r /= e.no;
    const int64_t a = r % e.nv; const int64_t i = r / e.nv;
    const double J = e.jov[t];
    const int64_t p = ((i * e.no + j) * e.nv + a) * e.nv + b;
    double wr = Tr[p], wi = Ti[p];
    // 1/2 (t_aa + t_bb) with the same-spin elements read from pair storage
    if (i != j && a != b) {
      const double sg = 0.5 * (i < j ? 1.0 : -1.0) * (a < b ? 1.0 : -1.0);
      const int64_t q = pidx(i < j ? i : j, i < j ? j : i, e.no) * e.npv + pidx(a < b ? a : b, a < b ? b : a, e.nv);
      wr += sg * (e.xr[e.off_aa + q] + e.xr[e.off_bb + q]);
      wi += sg * (e.xi[e.off_aa + q] + e.xi[e.off_bb + q]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int64_t o = s * e.n1;
      double xr1 = T1r[o + i * e.nv + a], xi1 = T1i[o + i * e.nv + a];
      double yr1 = T1r[o + j * e.nv + b], yi1 = T1i[o + j * e.nv + b];
      wr += 0.5 * (xr1 * yr1 - xi1 * yi1);
      wi += 0.5 * (xr1 * yi1 + xi1 * yr1);
      xr1 = T1r[o + i * e.nv + b]; xi1 = T1i[o + i * e.nv + b];
      yr1 = T1r[o + j * e.nv + a]; yi1 = T1i[o + j * e.nv + a];
      wr -= 0.5 * (xr1 * yr1 - xi1 * yi1);
      wi -= 0.5 * (xr1 * yi1 + xi1 * yr1);
    }
    {
      const double xr1 = T1r[i * e.nv + a], xi1 = T1i[i * e.nv + a];
      const double yr1 = T1r[e.n1 + j * e.nv + b], yi1 = T1i[e.n1 + j * e.nv + b];
      wr += xr1 * yr1 - xi1 * yi1;
      wi += xr1 * yi1 + xi1 * yr1;
    }
    accr += J * wr;
    acci += J * wi;
  }
  accr = wave_sum(accr);
  acci = wave_sum(acci);
  if ((threadIdx.x & 63) == 0) { sr[threadIdx.x >> 6] = accr; si[threadIdx.x >> 6] = acci; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += sr[w]; c += si[w]; }
    e.part[2 * blockIdx.x] = a;
    e.part[2 * blockIdx.x + 1] = c;
  }
}

__global__ __launch_bounds__(64) void energy_pass2(EnArgs e, int nparts) {
  // one wave: fixed-order sums, then the f_ia t_ia term
  double ar = 0.0, ai = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 64) { ar += e.part[2 * k]; ai += e.part[2 * k + 1]; }
  if (e.ft1) {
    for (int64_t k = threadIdx.x; k < 2 * e.n1; k += 64) {
      const int s = k >= e.n1;
      const int64_t r = k - s * e.n1, i = r / e.nv, a = r - i * e.nv;
      const double f = (s ? e.fov1 : e.fov0)[i * e.ld + a];
      ar += f * e.xr[k];
      ai += f * e.xi[k];
    }
  }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if (threadIdx.x == 0) { e.out[0] = ar; e.out[1] = ai; }
}

// sum_k a[k] b[k] in a fixed order: kEnergyBlocks block partials, then one wave.
__global__ __launch_bounds__(256) void dot_pass1(const double* a, const double* b, int64_t n, double* part) {
  __shared__ double sr[4];
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) acc += a[k] * b[k];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sr[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sr[0] + sr[1] + sr[2] + sr[3];
}

__global__ __launch_bounds__(64) void dot_pass2(const double* part, int nparts, double* out) {
  double acc = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 64) acc += part[k];
  acc = wave_sum(acc);
  if (threadIdx.x == 0) out[0] = acc;
}

__global__ void cumulant_kernel(double* c, double* e, const double* en, int64_t* step, double h, double* bad) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t k = *step;
    const double sr = e[2 * k] + en[0], si = e[2 * k + 1] + en[1];
    const double cr = c[2 * k] - h * si, ci = c[2 * k + 1] + h * sr;
    c[2 * (k + 1)] = cr;
    c[2 * (k + 1) + 1] = ci;
    e[2 * (k + 1)] = en[0];
    e[2 * (k + 1) + 1] = en[1];
    *step = k + 1;
    if (!isfinite(en[0]) || !isfinite(en[1]) || !isfinite(cr) || !isfinite(ci)) *bad = 1.0;
  }
}

// ---------------------------------------------------------------------------
// Spectral function (post-processing of C(t)).  G(t_k) = -i e^{-i s t_k} e^{C(t_k)}
// with s = eps_c + E_N^corr, times its trapezoid weight on the (possibly
// non-uniform) time grid; then A(w) = -(1/pi) Im sum_k wG_k e^{i w t_k - eta t_k},
// one frequency per thread, summed in k order; then the largest A on one block.
__global__ void green_kernel(const double* c, const double* t, int64_t n, double shift, double* wg) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double w = 0.0;
  if (n > 1) w = 0.5 * ((k + 1 < n ? t[k + 1] : t[k]) - (k > 0 ? t[k - 1] : t[k]));
  const double mag = exp(c[2 * k]) * w, ph = c[2 * k + 1] - shift * t[k];
  double sn, cs;
  sincos(ph, &sn, &cs);
  wg[2 * k] = mag * sn;          // -i e^{i ph}
  wg[2 * k + 1] = -mag * cs;
}

__global__ void spectrum_kernel(const double* wg, const double* t, int64_t n, double eta, const double* omega,
                                int64_t n_w, double* a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_w) return;
  const double w = omega[j];
  double im = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double sn, cs;
    sincos(w * t[k], &sn, &cs);
    im += exp(-eta * t[k]) * (wg[2 * k] * sn + wg[2 * k + 1] * cs);
  }
  a[j] = -im / M_PI;
}

constexpr int kPeakThreads = 1024;
constexpr int kMaxPeaks = 64;

// Local maxima of a, the largest first: k rounds of a block-wide arg-max over the local
// maxima not yet taken (ties: the first index).
__global__ __launch_bounds__(kPeakThreads) void peaks_kernel(const double* a, const double* omega, int64_t n_w,
                                                             int k, double* out) {
  __shared__ double sv[kPeakThreads];
  __shared__ int64_t si[kPeakThreads];
  __shared__ int64_t taken[kMaxPeaks];
  __shared__ int found;
  if (threadIdx.x == 0) found = 0;
  __syncthreads();
  for (int round = 0; round < k; ++round) {
    double best = -INFINITY;
    int64_t bi = -1;
    for (int64_t j = 1 + threadIdx.x; j + 1 < n_w; j += kPeakThreads) {
      if (!(a[j] > a[j - 1] && a[j] >= a[j + 1])) continue;
      bool used = false;
      for (int q = 0; q < found; ++q) used = used || taken[q] == j;
      if (used) continue;
      if (bi < 0 || a[j] > best) { best = a[j]; bi = j; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kPeakThreads / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        const double ov = sv[threadIdx.x + off];
        const int64_t oi = si[threadIdx.x + off];
        if (oi >= 0 && (si[threadIdx.x] < 0 || ov > sv[threadIdx.x] ||
                        (ov == sv[threadIdx.x] && oi < si[threadIdx.x]))) {
          sv[threadIdx.x] = ov;
          si[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    const int64_t j = si[0];
    if (j < 0) break;   // no local maximum left (uniform across the block)
    if (threadIdx.x == 0) {
      const double y0 = a[j - 1], y1 = a[j], y2 = a[j + 1], den = y0 - 2.0 * y1 + y2;
      const double sh = den != 0.0 ? 0.5 * (y0 - y2) / den : 0.0;
      out[2 * found] = omega[j] + sh * (omega[1] - omega[0]);
      out[2 * found + 1] = a[j];
      taken[found] = j;
      found = found + 1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[2 * k] = (double)found;
}
__global__ __launch_bounds__(kPeakThreads) void qp_kernel(const double* a, const double* omega, int64_t n_w,
                                                          double* qp) {
  __shared__ double sv[kPeakThreads];
  __shared__ int64_t si[kPeakThreads];
  double best = -INFINITY;
  int64_t bi = -1;
  for (int64_t j = threadIdx.x; j < n_w; j += kPeakThreads)
    if (a[j] > best || bi < 0) { best = a[j]; bi = j; }   // first index of the maximum in this stride
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = kPeakThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double ov = sv[threadIdx.x + off];
      const int64_t oi = si[threadIdx.x + off];
      if (oi >= 0 && (si[threadIdx.x] < 0 || ov > sv[threadIdx.x] ||
                      (ov == sv[threadIdx.x] && oi < si[threadIdx.x]))) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t k = si[0];
    double pos = omega[k];
    if (k > 0 && k + 1 < n_w) {
      const double y0 = a[k - 1], y1 = a[k], y2 = a[k + 1], den = y0 - 2.0 * y1 + y2;
      const double sh = den != 0.0 ? 0.5 * (y0 - y2) / den : 0.0;
      pos = omega[k] + sh * (omega[1] - omega[0]);
    }
    qp[0] = pos;
    qp[1] = a[k];
  }
}

// Tile shapes of gemm_mfma: 0 = 64x64, 1 = 64x128, 2 = 128x64, 3 = 128x128 (four
// waves), 4 = 64x128 and 5 = 128x64 with eight waves of 2 x 2 blocks.
constexpr int kTiles = 6;
constexpr int kTileM[kTiles] = {64, 64, 128, 128, 64, 128}, kTileN[kTiles] = {64, 128, 64, 128, 128, 64};

// Complex x complex keeps 64x64 (four MFMAs per staged fragment pair already).
// A complex x real product widens only the real operand's side: widening the
// complex side doubles two planes and leaves LDS for one work-group per CU.
// 128x128 holds 16 accumulator blocks: real x real in float32 only (in float64
// they exceed the registers of two waves per SIMD).  The bf16x3 kernel has one
// tile shape.
// The eight-wave shapes are built for float64 (the float32 path already keeps
// three or four waves per SIMD).
inline bool tile_allowed(int v, int prec, bool ac, bool bc) {
  if (v < 0 || v >= kTiles) return false;
  if (v >= 4 && prec != 0) return false;
  if (prec == 2 || (ac && bc)) return v == 0;
  if (ac) return v == 0 || v == 1 || v == 4;
  if (bc) return v == 0 || v == 2 || v == 5;
  return v != 3 || prec == 1;
}

// Launchers return false when no kernel is built for the requested tile shape and
// operand mix; the caller turns that into an error (never a silent fallback: the
// grid was sized for the requested shape).
template <typename T, bool AC, bool BC, int WM, int WN, int GM = 2, int GN = 2>
bool launch_mfma_tile(dim3 grid, hipStream_t st, const GemmArgs& g, bool akc, bool bkc) {
  constexpr int nt = 64 * GM * GN;
  if (akc && bkc) gemm_mfma<T, double, AC, BC, true, true, WM, WN, GM, GN><<<grid, nt, 0, st>>>(g);
  else if (akc) gemm_mfma<T, double, AC, BC, true, false, WM, WN, GM, GN><<<grid, nt, 0, st>>>(g);
  else if (bkc) gemm_mfma<T, double, AC, BC, false, true, WM, WN, GM, GN><<<grid, nt, 0, st>>>(g);
  else gemm_mfma<T, double, AC, BC, false, false, WM, WN, GM, GN><<<grid, nt, 0, st>>>(g);
  return true;
}

template <typename T, bool AC, bool BC>
bool launch_mfma(int v, dim3 grid, hipStream_t st, const GemmArgs& g, bool akc, bool bkc) {
  if (v == 0) return launch_mfma_tile<T, AC, BC, 2, 2>(grid, st, g, akc, bkc);
  if constexpr (!BC) {   // the real B side widens
    if (v == 1) return launch_mfma_tile<T, AC, BC, 2, 4>(grid, st, g, akc, bkc);
    if constexpr (sizeof(T) == 8) {
      if (v == 4) return launch_mfma_tile<T, AC, BC, 2, 2, 2, 4>(grid, st, g, akc, bkc);
    }
  }
  if constexpr (!AC) {   // the real A side widens
    if (v == 2) return launch_mfma_tile<T, AC, BC, 4, 2>(grid, st, g, akc, bkc);
    if constexpr (sizeof(T) == 8) {
      if (v == 5) return launch_mfma_tile<T, AC, BC, 2, 2, 4, 2>(grid, st, g, akc, bkc);
    }
  }
  if constexpr (sizeof(T) == 4 && !AC && !BC) {
    if (v == 3) return launch_mfma_tile<T, AC, BC, 4, 4>(grid, st, g, akc, bkc);
  }
  return false;
}

// float operands converted before the product: both k-contiguous
template <bool AC, bool BC>
bool launch_f32_converted(int v, dim3 grid, hipStream_t st, const GemmArgs& g) {
  if (v == 0) {
    gemm_mfma<float, float, AC, BC, true, true, 2, 2><<<grid, kThreads, 0, st>>>(g);
    return true;
  }
  if constexpr (!BC) {
    if (v == 1) {
      gemm_mfma<float, float, AC, BC, true, true, 2, 4><<<grid, kThreads, 0, st>>>(g);
      return true;
    }
  }
  if constexpr (!AC) {
    if (v == 2) {
      gemm_mfma<float, float, AC, BC, true, true, 4, 2><<<grid, kThreads, 0, st>>>(g);
      return true;
    }
  }
  if constexpr (!AC && !BC) {
    if (v == 3) {
      gemm_mfma<float, float, AC, BC, true, true, 4, 4><<<grid, kThreads, 0, st>>>(g);
      return true;
    }
  }
  return false;
}

bool launch_converted_gemm(int prec, int v, dim3 grid, hipStream_t st, const GemmArgs& g, bool ac, bool bc);

template <bool AC, bool BC>
void launch_bf16x3(dim3 grid, hipStream_t st, const GemmArgs& g, bool akc, bool bkc) {
  if (akc && bkc) gemm_bf16x3<AC, BC, true, true><<<grid, kThreads, 0, st>>>(g);
  else if (akc) gemm_bf16x3<AC, BC, true, false><<<grid, kThreads, 0, st>>>(g);
  else if (bkc) gemm_bf16x3<AC, BC, false, true><<<grid, kThreads, 0, st>>>(g);
  else gemm_bf16x3<AC, BC, false, false><<<grid, kThreads, 0, st>>>(g);
}

// Pre-split bf16x3 tile shapes: two LDS buffers of every hi/lo plane must fit
// 80 KB so that two work-groups share a CU.
constexpr int split_lds_bytes(bool ac, bool bc, int v, int nb, int bk = BKH) {
  return nb * ((ac ? 4 : 2) * kTileM[v] + (bc ? 4 : 2) * kTileN[v]) * (bk + PADH) * 2;
}
inline bool split_tile_allowed(int v, bool ac, bool bc) {
  return v >= 0 && v < 4 && split_lds_bytes(ac, bc, v, 2) <= 160 * 1024;
}

// Two LDS stages within 80 KiB: two work-groups per compute unit (two waves per SIMD).
// Larger tiles: complex x complex keeps two stages in up to the 160 KiB of a compute
// unit, one work-group with the whole register file per wave; the others keep two
// work-groups per compute unit with one stage.  (Measured on the ring and ladder
// shapes of the o=71, v=650 residual.)
template <typename E, bool AC, bool BC, int WM, int WN, int V>
bool launch_split_tile(dim3 grid, hipStream_t st, const GemmArgs& g) {
  if constexpr (split_lds_bytes(AC, BC, V, 2) <= 80 * 1024) {
    gemm_bf16x3_split<E, AC, BC, WM, WN, 2, 2, BKH><<<grid, kThreads, 0, st>>>(g);
    return true;
  } else if constexpr (AC && BC && split_lds_bytes(AC, BC, V, 2) <= 160 * 1024) {
    gemm_bf16x3_split<E, AC, BC, WM, WN, 2, 1, BKH><<<grid, kThreads, 0, st>>>(g);
    return true;
  } else if constexpr (!(AC && BC) && split_lds_bytes(AC, BC, V, 1) <= 80 * 1024) {
    gemm_bf16x3_split<E, AC, BC, WM, WN, 1, 2, BKH><<<grid, kThreads, 0, st>>>(g);
    return true;
  }
  return false;
}

template <typename E, bool AC, bool BC>
bool launch_split(int v, dim3 grid, hipStream_t st, const GemmArgs& g) {
  if (v == 0) return launch_split_tile<E, AC, BC, 1, 1, 0>(grid, st, g);
  if (v == 1) return launch_split_tile<E, AC, BC, 1, 2, 1>(grid, st, g);
  if (v == 2) return launch_split_tile<E, AC, BC, 2, 1, 2>(grid, st, g);
  if (v == 3) return launch_split_tile<E, AC, BC, 2, 2, 3>(grid, st, g);
  return false;
}

template <typename E>
bool launch_split_gemm(int v, dim3 grid, hipStream_t st, const GemmArgs& g, bool ac, bool bc) {
  if (ac && bc) return launch_split<E, true, true>(v, grid, st, g);
  if (ac) return launch_split<E, true, false>(v, grid, st, g);
  if (bc) return launch_split<E, false, true>(v, grid, st, g);
  return launch_split<E, false, false>(v, grid, st, g);
}

bool launch_converted_gemm(int prec, int v, dim3 grid, hipStream_t st, const GemmArgs& g, bool ac, bool bc) {
  if (prec == 2) return launch_split_gemm<SplitBf16>(v, grid, st, g, ac, bc);
  if (prec == 3) return launch_split_gemm<SplitF16>(v, grid, st, g, ac, bc);
  if (ac && bc) return launch_f32_converted<true, true>(v, grid, st, g);
  if (ac) return launch_f32_converted<true, false>(v, grid, st, g);
  if (bc) return launch_f32_converted<false, true>(v, grid, st, g);
  return launch_f32_converted<false, false>(v, grid, st, g);
}

template <bool AC, bool BC>
bool launch_prec(int prec, int v, dim3 grid, hipStream_t st, const GemmArgs& g, bool akc, bool bkc) {
  if (prec == 0) return launch_mfma<double, AC, BC>(v, grid, st, g, akc, bkc);
  if (prec == 1) return launch_mfma<float, AC, BC>(v, grid, st, g, akc, bkc);
  if (v != 0) return false;
  launch_bf16x3<AC, BC>(grid, st, g, akc, bkc);
  return true;
}

bool launch_gemm(int prec, int v, dim3 grid, hipStream_t st, const GemmArgs& g, bool ac, bool bc, bool akc,
                 bool bkc) {
  if (ac && bc) return launch_prec<true, true>(prec, v, grid, st, g, akc, bkc);
  if (ac) return launch_prec<true, false>(prec, v, grid, st, g, akc, bkc);
  if (bc) return launch_prec<false, true>(prec, v, grid, st, g, akc, bkc);
  return launch_prec<false, false>(prec, v, grid, st, g, akc, bkc);
}

// Fixed device scratch for entry points that must not allocate (rteom_spectral_noalloc):
// a file-scope device array, one copy per GPU, held until the process ends.  Host code
// never passes `scratch` itself (in host code it names a host-side stand-in): its device
// address is looked up once per device with hipGetSymbolAddress and kept.
constexpr int64_t kFixedScratchDoubles = int64_t(1) << 22;   // 32 MiB
static __device__ __align__(256) double scratch[kFixedScratchDoubles];

// Device address of `scratch` on the current device (looked up once per device; nullptr
// with a message if the lookup fails).
double* scratch_address(std::string* err) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    if (err) *err = "hipGetDevice failed";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    if (err) *err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
    return nullptr;
  }
  addr[dev] = static_cast<double*>(p);
  return addr[dev];
}

int grid_for(int64_t n, int per_block = 256) {
  int64_t g = (n + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

class HipBackend : public Backend {
 public:
  explicit HipBackend(hipStream_t s) : stream_(s) {
    // at set-up, with the context's device current: the fixed scratch's address
    std::string m;
    fixed_ = scratch_address(&m);
    if (!fixed_) set_err(m);
  }
  double* fixed_scratch(int64_t* doubles) override {
    if (doubles) *doubles = fixed_ ? kFixedScratchDoubles : 0;
    return fixed_;
  }
  double* fixed_ = nullptr;
  ~HipBackend() override {
    for (auto& e : done_) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (auto& e : pool_) (void)hipEventDestroy(e);
    for (auto& g : graphs_) (void)hipGraphDestroy(g);
    for (auto& e : graph_timed_) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    if (tune_a_) { (void)hipEventDestroy(tune_a_); (void)hipEventDestroy(tune_b_); }
    if (own_stream_) (void)hipStreamDestroy(stream_);
  }
  bool own_stream_ = false;

  void set_profile(unsigned mask) override { mask_ = mask; }
  double phase_ms(int ph, int64_t* ops) override {
    record(hipStreamSynchronize(stream_), "hipStreamSynchronize");
    double total = 0.0;
    int64_t n = 0;
    std::vector<Timed> keep;
    for (auto& e : done_) {
      if (e.ph != ph) { keep.push_back(e); continue; }
      float ms = 0.f;
      record(hipEventElapsedTime(&ms, e.a, e.b), "hipEventElapsedTime");
      total += ms;
      ++n;
      pool_.push_back(e.a);
      pool_.push_back(e.b);
    }
    done_.swap(keep);
    // operations inside captured graphs: their times in the most recent replay
    for (auto& e : graph_timed_) {
      if (e.ph != ph) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
        total += ms;
        ++n;
      } else {
        (void)hipGetLastError();   // graph not replayed yet
      }
    }
    if (ops) *ops = n;
    return total;
  }

  void* alloc(size_t bytes) override {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void release(void* p) override { record(hipFree(p), "hipFree"); }
  void h2d(void* d, const void* s, size_t b) override {
    record(hipMemcpyAsync(d, s, b, hipMemcpyHostToDevice, stream_), "hipMemcpyAsync H2D");
    record(hipStreamSynchronize(stream_), "hipStreamSynchronize");
  }
  void d2h(void* d, const void* s, size_t b) override {
    record(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToHost, stream_), "hipMemcpyAsync D2H");
    record(hipStreamSynchronize(stream_), "hipStreamSynchronize");
  }
  void d2d(void* d, const void* s, size_t b) override {
    record(hipMemcpyAsync(d, s, b, hipMemcpyDeviceToDevice, stream_), "hipMemcpyAsync D2D");
  }
  void fill(double* p, int64_t n, double v) override {
    if (n <= 0) return;
    begin();
    fill_kernel<<<grid_for(n), 256, 0, stream_>>>(p, n, v);
    launched("fill");
    end();
  }
  void sync() override { record(hipStreamSynchronize(stream_), "hipStreamSynchronize"); }
  bool ok(std::string* msg) override {
    if (!err_.empty()) {
      *msg = err_;
      return false;
    }
    return true;
  }
  int64_t energy_partials() const override { return 2 * kEnergyBlocks; }

  void gemm(const GemmOp& op) override {
    if (op.prec < 0 || op.prec > 3) {
      set_err("unknown contraction precision");
      return;
    }
    GemmArgs g;
    g.M = op.M; g.N = op.N; g.K = op.K; g.batch = op.batch;
    g.ar = op.a_re; g.ai = op.a_im; g.asm_ = op.a_sm; g.ask = op.a_sk; g.asb = op.a_sb;
    g.br = op.b_re; g.bi = op.b_im; g.bsk = op.b_sk; g.bsn = op.b_sn; g.bsb = op.b_sb;
    g.cr = op.c_re; g.ci = op.c_im; g.csm = op.c_sm; g.csn = op.c_sn; g.csb = op.c_sb;
    g.alpha = op.alpha;
    g.beta = op.beta;
    g.aext = 1 + (op.M - 1) * op.a_sm + (op.K - 1) * op.a_sk + (op.a_sb ? (op.batch - 1) * op.a_sb : 0);
    g.bext = 1 + (op.N - 1) * op.b_sn + (op.K - 1) * op.b_sk + (op.b_sb ? (op.batch - 1) * op.b_sb : 0);
    g.tiles_m = (op.M + BM - 1) / BM;
    g.tiles_n = (op.N + BN - 1) / BN;
    g.splitk = 1;
    g.kchunk = op.K;
    g.pr = g.pi = nullptr;
    const bool cplx = op.a_im != nullptr || op.b_im != nullptr;
    if (op.K <= 16) {
      const int n_inner = std::llabs(op.c_sn) <= std::llabs(op.c_sm) ? 1 : 0;
      const int64_t total = op.batch * op.M * op.N;
      begin();
      if (op.a_im && op.b_im) gemm_smallk<true, true><<<grid_for(total), 256, 0, stream_>>>(g, n_inner);
      else if (op.a_im) gemm_smallk<true, false><<<grid_for(total), 256, 0, stream_>>>(g, n_inner);
      else if (op.b_im) gemm_smallk<false, true><<<grid_for(total), 256, 0, stream_>>>(g, n_inner);
      else gemm_smallk<false, false><<<grid_for(total), 256, 0, stream_>>>(g, n_inner);
      launched("gemm_smallk");
      end();
      return;
    }
    // the larger operand is reused by neighbouring logical tiles
    g.m_fast = (op.K * op.N * (op.b_im ? 2 : 1) >= op.M * op.K * (op.a_im ? 2 : 1)) ? 1 : 0;
    if (op.splitk > 1 && op.partial && op.batch == 1) {
      g.kchunk = ((op.K + op.splitk - 1) / op.splitk + BKH - 1) / BKH * BKH;
      g.splitk = (int)((op.K + g.kchunk - 1) / g.kchunk);
      g.pr = op.partial;
      g.pi = cplx ? op.partial + (int64_t)g.splitk * op.M * op.N : nullptr;
    }
    // Wave priority: raised while a work-group's sum is shorter than 65536 k; longer
    // ones (the particle-particle ladder) keep the default, which lets the work-groups
    // sharing an operand panel stay closer in k, so that the XCD L2 serves more of it
    // (whole-step A/B: the long ladder 3.6 % faster without, the shorter products 1-3 %
    // faster with)
    g.prio = g.kchunk < 65536 ? 1 : 0;
    const bool ac = op.a_im != nullptr, bc = op.b_im != nullptr;
    const bool akc = op.a_sk == 1 && op.a_sm != 1, bkc = op.b_sk == 1 && op.b_sn != 1;
    const bool presplit = op.prec != 0 && op.split != nullptr;
    if (op.prec == 3 && (!presplit || op.b_conv)) {
      set_err("gemm: fp16x3 needs both operands converted before the product into the split scratch");
      return;
    }
    begin();   // one timed operation: operand conversion, product and split-K reduction
    if (presplit) {
      if (op.prec >= 2) split_operands(op, g, ac, bc);
      else f32_operands(op, g, ac, bc);
    }
    if (!(presplit && op.prec >= 2) && !windows_fit(g, op.prec == 0 || !presplit ? 8 : 4)) {
      set_err("gemm: an operand tile spans more than 2 GiB");
      end();
      return;
    }
    const int v = choose_tile(op, g, ac, bc, akc, bkc, presplit);
    if (v < 0) { end(); return; }
    dim3 grid;
    if (!shape_grid(g, v, op.batch, &grid)) { end(); return; }
    const bool ok = presplit ? launch_converted_gemm(op.prec, v, grid, stream_, g, ac, bc)
                             : launch_gemm(op.prec, v, grid, stream_, g, ac, bc, akc, bkc);
    if (!ok) {
      set_err("gemm: no kernel for tile shape " + std::to_string(v) + " with these operands");
      end();
      return;
    }
    launched("gemm");
    if (g.splitk > 1) {
      splitk_reduce<<<grid_for(op.M * op.N), 256, 0, stream_>>>(g, cplx ? 1 : 0);
      launched("splitk_reduce");
    }
    end();
  }

  // bf16 hi/lo planes of A ([batch][M][ld]) and B ([batch][N][ld]) in op.split.
  void split_operands(const GemmOp& op, GemmArgs& g, bool ac, bool bc) {
    const int64_t ld = split_ld(op.K), nba = op.a_sb ? op.batch : 1, nbb = op.b_sb ? op.batch : 1;
    const int64_t asz = nba * op.M * ld, bsz = nbb * op.N * ld;
    unsigned short* base = reinterpret_cast<unsigned short*>(op.split);
    const int pa = ac ? 4 : 2, pb = bc ? 4 : 2;
    unsigned short* bbase = op.b_conv ? reinterpret_cast<unsigned short*>(op.b_conv) : base + pa * asz;
    for (int p = 0; p < 4; ++p) {
      g.sa[p] = p < pa ? base + p * asz : nullptr;
      g.sb[p] = p < pb ? bbase + p * bsz : nullptr;
    }
    g.sld = ld;
    g.sab = op.a_sb ? op.M * ld : 0;
    g.sbb = op.b_sb ? op.N * ld : 0;
    if (op.prec == 3) {
      // fp16 planes scaled per row: row maxima of both planes, then the split.  The
      // scratch holds after the planes: A's and B's row maxima (uint) and inverse
      // scales (float), [batch][rows] each.
      unsigned int* amax = reinterpret_cast<unsigned int*>(base + pa * asz + pb * bsz);
      unsigned int* bmax = amax + nba * op.M;
      float* ainv = reinterpret_cast<float*>(bmax + nbb * op.N);
      float* binv = ainv + nba * op.M;
      g.sca = ainv;
      g.scb = binv;
      fill_kernel<<<grid_for((nba * op.M + nbb * op.N + 1) / 2), 256, 0, stream_>>>(
          reinterpret_cast<double*>(amax), (nba * op.M + nbb * op.N + 1) / 2, 0.0);
      launched("fill");
      auto rmax = [&](const double* src, int64_t rows, int64_t s_row, int64_t s_k, int64_t s_b, unsigned int* m) {
        dim3 grid((unsigned)((op.K + 63) / 64), (unsigned)((rows + 63) / 64), (unsigned)(s_b ? op.batch : 1));
        rowmax_kernel<<<grid, 256, 0, stream_>>>(src, rows, op.K, s_row, s_k, s_b, m);
        launched("row max");
      };
      auto run16 = [&](const double* src, int64_t rows, int64_t s_row, int64_t s_k, int64_t s_b, const unsigned int* m,
                       const unsigned short* h, const unsigned short* l, float* inv) {
        dim3 grid((unsigned)((ld + 63) / 64), (unsigned)((rows + 63) / 64), (unsigned)(s_b ? op.batch : 1));
        split_f16_kernel<<<grid, 256, 0, stream_>>>(src, rows, op.K, s_row, s_k, s_b, ld, m,
                                                     const_cast<unsigned short*>(h), const_cast<unsigned short*>(l), inv);
        launched("split f16");
      };
      rmax(op.a_re, op.M, op.a_sm, op.a_sk, op.a_sb, amax);
      if (ac) rmax(op.a_im, op.M, op.a_sm, op.a_sk, op.a_sb, amax);
      rmax(op.b_re, op.N, op.b_sn, op.b_sk, op.b_sb, bmax);
      if (bc) rmax(op.b_im, op.N, op.b_sn, op.b_sk, op.b_sb, bmax);
      run16(op.a_re, op.M, op.a_sm, op.a_sk, op.a_sb, amax, g.sa[0], g.sa[1], ainv);
      if (ac) run16(op.a_im, op.M, op.a_sm, op.a_sk, op.a_sb, amax, g.sa[2], g.sa[3], ainv);
      run16(op.b_re, op.N, op.b_sn, op.b_sk, op.b_sb, bmax, g.sb[0], g.sb[1], binv);
      if (bc) run16(op.b_im, op.N, op.b_sn, op.b_sk, op.b_sb, bmax, g.sb[2], g.sb[3], binv);
      return;
    }
    auto run = [&](const double* src, int64_t rows, int64_t s_row, int64_t s_k, int64_t s_b, const unsigned short* h,
                   const unsigned short* l) {
      dim3 grid((unsigned)((ld + 63) / 64), (unsigned)((rows + 63) / 64), (unsigned)(s_b ? op.batch : 1));
      split_kernel<<<grid, 256, 0, stream_>>>(src, rows, op.K, s_row, s_k, s_b, ld, const_cast<unsigned short*>(h),
                                               const_cast<unsigned short*>(l));
      launched("split");
    };
    run(op.a_re, op.M, op.a_sm, op.a_sk, op.a_sb, g.sa[0], g.sa[1]);
    if (ac) run(op.a_im, op.M, op.a_sm, op.a_sk, op.a_sb, g.sa[2], g.sa[3]);
    if (op.b_conv && !op.b_conv_fill) return;   // B converted by an earlier product
    run(op.b_re, op.N, op.b_sn, op.b_sk, op.b_sb, g.sb[0], g.sb[1]);
    if (bc) run(op.b_im, op.N, op.b_sn, op.b_sk, op.b_sb, g.sb[2], g.sb[3]);
  }

  // float planes of A ([batch][M][ld]) and B ([batch][N][ld]) in op.split; the
  // product then reads them through the double fields of g with float strides.
  void f32_operands(const GemmOp& op, GemmArgs& g, bool ac, bool bc) {
    const int64_t ld = split_ld(op.K), nba = op.a_sb ? op.batch : 1, nbb = op.b_sb ? op.batch : 1;
    const int64_t asz = nba * op.M * ld, bsz = nbb * op.N * ld;
    float* base = reinterpret_cast<float*>(op.split);
    float* pl[4] = {base, ac ? base + asz : nullptr, base + (ac ? 2 : 1) * asz, nullptr};
    if (op.b_conv) pl[2] = reinterpret_cast<float*>(op.b_conv);
    pl[3] = bc ? pl[2] + bsz : nullptr;
    auto run = [&](const double* src, int64_t rows, int64_t s_row, int64_t s_k, int64_t s_b, float* d) {
      dim3 grid((unsigned)((ld + 63) / 64), (unsigned)((rows + 63) / 64), (unsigned)(s_b ? op.batch : 1));
      f32_kernel<<<grid, 256, 0, stream_>>>(src, rows, op.K, s_row, s_k, s_b, ld, d);
      launched("f32 convert");
    };
    run(op.a_re, op.M, op.a_sm, op.a_sk, op.a_sb, pl[0]);
    if (ac) run(op.a_im, op.M, op.a_sm, op.a_sk, op.a_sb, pl[1]);
    if (!op.b_conv || op.b_conv_fill) {
      run(op.b_re, op.N, op.b_sn, op.b_sk, op.b_sb, pl[2]);
      if (bc) run(op.b_im, op.N, op.b_sn, op.b_sk, op.b_sb, pl[3]);
    }
    g.ar = reinterpret_cast<const double*>(pl[0]);
    g.ai = reinterpret_cast<const double*>(pl[1]);
    g.br = reinterpret_cast<const double*>(pl[2]);
    g.bi = reinterpret_cast<const double*>(pl[3]);
    g.asm_ = ld; g.ask = 1; g.asb = op.a_sb ? op.M * ld : 0;
    g.bsn = ld; g.bsk = 1; g.bsb = op.b_sb ? op.N * ld : 0;
    g.aext = nba * op.M * ld;
    g.bext = nbb * op.N * ld;
  }

  // The product kernels address one K tile of each operand through a buffer
  // resource with 32-bit offsets: the tile's extent must stay below 2 GiB.
  // (checked for the largest tile, 128 x 128, so that every candidate fits)
  static bool windows_fit(const GemmArgs& g, int64_t es) {
    const int64_t lim = int64_t(1) << 31;
    const int64_t wa = (127 * std::llabs(g.asm_) + (BK - 1) * std::llabs(g.ask) + 1) * es;
    const int64_t wb = (127 * std::llabs(g.bsn) + (BK - 1) * std::llabs(g.bsk) + 1) * es;
    return wa < lim && wb < lim;
  }

  void set_tuning(int on) override { tuning_ = on != 0; }
  void force_tile(int v) override { force_ = v; }

  int64_t tile_table(int64_t* rows, int64_t max) const override {
    int64_t n = 0;
    for (const auto& kv : tuned_) {
      if (rows && n < max) {
        for (int k = 0; k < kTileKey; ++k) rows[n * (kTileKey + 1) + k] = kv.first[k];
        rows[n * (kTileKey + 1) + kTileKey] = kv.second;
      }
      ++n;
    }
    return n;
  }
  bool load_tile_table(const int64_t* rows, int64_t n, std::string* err) override {
    std::map<std::array<int64_t, 10>, int> add;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t* r = rows + i * (kTileKey + 1);
      std::array<int64_t, 10> key;
      for (int k = 0; k < kTileKey; ++k) key[k] = r[k];
      // key: precision (+8 when the operands are converted first), M, N, K, batch,
      // A complex, B complex, A k-contiguous, B k-contiguous, split-K factor
      const int64_t pr = key[0] & 7, tile = r[kTileKey];
      const bool presplit = key[0] >= 8, ac = key[5] != 0, bc = key[6] != 0;
      const bool ok = key[0] >= 0 && key[0] < 16 && pr <= 3 && key[1] > 0 && key[2] > 0 && key[3] > 0 && key[4] > 0 &&
                      key[9] > 0 && tile >= 0 && tile < kTiles &&
                      ((presplit && pr >= 2) ? split_tile_allowed((int)tile, ac, bc)
                                             : tile_allowed((int)tile, (int)pr, ac, bc));
      if (!ok) {
        if (err) *err = "tile table entry " + std::to_string(i) + " is not a built tile shape for its product";
        return false;
      }
      add[key] = (int)tile;
    }
    for (const auto& kv : add) tuned_[kv.first] = kv.second;
    return true;
  }
  std::string device_arch() const override {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));   // the target without its feature flags
  }

  // Grid of tile shape v (tiles x split or batch); false on overflow.
  bool shape_grid(GemmArgs& g, int v, int64_t batch, dim3* grid) {
    g.tiles_m = (g.M + kTileM[v] - 1) / kTileM[v];
    g.tiles_n = (g.N + kTileN[v] - 1) / kTileN[v];
    const int64_t tiles = g.tiles_m * g.tiles_n;
    if (tiles > 0x7fffffffLL) {
      set_err("gemm: too many tiles");
      return false;
    }
    *grid = dim3((unsigned)tiles, (unsigned)(g.splitk > 1 ? g.splitk : std::min<int64_t>(batch, 65535)));
    return true;
  }

  // Rule used without timing: estimated time = rounds of work-groups over the
  // 256 CUs (two resident work-groups share one CU's matrix cores) times the
  // tile area over an efficiency that grows weakly with the MFMA products per
  // staged operand word (the complex x complex 64x64 tile runs at 64).  Wider
  // tiles only pay off over long sums, so they are considered from K >= 4096.
  static double rule_time(const GemmArgs& g, int v, int64_t batch, bool ac, bool bc) {
    const double tm = kTileM[v], tn = kTileN[v];
    const double prods = (ac && bc) ? 4.0 : ((ac || bc) ? 2.0 : 1.0);
    const double words = tm * (ac ? 2 : 1) + tn * (bc ? 2 : 1);
    const double eff = std::pow(std::min(1.0, tm * tn * prods / words / 64.0), 0.3);
    const double units = (double)((g.M + kTileM[v] - 1) / kTileM[v]) * ((g.N + kTileN[v] - 1) / kTileN[v]) *
                         (double)(g.splitk > 1 ? g.splitk : batch);
    return std::ceil(units / 256.0) * (tm * tn / 4096.0) / eff;
  }

  int choose_tile(const GemmOp& op, GemmArgs& g, bool ac, bool bc, bool akc, bool bkc, bool presplit) {
    auto allowed = [&](int v) {
      return (presplit && op.prec >= 2) ? split_tile_allowed(v, ac, bc) : tile_allowed(v, op.prec, ac, bc);
    };
    if (force_ >= 0) return allowed(force_) ? force_ : 0;
    int cand[kTiles], nc = 0;
    for (int v = 0; v < kTiles; ++v)
      if (allowed(v)) cand[nc++] = v;
    if (nc == 1) return cand[0];
    const std::array<int64_t, 10> key = {op.prec + (presplit ? 8 : 0), op.M, op.N, op.K, op.batch, (int64_t)ac,
                                         (int64_t)bc, (int64_t)akc, (int64_t)bkc, (int64_t)g.splitk};
    auto it = tuned_.find(key);
    if (it != tuned_.end()) return it->second;
    if (!tuning_ || capturing_) {
      if (presplit && op.prec >= 2 && g.kchunk >= 1024) {
        // split products (timed on the o=71, v=650 and o=95, v=561 residuals' shapes,
        // sums of 2000 and more).  Complex x complex: 128 x 128 (one work-group per
        // compute unit) unless its last round of tiles is mostly empty, where 64 x 64
        // (two per compute unit, a round taking 1/1.76 as long) wins.  Mixed products:
        // 128 x 128 with one short side or one very long one, else 64 x 128.
        const int64_t units = op.batch > 1 ? op.batch : g.splitk;
        int v;
        if (ac && bc) {
          const double r3 = std::ceil((double)((op.M + 127) / 128) * ((op.N + 127) / 128) * units / 256.0) * 1.76;
          const double r0 = std::ceil((double)((op.M + 63) / 64) * ((op.N + 63) / 64) * units / 512.0);
          v = r3 <= r0 ? 3 : 0;
        } else {
          v = std::min(op.M, op.N) <= 8192 || std::max(op.M, op.N) >= 131072 ? 3 : 1;
        }
        if (split_tile_allowed(v, ac, bc)) return v;
      }
      int best = cand[0];
      double bt = rule_time(g, cand[0], op.batch, ac, bc);
      // long sums weigh the tile shapes; so do float64 real products from sums of
      // 1024 on (the integral slabs: 64 x 128 measured 4.5 % faster than 64 x 64)
      const bool weigh = g.kchunk >= 4096 || (op.prec == 0 && !ac && !bc && g.kchunk >= 1024);
      for (int i = 1; i < nc && weigh; ++i) {
        const double t = rule_time(g, cand[i], op.batch, ac, bc);
        if (t < bt * 0.98) { bt = t; best = cand[i]; }
      }
      return best;
    }
    // Time every candidate on this product with alpha = 0: C (beta = 1) keeps
    // its value, a beta = 0 output and split partials are rewritten by the
    // launch that follows.  Short products are timed twice.
    if (!tune_a_) {
      record(hipEventCreate(&tune_a_), "hipEventCreate");
      record(hipEventCreate(&tune_b_), "hipEventCreate");
    }
    GemmArgs gt = g;
    gt.alpha = 0.0;
    float best_ms[kTiles];
    for (int i = 0; i < nc; ++i) best_ms[i] = 1e30f;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < nc; ++i) {
        dim3 grid;
        if (!shape_grid(gt, cand[i], op.batch, &grid)) return -1;
        record(hipEventRecord(tune_a_, stream_), "hipEventRecord");
        const bool ok = presplit ? launch_converted_gemm(op.prec, cand[i], grid, stream_, gt, ac, bc)
                                 : launch_gemm(op.prec, cand[i], grid, stream_, gt, ac, bc, akc, bkc);
        if (!ok) {
          set_err("gemm: no kernel for tile shape " + std::to_string(cand[i]) + " with these operands");
          return -1;
        }
        launched("gemm (tuning)");
        record(hipEventRecord(tune_b_, stream_), "hipEventRecord");
        record(hipEventSynchronize(tune_b_), "hipEventSynchronize");
        float ms = 0.f;
        record(hipEventElapsedTime(&ms, tune_a_, tune_b_), "hipEventElapsedTime");
        best_ms[i] = std::min(best_ms[i], ms);
      }
      float fastest = 1e30f;
      for (int i = 0; i < nc; ++i) fastest = std::min(fastest, best_ms[i]);
      if (fastest >= 2.0f) break;
    }
    int bi = 0;
    for (int i = 1; i < nc; ++i)
      if (best_ms[i] < best_ms[bi]) bi = i;
    tuned_[key] = cand[bi];
    return cand[bi];
  }

  void permute(const PermOp& op) override {
    PermArgs p;
    p.nd = op.nd;
    p.total = 1;
    for (int d = 0; d < kMaxDims; ++d) {
      p.dim[d] = d < op.nd ? op.dim[d] : 1;
      p.istr[d] = d < op.nd ? op.in_str[d] : 0;
      p.ostr[d] = d < op.nd ? op.out_str[d] : 0;
      p.sc[d] = d < op.nd ? op.scale[d] : nullptr;
      if (d < op.nd) p.total *= op.dim[d];
    }
    if (p.total == 0) return;
    p.ir = op.in_re; p.ii = op.in_im; p.orr = op.out_re; p.oi = op.out_im;
    p.ar = op.alpha_re; p.ai = op.alpha_im; p.beta = op.beta;
    // unit-stride dimension of each side (the innermost one if several)
    int din = -1, dout = -1;
    for (int d = 0; d < op.nd; ++d) {
      if (op.dim[d] > 1 && op.in_str[d] == 1) din = d;
      if (op.dim[d] > 1 && op.out_str[d] == 1) dout = d;
    }
    begin();
    if (din >= 0 && dout >= 0 && din != dout && op.dim[din] >= 8 && op.dim[dout] >= 8 && op.in_re != op.out_re) {
      const int64_t ti = (op.dim[din] + 31) / 32, to = (op.dim[dout] + 31) / 32;
      const int64_t nblocks = p.total / (op.dim[din] * op.dim[dout]) * ti * to;
      permute_tiled<<<(unsigned)std::min<int64_t>(nblocks, 1 << 18), 256, 0, stream_>>>(p, din, dout, ti, to, nblocks);
      launched("permute (tiled)");
    } else {
      permute_kernel<<<grid_for(p.total), 256, 0, stream_>>>(p);
      launched("permute");
    }
    end();
  }

  void ss(const SsOp& op) override {
    SsArgs g;
    g.n1 = op.n1; g.n2 = op.n2; g.np2 = op.n2 * (op.n2 - 1) / 2;
    g.i0 = op.i0; g.ci = op.ci; g.j0 = op.j0; g.cj = op.cj;
    g.pair2 = op.pair2; g.anti1 = op.anti1; g.anti2 = op.anti2; g.beta = op.beta; g.alpha = op.alpha;
    g.xr = op.x_re; g.xi = op.x_im; g.yr = op.y_re; g.yi = op.y_im;
    g.ur = op.u_re; g.ui = op.u_im; g.m1 = op.m1; g.m2 = op.m2;
    g.oi = op.pt.oi; g.oj = op.pt.oj; g.va = op.pt.va; g.vb = op.pt.vb;
    const int64_t np1 = op.n1 * (op.n1 - 1) / 2;
    switch (op.mode) {
      case SsOp::kExpand: case SsOp::kAccum: g.rows = op.ci * op.cj * op.n2; break;
      case SsOp::kAccumRows: g.rows = op.ci * op.n2; break;
      case SsOp::kT1T1: case SsOp::kMask: g.rows = np1 * op.n2; break;
      default: g.rows = op.ci * op.n1 * (op.pair2 ? op.n2 : 1); break;
    }
    if (g.rows <= 0 || op.n2 <= 0) return;
    begin();
    const unsigned grid = (unsigned)std::min<int64_t>(g.rows, 1 << 20);
    switch (op.mode) {
      case SsOp::kExpand: ss_expand<<<grid, 256, 0, stream_>>>(g); launched("pair expand"); break;
      case SsOp::kAccum: ss_accum<<<grid, 256, 0, stream_>>>(g); launched("pair accumulate"); break;
      case SsOp::kAccumRows: ss_accum_rows<<<grid, 256, 0, stream_>>>(g); launched("pair accumulate rows"); break;
      case SsOp::kT1T1: ss_pairwise<<<grid, 256, 0, stream_>>>(g, 0); launched("pair t1 t1"); break;
      case SsOp::kMask: ss_pairwise<<<grid, 256, 0, stream_>>>(g, 1); launched("pair mask"); break;
      default: ss_pack_slab<<<grid, 256, 0, stream_>>>(g); launched("pair pack"); break;
    }
    end();
  }

  void update(const UpdateOp& u) override {
    UpdArgs a;
    a.no = u.lay.no; a.nv = u.lay.nv; a.n1 = u.lay.n1(); a.nss = u.lay.nss(); a.npv = u.lay.npv();
    a.off_ab = u.lay.off_ab(); a.total = u.lay.size();
    a.oi = u.pt.oi; a.oj = u.pt.oj; a.va = u.pt.va; a.vb = u.pt.vb;
    a.xr = u.x_re; a.xi = u.x_im; a.rr = u.r_re; a.ri = u.r_im; a.hr_ = u.rhs_re; a.hi_ = u.rhs_im;
    a.h = u.h; a.mode = u.mode; a.start = u.start;
    for (int s = 0; s < 2; ++s) {
      a.mo[s] = u.sv.mo[s]; a.mv[s] = u.sv.mv[s]; a.fo[s] = u.sv.fo[s]; a.fv[s] = u.sv.fv[s];
    }
    a.delta = reinterpret_cast<unsigned long long*>(u.delta);
    begin();
    update_kernel<<<grid_for(a.total), 256, 0, stream_>>>(a);
    launched("update");
    end();
  }

  void energy(const EnergyOp& op) override {
    EnArgs e;
    e.no = op.lay.no; e.nv = op.lay.nv; e.n1 = op.lay.n1(); e.npv = op.lay.npv();
    e.off_aa = op.lay.off_ss(0); e.off_bb = op.lay.off_ss(1); e.off_ab = op.lay.off_ab();
    e.xr = op.x_re; e.xi = op.x_im; e.jov = op.jov;
    e.fov0 = op.fov[0]; e.fov1 = op.fov[1]; e.ld = op.fov_ld; e.ft1 = op.include_ft1;
    e.part = op.partial; e.out = op.e_out;
    begin();
    energy_pass1<<<kEnergyBlocks, 256, 0, stream_>>>(e);
    launched("energy_pass1");
    energy_pass2<<<1, 64, 0, stream_>>>(e, kEnergyBlocks);
    launched("energy_pass2");
    end();
  }

  void cumulant_append(double* c, double* e, const double* en, int64_t* step, double h, double* bad) override {
    begin();
    cumulant_kernel<<<1, 64, 0, stream_>>>(c, e, en, step, h, bad);
    launched("cumulant");
    end();
  }

  void dot(const double* a, const double* b, int64_t n, double* part, double* out) override {
    begin();
    dot_pass1<<<kEnergyBlocks, 256, 0, stream_>>>(a, b, n, part);
    launched("dot_pass1");
    dot_pass2<<<1, 64, 0, stream_>>>(part, kEnergyBlocks, out);
    launched("dot_pass2");
    end();
  }

  void spectral(const double* c_hist, const double* times, int64_t n, double shift, double eta, const double* omega,
                int64_t n_w, double* wg, double* a_out, double* qp_out) override {
    if (n < 1 || n_w < 1) return;
    green_kernel<<<grid_for(n), 256, 0, stream_>>>(c_hist, times, n, shift, wg);
    launched("green");
    spectrum_kernel<<<(unsigned)((n_w + 255) / 256), 256, 0, stream_>>>(wg, times, n, eta, omega, n_w, a_out);
    launched("spectrum");
    qp_kernel<<<1, kPeakThreads, 0, stream_>>>(a_out, omega, n_w, qp_out);
    launched("qp");
  }

  void spectral_peaks(const double* a, const double* omega, int64_t n_w, int k, double* out) override {
    begin();
    peaks_kernel<<<1, kPeakThreads, 0, stream_>>>(a, omega, n_w, k, out);
    launched("peaks");
    end();
  }

  void* stream() override { return stream_; }
  bool begin_capture() override {
    if (stream_ == nullptr) return false;   // the legacy null stream cannot be captured
    capturing_ = true;
    record(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    return err_.empty();
  }
  bool capturing() const override { return capturing_; }
  void* end_capture() override {
    hipGraph_t graph = nullptr;
    record(hipStreamEndCapture(stream_, &graph), "hipStreamEndCapture");
    capturing_ = false;
    if (!graph) return nullptr;
    hipGraphExec_t exec = nullptr;
    record(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    graphs_.push_back(graph);
    return exec;
  }
  void launch_graph(void* exec) override {
    record(hipGraphLaunch(static_cast<hipGraphExec_t>(exec), stream_), "hipGraphLaunch");
  }
  void destroy_graph(void* exec) override {
    if (exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(exec));
  }

 private:
  struct Timed { hipEvent_t a, b; int ph; };
  std::vector<hipGraph_t> graphs_;
  bool capturing_ = false;
  hipStream_t stream_;
  std::string err_;
  unsigned mask_ = 0;
  std::vector<Timed> done_;
  std::vector<Timed> graph_timed_;
  std::vector<hipEvent_t> pool_;
  std::map<std::array<int64_t, 10>, int> tuned_;   // tile shape per GEMM signature
  bool tuning_ = true;
  int force_ = -1;
  hipEvent_t tune_a_ = nullptr, tune_b_ = nullptr;
  hipEvent_t cur_a_ = nullptr;
  bool timing_ = false;
  hipEvent_t event() {
    if (!pool_.empty()) { hipEvent_t e = pool_.back(); pool_.pop_back(); return e; }
    hipEvent_t e = nullptr;
    record(hipEventCreate(&e), "hipEventCreate");
    return e;
  }
  void begin() {
    timing_ = ((mask_ >> phase_) & 1u) != 0;
    if (timing_) {
      cur_a_ = event();
      record(hipEventRecord(cur_a_, stream_), "hipEventRecord");
    }
  }
  void end() {
    if (!timing_) return;
    hipEvent_t b = event();
    record(hipEventRecord(b, stream_), "hipEventRecord");
    // recorded during capture: event nodes of the graph, re-recorded by every replay
    (capturing_ ? graph_timed_ : done_).push_back({cur_a_, b, phase_});
    timing_ = false;
  }
  void set_err(const std::string& m) {
    if (err_.empty()) err_ = m;
  }
  void record(hipError_t e, const char* what) {
    if (e != hipSuccess) set_err(std::string(what) + ": " + hipGetErrorString(e));
  }
  void launched(const char* what) { record(hipGetLastError(), what); }
};

}  // namespace

Backend* make_hip_backend(void* stream, std::string* err) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
    (void)hipGetLastError();
    if (err) *err = "no HIP device";
    return nullptr;
  }
  return new HipBackend(static_cast<hipStream_t>(stream));
}

}  // namespace rteom
