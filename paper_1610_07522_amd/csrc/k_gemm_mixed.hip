// Mixed-precision subspace products: complex64 operands on the FP16 matrix
// cores of gfx950 (v_mfma_f32_16x16x32_f16) with a two-term FP16 split.
//
// Each operand matrix gets one power-of-two scale 2^S, chosen from its largest
// component so that every scaled component is below 2^14.  Each scaled FP32
// component x is split once, in HBM, into x = h + l + r with h = fp16(x) and
// l = fp16(x - h) (round to nearest even; x - h is exact in FP32), so
// |r| <= 2^-22 |x| while h is normal and |r| <= 2^-25 below that (2^-39 of
// the largest component).  A real product keeps h h' + h l' + l h'; the
// dropped l l' is O(2^-22) relative.  The split planes hold (re h, re l,
// im h, im l) as FP16 bit patterns: 8 bytes per complex element, the size of
// the complex64 operand, and the GEMMs load their tiles from memory straight
// into LDS in 16-byte pieces.  MFMA accumulation is FP32 over each workgroup's contraction chunk
// (at most CHUNK_MAX elements); the overlap's split-K chunks are summed in
// FP64 and the scales removed exactly in FP64.  The overlap products are
// written in FP64 (they feed the FP64 subspace solve); the recombination
// (contraction = the state count) writes complex64 states.
//
// Workgroups are mapped to tiles so that the eight XCDs (workgroup i runs on
// XCD i mod 8) each stream their own slice of the data through their own L2.
//
// Sec. 3.3.1 (I and H, lower triangles, Fig. 3) and Sec. 3.3.3 (psi = phi U).
#include "sky_kernels.h"

namespace sky {

namespace {
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int KB = 32;       // contraction elements per MFMA step
constexpr int NP = 4;        // split planes: (part re/im) x (split h/l)
constexpr int NXCD = 8;      // XCDs of the MI355X

// Scale exponent S of a matrix whose largest |component| has the float bit
// pattern mx: max * 2^S lies in [2^13, 2^14).
__device__ inline int scale_exp(unsigned int mx) {
  const float m = __uint_as_float(mx);
  if (!(m > 0.0f) || m > 3.0e38f) return 0;
  int e;
  frexpf(m, &e);
  return 14 - e;
}

__device__ inline unsigned short f16_bits(_Float16 h) { return __builtin_bit_cast(unsigned short, h); }

// x -> (h, l) FP16 bit patterns (x already scaled).
__device__ inline void split2(float x, unsigned short& h, unsigned short& l) {
  const _Float16 a = (_Float16)x;
  const _Float16 b = (_Float16)(x - (float)a);
  h = f16_bits(a);
  l = f16_bits(b);
}

// Plane index: part (0 re, 1 im) * 2 + split (0 h, 1 l).
__device__ inline int plane(int part, int s) { return part * 2 + s; }

// Splits of 8 consecutive elements as four 16-byte vectors (one per plane).
__device__ inline void split8(const float2 (&z)[8], int S, u4 (&w)[NP]) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    unsigned short a[2][2], b[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      split2(ldexpf(z[2 * h + u].x, S), a[u][0], a[u][1]);
      split2(ldexpf(z[2 * h + u].y, S), b[u][0], b[u][1]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      w[plane(0, s)][h] = (unsigned int)a[0][s] | ((unsigned int)a[1][s] << 16);
      w[plane(1, s)][h] = (unsigned int)b[0][s] | ((unsigned int)b[1][s] << 16);
    }
  }
}

// Output tiles of BT x BT per workgroup.  Two wave layouts: 8 waves (4 x 2),
// each owning 32 rows x 64 columns (2 x 4 blocks of 16 x 16, two waves per
// SIMD), or 4 waves (2 x 2), each owning 64 x 64 (4 x 4 blocks, one wave per
// SIMD with the MFMA accumulators in the accumulation registers: two thirds
// of the LDS reads per MFMA).  Both load their tiles from memory straight
// into one of two alternating LDS buffers (buffer_load ... lds), the next
// step's buffer filling while this step's MFMAs read the other.  The MFMA
// accumulates in FP32 with a bias (its accumulator additions do not round
// to nearest: a 13824-long contraction in one accumulator is off by ~1e-5),
// so the MFMA accumulator is folded every FLUSH steps (256 contraction
// elements) into a second FP32 accumulator by ordinary round-to-nearest
// additions, whose errors are unbiased; workgroup chunks (at most CHUNK_MAX
// elements) are summed in FP64 afterwards.
constexpr int BT = 128;
constexpr int FLUSH = 8;
constexpr long CHUNK_MAX = 16384;

template <int NWM, int NWN> struct Lay {
  static constexpr int WAVES = NWM * NWN, THREADS = 64 * WAVES;
  static constexpr int WR = BT / NWM, WC = BT / NWN;   // rows, columns of a wave
  static constexpr int IB = WR / 16, JB = WC / 16;     // 16 x 16 blocks of a wave
};
using Lay8 = Lay<4, 2>;
using Lay4 = Lay<2, 2>;

// LDS tile of the direct loads: [plane][row][KB] fp16 bit patterns, 64-byte
// rows without padding (a direct load writes its 64 lanes' 16-byte pieces
// to consecutive LDS addresses).  The four 16-byte chunks of row r sit at
// slot c ^ swz(r), so that the fragment reads of eight consecutive rows at
// one chunk cover all 32 LDS banks.
struct TileD {
  unsigned short v[NP][BT][KB];
};
__device__ inline int swz(int r) { return (r >> 1) & 3; }

__device__ inline h8 ld8(const TileD& t, int p, int row, int k8) {
  u4 u = *reinterpret_cast<const u4*>(&t.v[p][row][((k8 >> 3) ^ swz(row)) * 8]);
  return __builtin_bit_cast(h8, u);
}

typedef __attribute__((address_space(3))) void lvoid;

// One step's tiles of the 4-wave layout by direct loads: 2 tiles x 4 planes
// x 8 blocks of 16 rows = 64 loads of 1 KB (16 bytes per lane), 16 per wave:
// waves 0-1 load A, waves 2-3 load B, two planes each.  Lane i of a load
// fills row i/4 of its block at slot i%4, i.e. chunk (i%4) ^ swz(row).
// Rows at or past R are clamped to R - 1: they only reach output rows (A)
// or columns (B) at or past R, which are never written.  Addresses are a
// wave-uniform base (matrix, plane, tile row, step) plus the lane's byte
// offset within the tile, fixed for the whole contraction (DmaLane); the
// offsets need BT * ld * 2 <= DMA_RANGE (checked by the launchers).
// Buffer resource of the direct loads: byte range DMA_RANGE from the tile
// base (every lane offset is below BT * ld * 2, which the launchers keep
// under it); BUF_WORD3 is the untyped-access word of gfx9 resources.
constexpr int DMA_RANGE = 0x7fffffff;
constexpr int BUF_WORD3 = 0x00020000;

// A wave-uniform pointer taken from the first lane (held in scalar registers).
__device__ inline const char* uniform_ptr(const char* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(v));
  const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(v >> 32));
  return reinterpret_cast<const char*>((static_cast<unsigned long long>(hi) << 32) | lo);
}

struct DmaLane {
  unsigned int off[BT / 16];
};

// The lane's offsets for the tile rows row0.. of a matrix with R rows and
// row pitch ld (in fp16 elements).
__device__ inline DmaLane dma_lane(int row0, int R, long ld, int lane) {
  DmaLane d;
  const int c = (lane & 3) ^ ((lane >> 3) & 3);   // (lane % 4) ^ swz(row) for every block
#pragma unroll
  for (int rb = 0; rb < BT / 16; ++rb) {
    const int rl = rb * 16 + (lane >> 2);
    const long r = min(row0 + rl, R - 1) - row0;
    d.off[rb] = unsigned((r * ld + c * 8) * 2);
  }
  return d;
}

// wave must be wave-uniform (read from the first lane); dl from dma_lane
// for this wave's matrix (A for the first half of the W waves, B for the
// second); 4 waves load two planes each, 8 waves one.
template <int W>
__device__ inline void dma_tiles(TileD& tA, TileD& tB, const unsigned short* __restrict__ PA,
                                 size_t pszA, long ldA, int rowA,
                                 const unsigned short* __restrict__ PB, size_t pszB, long ldB,
                                 int rowB, long k0, int wave, const DmaLane& dl) {
  constexpr int PPW = NP / (W / 2);   // planes per wave
  const bool isB = wave >= W / 2;
  const unsigned short* P = isB ? PB : PA;
  const size_t psz = isB ? pszB : pszA;
  const long ld = isB ? ldB : ldA;
  const int row0 = isB ? rowB : rowA;
  TileD& t = isB ? tB : tA;
#pragma unroll
  for (int q = 0; q < PPW; ++q) {
    const int p = (wave % (W / 2)) * PPW + q;
    // a buffer resource at the plane's tile base (scalar registers); each
    // load adds the lane's 32-bit offset, so no 64-bit per-lane addresses
    // are kept live across the contraction
    char* base = const_cast<char*>(
        uniform_ptr(reinterpret_cast<const char*>(P + p * psz + size_t(row0) * ld + k0)));
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(base, 0, DMA_RANGE, BUF_WORD3);
#pragma unroll
    for (int rb = 0; rb < BT / 16; ++rb)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lvoid*)&t.v[p][rb * 16][0], 16, dl.off[rb], 0,
                                               0, 0);
  }
}

__device__ inline h8 neg8(h8 x) {
  u4 u = __builtin_bit_cast(u4, x);
  u ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(h8, u);
}

template <int IB, int JB> struct Acc {
  f4 re[IB][JB], im[IB][JB];   // MFMA accumulators
  f4 hr[IB][JB], hi[IB][JB];   // folded sums
};

template <int IB, int JB>
__device__ inline void zero(Acc<IB, JB>& a) {
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      a.re[i][j] = f4{0, 0, 0, 0};
      a.im[i][j] = f4{0, 0, 0, 0};
      a.hr[i][j] = f4{0, 0, 0, 0};
      a.hi[i][j] = f4{0, 0, 0, 0};
    }
}

template <int IB, int JB>
__device__ inline void fold(Acc<IB, JB>& a) {
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j) {
      a.hr[i][j] += a.re[i][j];
      a.hi[i][j] += a.im[i][j];
      a.re[i][j] = f4{0, 0, 0, 0};
      a.im[i][j] = f4{0, 0, 0, 0};
    }
}

#define MF(a, b, c) c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0)

// acc += op(A) B^T over one KB step for the wave's block rows starting at
// row0 (of sA) and block columns starting at col0 (rows of sB); op(A) =
// conj(A) if CONJA.  Three split products per real product.  MFMA operands:
// lane l supplies 8 consecutive contraction elements starting at 8*(l/16) of
// row (or column) l%16.  The A fragments of the wave's row blocks stay in
// registers while its column blocks stream past.  The minus sign of the
// complex product goes on an A fragment at each use (NEGB false: measured
// 4% faster in the 8-wave layout) or once per column block on a B fragment
// (NEGB true: 2 instead of 3 IB negations per block, and no negated copies
// of the A fragments held, which the 64-row waves have no registers for).
template <bool CONJA, bool NEGB, int IB, int JB, typename TT>
__device__ inline void step(Acc<IB, JB>& acc, const TT& sA, const TT& sB, int row0, int col0,
                            int lane) {
  const int r = lane & 15, k8 = (lane >> 4) * 8;
  h8 ar[IB][2], ai[IB][2];
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      ar[i][s] = ld8(sA, plane(0, s), row0 + i * 16 + r, k8);
      ai[i][s] = ld8(sA, plane(1, s), row0 + i * 16 + r, k8);
      if (CONJA && !NEGB) ai[i][s] = neg8(ai[i][s]);
    }
  // split pairs (p, q): hh, hl, lh
  constexpr int P[3] = {0, 0, 1};
  constexpr int Q[3] = {0, 1, 0};
#pragma unroll
  for (int j = 0; j < JB; ++j) {
    h8 br[2], bi[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      br[s] = ld8(sB, plane(0, s), col0 + j * 16 + r, k8);
      bi[s] = ld8(sB, plane(1, s), col0 + j * 16 + r, k8);
    }
    // re += ar br - ai bi ; im += ar bi + ai br   (conj: re += ar br + ai bi ;
    // im += ar bi - ai br).  The row blocks i alternate innermost, so that
    // MFMAs into one accumulator are IB issues apart instead of back to back;
    // each accumulator still sums its products in the order hh, hl, lh with
    // the real part's two terms in a row.
    if constexpr (NEGB) {
      h8 nb[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) nb[s] = neg8(CONJA ? br[s] : bi[s]);
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int p = P[t], q = Q[t];
#pragma unroll
        for (int i = 0; i < IB; ++i) MF(ar[i][p], br[q], acc.re[i][j]);
#pragma unroll
        for (int i = 0; i < IB; ++i) MF(ar[i][p], bi[q], acc.im[i][j]);
#pragma unroll
        for (int i = 0; i < IB; ++i) MF(ai[i][p], CONJA ? bi[q] : nb[q], acc.re[i][j]);
#pragma unroll
        for (int i = 0; i < IB; ++i) MF(ai[i][p], CONJA ? nb[q] : br[q], acc.im[i][j]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int p = P[t], q = Q[t];
#pragma unroll
        for (int i = 0; i < IB; ++i) MF(ar[i][p], br[q], acc.re[i][j]);
#pragma unroll
        for (int i = 0; i < IB; ++i) MF(ar[i][p], bi[q], acc.im[i][j]);
#pragma unroll
        for (int i = 0; i < IB; ++i) MF(neg8(ai[i][p]), bi[q], acc.re[i][j]);
#pragma unroll
        for (int i = 0; i < IB; ++i) MF(ai[i][p], br[q], acc.im[i][j]);
      }
    }
  }
}
#undef MF

// Output element of register e of lane l in a 16x16 block (measured):
// row 4*(l/16) + e, column l%16.
template <int IB, int JB, typename F>
__device__ inline void foreach_out(const Acc<IB, JB>& acc, int row0, int col0, int lane, F f) {
#pragma unroll
  for (int i = 0; i < IB; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = row0 + i * 16 + 4 * (lane >> 4) + e;
        const int col = col0 + j * 16 + (lane & 15);
        f(row, col, acc.hr[i][j][e] + acc.re[i][j][e], acc.hi[i][j][e] + acc.im[i][j][e]);
      }
}

__device__ inline void tri_pair(int p, int& ta, int& tb) {
  int a = int((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= p) ++a;
  while (a * (a + 1) / 2 > p) --a;
  ta = a;
  tb = p - a * (a + 1) / 2;
}

// ------------------------------------------------------------------ scales
__global__ void k_clear_u32(unsigned int* __restrict__ w, int n, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = 0u;
}

// *mx = max(*mx, bits of the largest |component|) over n complex values
// (complex128 inputs are first rounded to complex64, as the split rounds them).
template <bool DOUBLE_IN>
__global__ void __launch_bounds__(256)
k_absmax(const void* __restrict__ xv, size_t n, unsigned int* __restrict__ mx, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  float m = 0.0f;
  for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256) {
    float a, b;
    if (DOUBLE_IN) {
      const double2 d = reinterpret_cast<const double2*>(xv)[i];
      a = float(d.x);
      b = float(d.y);
    } else {
      const float2 f = reinterpret_cast<const float2*>(xv)[i];
      a = f.x;
      b = f.y;
    }
    m = fmaxf(m, fmaxf(fabsf(a), fabsf(b)));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __shared__ float wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
    atomicMax(mx, __float_as_uint(m));
  }
}

// ------------------------------------------------------------------ split planes
// Row pitch of the NT planes: K + NT_PAD elements.  A state's plane row is
// K * 2 bytes long (442 368 at 48^3, a multiple of 2^14); unpadded, the same
// k offset of consecutive rows falls into 1 of 16 L2 sets, so the 128 rows
// of a tile thrash the L2 (measured: 12x the unique bytes fetched).  One
// extra 128-byte line per row spreads them over every set.
constexpr long NT_PAD = 64;

// Planes of an R x K complex64 matrix: P[p][r][k], row pitch K + NT_PAD
// (K % 8 == 0; the pad is never read).
__global__ void __launch_bounds__(256)
k_split_nt(const float2* __restrict__ x, int R, long K, const unsigned int* __restrict__ mx,
           unsigned short* __restrict__ P, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const long nk8 = K / 8;
  const size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= size_t(R) * nk8) return;
  const int S = scale_exp(*mx);
  const int r = int(t / nk8);
  const long k0 = (t % nk8) * 8;
  float2 z[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) z[e] = x[size_t(r) * K + k0 + e];
  u4 w[NP];
  split8(z, S, w);
  const long ld = K + NT_PAD;
  const size_t psz = size_t(R) * ld;
#pragma unroll
  for (int p = 0; p < NP; ++p) *reinterpret_cast<u4*>(P + p * psz + size_t(r) * ld + k0) = w[p];
}

// Transposed planes: input R x C (complex64 or, with DOUBLE_IN, complex128
// rounded to complex64), output P[p][c][r] with row length ldr (rows r >= R
// zero-filled up to ldr).
template <bool DOUBLE_IN>
__global__ void __launch_bounds__(256)
k_split_t(const void* __restrict__ xv, int R, long C, long ldr, const unsigned int* __restrict__ mx,
          unsigned short* __restrict__ P, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ float2 T[64][65];
  const long c0 = long(blockIdx.x) * 64;
  const int r0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  const int S = scale_exp(*mx);
  for (int e = tid; e < 64 * 64; e += 256) {
    const int rr = e / 64, cc = e % 64;
    float2 z = make_float2(0, 0);
    if (r0 + rr < R && c0 + cc < C) {
      if (DOUBLE_IN) {
        double2 d = reinterpret_cast<const double2*>(xv)[size_t(r0 + rr) * C + c0 + cc];
        z = make_float2(float(d.x), float(d.y));
      } else {
        z = reinterpret_cast<const float2*>(xv)[size_t(r0 + rr) * C + c0 + cc];
      }
    }
    T[cc][rr] = z;
  }
  __syncthreads();
  const size_t psz = size_t(C) * ldr;
  for (int g = tid; g < 64 * 8; g += 256) {
    const int cc = g / 8, rg = (g % 8) * 8;
    if (c0 + cc >= C || r0 + rg >= ldr) continue;
    float2 z[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = T[cc][rg + e];
    u4 w[NP];
    split8(z, S, w);
#pragma unroll
    for (int p = 0; p < NP; ++p)
      *reinterpret_cast<u4*>(P + p * psz + size_t(c0 + cc) * ldr + r0 + rg) = w[p];
  }
}

// Both plane layouts of an R x K complex64 matrix from one read of it: the
// row planes P[p][r][k] (pitch K + NT_PAD, rows r < R) and the transposed
// planes PT[p][k][r] (row length ldr, rows r >= R zero-filled), one 64 x 64
// tile per workgroup (grid K/64 x ldr/64).
__global__ void __launch_bounds__(256)
k_split_both(const float2* __restrict__ x, int R, long K, long ldr, const unsigned int* __restrict__ mx,
             unsigned short* __restrict__ P, unsigned short* __restrict__ PT,
             const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  __shared__ float2 T[64][65];
  const long c0 = long(blockIdx.x) * 64;
  const int r0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  const int S = scale_exp(*mx);
  for (int e = tid; e < 64 * 64; e += 256) {
    const int rr = e / 64, cc = e % 64;
    float2 z = make_float2(0, 0);
    if (r0 + rr < R && c0 + cc < K) z = x[size_t(r0 + rr) * K + c0 + cc];
    T[cc][rr] = z;
  }
  __syncthreads();
  const long ld = K + NT_PAD;
  const size_t psz = size_t(R) * ld;
  for (int g = tid; g < 64 * 8; g += 256) {   // row planes: row rr, 8 elements at cg
    const int rr = g / 8, cg = (g % 8) * 8;
    if (r0 + rr >= R || c0 + cg >= K) continue;
    float2 z[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = T[cg + e][rr];
    u4 w[NP];
    split8(z, S, w);
#pragma unroll
    for (int p = 0; p < NP; ++p)
      *reinterpret_cast<u4*>(P + p * psz + size_t(r0 + rr) * ld + c0 + cg) = w[p];
  }
  const size_t pszT = size_t(K) * ldr;
  for (int g = tid; g < 64 * 8; g += 256) {   // transposed planes: column cc, 8 rows at rg
    const int cc = g / 8, rg = (g % 8) * 8;
    if (c0 + cc >= K || r0 + rg >= ldr) continue;
    float2 z[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = T[cc][rg + e];
    u4 w[NP];
    split8(z, S, w);
#pragma unroll
    for (int p = 0; p < NP; ++p)
      *reinterpret_cast<u4*>(PT + p * pszT + size_t(c0 + cc) * ldr + r0 + rg) = w[p];
  }
}

// ------------------------------------------------------------------ products
// Workgroup w -> (chunk s, tile pair, z) of the overlap grid.
__device__ inline void overlap_work(int w, int npair, int split, int nz, int& s, int& pair, int& z) {
  const int T = npair * nz;
  int r;
  if (split % NXCD == 0) {
    const int j = w / NXCD;
    s = w % NXCD + NXCD * (j / T);
    r = j % T;
  } else {
    s = w / T;
    r = w % T;
  }
  pair = r / nz;
  z = r % nz;
}

// part[((z*npair + pair)*split + s)][BT*BT] (FP32, unscaled) = the chunk-s
// sum of conj(A) B^T over the lower tile pair; A, B0, B1 as planes
// [p][m][k].  One-dimensional grid of split*npair*nz workgroups; with
// split % 8 == 0, XCD x computes the chunks s = x mod 8, so that the tiles
// of one chunk are shared through that XCD's L2.  Each step: one barrier
// (which also waits for this wave's direct loads, so that after it the
// step's buffer is complete and every wave is done with the other buffer),
// the next step's loads into the other buffer, then this step's MFMAs.
// Steps run in pairs so that the two buffers are fixed LDS addresses.
template <int NWM, int NWN>
__global__ void __launch_bounds__(64 * NWM * NWN, 1)
k_overlap_planes(const unsigned short* __restrict__ PA, const unsigned short* __restrict__ PB0,
                     const unsigned short* __restrict__ PB1, int m, long k, int npair, int split,
                     int nz, float2* __restrict__ part, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using L = Lay<NWM, NWN>;
  constexpr int W = L::WAVES;
  constexpr bool NEGB = W == 4;
  __shared__ TileD sA0, sB0, sA1, sB1;
  int s, pair, z;
  overlap_work(blockIdx.x, npair, split, nz, s, pair, z);
  const unsigned short* PB = z ? PB1 : PB0;
  int ta, tb;
  tri_pair(pair, ta, tb);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = (wave / 2) * L::WR, col0 = (wave % 2) * L::WC;
  const long nst = k / KB;
  const long c0 = nst * s / split, c1 = nst * (s + 1) / split;
  const long ld = k + NT_PAD;
  const size_t psz = size_t(m) * ld;
  Acc<L::IB, L::JB> acc;
  zero(acc);
  int nacc = 0;
  const DmaLane dl = dma_lane(wave >= W / 2 ? tb * BT : ta * BT, m, ld, lane);
  if (c0 < c1)
    dma_tiles<W>(sA0, sB0, PA, psz, ld, ta * BT, PB, psz, ld, tb * BT, c0 * KB, wave, dl);
  for (long c = c0; c < c1; c += 2) {
    __syncthreads();
    if (c + 1 < c1)
      dma_tiles<W>(sA1, sB1, PA, psz, ld, ta * BT, PB, psz, ld, tb * BT, (c + 1) * KB, wave, dl);
    step<true, NEGB>(acc, sA0, sB0, row0, col0, lane);
    if (++nacc == FLUSH) { fold(acc); nacc = 0; }
    if (c + 1 >= c1) break;
    __syncthreads();
    if (c + 2 < c1)
      dma_tiles<W>(sA0, sB0, PA, psz, ld, ta * BT, PB, psz, ld, tb * BT, (c + 2) * KB, wave, dl);
    step<true, NEGB>(acc, sA1, sB1, row0, col0, lane);
    if (++nacc == FLUSH) { fold(acc); nacc = 0; }
  }
  float2* out = part + (size_t(z) * npair + pair) * split * BT * BT + size_t(s) * BT * BT;
  foreach_out(acc, row0, col0, lane, [&](int row, int col, float re, float im) {
    out[row * BT + col] = make_float2(re, im);
  });
}

// C_z[a][b] = scale 2^-(S_A + S_Bz) sum_s part (FP64) on the lower tiles.
// Grid (npair * RCH, nz): workgroup x handles slice x % RCH of tile pair
// x / RCH (BT*BT / RCH elements).
constexpr int RCH = 16;
__global__ void __launch_bounds__(256)
k_overlap_reduce_planes(const float2* __restrict__ part, int npair, int split, int m, double scale,
                        const unsigned int* __restrict__ mxA, const unsigned int* __restrict__ mxB0,
                        const unsigned int* __restrict__ mxB1, double2* __restrict__ C0,
                        double2* __restrict__ C1, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  const int pair = blockIdx.x / RCH, slice = blockIdx.x % RCH, z = blockIdx.y;
  double2* C = z ? C1 : C0;
  const double sc = ldexp(scale, -(scale_exp(*mxA) + scale_exp(*(z ? mxB1 : mxB0))));
  int ta, tb;
  tri_pair(pair, ta, tb);
  const float2* p = part + (size_t(z) * npair + pair) * split * BT * BT;
  constexpr int per = BT * BT / RCH;
  for (int e = slice * per + threadIdx.x; e < (slice + 1) * per; e += blockDim.x) {
    const int row = ta * BT + e / BT, col = tb * BT + e % BT;
    if (row >= m || col >= m) continue;
    double re = 0.0, im = 0.0;
    for (int q = 0; q < split; ++q) {
      const float2 v = p[size_t(q) * BT * BT + e];
      re += double(v.x);
      im += double(v.y);
    }
    C[size_t(row) * m + col] = make_double2(sc * re, sc * im);
  }
}

// Workgroup w -> (column tile vt, row tile bt) of the recombination grid.
__device__ inline void combine_work(long w, long nv, int nb, long& vt, int& bt) {
  if (nv % NXCD == 0) {
    const long j = w / NXCD;
    vt = w % NXCD + NXCD * (j / nb);
    bt = int(j % nb);
  } else {
    vt = w / nb;
    bt = int(w % nb);
  }
}

// Y[b][v] = sum_a U[a][b] X[a][v] from the planes of U^T (rows b) and of X^T
// (rows v), contraction length mpad (zero-padded), complex64 output.
// One-dimensional grid of nv*nb workgroups (nv = k/BT column tiles, nb row
// tiles); with nv % 8 == 0, XCD x computes the column tiles v = x mod 8, all
// row tiles of one column tile in a row, so that each X^T tile is fetched
// from HBM once.  Steps as in k_overlap_planes.
template <int NWM, int NWN>
__global__ void __launch_bounds__(64 * NWM * NWN, 1)
k_combine_planes(const unsigned short* __restrict__ PU, const unsigned short* __restrict__ PX,
                     const unsigned int* __restrict__ mxU, const unsigned int* __restrict__ mxX,
                     float2* __restrict__ Y, int m, long k, long mpad, int nb, const int* __restrict__ sky_gate) {
  if (sky_gate != nullptr && *sky_gate == 0) return;
  using L = Lay<NWM, NWN>;
  constexpr int W = L::WAVES;
  constexpr bool NEGB = W == 4;
  __shared__ TileD sA0, sB0, sA1, sB1;
  long vt;
  int bt;
  combine_work(blockIdx.x, k / BT, nb, vt, bt);
  const long v0 = vt * BT;
  const int b0 = bt * BT;
  const int SUX = scale_exp(*mxU) + scale_exp(*mxX);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row0 = (wave / 2) * L::WR, col0 = (wave % 2) * L::WC;
  const size_t pszU = size_t(m) * mpad, pszX = size_t(k) * mpad;
  const unsigned short* PXv = PX + size_t(v0) * mpad;
  Acc<L::IB, L::JB> acc;
  zero(acc);
  int nacc = 0;
  const DmaLane dl = wave >= W / 2 ? dma_lane(0, BT, mpad, lane) : dma_lane(b0, m, mpad, lane);
  dma_tiles<W>(sA0, sB0, PU, pszU, mpad, b0, PXv, pszX, mpad, 0, 0, wave, dl);
  for (long a0 = 0; a0 < mpad; a0 += 2 * KB) {
    __syncthreads();
    if (a0 + KB < mpad)
      dma_tiles<W>(sA1, sB1, PU, pszU, mpad, b0, PXv, pszX, mpad, 0, a0 + KB, wave, dl);
    step<false, NEGB>(acc, sA0, sB0, row0, col0, lane);
    if (++nacc == FLUSH) { fold(acc); nacc = 0; }
    if (a0 + KB >= mpad) break;
    __syncthreads();
    if (a0 + 2 * KB < mpad)
      dma_tiles<W>(sA0, sB0, PU, pszU, mpad, b0, PXv, pszX, mpad, 0, a0 + 2 * KB, wave, dl);
    step<false, NEGB>(acc, sA1, sB1, row0, col0, lane);
    if (++nacc == FLUSH) { fold(acc); nacc = 0; }
  }
  foreach_out(acc, row0, col0, lane, [&](int row, int col, float re, float im) {
    const int b = b0 + row;
    if (b < m)
      Y[size_t(b) * k + v0 + col] = make_float2(ldexpf(re, -SUX), ldexpf(im, -SUX));
  });
}

int overlap_split_mixed(int m, long k) {
  if (m <= 0) return 1;
  const int nt = (m + BT - 1) / BT;
  const int npair = nt * (nt + 1) / 2;
  const long nst = k / KB;
  int split = (2048 + 2 * npair - 1) / (2 * npair);
  const long need = (k + CHUNK_MAX - 1) / CHUNK_MAX;   // FP32 chunk length bound
  if (split < need) split = int(need);
  if (split > 64) split = 64;
  if (split > nst) split = int(nst);
  if (split < 1) split = 1;
  // whole XCD rounds: a multiple of 8 chunks where the contraction allows
  if (nst >= NXCD) split = (split + NXCD - 1) / NXCD * NXCD;
  if (split > nst) split = int(nst);
  return split;
}
}  // namespace

// Split-K factors tried by the autotuner: multiples of 8 (whole XCD rounds)
// from the FP32 chunk-length bound up to 64, around the default.
int overlap_split_candidates_mixed(int m, long k, int* out) {
  const long nst = k / KB;
  const int d = overlap_split_mixed(m, k);
  if (nst < NXCD) { out[0] = d; return 1; }
  const long need = (k + CHUNK_MAX - 1) / CHUNK_MAX;
  int n = 0;
  for (int c : {d / 2, d, 2 * d}) {
    c = (c + NXCD - 1) / NXCD * NXCD;
    if (c < need || c > 64 || c > nst) continue;
    if (n == 0 || out[n - 1] != c) out[n++] = c;
  }
  if (n == 0) out[n++] = d;
  return n;
}

size_t overlap_scratch_bytes_mixed(int m, long k) {
  const int nt = (m + BT - 1) / BT;
  const int npair = nt * (nt + 1) / 2;
  int c[3];
  const int nc = overlap_split_candidates_mixed(m, k, c);
  int split = overlap_split_mixed(m, k);
  for (int i = 0; i < nc; ++i) split = split > c[i] ? split : c[i];
  return size_t(split) * 2 * npair * BT * BT * sizeof(float2);
}

long planes_pad(int m) { return (long(m) + KB - 1) / KB * KB; }
size_t planes_bytes_nt(int rows, long k) { return size_t(NP) * rows * (k + NT_PAD) * 2; }
size_t planes_bytes_t(int m, long cols) { return size_t(NP) * cols * planes_pad(m) * 2; }

bool planes_direct_ok(int m, long k) {
  return long(BT) * (k + NT_PAD) * 2 <= DMA_RANGE && long(BT) * planes_pad(m) * 2 <= DMA_RANGE;
}

void plane_scale(const void* x, int x_is_c128, size_t n, unsigned int* mx, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, st, mx, 1, g_launch_gate);
  if (n == 0) return;
  size_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  if (x_is_c128)
    hipLaunchKernelGGL(k_absmax<true>, dim3(unsigned(nb)), dim3(256), 0, st, x, n, mx, g_launch_gate);
  else
    hipLaunchKernelGGL(k_absmax<false>, dim3(unsigned(nb)), dim3(256), 0, st, x, n, mx, g_launch_gate);
}

void clear_scales(unsigned int* mx, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_u32, dim3(1), dim3(64), 0, st, mx, n, g_launch_gate);
}

void split_planes_nt(const void* x, int rows, long k, const unsigned int* mx, void* P,
                     hipStream_t st) {
  if (rows <= 0) return;
  const size_t n = size_t(rows) * (k / 8);
  hipLaunchKernelGGL(k_split_nt, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st,
                     (const float2*)x, rows, k, mx, (unsigned short*)P, g_launch_gate);
}

void split_planes_both(const void* x, int rows, long k, const unsigned int* mx, void* P, void* PT,
                       hipStream_t st) {
  if (rows <= 0) return;
  const long ldr = planes_pad(rows);
  dim3 grid(unsigned((k + 63) / 64), unsigned((ldr + 63) / 64));
  hipLaunchKernelGGL(k_split_both, grid, dim3(256), 0, st, (const float2*)x, rows, k, ldr, mx,
                     (unsigned short*)P, (unsigned short*)PT, g_launch_gate);
}

void split_planes_t(const void* x, int x_is_c128, int rows, long cols, const unsigned int* mx,
                    void* P, hipStream_t st) {
  if (rows <= 0) return;
  const long ldr = planes_pad(rows);
  dim3 grid(unsigned((cols + 63) / 64), unsigned((ldr + 63) / 64));
  if (x_is_c128)
    hipLaunchKernelGGL((k_split_t<true>), grid, dim3(256), 0, st, x, rows, cols, ldr, mx,
                       (unsigned short*)P, g_launch_gate);
  else
    hipLaunchKernelGGL((k_split_t<false>), grid, dim3(256), 0, st, x, rows, cols, ldr, mx,
                       (unsigned short*)P, g_launch_gate);
}

void overlap_lower_planes(const void* PA, const void* PB0, const void* PB1,
                          const unsigned int* mxA, const unsigned int* mxB0,
                          const unsigned int* mxB1, int m, long k, double scale, void* C0,
                          void* C1, void* part, hipStream_t st, hipEvent_t* ev, int split_req,
                          int waves) {
  if (m <= 0) return;
  const int nt = (m + BT - 1) / BT;
  const int npair = nt * (nt + 1) / 2;
  const int split = split_req > 0 ? split_req : overlap_split_mixed(m, k);
  const int nz = PB1 ? 2 : 1;
  if (ev) hipEventRecord(ev[0], st);
  // every descriptor the library accepts (n <= 64) keeps a tile's byte span
  // far below DMA_RANGE (planes_direct_ok)
  if (waves == 4)
    hipLaunchKernelGGL((k_overlap_planes<2, 2>), dim3(unsigned(split * npair * nz)),
                       dim3(Lay4::THREADS), 0, st, (const unsigned short*)PA,
                       (const unsigned short*)PB0, (const unsigned short*)PB1, m, k, npair, split,
                       nz, (float2*)part, g_launch_gate);
  else
    hipLaunchKernelGGL((k_overlap_planes<4, 2>), dim3(unsigned(split * npair * nz)),
                       dim3(Lay8::THREADS), 0, st, (const unsigned short*)PA,
                       (const unsigned short*)PB0, (const unsigned short*)PB1, m, k, npair, split,
                       nz, (float2*)part, g_launch_gate);
  if (ev) hipEventRecord(ev[1], st);
  hipLaunchKernelGGL(k_overlap_reduce_planes, dim3(npair * RCH, nz), dim3(256), 0, st,
                     (const float2*)part, npair, split, m, scale, mxA, mxB0, PB1 ? mxB1 : mxB0,
                     (double2*)C0, (double2*)C1, g_launch_gate);
}

void combine_planes(const void* PU, const void* PX, const unsigned int* mxU,
                    const unsigned int* mxX, void* Y, int m, long k, hipStream_t st, int waves) {
  if (m <= 0) return;
  const int nb = (m + BT - 1) / BT;
  const long nv = k / BT;
  if (waves == 4)
    hipLaunchKernelGGL((k_combine_planes<2, 2>), dim3(unsigned(nv * nb)), dim3(Lay4::THREADS), 0,
                       st, (const unsigned short*)PU, (const unsigned short*)PX, mxU, mxX,
                       (float2*)Y, m, k, planes_pad(m), nb, g_launch_gate);
  else
    hipLaunchKernelGGL((k_combine_planes<4, 2>), dim3(unsigned(nv * nb)), dim3(Lay8::THREADS), 0,
                       st, (const unsigned short*)PU, (const unsigned short*)PX, mxU, mxX,
                       (float2*)Y, m, k, planes_pad(m), nb, g_launch_gate);
}

}  // namespace sky
