// Kernels of the learned Feldkamp filter (training and inference) for gfx950.
//
// The learned filter acts on detector rows: a long learned ramp (one
// channel, K = 2W-1 taps), a per-view weight, and a small 1D CNN (9-tap
// convolutions with 32 channels).  Everything is a batched row convolution
//   out[r][co][j] = bias[co] + sum_{ci,t} w(co,ci,t) in[r][ci][j + t - pad]
// (zero outside the row), its data gradient (the same convolution with the
// transposed, flipped weights), its weight/bias gradient (a reduction over
// rows and positions), plus elementwise helpers and Adam.
//
// conv_short_kernel: K <= 32, any channels.  A block covers 64 positions of
//   one row for all output channels; the input tile (cin x (64 + K - 1)) is
//   in LDS; wave w computes the output channels co = w, w + 4, ... so each
//   weight is wave-uniform (scalar loads) and every LDS value feeds all of a
//   wave's channels from registers.
// conv_long_kernel: cin = cout = 1, long K (the ramp).  A block covers 256
//   positions; FP64 accumulation (the ramp output is a small difference of
//   large terms).
// wgrad kernels: per-block partial sums over a strided set of rows, then a
//   fixed-order reduction over the blocks (deterministic).
#include "learn_internal.h"

#include <algorithm>
#include <cstdint>

namespace fdk {

constexpr int kShortTile = 64;
constexpr int kMaxShortK = 32;
constexpr int kMaxCh = 64;

__device__ __forceinline__ float conv_weight(const LearnConvArgs& a, int co, int ci, int t)
{
    // forward: weight[co][ci][t]; transposed: weight[ci][co][K-1-t] (stored
    // with the roles of cin and cout swapped)
    return a.transpose ? a.weight[((size_t)ci * a.cout + co) * a.K + (a.K - 1 - t)]
                       : a.weight[((size_t)co * a.cin + ci) * a.K + t];
}

__global__ __launch_bounds__(256) void conv_short_kernel(LearnConvArgs a)
{
    extern __shared__ float tile[];  // cin x (kShortTile + K - 1)
    const int row = blockIdx.y;
    const int j0 = blockIdx.x * kShortTile;
    const int span = kShortTile + a.K - 1;
    const float* in = a.in + (size_t)row * a.cin * a.W;
    for (int e = threadIdx.x; e < a.cin * span; e += 256) {
        const int ci = e / span, s = e - ci * span;
        const int j = j0 + s - a.pad;
        tile[e] = (j >= 0 && j < a.W) ? in[(size_t)ci * a.W + j] : 0.0f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j = j0 + lane;
    float* out = a.out + (size_t)row * a.cout * a.W;
    // up to kMaxCh / 4 output channels per wave, in registers
    float acc[kMaxCh / 4];
    const int nco = (a.cout - wave + 3) / 4;  // channels co = wave + 4 q, q < nco
#pragma unroll
    for (int q = 0; q < kMaxCh / 4; ++q)
        acc[q] = (q < nco && a.bias) ? a.bias[wave + 4 * q] : 0.0f;
    for (int ci = 0; ci < a.cin; ++ci) {
        const float* x = tile + ci * span + lane;
        for (int t = 0; t < a.K; ++t) {
            const float xv = x[t];
#pragma unroll
            for (int q = 0; q < kMaxCh / 4; ++q)
                if (q < nco) acc[q] = fmaf(conv_weight(a, wave + 4 * q, ci, t), xv, acc[q]);
        }
    }
    if (j < a.W) {
#pragma unroll
        for (int q = 0; q < kMaxCh / 4; ++q) {
            if (q < nco) {
                const int co = wave + 4 * q;
                float v = acc[q];
                float* o = out + (size_t)co * a.W + j;
                if (a.accumulate) v += *o;
                if (a.relu) v = fmaxf(v, 0.0f);
                if (a.mask) v = *o > 0.0f ? v : 0.0f;
                *o = v;
            }
        }
    }
}

__global__ __launch_bounds__(256) void conv_long_kernel(LearnConvArgs a)
{
    extern __shared__ float tile[];  // 256 + K - 1
    const int row = blockIdx.y;
    const int j0 = blockIdx.x * 256;
    const int span = 256 + a.K - 1;
    const float* in = a.in + (size_t)row * a.W;
    for (int s = threadIdx.x; s < span; s += 256) {
        const int j = j0 + s - a.pad;
        tile[s] = (j >= 0 && j < a.W) ? in[j] : 0.0f;
    }
    __syncthreads();
    const int j = j0 + threadIdx.x;
    if (j >= a.W) return;
    double acc = a.bias ? (double)a.bias[0] : 0.0;
    const float* x = tile + threadIdx.x;
    for (int t = 0; t < a.K; ++t) acc = fma((double)conv_weight(a, 0, 0, t), (double)x[t], acc);
    float* o = a.out + (size_t)row * a.W + j;
    float v = (float)acc;
    if (a.accumulate) v += *o;
    if (a.relu) v = fmaxf(v, 0.0f);
    if (a.mask) v = *o > 0.0f ? v : 0.0f;
    *o = v;
}

// ---------------------------------------------------------------------------
// MFMA path for the wide layers (cin = cout = 32, 9 taps)
// ---------------------------------------------------------------------------
// Both the convolution and its weight gradient are dense contractions:
//   out[co][j]   = sum over (ci, t) of W[co][ci][t] x[ci][j + t - pad]
//                  (M = cout, N = positions, K = cin * taps)
//   dW[co][ci][t] = sum over positions p of dy[co][p] x[ci][p + t - pad]
//                  (M = cout, N = cin * taps, K = positions)
// and run on v_mfma_f32_16x16x4_f32 (FP32 operands and accumulation, so the
// results keep FP32 accuracy).  Operand layout of that instruction: lane l
// holds A[m = l % 16][k = l / 16] and B[k = l / 16][n = l % 16]; the 4
// results of lane l are D[m = 4 (l / 16) + i][n = l % 16], i = 0..3.
typedef float mf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf4 mfma16x16x4(float a, float b, mf4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS pitch >= n that is 16 (mod 32) or 2 (mod 32): the fragment reads of a
// wave then touch distinct banks within each half-wave.
__host__ __device__ constexpr int pitch16(int n) { return ((n + 15) / 32) * 32 + 16; }
__host__ __device__ constexpr int pitch2(int n) { return ((n + 29) / 32) * 32 + 2; }

// A tile of ROWS x SPAN floats, row r taken from src + r * W at columns
// j_first .. j_first + SPAN - 1 (zero outside [0, W) and for rows >= VALID),
// moved into LDS (pitch PITCH) by 256 threads in two steps: fetch() issues
// all of a thread's global loads into registers, put() stores them.  A
// kernel that walks chunks fetches the next chunk before computing on the
// current one, so the loads' latency hides behind that work.
template <int ROWS, int VALID, int SPAN, int PITCH, int NTH = 256>
struct TileCopy {
    static constexpr int kN = (ROWS * SPAN + NTH - 1) / NTH;
    float r[kN];
    __device__ __forceinline__ void fetch(const float* src, int W, int j_first)
    {
#pragma unroll
        for (int k = 0; k < kN; ++k) {
            const int e = threadIdx.x + NTH * k;
            const int row = e / SPAN, sp = e - row * SPAN;
            const int j = j_first + sp;
            r[k] = (e < ROWS * SPAN && row < VALID && j >= 0 && j < W)
                       ? src[(size_t)row * W + j] : 0.0f;
        }
    }
    __device__ __forceinline__ void put(float* dst) const
    {
#pragma unroll
        for (int k = 0; k < kN; ++k) {
            const int e = threadIdx.x + NTH * k;
            const int row = e / SPAN, sp = e - row * SPAN;
            if (e < ROWS * SPAN) dst[row * PITCH + sp] = r[k];
        }
    }
};

// Convolution: a block of 8 waves owns 128 positions of one row at a time
// (wave w: positions 16 w .. 16 w + 15, one 16-wide n-tile) for all output
// channels (two 16-wide m-tiles); the weights, stored as A fragments, stay
// in LDS for the block's lifetime; it walks the chunks of all rows, with
// two input tiles in turn.  (Learned filter at 128^3, 32 -> 32 layer: 4
// waves with two n-tiles each and one tile, 3.55 ms; two tiles, 3.47; 8
// waves, 100 VGPRs, four per SIMD: 3.10-3.20.)
template <int CIN, int COUT, int KT>
struct ConvMfma {
    static constexpr int kWaves = 8;
    static constexpr int kChunk = 16 * kWaves;
    static constexpr int kMT = COUT / 16;
    static constexpr int kC4 = CIN / 4;
    static constexpr int kSteps = kC4 * KT;
    static constexpr int kSpan = kChunk + KT - 1;
    static constexpr int kPitch = pitch16(kSpan);
    static constexpr int kWeights = kMT * kSteps * 64;
    static constexpr size_t lds_bytes() { return (size_t)(kWeights + 2 * CIN * kPitch) * 4; }
    static_assert(CIN % 4 == 0 && COUT % 16 == 0, "channel counts");
};

// OLD: the call reads the output's values (mask or accumulate).
template <int CIN, int COUT, int KT, bool OLD>
__global__ __launch_bounds__((64 * ConvMfma<CIN, COUT, KT>::kWaves)) void conv_mfma_kernel(LearnConvArgs a, int chunks_per_row,
                                                        int total_chunks)
{
    using C = ConvMfma<CIN, COUT, KT>;
    constexpr int NT = 64 * C::kWaves;  // threads
    constexpr int NTW = 1;              // 16-wide n-tiles per wave
    extern __shared__ float lds[];
    float* wl = lds;                 // A fragments: [mt][step][lane]
    float* xs = lds + C::kWeights;   // two input tiles: [buffer][ci][kPitch]
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    for (int e = threadIdx.x; e < C::kWeights; e += NT) {
        const int ll = e & 63, f = e >> 6;
        const int mt = f / C::kSteps, st = f - mt * C::kSteps;
        const int c4 = st / KT, t = st - c4 * KT;
        wl[e] = conv_weight(a, mt * 16 + (ll & 15), 4 * c4 + (ll >> 4), t);
    }
    TileCopy<CIN, CIN, C::kSpan, C::kPitch, NT> tile;
    auto fetch = [&](int c) {
        const int row = c / chunks_per_row;
        const int j0 = (c - row * chunks_per_row) * C::kChunk;
        tile.fetch(a.in + (size_t)row * CIN * a.W, a.W, j0 - a.pad);
    };
    // the biases of the lane's output channels, read once (read per store,
    // the compiler waited for every outstanding load, the next tile's
    // included, at each)
    float bias[C::kMT][4];
#pragma unroll
    for (int mt = 0; mt < C::kMT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) bias[mt][i] = a.bias ? a.bias[mt * 16 + 4 * (l >> 4) + i] : 0.0f;
    // Double-buffered tiles: while the block computes chunk c from one
    // buffer, chunk c + grid (fetched into registers during chunk c - grid)
    // goes into the other, and chunk c + 2 grid is fetched; one barrier per
    // chunk.
    const int G = gridDim.x;  // <= total_chunks (the host's grid)
    fetch(blockIdx.x);
    tile.put(xs);
    fetch(min((int)blockIdx.x + G, total_chunks - 1));
    int buf = 0;
    for (int c = blockIdx.x; c < total_chunks; c += G, buf ^= 1) {
        const int row = c / chunks_per_row;
        const int j0 = (c - row * chunks_per_row) * C::kChunk;
        // values the output holds (mask, accumulate), used by the stores
        // only: read first, so that the stores wait for them and not for the
        // next tile's loads issued after; unguarded, with the column clamped
        // into the row (the stores skip the columns past W).  (Guarded per
        // load, after the tile's loads, the compiler waited for all of them
        // here: masked adjoint at 128^3, 4.2 against 3.3 ms unmasked.)
        float* out = a.out + (size_t)row * COUT * a.W;
        float old[C::kMT][NTW][4];
        if (OLD) {
#pragma unroll
            for (int mt = 0; mt < C::kMT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NTW; ++nt) {
                    const int jc = min(j0 + w * 16 * NTW + nt * 16 + (l & 15), a.W - 1);
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        old[mt][nt][i] = out[(size_t)(mt * 16 + 4 * (l >> 4) + i) * a.W + jc];
                }
        }
        // chunk c's tile is complete, and every wave is done with the other
        // buffer (chunk c - G's fragment reads)
        __syncthreads();
        // (the fetch is unconditional, of a valid chunk at the end: a load
        // under a branch makes the compiler wait for every outstanding load
        // where the branches join)
        if (c + G < total_chunks) tile.put(xs + (buf ^ 1) * CIN * C::kPitch);
        fetch(min(c + 2 * G, total_chunks - 1));
        const float* xb = xs + buf * CIN * C::kPitch + (l >> 4) * C::kPitch + w * 16 * NTW + (l & 15);
        mf4 acc[C::kMT][NTW];
#pragma unroll
        for (int mt = 0; mt < C::kMT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) acc[mt][nt] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c4 = 0; c4 < C::kC4; ++c4) {
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                const int st = c4 * KT + t;
                float bv[NTW];
#pragma unroll
                for (int nt = 0; nt < NTW; ++nt) bv[nt] = xb[c4 * 4 * C::kPitch + t + 16 * nt];
#pragma unroll
                for (int mt = 0; mt < C::kMT; ++mt) {
                    const float av = wl[(mt * C::kSteps + st) * 64 + l];
#pragma unroll
                    for (int nt = 0; nt < NTW; ++nt) acc[mt][nt] = mfma16x16x4(av, bv[nt], acc[mt][nt]);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < C::kMT; ++mt) {
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) {
                const int j = j0 + w * 16 * NTW + nt * 16 + (l & 15);
                if (j >= a.W) continue;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int co = mt * 16 + 4 * (l >> 4) + i;
                    float v = acc[mt][nt][i] + bias[mt][i];
                    if (OLD && a.accumulate) v += old[mt][nt][i];
                    if (a.relu) v = fmaxf(v, 0.0f);
                    if (OLD && a.mask) v = old[mt][nt][i] > 0.0f ? v : 0.0f;
                    out[(size_t)co * a.W + j] = v;
                }
            }
        }
    }
}

// Weight gradient: a block walks chunks of 64 positions (16 k-steps); the
// 32 x 288 result (columns n = t * CIN + ci) is split over the NW waves by
// n-tile (wave w: n-tiles w, w + NW, ...).  The MFMA accumulators are added
// into FP64 sums after every chunk, the bias gradient is summed in FP64,
// and the per-block sums go to the workspace for the fixed-order reduction.
// (32 -> 32 at 128^3: 4 waves at two per SIMD, 3.88 ms; 8 waves fitted to
// four per SIMD, 3.56 ms, bit-identical: each n-tile's sums stay in one
// wave.)
template <int CIN, int COUT, int KT, int NW = 4>
struct WgradMfma {
    static constexpr int kChunk = 64;
    static constexpr int kMT = (COUT + 15) / 16;       // m-tiles (rows past COUT are zero)
    static constexpr int kNN = CIN * KT;               // columns n = t * CIN + ci
    static constexpr int kNT = (kNN + 15) / 16;        // n-tiles (columns past kNN are zero)
    static constexpr int kNTW = (kNT + NW - 1) / NW;   // n-tiles per wave (at most)
    static constexpr int kSpan = kChunk + KT - 1;
    static constexpr int kPitchX = pitch2(kSpan);
    static constexpr int kPitchD = pitch2(kChunk);
    // waves per SIMD the register allocation aims at (fdk128 shapes, ms, in
    // 4-wave blocks: 32->32 6.2 at the default, 4.2 at two waves; 1->32 1.0,
    // 0.84; 32->1 2.7 at the default, 4.8 at two); 8-wave blocks aim at four
    static constexpr int kMinWaves = NW == 8 ? 4 : COUT == 1 ? 1 : 2;
    static constexpr size_t lds_bytes()
    {
        return (size_t)(16 * kMT * kPitchD + CIN * kPitchX) * 4 + 64 * NW * sizeof(double);
    }
};

template <int CIN, int COUT, int KT, int NW = 4>
__global__ __launch_bounds__(64 * NW, (WgradMfma<CIN, COUT, KT, NW>::kMinWaves)) void wgrad_mfma_kernel(LearnGradArgs a, int chunks_per_row,
                                                         int total_chunks)
{
    using G = WgradMfma<CIN, COUT, KT, NW>;
    extern __shared__ float lds[];
    float* dy = lds;                               // [co][kPitchD], 16 kMT rows
    float* xs = lds + 16 * G::kMT * G::kPitchD;    // [ci][kPitchX]
    double* red = (double*)(xs + CIN * G::kPitchX);
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    // per n-tile of this wave: offset of lane l's B fragment in the x tile
    int boff[G::kNTW];
    bool bvalid[G::kNTW];
#pragma unroll
    for (int k = 0; k < G::kNTW; ++k) {
        const int n = (w + NW * k) * 16 + (l & 15);
        bvalid[k] = n < G::kNN;
        const int t = n / CIN, ci = n - t * CIN;
        boff[k] = bvalid[k] ? ci * G::kPitchX + t + (l >> 4) : 0;
    }
    const int aoff = (l & 15) * G::kPitchD + (l >> 4);
    mf4 acc[G::kMT][G::kNTW];
    double sum[G::kMT][G::kNTW][4];
#pragma unroll
    for (int mt = 0; mt < G::kMT; ++mt)
#pragma unroll
        for (int k = 0; k < G::kNTW; ++k) {
            acc[mt][k] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < 4; ++i) sum[mt][k][i] = 0.0;
        }
    double accb = 0.0;  // bias gradient: thread sums co = tid / 8, positions (tid % 8) * 8 ..
    TileCopy<16 * G::kMT, COUT, G::kChunk, G::kPitchD, 64 * NW> dtile;
    TileCopy<CIN, CIN, G::kSpan, G::kPitchX, 64 * NW> xtile;
    auto fetch = [&](int c) {
        const int row = c / chunks_per_row;
        const int j0 = (c - row * chunks_per_row) * G::kChunk;
        dtile.fetch(a.dout + (size_t)row * COUT * a.W, a.W, j0);
        xtile.fetch(a.in + (size_t)row * CIN * a.W, a.W, j0 - a.pad);
    };
    if ((int)blockIdx.x < total_chunks) fetch(blockIdx.x);
    for (int c = blockIdx.x; c < total_chunks; c += gridDim.x) {
        __syncthreads();
        dtile.put(dy);
        xtile.put(xs);
        __syncthreads();
        if (c + (int)gridDim.x < total_chunks) fetch(c + gridDim.x);
#pragma unroll
        for (int st = 0; st < G::kChunk / 4; ++st) {
            float av[G::kMT];
#pragma unroll
            for (int mt = 0; mt < G::kMT; ++mt) av[mt] = dy[aoff + mt * 16 * G::kPitchD + 4 * st];
#pragma unroll
            for (int k = 0; k < G::kNTW; ++k) {
                if (w + NW * k < G::kNT) {
                    const float bv = bvalid[k] ? xs[boff[k] + 4 * st] : 0.0f;
#pragma unroll
                    for (int mt = 0; mt < G::kMT; ++mt) acc[mt][k] = mfma16x16x4(av[mt], bv, acc[mt][k]);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < G::kMT; ++mt)
#pragma unroll
            for (int k = 0; k < G::kNTW; ++k) {
#pragma unroll
                for (int i = 0; i < 4; ++i) sum[mt][k][i] += (double)acc[mt][k][i];
                acc[mt][k] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
            }
        if (threadIdx.x < COUT * 8) {
            const float* d = dy + (threadIdx.x >> 3) * G::kPitchD + (threadIdx.x & 7) * 8;
            double sb = 0.0;
#pragma unroll
            for (int p = 0; p < 8; ++p) sb += (double)d[p];
            accb += sb;
        }
    }
    const int nw = COUT * CIN * KT;
    double* part = a.part + (size_t)blockIdx.x * (nw + COUT);
#pragma unroll
    for (int mt = 0; mt < G::kMT; ++mt)
#pragma unroll
        for (int k = 0; k < G::kNTW; ++k) {
            if (w + NW * k >= G::kNT || !bvalid[k]) continue;
            const int n = (w + NW * k) * 16 + (l & 15);
            const int t = n / CIN, ci = n - t * CIN;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = mt * 16 + 4 * (l >> 4) + i;
                if (co < COUT) part[((size_t)co * CIN + ci) * KT + t] = sum[mt][k][i];
            }
        }
    red[threadIdx.x] = accb;
    __syncthreads();
    if (threadIdx.x < COUT) {
        double sb = 0.0;
        for (int q = 0; q < 8; ++q) sb += red[threadIdx.x * 8 + q];
        part[nw + threadIdx.x] = sb;
    }
}

// Weight gradient of a layer with one output channel: dW[ci][t] = sum_p
// x[ci][p] dy[p - t + pad] (the sum over j of dy[j] x[ci][j + t - pad] with
// p = j + t - pad).  With input channels as the MFMA's rows, the KT taps as
// its (one, zero-padded) column tile and positions as its k dimension, a
// k-step takes CIN / 16 MFMAs, where the general kernel's 16-row tile over
// the single output channel would take (CIN KT) / 16.  A block walks chunks
// of 256 positions (64 per wave), adds the accumulators into FP64 sums after
// each chunk, and combines its waves' sums in LDS for the fixed-order
// reduction.
template <int CIN, int KT>
struct WgradC1 {
    static constexpr int kChunk = 256;
    static constexpr int kMT = CIN / 16;
    static constexpr int kPitchX = kChunk + 4;  // rows 4 banks apart: conflict-free A reads
    static constexpr int kSpanD = kChunk + KT - 1;
    static constexpr int kNW = CIN * KT;
    static constexpr size_t lds_bytes()
    {
        return (size_t)(CIN * kPitchX + kSpanD) * 4 + (size_t)(4 * kNW + 256) * sizeof(double);
    }
    static_assert(CIN % 16 == 0 && KT <= 16, "shape");
    static_assert((CIN * kPitchX + kSpanD) % 2 == 0, "FP64 sums after the tiles stay aligned");
};

template <int CIN, int KT>
__global__ __launch_bounds__(256) void wgrad_c1_kernel(LearnGradArgs a, int chunks_per_row,
                                                       int total_chunks)
{
    using G = WgradC1<CIN, KT>;
    extern __shared__ float lds[];
    float* xt = lds;                          // [ci][kPitchX]
    float* dt = xt + CIN * G::kPitchX;        // kSpanD: position j0 + s - (KT - 1 - pad)
    double* red = (double*)(dt + G::kSpanD);  // [wave][ci * KT + t], then 256 bias sums
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int n = l & 15;  // tap of this lane's B column and D column
    const float* xa = xt + (l & 15) * G::kPitchX + w * 64 + (l >> 4);
    const float* db = dt + w * 64 + (l >> 4) + KT - 1 - n;
    mf4 acc[G::kMT];
    double sum[G::kMT][4];
#pragma unroll
    for (int mt = 0; mt < G::kMT; ++mt) {
        acc[mt] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < 4; ++i) sum[mt][i] = 0.0;
    }
    double accb = 0.0;
    TileCopy<CIN, CIN, G::kChunk, G::kPitchX> xtile;
    TileCopy<1, 1, G::kSpanD, G::kSpanD> dtile;
    auto fetch = [&](int c) {
        const int row = c / chunks_per_row;
        const int j0 = (c - row * chunks_per_row) * G::kChunk;
        xtile.fetch(a.in + (size_t)row * CIN * a.W, a.W, j0);
        dtile.fetch(a.dout + (size_t)row * a.W, a.W, j0 - (KT - 1 - a.pad));
    };
    if ((int)blockIdx.x < total_chunks) fetch(blockIdx.x);
    for (int c = blockIdx.x; c < total_chunks; c += gridDim.x) {
        __syncthreads();
        xtile.put(xt);
        dtile.put(dt);
        __syncthreads();
        if (c + (int)gridDim.x < total_chunks) fetch(c + gridDim.x);
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const float bv = n < KT ? db[4 * st] : 0.0f;
#pragma unroll
            for (int mt = 0; mt < G::kMT; ++mt)
                acc[mt] = mfma16x16x4(xa[mt * 16 * G::kPitchX + 4 * st], bv, acc[mt]);
        }
#pragma unroll
        for (int mt = 0; mt < G::kMT; ++mt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) sum[mt][i] += (double)acc[mt][i];
            acc[mt] = mf4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        accb += (double)dt[threadIdx.x + KT - 1 - a.pad];  // position j0 + threadIdx.x
    }
    // D[m][n] of lane l: rows m = 4 (l >> 4) + i, column n = l & 15
    if (n < KT) {
#pragma unroll
        for (int mt = 0; mt < G::kMT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                red[w * G::kNW + (mt * 16 + 4 * (l >> 4) + i) * KT + n] = sum[mt][i];
    }
    red[4 * G::kNW + threadIdx.x] = accb;
    __syncthreads();
    double* part = a.part + (size_t)blockIdx.x * (G::kNW + 1);
    for (int e = threadIdx.x; e < G::kNW; e += 256)
        part[e] = ((red[e] + red[G::kNW + e]) + red[2 * G::kNW + e]) + red[3 * G::kNW + e];
    if (threadIdx.x == 0) {
        double sb = 0.0;
        for (int q = 0; q < 256; ++q) sb += red[4 * G::kNW + q];
        part[G::kNW] = sb;
    }
}

// the shapes the MFMA path takes
__host__ __device__ constexpr bool mfma_shape(int cin, int cout, int K)
{
    return cin == 32 && cout == 32 && K == 9;
}

// The call's weights w(co, ci, t) into LDS at (co * CIN + ci) * KT + t and
// its biases (0 without) at co, for the block's threads to read at uniform
// addresses.  (Read from global memory per use, each weight's load was
// waited for before its FMAs: the narrow layers were bound by those waits.)
template <int CIN, int COUT, int KT>
__device__ __forceinline__ void stage_weights(const LearnConvArgs& a, float* wl, float* bl)
{
    for (int e = threadIdx.x; e < COUT * CIN * KT; e += blockDim.x) {
        const int co = e / (CIN * KT), r = e - co * CIN * KT;
        const int ci = r / KT, t = r - ci * KT;
        wl[e] = conv_weight(a, co, ci, t);
    }
    for (int e = threadIdx.x; e < COUT; e += blockDim.x) bl[e] = a.bias ? a.bias[e] : 0.0f;
}

// ---------------------------------------------------------------------------
// narrow layers (one channel in or out, 9 taps): memory-bound
// ---------------------------------------------------------------------------
// One thread per output position, 256 positions per block, the input tile
// (CIN x (256 + KT - 1)) in LDS, its global loads all issued before any is
// stored; the weights and biases staged in LDS (stage_weights).
// CIN = 1: the thread forms all COUT outputs from its KT inputs; COUT = 1: it
// sums CIN x KT products.  With a.mask or a.accumulate the COUT values the
// output holds are read up front, not one per output store.
template <int CIN, int COUT, int KT>
__global__ __launch_bounds__(256) void conv_narrow_kernel(LearnConvArgs a)
{
    constexpr int kSpan = 256 + KT - 1;
    __shared__ float tile[CIN * kSpan];
    __shared__ float wl[COUT * CIN * KT];  // w(co, ci, t) at (co * CIN + ci) * KT + t
    __shared__ float bl[COUT];
    const int row = blockIdx.y;
    const int j0 = blockIdx.x * 256;
    {
        TileCopy<CIN, CIN, kSpan, kSpan> tc;
        tc.fetch(a.in + (size_t)row * CIN * a.W, a.W, j0 - a.pad);
        tc.put(tile);
    }
    stage_weights<CIN, COUT, KT>(a, wl, bl);
    const int j = j0 + threadIdx.x;
    float* out = a.out + (size_t)row * COUT * a.W + j;
    float old[COUT];
    if ((a.mask || a.accumulate) && j < a.W) {
#pragma unroll
        for (int co = 0; co < COUT; ++co) old[co] = out[(size_t)co * a.W];
    }
    __syncthreads();
    if (j >= a.W) return;
    const float* x = tile + threadIdx.x;
    if (CIN == 1) {
        float xv[KT];
#pragma unroll
        for (int t = 0; t < KT; ++t) xv[t] = x[t];
#pragma unroll
        for (int co = 0; co < COUT; ++co) {
            float acc = bl[co];
#pragma unroll
            for (int t = 0; t < KT; ++t) acc = fmaf(wl[co * KT + t], xv[t], acc);
            if (a.accumulate) acc += old[co];
            if (a.relu) acc = fmaxf(acc, 0.0f);
            if (a.mask) acc = old[co] > 0.0f ? acc : 0.0f;
            out[(size_t)co * a.W] = acc;
        }
    } else {
        float acc = bl[0];
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
            for (int t = 0; t < KT; ++t) acc = fmaf(wl[ci * KT + t], x[ci * kSpan + t], acc);
        if (a.accumulate) acc += old[0];
        if (a.relu) acc = fmaxf(acc, 0.0f);
        if (a.mask) acc = old[0] > 0.0f ? acc : 0.0f;
        *out = acc;
    }
}

// One input channel with W a multiple of 4: a thread computes 4 consecutive
// positions from its KT + 3 taps (read straight from global memory, shared
// with its neighbours through the L1) and writes each output channel with
// one 16-byte store (4-byte stores measured 0.98 ms against 0.56 ms for the
// 32 channels of 128^3 x 62 views of 624-sample rows).
// OLD: the call reads the output's values (mask or accumulate).
template <int COUT, int KT, bool OLD>
__global__ __launch_bounds__(256) void conv_narrow1x4_kernel(LearnConvArgs a)
{
    __shared__ float wl[COUT * KT];  // w(co, 0, t) at co * KT + t
    __shared__ float bl[COUT];
    stage_weights<1, COUT, KT>(a, wl, bl);
    __syncthreads();
    const int row = blockIdx.y;
    const int j = (blockIdx.x * 256 + threadIdx.x) * 4;
    if (j >= a.W) return;
    const float* in = a.in + (size_t)row * a.W;
    float* out = a.out + (size_t)row * COUT * a.W + j;
    float xv[KT + 3];
#pragma unroll
    for (int t = 0; t < KT + 3; ++t) {
        const int p = j + t - a.pad;
        xv[t] = (p >= 0 && p < a.W) ? in[p] : 0.0f;
    }
    // the values the outputs hold (OLD: mask or accumulate), channel co + 1's
    // read while channel co is computed
    float4 next = OLD ? *(const float4*)out : float4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int co = 0; co < COUT; ++co) {
        const float4 old = next;
        if (OLD) next = *(const float4*)(out + (size_t)min(co + 1, COUT - 1) * a.W);
        const float b = bl[co];
        float acc[4] = {b, b, b, b};
#pragma unroll
        for (int t = 0; t < KT; ++t) {
            const float w = wl[co * KT + t];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = fmaf(w, xv[q + t], acc[q]);
        }
        const float ov[4] = {old.x, old.y, old.z, old.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (OLD && a.accumulate) acc[q] += ov[q];
            if (a.relu) acc[q] = fmaxf(acc[q], 0.0f);
            if (OLD && a.mask) acc[q] = ov[q] > 0.0f ? acc[q] : 0.0f;
        }
        *(float4*)(out + (size_t)co * a.W) = float4{acc[0], acc[1], acc[2], acc[3]};
    }
}

hipError_t launch_conv(const LearnConvArgs& a, hipStream_t s)
{
    if (a.K == 9 && ((a.cin == 1 && a.cout == 32) || (a.cin == 32 && a.cout == 1))) {
        // 16-byte stores need W a multiple of 4 and a 16-byte aligned output
        dim3 grid((a.W + 255) / 256, a.rows);
        if (a.cin == 1 && (a.W & 3) == 0 && ((uintptr_t)a.out & 15) == 0)
        {
            if (a.mask || a.accumulate)
                hipLaunchKernelGGL((conv_narrow1x4_kernel<32, 9, true>),
                                   dim3((a.W + 1023) / 1024, a.rows), dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((conv_narrow1x4_kernel<32, 9, false>),
                                   dim3((a.W + 1023) / 1024, a.rows), dim3(256), 0, s, a);
        }
        else if (a.cin == 1)
            hipLaunchKernelGGL((conv_narrow_kernel<1, 32, 9>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((conv_narrow_kernel<32, 1, 9>), grid, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (mfma_shape(a.cin, a.cout, a.K)) {
        using C = ConvMfma<32, 32, 9>;
        const int cpr = (a.W + C::kChunk - 1) / C::kChunk;
        const int total = a.rows * cpr;
        const int grid = total < 1024 ? total : 1024;
        if (a.mask || a.accumulate)
            hipLaunchKernelGGL((conv_mfma_kernel<32, 32, 9, true>), dim3(grid), dim3(64 * C::kWaves),
                               C::lds_bytes(), s, a, cpr, total);
        else
            hipLaunchKernelGGL((conv_mfma_kernel<32, 32, 9, false>), dim3(grid),
                               dim3(64 * C::kWaves), C::lds_bytes(), s, a, cpr, total);
    } else if (a.K <= kMaxShortK) {
        dim3 grid((a.W + kShortTile - 1) / kShortTile, a.rows);
        const size_t lds = (size_t)a.cin * (kShortTile + a.K - 1) * sizeof(float);
        hipLaunchKernelGGL(conv_short_kernel, grid, dim3(256), lds, s, a);
    } else {
        dim3 grid((a.W + 255) / 256, a.rows);
        const size_t lds = (size_t)(256 + a.K - 1) * sizeof(float);
        hipLaunchKernelGGL(conv_long_kernel, grid, dim3(256), lds, s, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// weight and bias gradients
// ---------------------------------------------------------------------------
// sum_p d[p] x[p] in FP64 with eight independent partial sums (the chains
// of dependent FMAs would otherwise bound the loop by their latency)
__device__ __forceinline__ double dot_f64(const float* d, const float* x, int n)
{
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int p = 0;
    for (; p + 8 <= n; p += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] = fma((double)d[p + u], (double)x[p + u], s[u]);
    }
    for (; p < n; ++p) s[0] = fma((double)d[p], (double)x[p], s[0]);
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Block b sums over rows b, b + B, b + 2B, ... into
//   part[b][(co*cin + ci)*K + t]  and  part_bias[b][co]
// in FP64; thread e owns entries e, e + 256, ...  For each row the block
// stages dout (cout x W) and in (cin x (W + K - 1), zero-padded) in LDS,
// in chunks of kGradChunk positions.
constexpr int kGradChunk = 128;

__global__ __launch_bounds__(256) void wgrad_partial_kernel(LearnGradArgs a)
{
    extern __shared__ float lds[];
    const int nw = a.cout * a.cin * a.K;
    const int span = kGradChunk + a.K - 1;
    float* dy = lds;                          // cout x kGradChunk
    float* x = lds + a.cout * kGradChunk;     // cin x span
    constexpr int kPer = 40;                  // entries per thread (<= 10240 total)
    double acc[kPer];
    double accb = 0.0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) acc[q] = 0.0;
    for (int row = blockIdx.x; row < a.rows; row += gridDim.x) {
        const float* drow = a.dout + (size_t)row * a.cout * a.W;
        const float* xrow = a.in + (size_t)row * a.cin * a.W;
        for (int j0 = 0; j0 < a.W; j0 += kGradChunk) {
            __syncthreads();
            for (int e = threadIdx.x; e < a.cout * kGradChunk; e += 256) {
                const int co = e / kGradChunk, s = e - co * kGradChunk;
                const int j = j0 + s;
                dy[e] = (j < a.W) ? drow[(size_t)co * a.W + j] : 0.0f;
            }
            for (int e = threadIdx.x; e < a.cin * span; e += 256) {
                const int ci = e / span, s = e - ci * span;
                const int j = j0 + s - a.pad;
                x[e] = (j >= 0 && j < a.W) ? xrow[(size_t)ci * a.W + j] : 0.0f;
            }
            __syncthreads();
            const int n = min(kGradChunk, a.W - j0);
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const int e = threadIdx.x + 256 * q;
                if (e < nw) {
                    const int t = e % a.K;
                    const int ci = (e / a.K) % a.cin;
                    const int co = e / (a.K * a.cin);
                    acc[q] += dot_f64(dy + co * kGradChunk, x + ci * span + t, n);
                }
            }
            if ((int)threadIdx.x < a.cout) {
                const float* d = dy + threadIdx.x * kGradChunk;
                double s = 0.0;
                for (int p = 0; p < n; ++p) s += (double)d[p];
                accb += s;
            }
        }
    }
    double* part = a.part + (size_t)blockIdx.x * (nw + a.cout);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e < nw) part[e] = acc[q];
    }
    if ((int)threadIdx.x < a.cout) part[nw + threadIdx.x] = accb;
}

__global__ __launch_bounds__(256) void wgrad_reduce_kernel(LearnGradArgs a, int nblocks)
{
    const int nw = a.cout * a.cin * a.K;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nw + a.cout) return;
    // eight interleaved partial sums (loads in flight), added in a fixed order
    const size_t stride = (size_t)nw + a.cout;
    double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = 0;
    for (; b + 8 <= nblocks; b += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) p[k] += a.part[(size_t)(b + k) * stride + e];
    }
    for (; b < nblocks; ++b) p[0] += a.part[(size_t)b * stride + e];
    const double s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    if (e < nw)
        a.dweight[e] = (float)s;
    else if (a.dbias)
        a.dbias[e - nw] = (float)s;
}

hipError_t launch_wgrad(const LearnGradArgs& a, int nblocks, hipStream_t s)
{
    const int cpr = (a.W + 63) / 64;  // 64-position chunks
    if (mfma_shape(a.cin, a.cout, a.K)) {
        hipLaunchKernelGGL((wgrad_mfma_kernel<32, 32, 9, 8>), dim3(nblocks), dim3(512),
                           (WgradMfma<32, 32, 9, 8>::lds_bytes()), s, a, cpr, a.rows * cpr);
    } else if (a.K == 9 && a.cin == 1 && a.cout == 32) {
        hipLaunchKernelGGL((wgrad_mfma_kernel<1, 32, 9>), dim3(nblocks), dim3(256),
                           (WgradMfma<1, 32, 9>::lds_bytes()), s, a, cpr, a.rows * cpr);
    } else if (a.K == 9 && a.cin == 32 && a.cout == 1 && a.pad <= 8) {
        // (its bias sum reads dy tile entries 8 - pad .. 263 - pad)
        const int cpr1 = (a.W + WgradC1<32, 9>::kChunk - 1) / WgradC1<32, 9>::kChunk;
        hipLaunchKernelGGL((wgrad_c1_kernel<32, 9>), dim3(nblocks), dim3(256),
                           (WgradC1<32, 9>::lds_bytes()), s, a, cpr1, a.rows * cpr1);
    } else if (a.K == 9 && a.cin == 32 && a.cout == 1) {
        hipLaunchKernelGGL((wgrad_mfma_kernel<32, 1, 9>), dim3(nblocks), dim3(256),
                           (WgradMfma<32, 1, 9>::lds_bytes()), s, a, cpr, a.rows * cpr);
    } else {
        const size_t lds =
            (size_t)(a.cout * kGradChunk + a.cin * (kGradChunk + a.K - 1)) * sizeof(float);
        hipLaunchKernelGGL(wgrad_partial_kernel, dim3(nblocks), dim3(256), lds, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = a.cout * a.cin * a.K + a.cout;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, nblocks);
    return hipGetLastError();
}

// Long-kernel (cin = cout = 1) weight gradient: dweight[t] = sum_r sum_j
// dout[r][j] in[r][j + t - pad].  Block b handles rows b, b + B, ...; each
// thread owns taps t = threadIdx.x + 256 q.
constexpr int kLongPer = 32;  // K <= 8192

__global__ __launch_bounds__(256) void wgrad_long_partial_kernel(LearnGradArgs a)
{
    extern __shared__ float lds[];
    float* dy = lds;          // W
    float* x = lds + a.W;     // W + K - 1
    double acc[kLongPer];
    double accb = 0.0;
#pragma unroll
    for (int q = 0; q < kLongPer; ++q) acc[q] = 0.0;
    const int span = a.W + a.K - 1;
    for (int row = blockIdx.x; row < a.rows; row += gridDim.x) {
        __syncthreads();
        for (int s = threadIdx.x; s < a.W; s += 256) dy[s] = a.dout[(size_t)row * a.W + s];
        for (int s = threadIdx.x; s < span; s += 256) {
            const int j = s - a.pad;
            x[s] = (j >= 0 && j < a.W) ? a.in[(size_t)row * a.W + j] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kLongPer; ++q) {
            const int t = threadIdx.x + 256 * q;
            if (t < a.K) acc[q] += dot_f64(dy, x + t, a.W);
        }
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int p = 0; p < a.W; ++p) s += (double)dy[p];
            accb += s;
        }
    }
    double* part = a.part + (size_t)blockIdx.x * (a.K + 1);
#pragma unroll
    for (int q = 0; q < kLongPer; ++q) {
        const int t = threadIdx.x + 256 * q;
        if (t < a.K) part[t] = acc[q];
    }
    if (threadIdx.x == 0) part[a.K] = accb;
}

hipError_t launch_wgrad_long(const LearnGradArgs& a, int nblocks, hipStream_t s)
{
    const size_t lds = (size_t)(2 * a.W + a.K - 1) * sizeof(float);
    hipLaunchKernelGGL(wgrad_long_partial_kernel, dim3(nblocks), dim3(256), lds, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = a.K + 1;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, s, a, nblocks);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise helpers
// ---------------------------------------------------------------------------
// y[g][i] = x[g][i] * scale[g] (+ y if accumulate)
__global__ __launch_bounds__(256) void scale_groups_kernel(float* y, const float* x,
                                                           const float* scale, size_t len,
                                                           int groups, int accumulate)
{
    const size_t n = len * groups;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        float v = x[i] * scale[i / len];
        if (accumulate) v += y[i];
        y[i] = v;
    }
}

// out[g] = sum_i a[g][i] * b[g][i] (FP64, one block per group)
// out[g] = sum_i a[g][i] b[g][i] in FP64: one 1024-thread block per group,
// eight partial sums per thread (loads in flight), then a fixed-order tree.
__global__ __launch_bounds__(1024) void group_dot_kernel(float* out, const float* a,
                                                         const float* b, size_t len)
{
    __shared__ double red[1024];
    const size_t base = (size_t)blockIdx.x * len;
    const float* pa = a + base;
    const float* pb = b + base;
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    size_t i = threadIdx.x;
    for (; i + 7 * 1024 < len; i += 8 * 1024) {
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += (double)pa[i + 1024 * k] * (double)pb[i + 1024 * k];
    }
    for (; i < len; i += 1024) s[0] += (double)pa[i] * (double)pb[i];
    red[threadIdx.x] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = (float)red[0];
}

// dx = dy where y > 0, else 0 (ReLU backward, y the ReLU output)
__global__ __launch_bounds__(256) void relu_backward_kernel(float* dx, const float* dy,
                                                            const float* y, size_t n)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        dx[i] = y[i] > 0.0f ? dy[i] : 0.0f;
}

// y = A x (A rows x cols, row-major) or y = A^T x; FP64 accumulation in a
// fixed order.  A x: one wave per output row, lane l taking the columns
// l + 64 k into four partial sums, the lanes then added by a butterfly (lane
// 0's result is stored).  A^T x: a block per 64 outputs (one per lane), its
// four waves taking the rows w + 4 k, added in wave order through LDS.
__global__ __launch_bounds__(256) void matvec_kernel(float* y, const float* A, const float* x,
                                                     int rows, int cols, int transpose)
{
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (!transpose) {
        const int i = blockIdx.x * 4 + w;
        if (i >= rows) return;
        const float* Ai = A + (size_t)i * cols;
        int c = l;
        for (; c + 192 < cols; c += 256) {
            s0 = fma((double)Ai[c], (double)x[c], s0);
            s1 = fma((double)Ai[c + 64], (double)x[c + 64], s1);
            s2 = fma((double)Ai[c + 128], (double)x[c + 128], s2);
            s3 = fma((double)Ai[c + 192], (double)x[c + 192], s3);
        }
        for (; c < cols; c += 64) s0 = fma((double)Ai[c], (double)x[c], s0);
        double t = (s0 + s1) + (s2 + s3);
        for (int m = 32; m > 0; m >>= 1) t += __shfl_xor(t, m);
        if (l == 0) y[i] = (float)t;
        return;
    }
    __shared__ double red[4][64];
    const int i = blockIdx.x * 64 + l;
    if (i < cols) {
        int r = w;
        for (; r + 12 < rows; r += 16) {
            s0 = fma((double)A[(size_t)r * cols + i], (double)x[r], s0);
            s1 = fma((double)A[(size_t)(r + 4) * cols + i], (double)x[r + 4], s1);
            s2 = fma((double)A[(size_t)(r + 8) * cols + i], (double)x[r + 8], s2);
            s3 = fma((double)A[(size_t)(r + 12) * cols + i], (double)x[r + 12], s3);
        }
        for (; r < rows; r += 4) s0 = fma((double)A[(size_t)r * cols + i], (double)x[r], s0);
    }
    red[w][l] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (w == 0 && i < cols) y[i] = (float)(((red[0][l] + red[1][l]) + red[2][l]) + red[3][l]);
}

// Adam (Kingma and Ba, 2015) with bias correction, step t >= 1
__global__ __launch_bounds__(256) void adam_kernel(float* p, float* m, float* v, const float* g,
                                                   int n, float lr, float b1, float b2, float eps,
                                                   float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// grad = 2 (a - b) / n, loss_part[block] = sum (a - b)^2 over the block's share
__global__ __launch_bounds__(256) void mse_kernel(float* grad, double* part, const float* a,
                                                  const float* b, size_t n)
{
    __shared__ double red[256];
    const size_t stride = (size_t)gridDim.x * 256;
    double s = 0.0;
    const float inv = 2.0f / (float)n;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const float d = a[i] - b[i];
        if (grad) grad[i] = d * inv;
        s += (double)d * (double)d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_parts_kernel(float* out, const double* part, int n, double scale)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    out[0] = (float)(s * scale);
}

static unsigned blocks_for(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > 256 * 64) b = 256 * 64;
    return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_scale_groups(float* y, const float* x, const float* scale, size_t len,
                               int groups, int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(scale_groups_kernel, dim3(blocks_for(len * groups)), dim3(256), 0, s, y, x,
                       scale, len, groups, accumulate);
    return hipGetLastError();
}

hipError_t launch_group_dot(float* out, const float* a, const float* b, size_t len, int groups,
                            hipStream_t s)
{
    hipLaunchKernelGGL(group_dot_kernel, dim3(groups), dim3(1024), 0, s, out, a, b, len);
    return hipGetLastError();
}

hipError_t launch_relu_backward(float* dx, const float* dy, const float* y, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(relu_backward_kernel, dim3(blocks_for(n)), dim3(256), 0, s, dx, dy, y, n);
    return hipGetLastError();
}

hipError_t launch_matvec(float* y, const float* A, const float* x, int rows, int cols,
                         int transpose, hipStream_t s)
{
    const int blocks = transpose ? (cols + 63) / 64 : (rows + 3) / 4;
    hipLaunchKernelGGL(matvec_kernel, dim3(blocks), dim3(256), 0, s, y, A, x, rows, cols,
                       transpose);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int n, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step);
    const float c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, m, v, g, n, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mse(float* grad, float* loss, double* part, int nparts, const float* a,
                      const float* b, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(mse_kernel, dim3(nparts), dim3(256), 0, s, grad, part, a, b, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, s, loss, part, nparts,
                       1.0 / (double)n);
    return hipGetLastError();
}

}  // namespace fdk
