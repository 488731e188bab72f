// Low-precision pieces of the inner operator for the mixed-precision mode.
//
// The W-sandwich products E Y E of the augmented operator (Section 5) run on
// the gfx950 matrix cores in FP32 (v_mfma_f32_16x16x4_f32) or BF16
// (v_mfma_f32_16x16x32_bf16), both accumulating in FP32; the dense constraint
// passes read an FP32 copy of the packed rows and accumulate in FP64.  The
// outer refinement that restores FP64 accuracy lives in the solver.
//
// MFMA 16x16 lane layout (both instructions, verified on gfx950): lane l
// supplies row l % 16 of A and column l % 16 of B at k-group l / 16; output
// element v of lane l is D[4 (l / 16) + v][l % 16].
#include "lowprec.hpp"

namespace wc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));
typedef double ld2 __attribute__((ext_vector_type(2)));
typedef float lf4 __attribute__((ext_vector_type(4)));
typedef float lf2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<unsigned short>((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<unsigned short>(u >> 16);
}

template <int BS>
__device__ __forceinline__ double lp_block_sum(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) s += sh[i];
    return s;
}

// ---- GEMM epilogue -----------------------------------------------------------------
template <LpOut OUT>
__device__ __forceinline__ void lp_store(void* C, long ldc, int M, int N, int r0, int c0, const v4f& acc) {
    const int lane = threadIdx.x & 63;
    const int col = c0 + (lane & 15);
    if (col >= N) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = r0 + 4 * (lane >> 4) + v;
        if (row >= M) continue;
        const long o = row + (long)col * ldc;
        if constexpr (OUT == LpOut::F32) static_cast<float*>(C)[o] = acc[v];
        else if constexpr (OUT == LpOut::BF16) static_cast<unsigned short*>(C)[o] = bf16_rne(acc[v]);
        else if constexpr (OUT == LpOut::F64) static_cast<double*>(C)[o] = static_cast<double>(acc[v]);
        else static_cast<double*>(C)[o] += static_cast<double>(acc[v]);
    }
}

// 64 x 64 output tile per workgroup, four waves in a 2 x 2 grid, each wave a
// 2 x 2 block of 16 x 16 MFMA tiles; K staged through LDS 32 at a time.
constexpr int LT = 64;
constexpr int LK = 32;

template <LpOut OUT>
__global__ __launch_bounds__(256) void sgemm_nn_kernel(int M, int N, int K, const float* __restrict__ A, long lda,
                                                       const float* __restrict__ B, long ldb, void* __restrict__ C,
                                                       long ldc) {
    __shared__ float As[LT][LK + 1];  // [row][k]
    __shared__ float Bs[LT][LK + 1];  // [col][k]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    const int row0 = blockIdx.x * LT, col0 = blockIdx.y * LT;
    v4f acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
    // the next K slice is fetched into registers while the current one is multiplied
    float ra[8], rb[8];
    const int ai = tid & 63, bk = tid & 31;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int kk = (tid >> 6) + 4 * t, gk = k0 + kk, gi = row0 + ai;
            ra[t] = (gi < M && gk < K) ? A[gi + (long)gk * lda] : 0.f;
            const int j = (tid >> 5) + 8 * t, gj = col0 + j, gkb = k0 + bk;
            rb[t] = (gkb < K && gj < N) ? B[gkb + (long)gj * ldb] : 0.f;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += LK) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            As[ai][(tid >> 6) + 4 * t] = ra[t];
            Bs[(tid >> 5) + 8 * t][bk] = rb[t];
        }
        __syncthreads();
        if (k0 + LK < K) fetch(k0 + LK);
#pragma unroll
        for (int s = 0; s < LK / 4; ++s) {
            const int kk = 4 * s + (lane >> 4);
            float a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) a[x] = As[wm * 32 + x * 16 + (lane & 15)][kk];
#pragma unroll
            for (int y = 0; y < 2; ++y) b[y] = Bs[wn * 32 + y * 16 + (lane & 15)][kk];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            lp_store<OUT>(C, ldc, M, N, row0 + wm * 32 + x * 16, col0 + wn * 32 + y * 16, acc[x][y]);
}

template <LpOut OUT>
__global__ __launch_bounds__(256) void bgemm_nn_kernel(int M, int N, int K, const unsigned short* __restrict__ A,
                                                       long lda, const unsigned short* __restrict__ B, long ldb,
                                                       void* __restrict__ C, long ldc) {
    // rows padded to 40 halves (80 bytes) so each lane's 8-element k-group is a 16-byte aligned read
    __shared__ __attribute__((aligned(16))) unsigned short As[LT][LK + 8];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[LT][LK + 8];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    const int row0 = blockIdx.x * LT, col0 = blockIdx.y * LT;
    v4f acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
    unsigned short ra[8], rb[8];
    const int ai = tid & 63, bk = tid & 31;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int kk = (tid >> 6) + 4 * t, gk = k0 + kk, gi = row0 + ai;
            ra[t] = (gi < M && gk < K) ? A[gi + (long)gk * lda] : static_cast<unsigned short>(0);
            const int j = (tid >> 5) + 8 * t, gj = col0 + j, gkb = k0 + bk;
            rb[t] = (gkb < K && gj < N) ? B[gkb + (long)gj * ldb] : static_cast<unsigned short>(0);
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += LK) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            As[ai][(tid >> 6) + 4 * t] = ra[t];
            Bs[(tid >> 5) + 8 * t][bk] = rb[t];
        }
        __syncthreads();
        if (k0 + LK < K) fetch(k0 + LK);
        const int kg = 8 * (lane >> 4);
        v8us a[2], b[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) a[x] = *reinterpret_cast<const v8us*>(&As[wm * 32 + x * 16 + (lane & 15)][kg]);
#pragma unroll
        for (int y = 0; y < 2; ++y) b[y] = *reinterpret_cast<const v8us*>(&Bs[wn * 32 + y * 16 + (lane & 15)][kg]);
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a[x]),
                                                                    __builtin_bit_cast(v8bf, b[y]), acc[x][y], 0, 0,
                                                                    0);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
            lp_store<OUT>(C, ldc, M, N, row0 + wm * 32 + x * 16, col0 + wn * 32 + y * 16, acc[x][y]);
}

// ---- BF16 product with a symmetric left operand ------------------------------------
// C = A B with A symmetric (M x M) and B (M x N), both column-major BF16.
// Because A is symmetric, A(i, k) = A[k + i lda]: row i of A is contiguous in k
// like column j of B, so both MFMA operands arrive as 16-byte (8 x BF16)
// k-contiguous loads and are stored to LDS as they are, without the
// transposition a general A needs.  128 x 128 output tile per workgroup, four
// waves in a 2 x 2 grid with 4 x 4 MFMA tiles (16 x 16 x 32) each; K advances
// 32 at a time through double-buffered LDS with one barrier per step, the next
// step's loads held in registers while the current one multiplies.  Requires
// lda and ldb multiples of 8 and 16-byte aligned A and B.
constexpr int ST = 128;  // output tile
constexpr int SK = 32;   // k per step (one MFMA k-extent)
constexpr int SP = SK + 8;  // LDS row pitch in halves (80 bytes: 16-byte aligned, spreads banks)

__device__ __forceinline__ v8us load8_guarded(const unsigned short* __restrict__ p, int k, int K) {
    if (k + 8 <= K) return *reinterpret_cast<const v8us*>(p);
    v8us v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (k + e < K) ? p[e] : static_cast<unsigned short>(0);
    return v;
}

template <LpOut OUT>
__global__ __launch_bounds__(256) void bgemm_sym_kernel(int M, int N, const unsigned short* __restrict__ A, long lda,
                                                        const unsigned short* __restrict__ B, long ldb,
                                                        void* __restrict__ C, long ldc) {
    __shared__ __attribute__((aligned(16))) unsigned short As[2][ST][SP];  // [buffer][row][k]
    __shared__ __attribute__((aligned(16))) unsigned short Bs[2][ST][SP];  // [buffer][col][k]
    const int K = M;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    const int row0 = blockIdx.x * ST, col0 = blockIdx.y * ST;
    // loader: vector q = tid + 256 h covers row (or column) q / 4 and k offset 8 (q % 4)
    v8us ra[2], rb[2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = tid + 256 * h, r = q >> 2, k = k0 + 8 * (q & 3);
            const int gi = row0 + r, gj = col0 + r;
            ra[h] = gi < M ? load8_guarded(A + k + (long)gi * lda, k, K) : v8us{0, 0, 0, 0, 0, 0, 0, 0};
            rb[h] = gj < N ? load8_guarded(B + k + (long)gj * ldb, k, K) : v8us{0, 0, 0, 0, 0, 0, 0, 0};
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = tid + 256 * h, r = q >> 2, k = 8 * (q & 3);
            *reinterpret_cast<v8us*>(&As[buf][r][k]) = ra[h];
            *reinterpret_cast<v8us*>(&Bs[buf][r][k]) = rb[h];
        }
    };
    v4f acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
    fetch(0);
    stash(0);
    __syncthreads();
    const int kg = 8 * (lane >> 4);
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += SK) {
        const bool more = k0 + SK < K;
        if (more) fetch(k0 + SK);
        v8us a[4], b[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) a[x] = *reinterpret_cast<const v8us*>(&As[buf][wm * 64 + x * 16 + (lane & 15)][kg]);
#pragma unroll
        for (int y = 0; y < 4; ++y) b[y] = *reinterpret_cast<const v8us*>(&Bs[buf][wn * 64 + y * 16 + (lane & 15)][kg]);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a[x]),
                                                                    __builtin_bit_cast(v8bf, b[y]), acc[x][y], 0, 0,
                                                                    0);
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
            lp_store<OUT>(C, ldc, M, N, row0 + wm * 64 + x * 16, col0 + wn * 64 + y * 16, acc[x][y]);
}

// The same BF16 product for large n: 256 x 256 output tile per workgroup,
// four waves in a 2 x 2 grid, each wave a 128 x 128 block of 8 x 8 MFMA tiles
// (16 x 16 x 32) whose accumulators take 256 registers per lane -- twice the
// flops per LDS byte of the 128 x 128 kernel.  With one wave per SIMD there
// is nothing to hide load latency behind, so the operands go from global
// memory straight into LDS (global_load_lds, 16 bytes per lane, no register
// staging) through a ring of BS = 4 stages: the loads of step k + 3 are in
// flight while step k multiplies, and each step ends with a wait for step
// k + 1's own loads (vmcnt) and a barrier for everyone else's.  A stage holds
// the step's 32 k-values of the 256 A rows and 256 B columns, 64 bytes per
// row, with the four 16-byte pieces of row r stored at position
// piece ^ ((r >> 1) & 3): the fragment reads (16 rows x 4 pieces per
// instruction) are then free of bank conflicts.  Rows past the matrix edge
// load a valid row (their outputs are not stored); a ragged K tail is
// multiplied after the loop from fragments loaded straight from global
// memory, zero past K.  Consecutive workgroups land on different XCDs (round
// robin), so the launch index is remapped to give each XCD a compact block of
// output tiles.  Requirements as for bgemm_sym_kernel.
constexpr int BT = 256;
constexpr int BS = 4;                 // stages in the LDS ring
constexpr int BSTAGE = 2 * BT * 32;   // halves per stage (A rows, then B columns)

__device__ __forceinline__ void xcd_tile(int tiles_m, int tiles_n, int& tm, int& tn) {
    const int total = tiles_m * tiles_n, id = blockIdx.x;
    int t = id;
    if (total % 8 == 0) t = (id % 8) * (total / 8) + id / 8;  // workgroups of one XCD become consecutive
    // walk the tiles in column panels of 4 tile rows (a compact block per XCD)
    const int panel = 4;
    const int full = tiles_m / panel * panel;
    const int per_panel = panel * tiles_n;
    if (t < full * tiles_n) {
        const int pnl = t / per_panel, w = t % per_panel;
        tm = pnl * panel + w % panel;
        tn = w / panel;
    } else {
        const int rest = tiles_m - full, w = t - full * tiles_n;
        tm = full + w % rest;
        tn = w / rest;
    }
}

// s_waitcnt vmcnt(n) for n in {0, 8, 16}, leaving expcnt and lgkmcnt alone (gfx9 encoding:
// vmcnt bits [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8])
__device__ __forceinline__ void wait_vmcnt(int n) {
    if (n >= 16) __builtin_amdgcn_s_waitcnt((1 << 14) | 0x0F70);
    else if (n >= 8) __builtin_amdgcn_s_waitcnt(0x0F70 | 8);
    else __builtin_amdgcn_s_waitcnt(0x0F70);
}
// s_waitcnt lgkmcnt(0) with vmcnt and expcnt left alone
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }

template <LpOut OUT>
__global__ __launch_bounds__(256) void bgemm_sym256_kernel(int M, int N, const unsigned short* __restrict__ A, long lda,
                                                           const unsigned short* __restrict__ B, long ldb,
                                                           void* __restrict__ C, long ldc, int tiles_m, int tiles_n) {
    extern __shared__ __attribute__((aligned(16))) unsigned short hsm[];
    const int K = M;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    int tm, tn;
    xcd_tile(tiles_m, tiles_n, tm, tn);
    const int row0 = tm * BT, col0 = tn * BT;
    const int full = K / 32;  // steps whose 32 k-values are all in range
    // load instruction h of wave wv covers c = wv + 4 h: A rows (c < 16) or B columns
    // 16 (c % 16) .. + 15; lane l fills row l / 4, stage position l % 4
    const unsigned short* src[8];
    {
        const int lrow = lane >> 2, lpos = lane & 3;
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int c = wv + 4 * h;
            const int isB = c >> 4, r = 16 * (c & 15) + lrow;
            const int piece = lpos ^ ((r >> 1) & 3);
            int g = (isB ? col0 : row0) + r;
            const int lim = isB ? N : M;
            g = g < lim ? g : lim - 1;
            src[h] = (isB ? B + (long)g * ldb : A + (long)g * lda) + 8 * piece;
        }
    }
    auto issue = [&](int st) {
        unsigned short* stage = hsm + (st % BS) * BSTAGE;
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            const int c = wv + 4 * h;
            __builtin_amdgcn_global_load_lds(src[h] + st * 32, stage + (c >> 4) * BT * 32 + (c & 15) * 16 * 32, 16,
                                             0, 0);
        }
    };
    v4f acc[8][8];
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) acc[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
    const int pos = (lane >> 4) ^ ((lane >> 1) & 3);
    const int aoff = (wm * 128 + (lane & 15)) * 32 + 8 * pos;
    const int boff = BT * 32 + (wn * 128 + (lane & 15)) * 32 + 8 * pos;
    v8us a[8], b[8];
    int issued = 0;
    for (; issued < BS - 1 && issued < full; ++issued) issue(issued);
    if (full > 0) {
        wait_vmcnt(8 * (issued - 1));
        __builtin_amdgcn_s_barrier();
    }
    for (int st = 0; st < full; ++st) {
        // the stage about to be refilled was last read in step st - 1, before its barrier
        if (issued < full) {
            issue(issued);
            ++issued;
        }
        const unsigned short* stage = hsm + (st % BS) * BSTAGE;
#pragma unroll
        for (int y = 0; y < 8; ++y) b[y] = *reinterpret_cast<const v8us*>(stage + boff + y * 16 * 32);
#pragma unroll
        for (int x = 0; x < 8; ++x) a[x] = *reinterpret_cast<const v8us*>(stage + aoff + x * 16 * 32);
        __builtin_amdgcn_sched_barrier(0);  // every fragment load ahead of the first product
#pragma unroll
        for (int x = 0; x < 8; ++x)
#pragma unroll
            for (int y = 0; y < 8; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a[x]),
                                                                    __builtin_bit_cast(v8bf, b[y]), acc[x][y], 0, 0,
                                                                    0);
        // step st + 1's loads (this wave's) done, this step's fragment reads done, then everyone's
        const int ahead = issued - st - 2;
        wait_vmcnt(8 * (ahead > 0 ? ahead : 0));
        wait_lgkm0();
        __builtin_amdgcn_s_barrier();
    }
    if (K > 32 * full) {
        // ragged K tail: fragments straight from global memory, zero past K
        const int k = 32 * full + 8 * (lane >> 4);
#pragma unroll
        for (int y = 0; y < 8; ++y) {
            const int g = col0 + wn * 128 + y * 16 + (lane & 15);
            b[y] = g < N ? load8_guarded(B + (long)g * ldb + k, k, K) : v8us{0, 0, 0, 0, 0, 0, 0, 0};
        }
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            const int g = row0 + wm * 128 + x * 16 + (lane & 15);
            a[x] = g < M ? load8_guarded(A + (long)g * lda + k, k, K) : v8us{0, 0, 0, 0, 0, 0, 0, 0};
        }
#pragma unroll
        for (int x = 0; x < 8; ++x)
#pragma unroll
            for (int y = 0; y < 8; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a[x]),
                                                                    __builtin_bit_cast(v8bf, b[y]), acc[x][y], 0, 0,
                                                                    0);
    }
#pragma unroll
    for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y)
            lp_store<OUT>(C, ldc, M, N, row0 + wm * 128 + x * 16, col0 + wn * 128 + y * 16, acc[x][y]);
}

// FP32 form of the same product: 128 x 128 tiles, four waves of 4 x 4 MFMA
// tiles (16 x 16 x 4, FP32).  Within a 32-deep K step, lane group g (= lane /
// 16) owns the k-run 8g .. 8g + 7 and feeds k = 8g + j to MFMA step j, so the
// four k-slots of step j are 8g + j (g = 0..3) and the eight steps cover the
// 32 values of k once each -- every lane reads its A row and B column as two
// 16-byte LDS loads.  K advances through double-buffered dynamic LDS
// (2 x 2 x 128 x 36 floats) with one barrier per step.  Requires lda and ldb
// multiples of 4 and 16-byte aligned A and B.
constexpr int FP = SK + 4;  // LDS row pitch in floats (144 bytes)
typedef float lf4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ lf4v load4_guarded(const float* __restrict__ p, int k, int K) {
    if (k + 4 <= K) return *reinterpret_cast<const lf4v*>(p);
    lf4v v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (k + e < K) ? p[e] : 0.f;
    return v;
}

template <LpOut OUT>
__global__ __launch_bounds__(256) void sgemm_sym_kernel(int M, int N, const float* __restrict__ A, long lda,
                                                        const float* __restrict__ B, long ldb, void* __restrict__ C,
                                                        long ldc) {
    extern __shared__ float fsm[];
    float (*As)[ST][FP] = reinterpret_cast<float (*)[ST][FP]>(fsm);             // [buffer][row][k]
    float (*Bs)[ST][FP] = reinterpret_cast<float (*)[ST][FP]>(fsm + 2 * ST * FP);  // [buffer][col][k]
    const int K = M;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    const int row0 = blockIdx.x * ST, col0 = blockIdx.y * ST;
    // loader: vector q = tid + 256 h covers row (column) q / 8 and k offset 4 (q % 8)
    lf4v ra[4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int q = tid + 256 * h, r = q >> 3, k = k0 + 4 * (q & 7);
            const int gi = row0 + r, gj = col0 + r;
            ra[h] = gi < M ? load4_guarded(A + k + (long)gi * lda, k, K) : lf4v{0.f, 0.f, 0.f, 0.f};
            rb[h] = gj < N ? load4_guarded(B + k + (long)gj * ldb, k, K) : lf4v{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int q = tid + 256 * h, r = q >> 3, k = 4 * (q & 7);
            *reinterpret_cast<lf4v*>(&As[buf][r][k]) = ra[h];
            *reinterpret_cast<lf4v*>(&Bs[buf][r][k]) = rb[h];
        }
    };
    v4f acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = v4f{0.f, 0.f, 0.f, 0.f};
    fetch(0);
    stash(0);
    __syncthreads();
    const int kg = 8 * (lane >> 4);
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += SK) {
        const bool more = k0 + SK < K;
        if (more) fetch(k0 + SK);
        lf4v a[4][2], b[4][2];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const float* pa = &As[buf][wm * 64 + x * 16 + (lane & 15)][kg];
            a[x][0] = *reinterpret_cast<const lf4v*>(pa);
            a[x][1] = *reinterpret_cast<const lf4v*>(pa + 4);
        }
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const float* pb = &Bs[buf][wn * 64 + y * 16 + (lane & 15)][kg];
            b[y][0] = *reinterpret_cast<const lf4v*>(pb);
            b[y][1] = *reinterpret_cast<const lf4v*>(pb + 4);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x][j >> 2][j & 3], b[y][j >> 2][j & 3],
                                                                     acc[x][y], 0, 0, 0);
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
            lp_store<OUT>(C, ldc, M, N, row0 + wm * 64 + x * 16, col0 + wn * 64 + y * 16, acc[x][y]);
}

bool lp_gemm_sym(hipStream_t st, Lp in, LpOut out, int M, int N, const void* A, long lda, const void* B, long ldb,
                 void* C, long ldc) {
    require(M >= 0 && N >= 0, "lp_gemm_sym: negative size");
    require(lda >= std::max(1, M) && ldb >= std::max(1, M) && ldc >= std::max(1, M),
            "lp_gemm_sym: bad leading dimension");
    if (M == 0 || N == 0) return true;
    const int vec = in == Lp::BF16 ? 8 : 4;  // elements per 16-byte load
    const bool aligned = (lda % vec == 0) && (ldb % vec == 0) && (reinterpret_cast<uintptr_t>(A) % 16 == 0) &&
                         (reinterpret_cast<uintptr_t>(B) % 16 == 0);
    // the 128 x 128 tiles only pay once there are enough of them (n >~ 1000);
    // smaller products keep the 64 x 64 kernel's parallelism
    if (!aligned || cdiv(N, ST) > 65535 || (long)cdiv(M, ST) * cdiv(N, ST) < 64) return false;
    dim3 grid(cdiv(M, ST), cdiv(N, ST));
    if (in == Lp::F32) {
        const auto* a = static_cast<const float*>(A);
        const auto* b = static_cast<const float*>(B);
        const size_t lds = sizeof(float) * 2 * 2 * ST * FP;
        switch (out) {
            case LpOut::F32: hipLaunchKernelGGL(sgemm_sym_kernel<LpOut::F32>, grid, dim3(256), lds, st, M, N, a, lda, b, ldb, C, ldc); break;
            case LpOut::BF16: hipLaunchKernelGGL(sgemm_sym_kernel<LpOut::BF16>, grid, dim3(256), lds, st, M, N, a, lda, b, ldb, C, ldc); break;
            case LpOut::F64: hipLaunchKernelGGL(sgemm_sym_kernel<LpOut::F64>, grid, dim3(256), lds, st, M, N, a, lda, b, ldb, C, ldc); break;
            case LpOut::ADD_F64: hipLaunchKernelGGL(sgemm_sym_kernel<LpOut::ADD_F64>, grid, dim3(256), lds, st, M, N, a, lda, b, ldb, C, ldc); break;
        }
        WC_LAUNCH_CHECK();
        return true;
    }
    const auto* a = static_cast<const unsigned short*>(A);
    const auto* b = static_cast<const unsigned short*>(B);
    const int tm = cdiv(M, BT), tn = cdiv(N, BT);
    if ((long)tm * tn >= 200) {
        // enough 256 x 256 tiles to fill the chip (n >~ 3600)
        const size_t lds = sizeof(unsigned short) * BS * BSTAGE;  // 128 KB
        const dim3 g1(static_cast<unsigned>(tm * tn));
        switch (out) {
            case LpOut::F32: hipLaunchKernelGGL(bgemm_sym256_kernel<LpOut::F32>, g1, dim3(256), lds, st, M, N, a, lda, b, ldb, C, ldc, tm, tn); break;
            case LpOut::BF16: hipLaunchKernelGGL(bgemm_sym256_kernel<LpOut::BF16>, g1, dim3(256), lds, st, M, N, a, lda, b, ldb, C, ldc, tm, tn); break;
            case LpOut::F64: hipLaunchKernelGGL(bgemm_sym256_kernel<LpOut::F64>, g1, dim3(256), lds, st, M, N, a, lda, b, ldb, C, ldc, tm, tn); break;
            case LpOut::ADD_F64: hipLaunchKernelGGL(bgemm_sym256_kernel<LpOut::ADD_F64>, g1, dim3(256), lds, st, M, N, a, lda, b, ldb, C, ldc, tm, tn); break;
        }
        WC_LAUNCH_CHECK();
        return true;
    }
    switch (out) {
        case LpOut::F32: hipLaunchKernelGGL(bgemm_sym_kernel<LpOut::F32>, grid, dim3(256), 0, st, M, N, a, lda, b, ldb, C, ldc); break;
        case LpOut::BF16: hipLaunchKernelGGL(bgemm_sym_kernel<LpOut::BF16>, grid, dim3(256), 0, st, M, N, a, lda, b, ldb, C, ldc); break;
        case LpOut::F64: hipLaunchKernelGGL(bgemm_sym_kernel<LpOut::F64>, grid, dim3(256), 0, st, M, N, a, lda, b, ldb, C, ldc); break;
        case LpOut::ADD_F64: hipLaunchKernelGGL(bgemm_sym_kernel<LpOut::ADD_F64>, grid, dim3(256), 0, st, M, N, a, lda, b, ldb, C, ldc); break;
    }
    WC_LAUNCH_CHECK();
    return true;
}

template <LpOut OUT>
static void lp_gemm_launch(hipStream_t st, Lp in, int M, int N, int K, const void* A, long lda, const void* B,
                           long ldb, void* C, long ldc) {
    dim3 grid(cdiv(M, LT), cdiv(N, LT));
    if (in == Lp::F32)
        hipLaunchKernelGGL(sgemm_nn_kernel<OUT>, grid, dim3(256), 0, st, M, N, K, static_cast<const float*>(A), lda,
                           static_cast<const float*>(B), ldb, C, ldc);
    else
        hipLaunchKernelGGL(bgemm_nn_kernel<OUT>, grid, dim3(256), 0, st, M, N, K,
                           static_cast<const unsigned short*>(A), lda, static_cast<const unsigned short*>(B), ldb, C,
                           ldc);
    WC_LAUNCH_CHECK();
}

void lp_gemm_nn(hipStream_t st, Lp in, LpOut out, int M, int N, int K, const void* A, long lda, const void* B,
                long ldb, void* C, long ldc) {
    require(M >= 0 && N >= 0 && K >= 0, "lp_gemm: negative size");
    require(lda >= std::max(1, M) && ldb >= std::max(1, K) && ldc >= std::max(1, M), "lp_gemm: bad leading dimension");
    if (M == 0 || N == 0) return;
    require(cdiv(N, LT) <= 65535, "lp_gemm: N too large for the grid");
    switch (out) {
        case LpOut::F32: lp_gemm_launch<LpOut::F32>(st, in, M, N, K, A, lda, B, ldb, C, ldc); break;
        case LpOut::BF16: lp_gemm_launch<LpOut::BF16>(st, in, M, N, K, A, lda, B, ldb, C, ldc); break;
        case LpOut::F64: lp_gemm_launch<LpOut::F64>(st, in, M, N, K, A, lda, B, ldb, C, ldc); break;
        case LpOut::ADD_F64: lp_gemm_launch<LpOut::ADD_F64>(st, in, M, N, K, A, lda, B, ldb, C, ldc); break;
    }
}

// ---- entry-sampling pieces of the low-precision operator -----------------------------
// Y = A^T(u) = sum_i u_i sym(e_j e_k^T) written straight into a zeroed
// low-precision n x n matrix (the pairs are distinct, so every entry is one
// u_i or u_i / 2, rounded as to_lowp would round it).
template <Lp P>
__global__ void entry_scatter_lp_kernel(int m, const int* __restrict__ jk, const double* __restrict__ u,
                                        void* __restrict__ Y, long ldy) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int j = jk[2 * i], k = jk[2 * i + 1];
    const float v = static_cast<float>(j == k ? u[i] : 0.5 * u[i]);
    if constexpr (P == Lp::F32) {
        static_cast<float*>(Y)[j + (long)k * ldy] = v;
        static_cast<float*>(Y)[k + (long)j * ldy] = v;
    } else {
        const unsigned short h = bf16_rne(v);
        static_cast<unsigned short*>(Y)[j + (long)k * ldy] = h;
        static_cast<unsigned short*>(Y)[k + (long)j * ldy] = h;
    }
}
void entry_scatter_lp(hipStream_t st, Lp p, int m, const int* jk, const double* u, void* Y, long ldy) {
    if (m <= 0) return;
    if (p == Lp::F32)
        hipLaunchKernelGGL(entry_scatter_lp_kernel<Lp::F32>, dim3(cdiv(m, 256)), dim3(256), 0, st, m, jk, u, Y, ldy);
    else
        hipLaunchKernelGGL(entry_scatter_lp_kernel<Lp::BF16>, dim3(cdiv(m, 256)), dim3(256), 0, st, m, jk, u, Y, ldy);
    WC_LAUNCH_CHECK();
}

// count elements of `bytes` bytes each set to zero (16-byte stores, then the tail)
__global__ void zero_bytes_kernel(long n16, long nbytes, unsigned char* __restrict__ p) {
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t < n16) {
        reinterpret_cast<uint4*>(p)[t] = uint4{0u, 0u, 0u, 0u};
    } else if (t == n16) {
        for (long b = 16 * n16; b < nbytes; ++b) p[b] = 0;
    }
}
void zero_lowp(hipStream_t st, Lp p, long count, void* X) {
    const long nbytes = count * lp_bytes(p);
    if (nbytes <= 0) return;
    require(reinterpret_cast<uintptr_t>(X) % 16 == 0, "zero_lowp: buffer must be 16-byte aligned");
    const long n16 = nbytes / 16;
    hipLaunchKernelGGL(zero_bytes_kernel, dim3(cdiv(n16 + 1, 256)), dim3(256), 0, st, n16, nbytes,
                       static_cast<unsigned char*>(X));
    WC_LAUNCH_CHECK();
}

// out_i = alpha (M_jk + M_kj) / 2 + beta out_i for an FP32 n x n M at the sampled pairs
__global__ void entry_gather_f32_kernel(int m, const int* __restrict__ jk, const float* __restrict__ M, long ldm,
                                        double* __restrict__ out, double alpha, double beta) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int j = jk[2 * i], k = jk[2 * i + 1];
    const double v = 0.5 * (static_cast<double>(M[j + (long)k * ldm]) + static_cast<double>(M[k + (long)j * ldm]));
    out[i] = (beta == 0.0) ? alpha * v : alpha * v + beta * out[i];
}
void entry_gather_f32(hipStream_t st, int m, const int* jk, const float* M, long ldm, double* out, double alpha,
                      double beta) {
    if (m <= 0) return;
    hipLaunchKernelGGL(entry_gather_f32_kernel, dim3(cdiv(m, 256)), dim3(256), 0, st, m, jk, M, ldm, out, alpha, beta);
    WC_LAUNCH_CHECK();
}

// ---- conversions ---------------------------------------------------------------------
template <Lp P>
__global__ void to_lowp_kernel(int rows, int cols, const double* __restrict__ A, long lda, void* __restrict__ B,
                               long ldb) {
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t >= (long)rows * cols) return;
    const int i = static_cast<int>(t % rows), j = static_cast<int>(t / rows);
    const double v = A[i + (long)j * lda];
    if constexpr (P == Lp::F32) static_cast<float*>(B)[i + (long)j * ldb] = static_cast<float>(v);
    else static_cast<unsigned short*>(B)[i + (long)j * ldb] = bf16_rne(static_cast<float>(v));
}
void to_lowp(hipStream_t st, Lp p, int rows, int cols, const double* A, long lda, void* B, long ldb) {
    const long cnt = (long)rows * cols;
    if (cnt <= 0) return;
    // double -> float rounds to nearest; float -> bf16 rounds to nearest even.
    // (The two-step rounding to BF16 can differ from a direct one only on
    // exact float ties, which does not matter for an approximate operator.)
    if (p == Lp::F32)
        hipLaunchKernelGGL(to_lowp_kernel<Lp::F32>, dim3(cdiv(cnt, 256)), dim3(256), 0, st, rows, cols, A, lda, B, ldb);
    else
        hipLaunchKernelGGL(to_lowp_kernel<Lp::BF16>, dim3(cdiv(cnt, 256)), dim3(256), 0, st, rows, cols, A, lda, B,
                           ldb);
    WC_LAUNCH_CHECK();
}

__global__ void to_f32_kernel(long n, const double* __restrict__ x, float* __restrict__ y) {
    const long t = blockIdx.x * 256L + threadIdx.x;
    if (t < n) y[t] = static_cast<float>(x[t]);
}
void to_f32(hipStream_t st, long count, const double* x, float* y) {
    if (count <= 0) return;
    hipLaunchKernelGGL(to_f32_kernel, dim3(cdiv(count, 256)), dim3(256), 0, st, count, x, y);
    WC_LAUNCH_CHECK();
}

// ---- packed constraint passes over FP32 rows ---------------------------------------------
constexpr int PF_ROWS = 4;     // rows per workgroup of the A(M) pass
constexpr int PF_SLAB = 64;    // row slab of the A^T(u) pass
constexpr int PF_UNROLL = 8;   // rows in flight per thread in the A^T(u) pass

__global__ __launch_bounds__(256) void packed_rows_f32_kernel(int m, int k4, const float* __restrict__ P, long ldp,
                                                              const float* __restrict__ x, double* __restrict__ y,
                                                              double alpha, double beta) {
    __shared__ double sh[4];
    const int row0 = blockIdx.x * PF_ROWS;
    double acc[PF_ROWS];
#pragma unroll
    for (int r = 0; r < PF_ROWS; ++r) acc[r] = 0.0;
    const lf4* x4 = reinterpret_cast<const lf4*>(x);
    const lf4* arow[PF_ROWS];
#pragma unroll
    for (int r = 0; r < PF_ROWS; ++r) {
        const int row = row0 + r < m ? row0 + r : m - 1;
        arow[r] = reinterpret_cast<const lf4*>(P + (long)row * ldp);
    }
    for (int c = threadIdx.x; c < k4; c += 256) {
        const lf4 xv = x4[c];
#pragma unroll
        for (int r = 0; r < PF_ROWS; ++r) {
            const lf4 av = __builtin_nontemporal_load(&arow[r][c]);
            acc[r] += (double)av.x * xv.x + (double)av.y * xv.y + (double)av.z * xv.z + (double)av.w * xv.w;
        }
    }
#pragma unroll
    for (int r = 0; r < PF_ROWS; ++r) {
        const double s = lp_block_sum<256>(acc[r], sh);
        if (threadIdx.x == 0 && row0 + r < m) {
            const double v = alpha * s;
            y[row0 + r] = (beta == 0.0) ? v : v + beta * y[row0 + r];
        }
    }
}

__global__ __launch_bounds__(256) void packed_cols_partial_f32_kernel(int m, int k4, const float* __restrict__ P,
                                                                      long ldp, const double* __restrict__ x,
                                                                      double* __restrict__ part, long pstride) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int i0 = blockIdx.y * PF_SLAB;
    const int i1 = min(m, i0 + PF_SLAB);
    if (c >= k4) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = i0;
    for (; i + PF_UNROLL <= i1; i += PF_UNROLL) {
        lf4 a[PF_UNROLL];
#pragma unroll
        for (int u = 0; u < PF_UNROLL; ++u)
            a[u] = __builtin_nontemporal_load(reinterpret_cast<const lf4*>(P + (long)(i + u) * ldp) + c);
#pragma unroll
        for (int u = 0; u < PF_UNROLL; ++u) {
            const double xv = x[i + u];
            a0 += a[u].x * xv;
            a1 += a[u].y * xv;
            a2 += a[u].z * xv;
            a3 += a[u].w * xv;
        }
    }
    for (; i < i1; ++i) {
        const lf4 a = reinterpret_cast<const lf4*>(P + (long)i * ldp)[c];
        const double xv = x[i];
        a0 += a.x * xv;
        a1 += a.y * xv;
        a2 += a.z * xv;
        a3 += a.w * xv;
    }
    ld2* out = reinterpret_cast<ld2*>(part + blockIdx.y * pstride + 4L * c);
    out[0] = ld2{a0, a1};
    out[1] = ld2{a2, a3};
}

int packed_cols_parts_f32(int m) { return cdiv(m, PF_SLAB); }

void packed_rows_f32(hipStream_t st, int m, int k, const float* P, long ldp, const float* x, double* y,
                     double alpha, double beta) {
    if (m <= 0) return;
    require(ldp % 4 == 0, "packed_rows_f32: row pitch must be a multiple of 4");
    const int k4 = static_cast<int>(round_up(k, 4) / 4);
    hipLaunchKernelGGL(packed_rows_f32_kernel, dim3(cdiv(m, PF_ROWS)), dim3(256), 0, st, m, k4, P, ldp, x, y, alpha,
                       beta);
    WC_LAUNCH_CHECK();
}

void packed_cols_partial_f32(hipStream_t st, int m, int k, const float* P, long ldp, const double* x, double* part) {
    if (k <= 0 || m <= 0) return;
    require(ldp % 4 == 0, "packed_cols_partial_f32: row pitch must be a multiple of 4");
    const int k4 = static_cast<int>(round_up(k, 4) / 4);
    hipLaunchKernelGGL(packed_cols_partial_f32_kernel, dim3(cdiv(k4, 256), packed_cols_parts_f32(m)), dim3(256), 0,
                       st, m, k4, P, ldp, x, part, round_up(k, 4));
    WC_LAUNCH_CHECK();
}

__global__ void pack_weighted_f32_kernel(long N2, long ldp, const double* __restrict__ M, long ldm,
                                         const int* __restrict__ pj, const int* __restrict__ pk,
                                         float* __restrict__ mw) {
    const long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= ldp) return;
    double v = 0.0;
    if (p < N2) {
        const int j = pj[p], k = pk[p];
        v = (j == k) ? M[j + (long)j * ldm] : (M[j + (long)k * ldm] + M[k + (long)j * ldm]);
    }
    mw[p] = static_cast<float>(v);
}
void pack_weighted_f32(hipStream_t st, long N2, long ldp, const double* M, long ldm, const int* pj, const int* pk,
                       float* mw) {
    hipLaunchKernelGGL(pack_weighted_f32_kernel, dim3(cdiv(ldp, 256)), dim3(256), 0, st, N2, ldp, M, ldm, pj, pk, mw);
    WC_LAUNCH_CHECK();
}

template <Lp P>
__global__ void at_reduce_unpack_lp_kernel(long N2, int nparts, const double* __restrict__ part, long pstride,
                                           const int* __restrict__ pj, const int* __restrict__ pk,
                                           double* __restrict__ Y, long ldy, void* __restrict__ Ylp) {
    const long p = blockIdx.x * 256L + threadIdx.x;
    if (p >= N2) return;
    // fixed part order; the loads of a batch are issued before their sums
    double s = 0.0;
    int q = 0;
    for (; q + 8 <= nparts; q += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = part[(q + u) * pstride + p];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += x[u];
    }
    for (; q < nparts; ++q) s += part[q * pstride + p];
    const int j = pj[p], k = pk[p];
    const long o1 = j + (long)k * ldy, o2 = k + (long)j * ldy;
    if (Y) {
        Y[o1] = s;
        Y[o2] = s;
    }
    if constexpr (P == Lp::F32) {
        static_cast<float*>(Ylp)[o1] = static_cast<float>(s);
        static_cast<float*>(Ylp)[o2] = static_cast<float>(s);
    } else {
        const unsigned short h = bf16_rne(static_cast<float>(s));
        static_cast<unsigned short*>(Ylp)[o1] = h;
        static_cast<unsigned short*>(Ylp)[o2] = h;
    }
}
void at_reduce_unpack_lp(hipStream_t st, Lp p, long N2, int nparts, const double* part, long pstride, const int* pj,
                         const int* pk, double* Y, long ldy, void* Ylp) {
    if (N2 <= 0) return;
    if (p == Lp::F32)
        hipLaunchKernelGGL(at_reduce_unpack_lp_kernel<Lp::F32>, dim3(cdiv(N2, 256)), dim3(256), 0, st, N2, nparts,
                           part, pstride, pj, pk, Y, ldy, Ylp);
    else
        hipLaunchKernelGGL(at_reduce_unpack_lp_kernel<Lp::BF16>, dim3(cdiv(N2, 256)), dim3(256), 0, st, N2, nparts,
                           part, pstride, pj, pk, Y, ldy, Ylp);
    WC_LAUNCH_CHECK();
}

}  // namespace wc
