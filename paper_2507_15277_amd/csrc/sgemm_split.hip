// Single-precision GEMM through 16-bit MFMA with FP32 accumulation (gfx950).
//
//   C = alpha * A * B + beta * C      A: M x K, B: K x N, C: M x N, row-major FP32
//
// The operands are FP32; each is split on the fly into T 16-bit terms and
// the product is formed from the term products that matter, accumulated in
// FP32 by v_mfma_f32_32x32x16_{bf16,f16} / v_mfma_f32_16x16x32_{bf16,f16}:
//
//   FF_PREC 1 (bf16x3): x = hi + lo + O(2^-16 x), hi = bf16(x), lo = bf16(x - hi);
//                       A*B ~ lo_A hi_B + hi_A lo_B + hi_A hi_B
//   FF_PREC 2 (bf16x6): x = hi + mid + lo + O(2^-24 x), mid = bf16(x - hi),
//                       lo = bf16(x - hi - mid); the six products of total
//                       order <= 2 (lo hi, hi lo, mid mid, mid hi, hi mid, hi hi)
//   FF_PREC 3 (fp16s):  x * 2^e rounded to FP16, with e per matrix such that
//                       max |x| * 2^e lies in [2^14, 2^15); one product,
//                       unscaled by 2^-(eA+eB) with one ldexp (a single
//                       rounding, exact while the result is a normal FP32)
//   FF_PREC 4 (fp16x3): the same scaled value s = x * 2^e split into two FP16
//                       pieces, hi = fp16(s), lo = fp16(s - hi), so
//                       s = hi + lo + O(2^-22 s); A*B ~ lo_A hi_B + hi_A lo_B
//                       + hi_A hi_B (11-bit pieces: the dropped terms are
//                       2^-22 relative, against bf16x3's 2^-16), unscaled as
//                       in fp16s
//
// Residuals x - hi and x - hi - mid are exact in FP32, and every term
// product is exact in the FP32 accumulator's input, so the only roundings
// are the splits themselves and the FP32 accumulation.  Term products are
// issued smallest first.  The alpha/beta epilogue stays in FP32.
//
// Compile-time parameters: FF_MWG, FF_NWG (work-group tile), FF_KWG (slab
// depth, a multiple of the MFMA k: 16 for MI 32, 32 for MI 16), FF_MI
// (MFMA block edge 32 or 16), FF_WM x FF_WN (wave grid), FF_PREC, FF_GM
// (tile-order group height), FF_SG (largest number of work-groups that
// split one tile's K range; 1: no split), FF_NAME (kernel symbol;
// FF_NAME##_v1 is the scalar-load kernel of the same configuration).
//
// FF_LDS 2 (pre-split): two small kernels of the same code object first form
// the 16-bit pieces of A and B once per call into a workspace, K-major and
// zero-padded to whole tiles and to a multiple of 64 in K (FF_NAME##_pa
// for A, FF_NAME##_pb for B, which also transposes B to [n][k]); the GEMM
// kernel then copies slabs of pieces straight into LDS with load-to-LDS
// copies (16 bytes = 8 pieces per lane) and runs only the MFMAs, with no
// splitting, masking or register staging in its loop.
//
// With the K range split over work-groups (splits > 1, at most FF_SG), each
// work-group takes a contiguous range of slabs and writes its raw partial
// product (after the FP16 form's exact unscale) to its split's M x N slice
// of the workspace; the runtime's reduction adds the slices in split order
// and applies alpha and beta, as for the FP32 variants.
//
// Data flow: each slab of A (M rows, 8 consecutive k per item) and of B (8
// consecutive k of one column per item; consecutive threads take
// consecutive columns, so each load instruction is coalesced) is loaded in
// FP32, split, and stored in LDS as [term][row][k] for A and [term][n][k]
// for B, so that both MFMA operands are one 16-byte LDS read per lane: lane
// l supplies 8 consecutive k of row / column (l % MI) at k offset 8*(l/MI).
// As in the FP32 kernel the MFMA's first operand comes from B and its second
// from A, so each lane's accumulators hold one row of C and runs of four
// consecutive columns.  Double-buffered LDS, one barrier per slab, the next
// slab's global loads in flight during the MFMAs.

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef FF_MWG
#define FF_MWG 128
#define FF_NWG 128
#define FF_KWG 32
#define FF_MI 32
#define FF_WM 2
#define FF_WN 2
#define FF_PREC 1
#define FF_GM 8
#define FF_NAME sgemmx_bf16x3_m128n128k32_i32_w2x2
#endif
#ifndef FF_SG
#define FF_SG 1
#endif
#ifndef FF_LDS
#define FF_LDS 1
#endif
#ifndef FF_PD
#define FF_PD 1
#endif

#define FF_CAT2(a, b) a##b
#define FF_CAT(a, b) FF_CAT2(a, b)

namespace {

constexpr int MWG = FF_MWG, NWG = FF_NWG, KWG = FF_KWG, MI = FF_MI;
constexpr int WM = FF_WM, WN = FF_WN, PREC = FF_PREC, GM = FF_GM, SG = FF_SG;
constexpr bool PRESPLIT = FF_LDS == 2;
constexpr int NS = PRESPLIT ? FF_PD + 1 : 2;            // LDS stages (pre-split: PD slabs in flight)
constexpr int TERMS = PREC == 2 ? 3 : (PREC == 3 ? 1 : 2);
constexpr bool SCALED = PREC >= 3;       // FP16 pieces of the power-of-two scaled operands
constexpr int KB = 8 * (64 / MI);        // MFMA k depth: 16 (MI 32) or 32 (MI 16)
constexpr int WTM = MWG / WM, WTN = NWG / WN;
constexpr int RM = WTM / MI, RN = WTN / MI;
constexpr int NT = 64 * WM * WN;
constexpr int S = KWG / KB;              // MFMA k steps per slab
constexpr int ACC = MI * MI / 64;
// LDS rows of 16-bit values padded by 8: the row stride in dwords,
// (KWG + 8) / 2, is an odd multiple of 4 for KWG in {16, 32, 64}, so 16-byte
// reads of 8 consecutive rows fall in disjoint banks.
constexpr int LDK = KWG + 8;
constexpr int A_TERM = MWG * LDK, B_TERM = NWG * LDK;   // 16-bit elements
constexpr int STAGE_RAW = TERMS * (A_TERM + B_TERM);
// Pre-split: a stage is rounded up to whole wave copies (64 lanes x 8
// pieces); surplus copies land in a 1 KB scratch area after the stages.
constexpr int STAGE = PRESPLIT ? (STAGE_RAW + 511) / 512 * 512 : STAGE_RAW;
constexpr int NWI = STAGE / 512;                         // wave copies per stage
constexpr int NWAVE = WM * WN;
constexpr int DPS = (NWI + NWAVE - 1) / NWAVE;           // copies per wave per slab
constexpr int LDS_ELEMS = NS * STAGE + (PRESPLIT ? 512 : 0);
constexpr int KPAD = 64;                                 // pre-split pieces: K padded to this

static_assert(PREC >= 1 && PREC <= 4, "precision form");
static_assert(MI == 32 || MI == 16, "MFMA block edge");
static_assert(MWG % (WM * MI) == 0 && NWG % (WN * MI) == 0, "tile must split into MFMA blocks");
static_assert(KWG % KB == 0, "slab depth must be a multiple of the MFMA k");
static_assert(NT <= 1024, "work-group size");
static_assert(SG >= 1, "split count");
static_assert(FF_LDS == 1 || FF_LDS == 2, "staging mode");
static_assert(KPAD % KWG == 0, "pre-split K padding must be whole slabs");
static_assert((NS - 1) * DPS <= 63, "wait count range");
static_assert(FF_PD == 1 || (PRESPLIT && FF_PD == 2), "prefetch depth");

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

template <int E> struct AccT;
template <> struct AccT<16> { typedef f32x16 T; };
template <> struct AccT<4> { typedef f32x4 T; };
typedef typename AccT<ACC>::T acc_t;

// One MFMA on 8 16-bit values per lane, kept as raw 16-bit patterns.
__device__ __forceinline__ f32x16 mfma16(i16x8 x, i16x8 y, f32x16 c)
{
    if constexpr (SCALED)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, x), __builtin_bit_cast(f16x8, y),
                                                      c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, x),
                                                       __builtin_bit_cast(bf16x8, y), c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(i16x8 x, i16x8 y, f32x4 c)
{
    if constexpr (SCALED)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, x), __builtin_bit_cast(f16x8, y),
                                                      c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, x),
                                                       __builtin_bit_cast(bf16x8, y), c, 0, 0, 0);
}

// Split 8 FP32 values into TERMS vectors of 8 16-bit patterns.  `ex` is
// the FP16 form's prescale exponent (unused otherwise): x * 2^ex by ldexp,
// exact for any exponent while the result stays a normal FP32.
__device__ __forceinline__ void split8(const float (&x)[8], int ex, i16x8 (&out)[TERMS])
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if constexpr (SCALED) {
            float r = __builtin_amdgcn_ldexpf(x[e], ex);
#pragma unroll
            for (int t = 0; t < TERMS; ++t) {
                const _Float16 h = (_Float16)r;
                out[t][e] = __builtin_bit_cast(short, h);
                r -= (float)h;                  // exact: the residual fits in FP32
            }
        } else {
            float r = x[e];
#pragma unroll
            for (int t = 0; t < TERMS; ++t) {
                const __bf16 b = (__bf16)r;
                out[t][e] = __builtin_bit_cast(short, b);
                r -= (float)b;          // exact: the residual fits in FP32
            }
        }
    }
}

// Work-group index -> (tile row, tile column, K split): work-groups are
// dealt to the 8 XCDs round-robin and renumbered so that each XCD owns a
// contiguous range (the splits of one tile, then neighbouring tiles in
// groups of GM tile rows).
__device__ __forceinline__ void tile_of(int bid, int nbm, int nbn, int splits, int& tm, int& tn, int& part)
{
    const int nb = nbm * nbn * splits;
    const int q = nb >> 3, r = nb & 7;
    const int x = bid & 7, i = bid >> 3;
    const int lin2 = (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
    const int lin = lin2 / splits;
    part = lin2 - lin * splits;
    const int width = GM * nbn;
    const int grp = lin / width;
    const int first = grp * GM;
    const int gsz = min(nbm - first, GM);
    const int w = lin - grp * width;
    tm = first + w % gsz;
    tn = w / gsz;
}

// Term products (A term, B term), smallest first.
struct Pair { int a, b; };
__device__ constexpr Pair kPairs3[3] = {{1, 0}, {0, 1}, {0, 0}};
__device__ constexpr Pair kPairs6[6] = {{2, 0}, {0, 2}, {1, 1}, {1, 0}, {0, 1}, {0, 0}};
__device__ constexpr Pair kPairs1[1] = {{0, 0}};
constexpr int NPAIRS = PREC == 2 ? 6 : (PREC == 3 ? 1 : 3);

// The MFMAs of one LDS slab: every kept term product of the lane's A rows
// and B columns, smallest first.
// The fragments of step s + 1 are read while the products of step s issue.
__device__ __forceinline__ void mma_slab(const short* sA, const short* sB, int arow, int bcol,
                                         acc_t (&acc)[RM][RN])
{
    i16x8 av[2][TERMS][RM], bv[2][TERMS][RN];
    auto fragments = [&](int s, int buf) {
#pragma unroll
        for (int q = 0; q < TERMS; ++q) {
#pragma unroll
            for (int i = 0; i < RM; ++i)
                av[buf][q][i] = *reinterpret_cast<const i16x8*>(sA + q * A_TERM + arow + i * MI * LDK + s * KB);
#pragma unroll
            for (int j = 0; j < RN; ++j)
                bv[buf][q][j] = *reinterpret_cast<const i16x8*>(sB + q * B_TERM + bcol + j * MI * LDK + s * KB);
        }
    };
    fragments(0, 0);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (s + 1 < S) fragments(s + 1, (s + 1) & 1);
#pragma unroll
        for (int p = 0; p < NPAIRS; ++p) {
            const Pair pr = PREC == 2 ? kPairs6[p] : (PREC == 3 ? kPairs1[p] : kPairs3[p]);
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j)
                    acc[i][j] = mfma16(bv[s & 1][pr.b][j], av[s & 1][pr.a][i], acc[i][j]);
        }
    }
}

// Epilogue as in the FP32 kernel; the FP16 form first removes its prescale
// by ldexp with the exponent -(eA + eB) (one rounding, exact while the
// result is a normal FP32).  A split tile writes its raw partial to its
// slice of the workspace (alpha 1, beta 0).
__device__ __forceinline__ void store_tile(const acc_t (&acc)[RM][RN], int M, int N, float alpha, float beta,
                                           float* __restrict__ C, long ldc, int unscale, float* __restrict__ ws,
                                           int splits, int part, int m0, int n0, int wm, int wn, int lr, int lh)
{
    if constexpr (SG > 1) {
        if (splits > 1) {
            C = ws + (size_t)part * (size_t)M * (size_t)N;
            ldc = N;
            alpha = 1.0f;
            beta = 0.0f;
        }
    }
    const bool cvec = ((reinterpret_cast<uintptr_t>(C) & 15) == 0) && ((ldc & 3) == 0);
    const bool use_beta = (beta != 0.0f);
#pragma unroll
    for (int i = 0; i < RM; ++i) {
        const int m = m0 + wm * WTM + i * MI + lr;
        if (m >= M) continue;
        float* crow = C + (long)m * ldc;
#pragma unroll
        for (int j = 0; j < RN; ++j) {
#pragma unroll
            for (int g = 0; g < ACC / 4; ++g) {
                const int n = n0 + wn * WTN + j * MI + (MI == 32 ? 8 * g : 0) + 4 * lh;
                f32x4 v;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    v[c] = SCALED ? __builtin_amdgcn_ldexpf(acc[i][j][4 * g + c], unscale) : acc[i][j][4 * g + c];
                if (cvec && n + 4 <= N) {
                    f32x4 o = alpha * v;
                    if (use_beta) o += beta * *reinterpret_cast<const f32x4*>(crow + n);
                    *reinterpret_cast<f32x4*>(crow + n) = o;
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (n + c < N) {
                            float o = alpha * v[c];
                            if (use_beta) o += beta * crow[n + c];
                            crow[n + c] = o;
                        }
                    }
                }
            }
        }
    }
}

template <bool VEC>
__device__ __forceinline__ void body(int M, int N, int K, float alpha, const float* __restrict__ A, long lda,
                                     const float* __restrict__ B, long ldb, float beta, float* __restrict__ C,
                                     long ldc, float* __restrict__ ws, int splits, int kper,
                                     const int* __restrict__ pexp, short* smem)
{
    const int nbm = (M + MWG - 1) / MWG, nbn = (N + NWG - 1) / NWG;
    int tm, tn, part;
    tile_of(blockIdx.x, nbm, nbn, SG > 1 ? splits : 1, tm, tn, part);
    const int m0 = tm * MWG, n0 = tn * NWG;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    const int lr = lane % MI, lh = lane / MI;

    int sa = 0, sb = 0, unscale = 0;
    if constexpr (SCALED) {
        sa = pexp[0];
        sb = pexp[1];
        unscale = -(sa + sb);
    }

    acc_t acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) acc[i][j] = acc_t{};

    // Load items: 8 consecutive k of one A row, or of one B column.
    constexpr int KC = KWG / 8;
    constexpr int NA = MWG * KC, NB = NWG * KC;
    constexpr int LA = (NA + NT - 1) / NT, LB = (NB + NT - 1) / NT;
    float ra[LA][8], rb[LB][8];
    // This work-group's slabs [kt0, kt1): all of K unless the tile is split.
    const int nkt = (K + KWG - 1) / KWG;
    const int kt0 = (SG > 1) ? part * kper : 0;
    const int kt1 = (SG > 1) ? min(nkt, kt0 + kper) : nkt;

    // Loads read clamped addresses and keep raw values; validity is
    // recomputed and applied when the slab is split into LDS, so the loads of
    // the next slab stay in flight during the MFMAs.
    auto gload = [&](int kt) {
        const int kb = kt * KWG;
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int item = tid + i * NT;
            if (NA % NT == 0 || item < NA) {
                const int row = item / KC, kk = (item % KC) * 8;
                const int m = m0 + row, k = kb + kk;
                const bool rok = m < M;
                const float* p = A + (long)(rok ? m : 0) * lda + k;
                if constexpr (VEC) {
                    // K % 4 == 0 and 16-byte aligned rows: two whole vectors.
                    const f32x4 v0 = *reinterpret_cast<const f32x4*>(rok && k < K ? p : A);
                    const f32x4 v1 = *reinterpret_cast<const f32x4*>(rok && k + 4 < K ? p + 4 : A);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        ra[i][e] = v0[e];
                        ra[i][4 + e] = v1[e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e) ra[i][e] = *(rok && k + e < K ? p + e : A);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int item = tid + i * NT;
            if (NB % NT == 0 || item < NB) {
                const int col = item % NWG, kk = (item / NWG) * 8;
                const int n = n0 + col, k = kb + kk;
                const bool cok = n < N;
#pragma unroll
                for (int e = 0; e < 8; ++e) rb[i][e] = *(cok && k + e < K ? B + (long)(k + e) * ldb + n : B);
            }
        }
    };
    auto sstore = [&](int st, int kt) {
        const int kb = kt * KWG;
        short* sA = smem + st * STAGE;
        short* sB = sA + TERMS * A_TERM;
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int item = tid + i * NT;
            if (NA % NT == 0 || item < NA) {
                const int row = item / KC, kk = (item % KC) * 8;
                const bool rok = m0 + row < M;
                float x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = (rok && kb + kk + e < K) ? ra[i][e] : 0.0f;
                i16x8 t[TERMS];
                split8(x, sa, t);
#pragma unroll
                for (int q = 0; q < TERMS; ++q)
                    *reinterpret_cast<i16x8*>(sA + q * A_TERM + row * LDK + kk) = t[q];
            }
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int item = tid + i * NT;
            if (NB % NT == 0 || item < NB) {
                const int col = item % NWG, kk = (item / NWG) * 8;
                const bool cok = n0 + col < N;
                float x[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) x[e] = (cok && kb + kk + e < K) ? rb[i][e] : 0.0f;
                i16x8 t[TERMS];
                split8(x, sb, t);
#pragma unroll
                for (int q = 0; q < TERMS; ++q)
                    *reinterpret_cast<i16x8*>(sB + q * B_TERM + col * LDK + kk) = t[q];
            }
        }
    };

    gload(kt0);
    sstore(0, kt0);
    __syncthreads();
    const int arow = (wm * WTM + lr) * LDK + lh * 8;
    const int bcol = (wn * WTN + lr) * LDK + lh * 8;
    for (int kt = kt0; kt < kt1; ++kt) {
        const int st = (kt - kt0) & 1;
        if (kt + 1 < kt1) gload(kt + 1);
        const short* sA = smem + st * STAGE;
        mma_slab(sA, sA + TERMS * A_TERM, arow, bcol, acc);
        if (kt + 1 < kt1) sstore(st ^ 1, kt + 1);
        __syncthreads();
    }
    store_tile(acc, M, N, alpha, beta, C, ldc, unscale, ws, splits, part, m0, n0, wm, wn, lr, lh);
}

// ---- pre-split mode --------------------------------------------------------

// s_waitcnt immediate (gfx9 encoding): at most `vm` vector-memory operations
// outstanding, no LDS/scalar-memory operations outstanding, exports untouched.
constexpr int waitcnt_vm(int vm) { return (vm & 15) | (((vm >> 4) & 3) << 14) | (7 << 4); }
typedef __attribute__((address_space(3))) void* lds_ptr;

// GEMM on pieces formed by the split-pass kernels: PA holds TERMS planes of
// Mp x Kp pieces of A (row m, k contiguous), PB TERMS planes of Np x Kp
// pieces of B (row n, k contiguous), zero past M, N and K, so every copy is
// in bounds and every slab is whole.  Slabs are copied into LDS with
// load-to-LDS copies, NS = PD + 1 stages deep; unit u (16 bytes) of a stage holds
// pieces 8u..8u+7 of the stage image [term][row][LDK] (A rows, then B rows);
// units in the row padding or past the image copy from PA itself.
__device__ __forceinline__ void body_pieces(int M, int N, int Kp, float alpha, const short* __restrict__ PA,
                                            long pa_plane, const short* __restrict__ PB, long pb_plane,
                                            float beta, float* __restrict__ C, long ldc, float* __restrict__ ws,
                                            int splits, int kper, const int* __restrict__ pexp, short* smem)
{
    const int nbm = (M + MWG - 1) / MWG, nbn = (N + NWG - 1) / NWG;
    int tm, tn, part;
    tile_of(blockIdx.x, nbm, nbn, SG > 1 ? splits : 1, tm, tn, part);
    const int m0 = tm * MWG, n0 = tn * NWG;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wm = wid / WN, wn = wid % WN;
    const int lr = lane % MI, lh = lane / MI;
    const int unscale = SCALED ? -(pexp[0] + pexp[1]) : 0;

    acc_t acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) acc[i][j] = acc_t{};

    const int nkt = Kp / KWG;
    const int kt0 = (SG > 1) ? part * kper : 0;
    const int kt1 = (SG > 1) ? min(nkt, kt0 + kper) : nkt;

    // Per copy slot: the unit's source at k = 0 (pieces advance by KWG per slab).
    constexpr int RU = LDK / 8;                          // units per LDS row
    constexpr int UA = TERMS * MWG * RU;
    constexpr int UB = TERMS * NWG * RU;
    const short* base[DPS];
    bool real[DPS];
#pragma unroll
    for (int j = 0; j < DPS; ++j) {
        const int wi = wid + j * NWAVE;
        const int u = wi * 64 + lane;
        base[j] = PA;
        real[j] = false;
        if (wi < NWI && u < UA) {
            const int q = u / (MWG * RU), rem = u % (MWG * RU), row = rem / RU, c = rem % RU;
            if (c < KWG / 8) {
                base[j] = PA + q * pa_plane + (long)(m0 + row) * Kp + 8 * c;
                real[j] = true;
            }
        } else if (wi < NWI && u < UA + UB) {
            const int v = u - UA;
            const int q = v / (NWG * RU), rem = v % (NWG * RU), row = rem / RU, c = rem % RU;
            if (c < KWG / 8) {
                base[j] = PB + q * pb_plane + (long)(n0 + row) * Kp + 8 * c;
                real[j] = true;
            }
        }
    }
    auto issue = [&](int kt, int st) {
#pragma unroll
        for (int j = 0; j < DPS; ++j) {
            const int wi = wid + j * NWAVE;
            const short* src = base[j] + (real[j] ? kt * KWG : 0);
            short* dst = (wi < NWI) ? smem + st * STAGE + wi * 512 : smem + NS * STAGE;
            __builtin_amdgcn_global_load_lds(src, (lds_ptr)dst, 16, 0, 0);
        }
    };

    const int arow = (wm * WTM + lr) * LDK + lh * 8;
    const int bcol = (wn * WTN + lr) * LDK + lh * 8;
#pragma unroll
    for (int p = 0; p < NS - 1; ++p)
        if (kt0 + p < kt1) issue(kt0 + p, p);
    int st = 0;
    for (int kt = kt0; kt < kt1; ++kt) {
        // This slab's copies are done when at most the later slabs' copies are
        // outstanding (every wave issues DPS per slab), every wave's are after
        // the barrier, and every wave is then done with the stage refilled next
        // (the empty asm statements keep LDS accesses from moving across).
        asm volatile("" ::: "memory");
        if (kt + NS - 2 < kt1)
            __builtin_amdgcn_s_waitcnt(waitcnt_vm((NS - 2) * DPS));
        else
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (kt + NS - 1 < kt1) {
            int nx = st + NS - 1;
            if (nx >= NS) nx -= NS;
            issue(kt + NS - 1, nx);
        }
        const short* sA = smem + st * STAGE;
        mma_slab(sA, sA + TERMS * A_TERM, arow, bcol, acc);
        if (++st == NS) st = 0;
    }
    __syncthreads();
    store_tile(acc, M, N, alpha, beta, C, ldc, unscale, ws, splits, part, m0, n0, wm, wn, lr, lh);
}

// Pieces of one 8-value chunk of k.  `x` holds the FP32 values (0 past the
// matrix), written as TERMS 16-byte vectors to planes of `plane` elements.
__device__ __forceinline__ void put_pieces(const float (&x)[8], int ex, short* __restrict__ out, long plane)
{
    i16x8 t[TERMS];
    split8(x, ex, t);
#pragma unroll
    for (int q = 0; q < TERMS; ++q) *reinterpret_cast<i16x8*>(out + q * plane) = t[q];
}

}  // namespace

#if FF_LDS == 2
// Split pass over A (M x K, row stride lda): item (m, k8) writes pieces of
// A[m][8 k8 .. 8 k8 + 7] to row m of the Mp x Kp planes; zeros past M and K.
// vec: K and lda multiples of 4 and A 16-byte aligned (two vector loads).
extern "C" __global__ void __launch_bounds__(256)
FF_CAT(FF_NAME, _pa)(int M, int K, const float* __restrict__ A, long lda, int vec,
                     const int* __restrict__ pexp, short* __restrict__ P, int Mp, int Kp, long plane)
{
    const long items = (long)Mp * (Kp / 8);
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= items) return;
    const int m = (int)(idx / (Kp / 8)), k = (int)(idx % (Kp / 8)) * 8;
    float x[8];
    const float* p = A + (long)m * lda + k;
    if (vec && m < M && k + 8 <= K) {
        const f32x4 v0 = *reinterpret_cast<const f32x4*>(p);
        const f32x4 v1 = *reinterpret_cast<const f32x4*>(p + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            x[e] = v0[e];
            x[4 + e] = v1[e];
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = (m < M && k + e < K) ? p[e] : 0.0f;
    }
    put_pieces(x, SCALED ? pexp[0] : 0, P + (long)m * Kp + k, plane);
}

// Split pass over B (K x N, row stride ldb), transposed to row n of the
// Np x Kp planes; zeros past N and K.  One block moves a 64 (k) x 64 (n)
// tile through LDS: it reads rows of B with consecutive threads on
// consecutive n, and writes with 8 consecutive threads covering 64
// consecutive k of one n (128 contiguous bytes per piece plane).  Grid:
// ceil(Np / 64) x (Kp / 64) blocks, n tiles fastest.
extern "C" __global__ void __launch_bounds__(256)
FF_CAT(FF_NAME, _pb)(int K, int N, const float* __restrict__ B, long ldb, const int* __restrict__ pexp,
                     short* __restrict__ P, int Np, int Kp, long plane)
{
    __shared__ float tile[64][65];
    const int ntiles = (Np + 63) / 64;
    const int n0 = (blockIdx.x % ntiles) * 64, k0 = (blockIdx.x / ntiles) * 64;
    const int t = threadIdx.x;
    {
        const int nl = t & 63, kb = t >> 6;
        const int n = n0 + nl;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int kl = kb + 4 * i, k = k0 + kl;
            tile[kl][nl] = (n < N && k < K) ? B[(long)k * ldb + n] : 0.0f;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int item = t + 256 * j;
        const int nl = item >> 3, kc = item & 7;
        if (n0 + nl < Np) {
            float x[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = tile[8 * kc + e][nl];
            put_pieces(x, SCALED ? pexp[1] : 0, P + (long)(n0 + nl) * Kp + k0 + 8 * kc, plane);
        }
    }
}

// GEMM on the pieces (see body_pieces).
extern "C" __global__ void __launch_bounds__(NT)
FF_NAME(int M, int N, int Kp, float alpha, const short* __restrict__ PA, long pa_plane,
        const short* __restrict__ PB, long pb_plane, float beta, float* __restrict__ C, long ldc,
        float* __restrict__ ws, int splits, int kper, const int* __restrict__ pexp)
{
    __shared__ __attribute__((aligned(16))) short smem[LDS_ELEMS];
    body_pieces(M, N, Kp, alpha, PA, pa_plane, PB, pb_plane, beta, C, ldc, ws, splits, kper, pexp, smem);
}
#else
// Same argument list as the FP32 variants; `pexp` (FP16 form only) points
// to the per-matrix exponents {eA, eB}.
extern "C" __global__ void __launch_bounds__(NT)
FF_NAME(int M, int N, int K, float alpha, const float* __restrict__ A, long lda, const float* __restrict__ B,
        long ldb, float beta, float* __restrict__ C, long ldc, float* __restrict__ ws, int splits, int kper,
        const int* __restrict__ pexp)
{
    __shared__ __attribute__((aligned(16))) short smem[LDS_ELEMS];
    body<true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, kper, pexp, smem);
}

extern "C" __global__ void __launch_bounds__(NT)
FF_CAT(FF_NAME, _v1)(int M, int N, int K, float alpha, const float* __restrict__ A, long lda,
                     const float* __restrict__ B, long ldb, float beta, float* __restrict__ C, long ldc,
                     float* __restrict__ ws, int splits, int kper, const int* __restrict__ pexp)
{
    __shared__ __attribute__((aligned(16))) short smem[LDS_ELEMS];
    body<false>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, kper, pexp, smem);
}
#endif
