// Parameterised single-precision GEMM variant for gfx950 (CDNA4).
//
//   C = alpha * A * B + beta * C      A: M x K, B: K x N, C: M x N, row-major FP32
//
// The paper's premise (Sec. III-A, Sec. III-B) is a kernel whose tuning
// parameters are compile-time constants, compiled ahead of time into a family
// of code variants from which a few are kept.  This file is that kernel: it is
// compiled once per parameter configuration (the FF_* macros below) into its
// own code object, which the runtime loads on demand.
//
// Parameters (compile-time):
//   FF_MWG, FF_NWG   work-group tile of C (rows x columns)
//   FF_KWG           K extent of one pipeline stage (slab)
//   FF_MI            MFMA block edge: 32 -> v_mfma_f32_32x32x2_f32,
//                                      16 -> v_mfma_f32_16x16x4_f32
//   FF_WM, FF_WN     wave grid over the tile (each wave owns a
//                    (MWG/WM) x (NWG/WN) sub-tile of RM x RN MFMA blocks)
//   FF_SK            intra-work-group split of each slab's K range over SK
//                    groups of waves, reduced through LDS at the end
//   FF_VW            global-load vector width in floats (1, 2, 4)
//   FF_LDS           1: slabs staged through double-buffered LDS shared by all
//                    waves; 0: each wave loads its own operands straight from
//                    global memory into registers (no LDS, no barriers)
//   FF_GM            tile-order group height (tiles of M per group)
//                    (FF_LDS 2: slabs are copied from global memory straight
//                    into LDS by the load-to-LDS instruction, each lane one
//                    16-byte unit of the padded slab image, with PD + 1 LDS
//                    stages in flight; no register staging.  Needs the
//                    vector kernel's conditions; the scalar-load kernel of
//                    the same code object stages through registers.)
//   FF_PD            LDS variants: prefetch depth in slabs (1: the next
//                    slab's global loads are in flight while the current one
//                    is computed; 2: the one after next, through a second
//                    register staging buffer, to cover longer load latency)
//   FF_SG            largest number of work-groups that split one tile's K
//                    range (1: no split).  The runtime passes the split count
//                    actually used (<= FF_SG); with more than one split each
//                    work-group writes its raw partial product (row-major,
//                    M x N per split) to a workspace instead of C, and a
//                    separate reduction kernel of the runtime sums the splits
//                    in a fixed order (deterministic) and applies alpha, beta
//   FF_NAME          kernel symbol; a second kernel FF_NAME##_v1 is the same
//                    configuration with scalar loads, for operands whose
//                    alignment or leading dimension rules out vector loads;
//                    FF_NAME##_g and FF_NAME##_g1 are the grouped persistent
//                    forms (many independent problems in one launch)
//
// Operand roles inside the MFMA.  The MFMA computes D[i][j] += sum_k X[i][k]
// Y[k][j] with X held one value per lane as X[lane%MI][lane/MI] and Y as
// Y[lane/MI][lane%MI].  The kernel feeds X from B (i indexes columns n of C)
// and Y from A (j indexes rows m of C), so that each lane's accumulator
// holds one row of C and runs of four consecutive columns, which are stored
// as 16-byte vectors.  Within one slab the k values are assigned to lanes as
// k = kgroup_base + (lane/MI)*S + s for step s < S: both operands use the
// same assignment, so every product A[m][k]B[k][n] is formed once, and each
// lane reads S consecutive k values of its A row as wide LDS reads.
//
// Edges: loads outside the matrices are replaced by zeros and stores are
// masked, so M, N and K are arbitrary.  The vector-load kernel requires
// K % VW == 0, N % VW == 0, lda % VW == 0, ldb % VW == 0 and VW-aligned A
// and B; the runtime launches the scalar kernel otherwise.  alpha == 0 and K == 0 never reach
// this kernel (the runtime handles them without reading A and B).  beta == 0
// never reads C.

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef FF_MWG
#define FF_MWG 64
#define FF_NWG 64
#define FF_KWG 16
#define FF_MI 32
#define FF_WM 2
#define FF_WN 2
#define FF_SK 1
#define FF_VW 4
#define FF_LDS 1
#define FF_GM 8
#define FF_SG 1
#define FF_NAME sgemm_m64n64k16_i32_w2x2_s1_v4_l1
#endif
#ifndef FF_PD
#define FF_PD 1
#endif

#define FF_CAT2(a, b) a##b
#define FF_CAT(a, b) FF_CAT2(a, b)

namespace {

constexpr int MWG = FF_MWG, NWG = FF_NWG, KWG = FF_KWG, MI = FF_MI;
constexpr int WM = FF_WM, WN = FF_WN, SK = FF_SK, VW = FF_VW, GM = FF_GM, SG = FF_SG, PD = FF_PD;
constexpr bool USE_LDS = FF_LDS != 0;
constexpr bool DMA = FF_LDS == 2;        // load-to-LDS staging (vector kernel only)

constexpr int MK = (MI == 32) ? 2 : 4;   // k per MFMA instruction
constexpr int WTM = MWG / WM;            // wave sub-tile rows
constexpr int WTN = NWG / WN;            // wave sub-tile columns
constexpr int RM = WTM / MI;             // MFMA blocks per wave along M
constexpr int RN = WTN / MI;             // MFMA blocks per wave along N
constexpr int NWAVE = WM * WN * SK;
constexpr int NT = 64 * NWAVE;           // threads per work-group
constexpr int KG = KWG / SK;             // k per split group per slab
constexpr int S = KG / MK;               // MFMA steps per split group per slab
constexpr int ACC = MI * MI / 64;        // accumulator floats per lane per block
constexpr int AV = (S % 4 == 0) ? 4 : ((S % 2 == 0) ? 2 : 1);  // A read width
// LDS fragment order of 16x16 blocks.  The four lane groups of an MFMA read
// B rows (their k) in the same instruction.  With each group owning S
// consecutive k, the groups sit S rows apart; for S = 8 and more that is a
// multiple of 32 words, so the 16 columns of two groups in one half-wave
// share banks (the LDS bank-conflict counter shows it).  When a group has
// more than one chunk of AV steps, the chunks of the four groups are
// interleaved instead (group h, chunk q owns k = (q*4 + h)*AV + t): the
// groups sit AV rows apart, 16 words modulo 32, in disjoint banks, and A
// reads stay AV-wide vectors.  32x32 blocks (two lane groups, one per
// half-wave) keep the contiguous order.
constexpr bool KIL = (MI == 16) && (S > AV);
constexpr int KQS = KIL ? (64 / MI) * AV : AV;    // k distance between a group's chunks

// LDS rows are padded by 4 floats: the A row stride (KWG+4) is an odd
// multiple of 4 floats for KWG in {8,16,32}, so 16-byte reads of 8
// consecutive rows fall in disjoint banks.
constexpr int PA = 4, PB = 4;
constexpr int LDA_S = KWG + PA;          // LDS row stride of the A slab [m][k]
constexpr int LDB_S = NWG + PB;          // LDS row stride of the B slab [k][n]
constexpr int STAGE_FLOATS = MWG * LDA_S + KWG * LDB_S;
constexpr int RED_FLOATS = (SK - 1) * MWG * NWG;

// Load-to-LDS staging: a stage is the padded slab image (A then B) rounded
// up to whole wave copies of 64 x 16 bytes; the wave copies of a stage are
// dealt to the waves round-robin, DPS per wave (the surplus copies of the
// last round land in a 1 KB scratch area after the stages), so every wave
// issues the same number of copies per slab and the wait counts are exact.
constexpr int NS = PD + 1;                               // LDS stages in flight
constexpr int STAGE_UNITS = (STAGE_FLOATS / 4 + 63) / 64 * 64;   // 16-byte units
constexpr int STAGE_DMA = STAGE_UNITS * 4;               // floats per stage
constexpr int NWI = STAGE_UNITS / 64;                    // wave copies per stage
constexpr int DPS = (NWI + NWAVE - 1) / NWAVE;           // copies per wave per slab
constexpr int STAGE_STRIDE = DMA ? STAGE_DMA : STAGE_FLOATS;
constexpr int STAGE_AREA = DMA ? NS * STAGE_DMA + 256 : 2 * STAGE_FLOATS;
constexpr int LDS_FLOATS = USE_LDS ? (STAGE_AREA > RED_FLOATS ? STAGE_AREA : RED_FLOATS)
                                   : (RED_FLOATS > 0 ? RED_FLOATS : 1);

static_assert(MI == 32 || MI == 16, "MFMA block edge must be 16 or 32");
static_assert(MWG % (WM * MI) == 0 && NWG % (WN * MI) == 0, "tile must split into MFMA blocks");
static_assert(KWG % (SK * MK) == 0, "slab must split over groups and MFMA k");
static_assert(VW == 1 || VW == 2 || VW == 4, "vector width");
static_assert(NT <= 1024, "work-group size");
static_assert(KWG % 4 == 0 && NWG % 4 == 0, "LDS vector alignment");
static_assert(SG >= 1, "split count");
static_assert(PD == 1 || PD == 2, "prefetch depth");
static_assert(FF_LDS >= 0 && FF_LDS <= 2, "LDS staging mode");
static_assert(!DMA || VW == 4, "load-to-LDS staging moves 16-byte units");
static_assert(!DMA || (NS - 2) * DPS <= 63, "wait count range");

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <int E> struct AccT;
template <> struct AccT<16> { typedef f32x16 T; };
template <> struct AccT<4> { typedef f32x4 T; };
typedef typename AccT<ACC>::T acc_t;

__device__ __forceinline__ f32x16 mfma(float x, float y, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(x, y, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(float x, float y, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
}

template <int V> struct VecT { typedef float T __attribute__((ext_vector_type(V))); };
template <> struct VecT<1> { typedef float T; };

template <int V>
__device__ __forceinline__ float vget(const typename VecT<V>::T& v, int e)
{
    if constexpr (V == 1) { (void)e; return v; } else { return v[e]; }
}
template <int V>
__device__ __forceinline__ void vset(typename VecT<V>::T& v, int e, float x)
{
    if constexpr (V == 1) { (void)e; v = x; } else { v[e] = x; }
}
// Element j of the result is element j + s of v (0 <= s < V); the last s
// elements keep v's last one.
template <int V>
__device__ __forceinline__ typename VecT<V>::T vshift(const typename VecT<V>::T& v, int s)
{
    typename VecT<V>::T w = v;
    if constexpr (V > 1) {
#pragma unroll
        for (int j = 0; j < V - 1; ++j) {
            float x = v[V - 1];
#pragma unroll
            for (int t = V - 2; t >= j; --t) x = (j + s == t) ? v[t] : x;
            w[j] = x;
        }
    }
    return w;
}

// Edge handling is branch-free: an invalid lane loads V floats from `safe`
// (any readable address aligned for V) instead of p, and the value is
// replaced by zeros only where it is consumed (zsel), so that the loads of
// the next slab stay in flight while the current slab is computed.  Vector
// kernels (V > 1) are launched only when K and N are multiples of V and rows
// are V-aligned, so a vector never straddles the edge of a matrix.
template <int V>
__device__ __forceinline__ typename VecT<V>::T load_raw(const float* p, bool ok, const float* safe)
{
    return *reinterpret_cast<const typename VecT<V>::T*>(ok ? p : safe);
}
template <int V>
__device__ __forceinline__ typename VecT<V>::T zsel(const typename VecT<V>::T& v, bool ok)
{
    return ok ? v : typename VecT<V>::T(0.0f);
}

// Work-group index -> (tile row, tile column, K split).  Work-groups are
// handed to the 8 XCDs round-robin; the first step renumbers them so that
// each XCD gets a contiguous range, whose consecutive entries are the splits
// of one tile and then neighbouring tiles, walked in groups of GM tile rows
// (column-major inside a group) so that neighbours share A rows and B
// columns in the XCD's L2.
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

// s_waitcnt immediate (gfx9 encoding): at most `vm` vector-memory operations
// outstanding, no LDS/scalar-memory operations outstanding, exports untouched.
constexpr int waitcnt_vm(int vm) { return (vm & 15) | (((vm >> 4) & 3) << 14) | (7 << 4); }

typedef __attribute__((address_space(3))) void* lds_ptr;

// Slabs [kt0, kt1) of one tile through load-to-LDS copies, NS stages deep,
// calling compute(stage) for each.  Unit u of a stage (16 bytes) holds floats
// 4u..4u+3 of the padded slab image: A rows of LDA_S floats, then B rows of
// LDB_S floats; units in the row padding or past the image copy from a safe
// address.  Rows past M and columns past N copy a clamped row or column:
// they only reach C rows and columns that are never stored.  Units past K
// also copy a clamped address and are zeroed in LDS before the slab is used,
// so the tail slab contributes exact zeros.  Needs K, N, lda, ldb multiples
// of 4 and 16-byte aligned A and B (the vector kernel's conditions).
template <typename Compute>
__device__ __forceinline__ void dma_slabs(int M, int N, int K, const float* __restrict__ A, long lda,
                                          const float* __restrict__ B, long ldb, int m0, int n0, int kt0,
                                          int kt1, int wid, int lane, float* smem, Compute&& compute)
{
    constexpr int UA = MWG * LDA_S / 4, UB = KWG * LDB_S / 4;
    constexpr int RA = LDA_S / 4, RB = LDB_S / 4;        // units per LDS row
    // Per copy slot: the unit's source without the slab's k offset, its k
    // within the slab, and the source step per unit of k (1 along an A row,
    // ldb down the B rows, 0 for padding units, which copy from A itself).
    const float* base[DPS];
    int kl[DPS];
    long step[DPS];
#pragma unroll
    for (int j = 0; j < DPS; ++j) {
        const int wi = wid + j * NWAVE;
        const int u = wi * 64 + lane;
        base[j] = A;
        kl[j] = 0;
        step[j] = 0;
        if (wi < NWI && u < UA) {
            const int row = u / RA, c = u % RA;
            if (c < KWG / 4) {
                base[j] = A + (long)min(m0 + row, M - 1) * lda;
                kl[j] = 4 * c;
                step[j] = 1;
            }
        } else if (wi < NWI && u < UA + UB) {
            const int v = u - UA;
            const int row = v / RB, c = v % RB;
            if (c < NWG / 4) {
                base[j] = B + min(n0 + 4 * c, N - 4);
                kl[j] = row;
                step[j] = ldb;
            }
        }
    }
    auto issue = [&](int kt, int st) {
        const int kb = kt * KWG;
#pragma unroll
        for (int j = 0; j < DPS; ++j) {
            const int wi = wid + j * NWAVE;
            const int k = kb + kl[j];
            const float* src = base[j] + ((k < K) ? (long)k * step[j] : 0L);
            float* dst = (wi < NWI) ? smem + st * STAGE_DMA + wi * 256 : smem + NS * STAGE_DMA;
            __builtin_amdgcn_global_load_lds(src, (lds_ptr)dst, 16, 0, 0);
        }
    };
    // Zero the k >= K part of a tail slab's A columns and B rows.
    auto zero_tail = [&](int kt, int st) {
        const int kv = K - kt * KWG;                     // valid k in this slab, 0 < kv < KWG
        float* sA = smem + st * STAGE_DMA;
        float* sB = sA + MWG * LDA_S;
        const int tid = wid * 64 + lane;
        for (int e = tid; e < MWG * (KWG - kv); e += NT) {
            const int r = e / (KWG - kv), c = kv + e % (KWG - kv);
            sA[r * LDA_S + c] = 0.0f;
        }
        for (int e = tid; e < (KWG - kv) * NWG; e += NT) {
            const int r = kv + e / NWG, c = e % NWG;
            sB[r * LDB_S + c] = 0.0f;
        }
    };

#pragma unroll
    for (int p = 0; p < NS - 1; ++p)
        if (kt0 + p < kt1) issue(kt0 + p, p);
    int st = 0;
    for (int kt = kt0; kt < kt1; ++kt) {
        // This slab's copies are done when only the later slabs' copies may
        // still be outstanding; then every wave's copies are (barrier), and
        // every wave has finished the slab before (so its stage is free).
        // (The empty asm statements keep the compiler from moving LDS
        // accesses across the wait and barrier; a fenced barrier would also
        // wait for the copies still in flight.)
        asm volatile("" ::: "memory");
        if (kt + NS - 2 < kt1)
            __builtin_amdgcn_s_waitcnt(waitcnt_vm((NS - 2) * DPS));
        else
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if ((kt + 1) * KWG > K) {                        // tail slab (uniform)
            zero_tail(kt, st);
            __syncthreads();
        }
        if (kt + NS - 1 < kt1) {
            int nx = st + NS - 1;
            if (nx >= NS) nx -= NS;
            issue(kt + NS - 1, nx);
        }
        compute(st);
        if (++st == NS) st = 0;
    }
    __syncthreads();                                     // LDS reused by the caller
}

// Variants with an unmasked copy of the slab loop for interior tiles.
template <int V> constexpr bool kUnmasked = USE_LDS && !(DMA && V == 4);

template <int V, bool EDGE, bool ONE = false, bool NS = false>
__device__ __forceinline__ void tile_loop(acc_t (&acc)[RM][RN], int M, int N, int K,
                                          const float* __restrict__ A, long lda,
                                          const float* __restrict__ B, long ldb,
                                          int kt0, int kt1, int tm, int tn, float* smem);

// Slabs [kt0, kt1) with every load masked.  The vector kernels of the
// register-staged variants also run where K or N is not a multiple of V
// (their rows need only be 4-byte aligned); there the slabs go element by
// element.
template <int V>
__device__ __forceinline__ void masked_slabs(acc_t (&acc)[RM][RN], int M, int N, int K,
                                             const float* __restrict__ A, long lda,
                                             const float* __restrict__ B, long ldb,
                                             int kt0, int kt1, int tm, int tn, float* smem)
{
    if constexpr (V > 1 && kUnmasked<V>) {
        if (K % V != 0 || N % V != 0) {
            tile_loop<V, true, true>(acc, M, N, K, A, lda, B, ldb, kt0, kt1, tm, tn, smem);
            return;
        }
    }
    tile_loop<V, true>(acc, M, N, K, A, lda, B, ldb, kt0, kt1, tm, tn, smem);
}

// One work-group adds the products of slabs [kt0, kt1) of K for tile
// (tm, tn) of C to its accumulators.  Every wave reaches every barrier, the
// loop ends with one (its LDS is free again afterwards), and no wave returns
// early.  EDGE false: slabs [kt0, kt1) lie inside K, so no load needs a
// per-element bounds test or select.  Rows of the tile past M read row M - 1
// instead, and load vectors that run past N read the row's last V columns
// (N >= V): those wholly past N only feed outputs past N, and the one that
// straddles N (N not a multiple of V; NS true, for the tile that holds it)
// has its valid part moved into place when it is staged.  Outputs past M or
// N are never stored.
// Only the prefetch of a slab past kt1 (issued unconditionally by the
// two-deep loop and never staged) is sent to the safe address, by one
// uniform test of the slab index.  ONE (with EDGE): every element is loaded
// on its own, with all three bounds tested, straight into the first LDS
// stage, one slab at a time; for a last slab that ends inside a load vector
// (K not a multiple of V).
template <int V, bool EDGE, bool ONE, bool NS>
__device__ __forceinline__ void tile_loop(acc_t (&acc)[RM][RN], int M, int N, int K,
                                          const float* __restrict__ A, long lda,
                                          const float* __restrict__ B, long ldb,
                                          int kt0, int kt1, int tm, int tn, float* smem)
{
    const int m0 = tm * MWG, n0 = tn * NWG;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int grp = wid / (WM * WN);      // split-K group
    const int wq = wid % (WM * WN);
    const int wm = wq / WN, wn = wq % WN;
    const int lr = lane % MI;             // lane's row within an MFMA block
    const int lh = lane / MI;             // lane's k group
    const int kg0 = grp * KG + lh * S;    // first k of this lane within a slab

    if constexpr (USE_LDS) {
        // ---- cooperative slab loads: global -> registers -> LDS ----------
        constexpr int AVEC_ROW = KWG / V;
        constexpr int NVA = MWG * AVEC_ROW;
        constexpr int LA = (NVA + NT - 1) / NT;
        constexpr int BVEC_ROW = NWG / V;
        constexpr int NVB = KWG * BVEC_ROW;
        constexpr int LB = (NVB + NT - 1) / NT;
        typedef typename VecT<V>::T vt;
        vt ra[PD][LA], rb[PD][LB];     // register staging, one set per slab in flight
        bool oka[PD][LA], okb[PD][LB];

        float* sA0 = smem;
        float* sB0 = smem + MWG * LDA_S;

        auto gload = [&](int kt, int rbuf) {
            const int kb = kt * KWG;
#pragma unroll
            for (int i = 0; i < LA; ++i) {
                const int v = tid + i * NT;
                if (NVA % NT == 0 || v < NVA) {
                    const int row = v / AVEC_ROW, kk = (v % AVEC_ROW) * V;
                    const int m = m0 + row, k = kb + kk;
                    const int mr = EDGE ? m : min(m, M - 1);
                    oka[rbuf][i] = EDGE ? ((m < M) && (k < K)) : (kt < kt1);
                    ra[rbuf][i] = load_raw<V>(A + (long)mr * lda + k, oka[rbuf][i], A);
                }
            }
#pragma unroll
            for (int i = 0; i < LB; ++i) {
                const int v = tid + i * NT;
                if (NVB % NT == 0 || v < NVB) {
                    const int row = v / BVEC_ROW, nn = (v % BVEC_ROW) * V;
                    const int k = kb + row, n = n0 + nn;
                    const int nr = (EDGE || n + V <= N) ? n : N - V;
                    okb[rbuf][i] = EDGE ? ((k < K) && (n < N)) : (kt < kt1);
                    rb[rbuf][i] = load_raw<V>(B + (long)k * ldb + nr, okb[rbuf][i], B);
                }
            }
        };
        auto sstore = [&](int st, int rbuf) {
            float* sA = sA0 + st * STAGE_STRIDE;
            float* sB = sB0 + st * STAGE_STRIDE;
#pragma unroll
            for (int i = 0; i < LA; ++i) {
                const int v = tid + i * NT;
                if (NVA % NT == 0 || v < NVA) {
                    const int row = v / AVEC_ROW, kk = (v % AVEC_ROW) * V;
                    *reinterpret_cast<vt*>(sA + row * LDA_S + kk) = EDGE ? zsel<V>(ra[rbuf][i], oka[rbuf][i]) : ra[rbuf][i];
                }
            }
#pragma unroll
            for (int i = 0; i < LB; ++i) {
                const int v = tid + i * NT;
                if (NVB % NT == 0 || v < NVB) {
                    const int row = v / BVEC_ROW, nn = (v % BVEC_ROW) * V;
                    vt x = EDGE ? zsel<V>(rb[rbuf][i], okb[rbuf][i]) : rb[rbuf][i];
                    if constexpr (NS && !EDGE) {
                        // The straddling vector was read from N - V.
                        const int n = n0 + nn;
                        x = vshift<V>(x, (n < N && n + V > N) ? n - (N - V) : 0);
                    }
                    *reinterpret_cast<vt*>(sB + row * LDB_S + nn) = x;
                }
            }
        };

        const int kq0 = KIL ? grp * KG + lh * AV : kg0;   // first k of the lane's chunk 0
        const int arow0 = (wm * WTM + lr) * LDA_S + kq0;
        const int bcol0 = wn * WTN + lr;
        // One slab from LDS: the steps go in chunks of AV (one A vector read
        // per MFMA row block); the fragments of chunk q + 1 are read while
        // the MFMAs of chunk q run, so LDS latency overlaps matrix work.
        auto compute = [&](int st) {
            const float* sA = sA0 + st * STAGE_STRIDE;
            const float* sB = sB0 + st * STAGE_STRIDE;
            typedef typename VecT<AV>::T avt;
            avt av[2][RM];
            float bv[2][AV][RN];
            auto fragments = [&](int q, int buf) {
#pragma unroll
                for (int i = 0; i < RM; ++i)
                    av[buf][i] = *reinterpret_cast<const avt*>(sA + arow0 + i * MI * LDA_S + q * KQS);
#pragma unroll
                for (int t = 0; t < AV; ++t)
#pragma unroll
                    for (int j = 0; j < RN; ++j)
                        bv[buf][t][j] = sB[(kq0 + q * KQS + t) * LDB_S + bcol0 + j * MI];
            };
            fragments(0, 0);
#pragma unroll
            for (int q = 0; q < S / AV; ++q) {
                if (q + 1 < S / AV) fragments(q + 1, (q + 1) & 1);
#pragma unroll
                for (int t = 0; t < AV; ++t)
#pragma unroll
                    for (int i = 0; i < RM; ++i)
#pragma unroll
                        for (int j = 0; j < RN; ++j)
                            acc[i][j] = mfma(bv[q & 1][t][j], vget<AV>(av[q & 1][i], t), acc[i][j]);
            }
        };

        if constexpr (ONE) {
            for (int kt = kt0; kt < kt1; ++kt) {
                const int kb = kt * KWG;
                for (int e = tid; e < MWG * KWG; e += NT) {
                    const int r = e / KWG, c = e - r * KWG;
                    const int m = m0 + r, k = kb + c;
                    sA0[r * LDA_S + c] = (m < M && k < K) ? A[(long)m * lda + k] : 0.0f;
                }
                for (int e = tid; e < KWG * NWG; e += NT) {
                    const int r = e / NWG, c = e - r * NWG;
                    const int k = kb + r, n = n0 + c;
                    sB0[r * LDB_S + c] = (k < K && n < N) ? B[(long)k * ldb + n] : 0.0f;
                }
                __syncthreads();
                compute(0);
                __syncthreads();
            }
        } else if constexpr (DMA && V == 4) {
            dma_slabs(M, N, K, A, lda, B, ldb, m0, n0, kt0, kt1, wid, lane, smem, compute);
        } else if constexpr (PD == 1) {
            gload(kt0, 0);
            sstore(0, 0);
            __syncthreads();
            for (int kt = kt0; kt < kt1; ++kt) {
                const int st = (kt - kt0) & 1;
                if (kt + 1 < kt1) gload(kt + 1, 0);
                compute(st);
                if (kt + 1 < kt1) sstore(st ^ 1, 0);
                __syncthreads();
            }
        } else {
            // Slab j is loaded into register set (j - kt0) & 1 two slabs ahead
            // and staged into LDS stage (j - kt0) & 1 one slab ahead.  Two
            // slabs per trip keep the register sets statically indexed.  The
            // loads are issued unconditionally (slabs past the end read the
            // clamped safe address and are never staged): a conditional load
            // makes the compiler wait for all loads before the next LDS store,
            // which would take the second slab of prefetch away.
            // The last one or two slabs are peeled off so that every trip of
            // the steady loop stages both of its successors: with a stage
            // under a branch, the compiler's wait counts merge over the
            // path that skips it and it waits for all loads at the top of
            // the loop.
            gload(kt0, 0);
            gload(kt0 + 1, 1);
            sstore(0, 0);
            __syncthreads();
            // A scheduling barrier keeps each stage after its MFMAs: without
            // it the (branch-free) loop lets the scheduler hoist the stage's
            // selects and stores above the MFMAs, which then wait on loads
            // issued a moment earlier.
            int kt = kt0;
            for (; kt + 2 < kt1; kt += 2) {
                gload(kt + 2, 0);
                compute(0);
                __builtin_amdgcn_sched_barrier(0);
                sstore(1, 1);
                __syncthreads();
                gload(kt + 3, 1);
                compute(1);
                __builtin_amdgcn_sched_barrier(0);
                sstore(0, 0);
                __syncthreads();
            }
            compute(0);
            if (kt + 1 < kt1) {
                sstore(1, 1);
                __syncthreads();
                compute(1);
            }
            __syncthreads();
        }
    } else {
        // ---- direct loads: every wave fetches its own operands -------------
        // A operand: S consecutive k of one row per lane (vector loads);
        // B operand: one column per lane for each of the S steps.
        constexpr int AVV = (S % V == 0) ? V : 1;
        typedef typename VecT<AVV>::T avt;
        avt ra[2][RM][S / AVV];
        float rb[2][RN][S];
        bool oka[2][RM][S / AVV], okb[2][RN][S];
        const int mrow = m0 + wm * WTM + lr;
        const int ncol = n0 + wn * WTN + lr;

        auto gload = [&](int kt, int b) {
            const int kbase = kt * KWG + kg0;
#pragma unroll
            for (int i = 0; i < RM; ++i) {
                const int m = mrow + i * MI;
#pragma unroll
                for (int q = 0; q < S / AVV; ++q) {
                    const int k = kbase + q * AVV;
                    oka[b][i][q] = (m < M) && (k < K);
                    ra[b][i][q] = load_raw<AVV>(A + (long)m * lda + k, oka[b][i][q], A);
                }
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = kbase + s;
#pragma unroll
                for (int j = 0; j < RN; ++j) {
                    const int n = ncol + j * MI;
                    okb[b][j][s] = (k < K) && (n < N);
                    rb[b][j][s] = load_raw<1>(B + (long)k * ldb + n, okb[b][j][s], B);
                }
            }
        };

        gload(kt0, 0);
        for (int kt = kt0; kt < kt1; kt += 2) {
            // Two slabs per trip so that the register buffers are indexed by
            // constants after unrolling.
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                if (kt + b < kt1) {
                    if (kt + b + 1 < kt1) gload(kt + b + 1, b ^ 1);
#pragma unroll
                    for (int s = 0; s < S; ++s) {
#pragma unroll
                        for (int i = 0; i < RM; ++i) {
                            const float y = oka[b][i][s / AVV] ? vget<AVV>(ra[b][i][s / AVV], s % AVV) : 0.0f;
#pragma unroll
                            for (int j = 0; j < RN; ++j)
                                acc[i][j] = mfma(okb[b][j][s] ? rb[b][j][s] : 0.0f, y, acc[i][j]);
                        }
                    }
                }
            }
        }
    }

}

// One work-group computes tile (tm, tn) of C over slabs [kt0, kt1) of K
// (split `part` of `splits` when the K range is split over work-groups).
// Every wave reaches every barrier and no wave returns before the epilogue,
// so the grouped kernel can call this once per tile in a loop.  EDGE false:
// all the tile's slabs lie inside K and N >= V (the loads of the loop
// without masks above).  TAIL (with
// EDGE false): the same, except that the last slab runs past K; the full
// slabs run the loop without masks and only the last one the masked loop.
// The epilogue tests every row and column in all three cases.
template <int V, bool EDGE = true, bool TAIL = false, bool NS = false>
__device__ __forceinline__ void tile_gemm(int M, int N, int K, float alpha,
                                          const float* __restrict__ A, long lda,
                                          const float* __restrict__ B, long ldb,
                                          float beta, float* __restrict__ C, long ldc,
                                          float* __restrict__ ws, int splits, int part,
                                          int kt0, int kt1, int tm, int tn, float* smem)
{
    const int m0 = tm * MWG, n0 = tn * NWG;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int grp = wid / (WM * WN);      // split-K group
    const int wq = wid % (WM * WN);
    const int wm = wq / WN, wn = wq % WN;
    const int lr = lane % MI;             // lane's row within an MFMA block
    const int lh = lane / MI;             // lane's k group

    acc_t acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j)
            acc[i][j] = acc_t{};

    if constexpr (TAIL) {
        tile_loop<V, false, false, NS>(acc, M, N, K, A, lda, B, ldb, kt0, kt1 - 1, tm, tn, smem);
        masked_slabs<V>(acc, M, N, K, A, lda, B, ldb, kt1 - 1, kt1, tm, tn, smem);
    } else {
        if constexpr (EDGE)
            masked_slabs<V>(acc, M, N, K, A, lda, B, ldb, kt0, kt1, tm, tn, smem);
        else
            tile_loop<V, false, false, NS>(acc, M, N, K, A, lda, B, ldb, kt0, kt1, tm, tn, smem);
    }

    // ---- reduce split-K groups through LDS ---------------------------------
    if constexpr (SK > 1) {
        if constexpr (USE_LDS) __syncthreads();
        constexpr int PER_WAVE = RM * RN * ACC * 64;
        if (grp > 0) {
            float* dst = smem + ((grp - 1) * (WM * WN) + wq) * PER_WAVE;
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j)
#pragma unroll
                    for (int e = 0; e < ACC; ++e)
                        dst[((i * RN + j) * ACC + e) * 64 + lane] = acc[i][j][e];
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
        for (int g = 1; g < SK; ++g) {
            const float* src = smem + ((g - 1) * (WM * WN) + wq) * PER_WAVE;
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j)
#pragma unroll
                    for (int e = 0; e < ACC; ++e)
                        acc[i][j][e] += src[((i * RN + j) * ACC + e) * 64 + lane];
        }
        }
    }

    if (grp > 0) return;   // waves of split groups > 0 hold no result

    // ---- epilogue: C = alpha*acc + beta*C ----------------------------------
    // With the K range split over work-groups the raw partial goes to this
    // split's M x N slice of the workspace instead (alpha 1, beta 0).
    if constexpr (SG > 1) {
        if (splits > 1) {
            C = ws + (size_t)part * (size_t)M * (size_t)N;
            ldc = N;
            alpha = 1.0f;
            beta = 0.0f;
        }
    }
    // Lane holds row m0+wm*WTM+i*MI+lr and, per group of 4 accumulators, the
    // columns n0+wn*WTN+j*MI + (MI==32 ? 8*g : 0) + 4*lh + {0,1,2,3}.
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
                v[0] = acc[i][j][4 * g + 0];
                v[1] = acc[i][j][4 * g + 1];
                v[2] = acc[i][j][4 * g + 2];
                v[3] = acc[i][j][4 * g + 3];
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

// Tile (tm, tn) over slabs [kt0, kt1) on the loop without masks, if it can
// take it (true), else nothing (false).  The register-staged variants run it
// for every tile (rows past M and load vectors past N read clamped
// addresses) while N >= V; a tile whose last slab runs past K runs its full
// slabs so and masks only the last one.  The tile that holds a load vector
// straddling N gets the copy of the loop that moves it into place, so the
// others run the loop unchanged.  The load-to-LDS path clamps addresses
// instead; the direct-load path measured slower without its selects.
template <int V>
__device__ __forceinline__ bool tile_unmasked(int M, int N, int K, float alpha,
                                              const float* __restrict__ A, long lda,
                                              const float* __restrict__ B, long ldb,
                                              float beta, float* __restrict__ C, long ldc,
                                              float* __restrict__ ws, int splits, int part,
                                              int kt0, int kt1, int tm, int tn, float* smem)
{
    if constexpr (kUnmasked<V>) {
        if (N < V) return false;
        const bool full = kt1 * KWG <= K;
        if (!full && kt1 - 1 <= kt0) return false;
        if constexpr (V > 1) {
            if ((tn + 1) * NWG > N && N % V != 0) {
                if (full)
                    tile_gemm<V, false, false, true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, part,
                                                     kt0, kt1, tm, tn, smem);
                else
                    tile_gemm<V, false, true, true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, part,
                                                    kt0, kt1, tm, tn, smem);
                return true;
            }
        }
        if (full)
            tile_gemm<V, false>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, part, kt0, kt1, tm, tn,
                                smem);
        else
            tile_gemm<V, false, true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, part, kt0, kt1, tm,
                                      tn, smem);
        return true;
    }
    return false;
}

template <int V>
__device__ __forceinline__ void gemm_body(int M, int N, int K, float alpha,
                                          const float* __restrict__ A, long lda,
                                          const float* __restrict__ B, long ldb,
                                          float beta, float* __restrict__ C, long ldc,
                                          float* __restrict__ ws, int splits, int kper, float* smem)
{
    const int nbm = (M + MWG - 1) / MWG, nbn = (N + NWG - 1) / NWG;
    int tm, tn, part;
    tile_of(blockIdx.x, nbm, nbn, SG > 1 ? splits : 1, tm, tn, part);
    const int nkt = (K + KWG - 1) / KWG;
    // This work-group's slabs [kt0, kt1): all of K unless the tile is split.
    const int kt0 = (SG > 1) ? part * kper : 0;
    const int kt1 = (SG > 1) ? min(nkt, kt0 + kper) : nkt;
    if (tile_unmasked<V>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, part, kt0, kt1, tm, tn, smem))
        return;
    tile_gemm<V, true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, part, kt0, kt1, tm, tn, smem);
}

// One problem of a grouped launch (layout shared with the runtime).
struct GemmDesc {
    const float* A;
    const float* B;
    float* C;
    long lda, ldb, ldc;
    int M, N, K, tiles;
};

// Grouped persistent launch: the tiles of `count` independent problems form
// one work list (prefix[g] = tiles before problem g, total = all tiles),
// walked in rounds of G = gridDim.x tiles: in round r work-group w takes
// tile r G + w when r is even and r G + (G - 1 - w) when r is odd, so with
// the list ordered heaviest first (as the runtime's caller orders it) the
// work-groups that took the heavier tiles of one round take the lighter
// ones of the next.  A work-group stops at its first tile past the list
// (later rounds only hold later tiles).  Each problem's tiles are walked
// row by row.  K is never split here.
template <int V>
__device__ __forceinline__ void grouped_body(const GemmDesc* __restrict__ d, const int* __restrict__ prefix,
                                             int count, int total, float alpha, float beta, float* smem)
{
    const int G = gridDim.x;
    for (int r = 0;; ++r) {
        const int t = r * G + ((r & 1) ? G - 1 - (int)blockIdx.x : (int)blockIdx.x);
        if (t >= total) break;
        int lo = 0, hi = count - 1;   // last problem whose first tile is <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const GemmDesc p = d[lo];
        const int local = t - prefix[lo];
        const int nbn = (p.N + NWG - 1) / NWG;
        const int tm = local / nbn, tn = local - tm * nbn;
        __syncthreads();   // the previous tile is done with LDS
        const int nkt = (p.K + KWG - 1) / KWG;
        if (tile_unmasked<V>(p.M, p.N, p.K, alpha, p.A, p.lda, p.B, p.ldb, beta, p.C, p.ldc, nullptr, 1, 0, 0, nkt,
                             tm, tn, smem))
            continue;
        tile_gemm<V, true>(p.M, p.N, p.K, alpha, p.A, p.lda, p.B, p.ldb, beta, p.C, p.ldc, nullptr, 1, 0, 0,
                           nkt, tm, tn, smem);
    }
}

}  // namespace

extern "C" __global__ void __launch_bounds__(NT)
FF_NAME(int M, int N, int K, float alpha, const float* __restrict__ A, long lda,
        const float* __restrict__ B, long ldb, float beta, float* __restrict__ C, long ldc,
        float* __restrict__ ws, int splits, int kper)
{
    __shared__ __attribute__((aligned(16))) float smem[LDS_FLOATS];
    gemm_body<VW>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, kper, smem);
}

extern "C" __global__ void __launch_bounds__(NT)
FF_CAT(FF_NAME, _v1)(int M, int N, int K, float alpha, const float* __restrict__ A, long lda,
                     const float* __restrict__ B, long ldb, float beta, float* __restrict__ C, long ldc,
                     float* __restrict__ ws, int splits, int kper)
{
    __shared__ __attribute__((aligned(16))) float smem[LDS_FLOATS];
    gemm_body<1>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, splits, kper, smem);
}

extern "C" __global__ void __launch_bounds__(NT)
FF_CAT(FF_NAME, _g)(const GemmDesc* __restrict__ d, const int* __restrict__ prefix, int count, int total,
                    float alpha, float beta)
{
    __shared__ __attribute__((aligned(16))) float smem[LDS_FLOATS];
    grouped_body<VW>(d, prefix, count, total, alpha, beta, smem);
}

extern "C" __global__ void __launch_bounds__(NT)
FF_CAT(FF_NAME, _g1)(const GemmDesc* __restrict__ d, const int* __restrict__ prefix, int count, int total,
                     float alpha, float beta)
{
    __shared__ __attribute__((aligned(16))) float smem[LDS_FLOATS];
    grouped_body<1>(d, prefix, count, total, alpha, beta, smem);
}
