// libfewfit runtime: variant registry, variant-set files, dispatch, launch,
// timing and the correctness screen.  C ABI declared in include/fewfit.h.
//
// Variants are separate code objects (one per parameter configuration, built
// ahead of time from sgemm_variant.hip) loaded with hipModuleLoad; only the
// members of the active set need to be loaded for sgemm() (Sec. III-B: the
// full variant space is too large to precompile and ship, so a few are
// pre-selected).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/fewfit.h"
#include "ptune_internal.h"
#include "runtime_internal.h"
#include "setfile.h"

#define FF_EXPORT extern "C" __attribute__((visibility("default")))

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(FF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Variant descriptors and registry

struct Variant : FfDesc {
    Variant() = default;
    explicit Variant(const FfDesc& d) : FfDesc(d) {}
    hipModule_t mod = nullptr;
    hipFunction_t fvec = nullptr;  // VW-wide loads
    hipFunction_t fsca = nullptr;  // scalar loads
    hipFunction_t fgrp = nullptr;  // grouped persistent, VW-wide loads (FP32 variants)
    hipFunction_t fgrp1 = nullptr; // grouped persistent, scalar loads
    int grp_blocks = 0;            // grouped grid: resident work-groups per device
    hipFunction_t fpa = nullptr;   // pre-split forms (LDS mode 2): pieces of A
    hipFunction_t fpb = nullptr;   // pre-split forms: pieces of B, transposed
};

struct VarSet {
    std::vector<int> ids;                        // members
    std::vector<std::array<int64_t, 3>> shapes;  // training shapes, file order
    std::vector<int64_t> flat;                   // the same, as M,N,K triples
    std::vector<int> winners;                    // member chosen per training shape
    std::vector<double> cost;                    // ntrain x k log-slowdowns of the members
    std::vector<Variant> members;                // descriptors, in member order
    // Wave correction of the dispatch, for the device the set was loaded on:
    // its compute-unit count and the log wave efficiency of every member's
    // launch on every training shape (ntrain x k).
    int dev = -1, cus = 0;
    std::vector<double> lw_train;
    std::vector<double> train_lg;                // log2 sizes of the training shapes
};

constexpr int kForms = kFfForms;
constexpr int kMaxMembers = kFfMaxMembers;  // variants in one set
std::mutex g_mu;
std::map<int, std::shared_ptr<Variant>> g_variants;
std::shared_ptr<const VarSet> g_set[kForms];  // one loaded set per precision form

// Workspace of the K-split variants: one M x N slice of partial products per
// split, per device.  Allocated once, when the first K-split variant is
// registered on that device (never inside sgemm()).
constexpr size_t kWsBytes = size_t(128) << 20;
constexpr int kMaxDevices = 16;
struct Workspace {
    float* ws = nullptr;
    float* scale = nullptr;  // FP16 forms: block maxima of |A| and |B|, then the exponents {eA, eB}
    short* pieces = nullptr; // pre-split forms: 16-bit pieces of A and B
    // Order of the calls that use these buffers, across streams: the stream
    // of the latest such call (`last_stream`); a call on another stream
    // records `last` on it and waits for that event first.  `mu` keeps the
    // ordering and the launches of one call together.
    std::mutex mu;
    hipEvent_t last = nullptr;
    hipStream_t last_stream = nullptr;
    bool last_valid = false;
};
// Pieces of the pre-split forms: TERMS planes of A (Mp x Kp) and of B
// (Np x Kp) 16-bit values, Mp, Np rounded up to the tile and Kp to 64.
constexpr size_t kPieceBytes = size_t(1) << 30;
constexpr int kPieceKPad = 64;
Workspace g_ws[kMaxDevices];
constexpr int kMaxBlocks = 1024;  // per matrix, for the |A|, |B| maxima
// Maxima of both matrices, then the two exponents.
constexpr size_t kScaleBytes = (2 * kMaxBlocks + 4) * sizeof(float);

int ensure_workspace()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FF_ERR_ARG, "device %d beyond the supported %d", dev, kMaxDevices);
    Workspace& w = g_ws[dev];
    if (w.ws != nullptr) return FF_OK;
    e = hipMalloc(&w.ws, kWsBytes);
    if (e == hipSuccess) e = hipMalloc(&w.scale, kScaleBytes);
    if (e == hipSuccess && w.last == nullptr) e = hipEventCreateWithFlags(&w.last, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (w.ws) (void)hipFree(w.ws);
        if (w.scale) (void)hipFree(w.scale);
        w.ws = nullptr;
        w.scale = nullptr;
        return hip_fail(e, "allocate workspace");
    }
    return FF_OK;
}

int ensure_pieces()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FF_ERR_ARG, "device %d beyond the supported %d", dev, kMaxDevices);
    if (g_ws[dev].pieces != nullptr) return FF_OK;
    if (g_ws[dev].last == nullptr) {
        e = hipEventCreateWithFlags(&g_ws[dev].last, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "create the workspace event");
    }
    e = hipMalloc(&g_ws[dev].pieces, kPieceBytes);
    if (e != hipSuccess) {
        g_ws[dev].pieces = nullptr;
        return hip_fail(e, "allocate the pieces workspace");
    }
    return FF_OK;
}

int load_code_object(Variant& v, const std::string& path)
{
    {
        std::ifstream f(path, std::ios::binary);
        if (!f) return fail(FF_ERR_IO, "cannot open code object %s", path.c_str());
    }
    hipModule_t mod = nullptr;
    hipError_t e = hipModuleLoad(&mod, path.c_str());
    if (e != hipSuccess) return hip_fail(e, ("hipModuleLoad " + path).c_str());
    hipFunction_t fv = nullptr, fs = nullptr;
    e = hipModuleGetFunction(&fv, mod, v.name.c_str());
    if (v.presplit()) {
        // One GEMM kernel (pieces are always aligned and padded) and the two
        // split passes.
        fs = fv;
        if (e == hipSuccess) e = hipModuleGetFunction(&v.fpa, mod, (v.name + "_pa").c_str());
        if (e == hipSuccess) e = hipModuleGetFunction(&v.fpb, mod, (v.name + "_pb").c_str());
    } else if (e == hipSuccess) {
        e = hipModuleGetFunction(&fs, mod, (v.name + "_v1").c_str());
    }
    if (e != hipSuccess) {
        (void)hipModuleUnload(mod);
        return hip_fail(e, ("hipModuleGetFunction " + v.name).c_str());
    }
    v.mod = mod;
    v.fvec = fv;
    v.fsca = fs;
    // Grouped forms are optional (the split-precision family has none).
    hipFunction_t g = nullptr, g1 = nullptr;
    if (hipModuleGetFunction(&g, mod, (v.name + "_g").c_str()) == hipSuccess &&
        hipModuleGetFunction(&g1, mod, (v.name + "_g1").c_str()) == hipSuccess) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, g1, v.threads(), 0) == hipSuccess &&
            hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            per_cu > 0 && cus > 0) {
            v.fgrp = g;
            v.fgrp1 = g1;
            v.grp_blocks = per_cu * cus;
        }
    }
    (void)hipGetLastError();
    return FF_OK;
}

// Register a variant, loading its code object unless an identical
// descriptor is already loaded under the same id.
int register_variant(const Variant& d, const std::string& dir)
{
    auto it = g_variants.find(d.id);
    if (it != g_variants.end()) {
        const Variant& o = *it->second;
        if (o.name == d.name) return FF_OK;
        return fail(FF_ERR_PARSE, "variant id %d already registered as %s, not %s", d.id, o.name.c_str(),
                    d.name.c_str());
    }
    auto v = std::make_shared<Variant>(d);
    int rc = load_code_object(*v, dir + "/" + d.name + ".co");
    if (rc != FF_OK) return rc;
    if (d.sg > 1 || d.scaled()) {
        rc = ensure_workspace();
        if (rc != FF_OK) return rc;
    }
    if (d.presplit()) {
        rc = ensure_pieces();
        if (rc != FF_OK) return rc;
    }
    g_variants[d.id] = v;
    return FF_OK;
}

std::string dirname_of(const std::string& path)
{
    size_t p = path.find_last_of('/');
    return p == std::string::npos ? std::string(".") : path.substr(0, p);
}

int device_arch(std::string& arch)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    arch = prop.gcnArchName;
    size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return FF_OK;
}

// ---------------------------------------------------------------------------
// Argument validation shared by sgemm() and sgemm_variant(): reference-BLAS
// order, before any HIP call.

int validate(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda, const float* B,
             int64_t ldb, float beta, const float* C, int64_t ldc)
{
    (void)beta;
    if (M < 0) return fail(FF_ERR_M, "sgemm: M=%lld < 0", (long long)M);
    if (N < 0) return fail(FF_ERR_N, "sgemm: N=%lld < 0", (long long)N);
    if (K < 0) return fail(FF_ERR_K, "sgemm: K=%lld < 0", (long long)K);
    const bool reads_ab = (alpha != 0.0f) && K > 0 && M > 0 && N > 0;
    if (reads_ab && A == nullptr) return fail(FF_ERR_A, "sgemm: A is NULL");
    if (lda < std::max<int64_t>(1, K)) return fail(FF_ERR_LDA, "sgemm: lda=%lld < max(1,K)", (long long)lda);
    if (reads_ab && B == nullptr) return fail(FF_ERR_B, "sgemm: B is NULL");
    if (ldb < std::max<int64_t>(1, N)) return fail(FF_ERR_LDB, "sgemm: ldb=%lld < max(1,N)", (long long)ldb);
    if (M > 0 && N > 0 && C == nullptr) return fail(FF_ERR_C, "sgemm: C is NULL");
    if (ldc < std::max<int64_t>(1, N)) return fail(FF_ERR_LDC, "sgemm: ldc=%lld < max(1,N)", (long long)ldc);
    if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX)
        return fail(FF_ERR_TOO_LARGE, "sgemm: sizes must fit in int32");
    return FF_OK;
}

// C <- beta * C (beta == 0 writes zeros without reading C).
__global__ void ff_scale_c(int64_t M, int64_t N, float beta, float* C, int64_t ldc)
{
    const int64_t total = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / N, j = idx - i * N;
        float* p = C + i * ldc + j;
        *p = (beta == 0.0f) ? 0.0f : beta * *p;
    }
}

int launch_scale(int64_t M, int64_t N, float beta, float* C, int64_t ldc, hipStream_t s)
{
    const int64_t total = M * N;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(ff_scale_c, dim3((unsigned)blocks), dim3(256), 0, s, M, N, beta, C, ldc);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FF_OK : hip_fail(e, "launch scale kernel");
}

bool aligned_for(const void* p, int vw) { return (reinterpret_cast<uintptr_t>(p) % (4u * vw)) == 0; }

// Whether the vector-load kernel of FP32 variant v can run a problem.  The
// variants that stage through registers load A along K and B along N in
// VW-wide vectors that need only 4-byte alignment (the hardware takes
// multi-dword accesses at any dword address); a load vector that would run
// past N reads the row's last VW columns instead (N >= VW), and a last slab
// that ends inside a vector goes element by element.  The load-to-LDS and
// direct-load variants need K, N, lda and ldb multiples of VW and 16-byte
// aligned A and B.
bool fp32_vector_ok(const FfDesc& v, int64_t N, int64_t K, int64_t lda, int64_t ldb, const void* A,
                    const void* B)
{
    const int w = v.vw;
    if (w <= 1) return false;
    if (v.lds == 1) return N >= w && aligned_for(A, 1) && aligned_for(B, 1);
    return K % w == 0 && N % w == 0 && lda % w == 0 && ldb % w == 0 && aligned_for(A, w) && aligned_for(B, w);
}

// C = alpha * sum_{q < splits} P[q] + beta * C, P[q] the q-th M x N slice of
// partial products; the splits are added in index order (deterministic).
// Each thread handles four consecutive columns of one row, with 16-byte
// accesses when N and ldc are multiples of 4 and C is 16-byte aligned.
template <bool VEC>
__global__ void __launch_bounds__(256)
ff_splitk_reduce(int64_t M, int64_t N, int splits, const float* __restrict__ P, float alpha, float beta,
                 float* __restrict__ C, int64_t ldc)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int64_t nq = (N + 3) / 4;
    const int64_t total = M * nq;
    const int64_t slice = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / nq, j0 = (idx - i * nq) * 4;
        if constexpr (VEC) {
            const f4* p = reinterpret_cast<const f4*>(P + i * N + j0);
            const int64_t step = slice / 4;
            f4 s = p[0];
            for (int q = 1; q < splits; ++q) s += p[q * step];
            f4* c = reinterpret_cast<f4*>(C + i * ldc + j0);
            f4 o = alpha * s;
            if (beta != 0.0f) o += beta * *c;
            *c = o;
        } else {
            const int w = (int)(N - j0 < 4 ? N - j0 : 4);
            float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int q = 0; q < splits; ++q) {
                const float* p = P + q * slice + i * N + j0;
                for (int c = 0; c < w; ++c) s[c] += p[c];
            }
            float* crow = C + i * ldc + j0;
            for (int c = 0; c < w; ++c) {
                float o = alpha * s[c];
                if (beta != 0.0f) o += beta * crow[c];
                crow[c] = o;
            }
        }
    }
}

// Maximum of a non-negative float over the 64 lanes of a wave, by DPP
// row shifts and row broadcasts: within each row of 16 lanes the maximum
// collects in lane 15 (shifts by 1, 2, 4, 8; lanes shifted in from outside
// the row read 0, the identity for non-negative values), row_bcast:15 folds
// row 0 into row 1 and row 2 into row 3, and row_bcast:31 folds lane 31
// into rows 2 and 3, leaving the wave's maximum in lane 63, which is read
// back as a wave-uniform value.  fmaxf ignores a NaN operand, as the
// per-lane loop does.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_max(float v)
{
    const int x = __float_as_int(v);
    const int y = __builtin_amdgcn_update_dpp(x, x, CTRL, ROW_MASK, 0xf, true);
    return fmaxf(v, __int_as_float(y));
}

__device__ __forceinline__ float wave_max(float v)
{
    v = dpp_max<0x111, 0xf>(v);   // row_shr:1
    v = dpp_max<0x112, 0xf>(v);   // row_shr:2
    v = dpp_max<0x114, 0xf>(v);   // row_shr:4
    v = dpp_max<0x118, 0xf>(v);   // row_shr:8
    v = dpp_max<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_max<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Maximum over a 256-thread work-group: one wave maximum per wave, then
// the four through LDS.  Every thread returns the result.
__device__ __forceinline__ float block_max256(float v)
{
    __shared__ float part[4];
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
}

// Scaled FP16 forms, step 1: block maxima of |A| (blocks [0, nb)) and |B|
// (blocks [nb, 2 nb)).  A matrix is cut into units of one row by kAbsCols
// columns; block b takes units b, b + nb, ... of its matrix, and its threads
// read each unit's columns in coalesced strides (no division per element).
constexpr int kAbsCols = 2048;

__global__ void __launch_bounds__(256)
ff_absmax_blocks(int64_t M, int64_t K, const float* __restrict__ A, int64_t lda, int64_t N,
                 const float* __restrict__ B, int64_t ldb, int nb, float* __restrict__ out)
{
    const bool isA = (int)blockIdx.x < nb;
    const int blk = isA ? blockIdx.x : blockIdx.x - nb;
    const int64_t rows = isA ? M : K, cols = isA ? K : N, ld = isA ? lda : ldb;
    const float* X = isA ? A : B;
    const int64_t chunks = (cols + kAbsCols - 1) / kAbsCols;
    const int64_t units = rows * chunks;
    float m = 0.0f;
    for (int64_t u = blk; u < units; u += nb) {
        const int64_t i = u / chunks;
        const int64_t c0 = (u - i * chunks) * kAbsCols;
        const int64_t c1 = min(cols, c0 + (int64_t)kAbsCols);
        const float* row = X + i * ld;
#pragma unroll 8
        for (int64_t j = c0 + threadIdx.x; j < c1; j += 256) m = fmaxf(m, fabsf(row[j]));
    }
    m = block_max256(m);
    if (threadIdx.x == 0) out[blockIdx.x] = m;
}

// Step 2: exponents e with max * 2^e in [2^14, 2^15) (0 for an all-zero
// matrix); writes the integers {eA, eB} after the block maxima (the GEMM
// kernels scale by ldexp, so any exponent a finite FP32 maximum needs is
// exact).  One work-group of 256 threads reduces the block maxima.
__global__ void __launch_bounds__(256) ff_fp16_prescale(int nb, float* __restrict__ buf)
{
    float ma = 0.0f, mb = 0.0f;
    for (int i = threadIdx.x; i < nb; i += 256) {
        ma = fmaxf(ma, buf[i]);
        mb = fmaxf(mb, buf[nb + i]);
    }
    ma = block_max256(ma);
    __syncthreads();                      // the partials are reused
    mb = block_max256(mb);
    if (threadIdx.x != 0) return;
    int ea = 0, eb = 0;
    if (ma > 0.0f) { int E; frexpf(ma, &E); ea = 15 - E; }
    if (mb > 0.0f) { int E; frexpf(mb, &E); eb = 15 - E; }
    int* o = reinterpret_cast<int*>(buf + 2 * kMaxBlocks);
    o[0] = ea;
    o[1] = eb;
}

// The current device's K-split workspace, or nullptr if it has none.
float* current_workspace()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    return g_ws[dev].ws;
}

// K split over work-groups: as many as the variant allows, no more than
// there are slabs, every split non-empty, and within the workspace.  M, N >= 1.
// K as the GEMM kernel sees it: pre-split forms run over K padded to 64.
int64_t launch_k(const Variant& v, int64_t K)
{
    return v.presplit() ? (K + kPieceKPad - 1) / kPieceKPad * kPieceKPad : K;
}

int split_count(const Variant& v, int64_t M, int64_t N, int64_t K, bool have_ws)
{
    K = launch_k(v, K);
    const int64_t nkt = (K + v.kwg - 1) / v.kwg;
    if (!(v.sg > 1 && nkt > 1 && have_ws)) return 1;
    const int64_t nb = ((M + v.mwg - 1) / v.mwg) * ((N + v.nwg - 1) / v.nwg);
    int64_t sp = std::min<int64_t>(v.sg, nkt);
    sp = std::min<int64_t>(sp, (int64_t)(kWsBytes / 4) / (M * N));   // slices that fit the workspace
    if (sp < 2 || nb * sp > INT32_MAX) return 1;
    const int64_t per = (nkt + sp - 1) / sp;
    return (int)((nkt + per - 1) / per);
}

// Work-groups of the GEMM kernel launch of variant v on (M, N, K): tiles
// times K splits; 0 for an empty product (nothing is launched).
int64_t launch_groups(const Variant& v, int64_t M, int64_t N, int64_t K, bool have_ws)
{
    if (M <= 0 || N <= 0) return 0;
    const int64_t nb = ((M + v.mwg - 1) / v.mwg) * ((N + v.nwg - 1) / v.nwg);
    return nb * split_count(v, M, N, K, have_ws);
}

// Device buffers one call may use, and their sizes: the K-split slices, the
// FP16 maxima and exponents, the pieces of the pre-split forms.  Null where
// absent.
struct Buffers {
    float* ws = nullptr;
    size_t ws_bytes = 0;
    float* scale = nullptr;
    short* pieces = nullptr;
    size_t pieces_bytes = 0;
};

// Bytes of pieces a pre-split variant forms for (M, N, K): T planes of A
// (Mp x Kp) and of B (Np x Kp) 16-bit values.
size_t presplit_bytes(const Variant& v, int64_t M, int64_t N, int64_t K)
{
    const int64_t Mp = (M + v.mwg - 1) / v.mwg * v.mwg, Np = (N + v.nwg - 1) / v.nwg * v.nwg;
    return (size_t)(2 * (int64_t)v.terms() * (Mp + Np) * launch_k(v, K));
}

int launch_variant(const Variant& v, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                   int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc, const Buffers& buf,
                   hipStream_t s)
{
    const int64_t nbm = (M + v.mwg - 1) / v.mwg, nbn = (N + v.nwg - 1) / v.nwg;
    const int64_t nb = nbm * nbn;
    if (nb > INT32_MAX) return fail(FF_ERR_TOO_LARGE, "sgemm: %lld tiles exceed the grid limit", (long long)nb);
    // The vector-load kernel where its loads allow (fp32_vector_ok);
    // otherwise the scalar-load kernel of the same variant.  Split-precision
    // variants load B by columns (scalar) and A in 16-byte vectors.
    const bool vec = v.prec > 0 ? (K % 4 == 0 && lda % 4 == 0 && aligned_for(A, 4))
                                : fp32_vector_ok(v, N, K, lda, ldb, A, B);
    hipFunction_t f = vec ? v.fvec : v.fsca;
    const float* prescale = nullptr;
    // Every check that can fail comes before the first launch.
    const int64_t nkt = (launch_k(v, K) + v.kwg - 1) / v.kwg;
    float* ws = buf.ws;
    int splits = split_count(v, M, N, K, ws != nullptr);
    if (splits == 1) ws = nullptr;
    if (splits > 1 && (size_t)splits * (size_t)(M * N) * sizeof(float) > buf.ws_bytes)
        return fail(FF_ERR_TOO_LARGE, "%d K splits of %lld x %lld exceed the %zu-byte workspace", splits,
                    (long long)M, (long long)N, buf.ws_bytes);
    if (v.scaled() && buf.scale == nullptr) return fail(FF_ERR_HIP, "fp16 form: no scale buffer on this device");
    if (v.presplit()) {
        if (buf.pieces == nullptr) return fail(FF_ERR_HIP, "pre-split form: no pieces workspace on this device");
        const size_t need = presplit_bytes(v, M, N, K);
        if (need > buf.pieces_bytes)
            return fail(FF_ERR_TOO_LARGE, "pre-split form: %zu bytes of pieces exceed the %zu-byte workspace", need,
                        buf.pieces_bytes);
    }
    if (v.scaled()) {
        float* sbuf = buf.scale;
        // One block per row unit (a row, or kAbsCols columns of it), at
        // most kMaxBlocks blocks per matrix.
        const int64_t units = std::max(M * ((K + kAbsCols - 1) / kAbsCols), K * ((N + kAbsCols - 1) / kAbsCols));
        const int nbk = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxBlocks, units));
        hipLaunchKernelGGL(ff_absmax_blocks, dim3(2 * nbk), dim3(256), 0, s, M, K, A, lda, N, B, ldb, nbk, sbuf);
        hipLaunchKernelGGL(ff_fp16_prescale, dim3(1), dim3(256), 0, s, nbk, sbuf);
        hipError_t e0 = hipGetLastError();
        if (e0 != hipSuccess) return hip_fail(e0, "launch fp16 prescale");
        prescale = sbuf + 2 * kMaxBlocks;
    }
    int kper = (int)((nkt + splits - 1) / splits);
    int Mi = (int)M, Ni = (int)N, Ki = (int)K;
    long la = (long)lda, lb = (long)ldb, lc = (long)ldc;
    hipError_t e;
    if (v.presplit()) {
        // Form the pieces of A and B, then the GEMM on them.
        int Mp = (int)(nbm * v.mwg), Np = (int)(nbn * v.nwg), Kp = (int)launch_k(v, K);
        const int64_t T = v.terms();
        short* PA = buf.pieces;
        short* PB = PA + T * (int64_t)Mp * Kp;
        long pa_plane = (long)Mp * Kp, pb_plane = (long)Np * Kp;
        int vecA = (K % 4 == 0 && lda % 4 == 0 && aligned_for(A, 4)) ? 1 : 0;
        void* aa[] = {&Mi, &Ki, (void*)&A, &la, &vecA, (void*)&prescale, (void*)&PA, &Mp, &Kp, &pa_plane};
        void* ab[] = {&Ki, &Ni, (void*)&B, &lb, (void*)&prescale, (void*)&PB, &Np, &Kp, &pb_plane};
        const int64_t ia = (int64_t)Mp * (Kp / 8);
        const int64_t gb = (int64_t)((Np + 63) / 64) * (Kp / 64);     // 64 x 64 tiles of B
        e = hipModuleLaunchKernel(v.fpa, (unsigned)((ia + 255) / 256), 1, 1, 256, 1, 1, 0, s, aa, nullptr);
        if (e == hipSuccess)
            e = hipModuleLaunchKernel(v.fpb, (unsigned)gb, 1, 1, 256, 1, 1, 0, s, ab, nullptr);
        if (e != hipSuccess) return hip_fail(e, ("launch split passes of " + v.name).c_str());
        void* ag[] = {&Mi, &Ni, &Kp, &alpha, (void*)&PA, &pa_plane, (void*)&PB, &pb_plane, &beta, (void*)&C, &lc,
                      (void*)&ws, &splits, &kper, (void*)&prescale};
        e = hipModuleLaunchKernel(v.fvec, (unsigned)(nb * splits), 1, 1, (unsigned)v.threads(), 1, 1, 0, s, ag,
                                  nullptr);
    } else {
        // FP32 variants take 14 arguments; split-precision variants add the
        // FP16 prescale pointer.
        void* args[] = {&Mi, &Ni, &Ki, &alpha, (void*)&A, &la, (void*)&B, &lb, &beta, (void*)&C, &lc,
                        (void*)&ws, &splits, &kper, (void*)&prescale};
        e = hipModuleLaunchKernel(f, (unsigned)(nb * splits), 1, 1, (unsigned)v.threads(), 1, 1, 0, s, args,
                                  nullptr);
    }
    if (e != hipSuccess) return hip_fail(e, ("launch " + v.name).c_str());
    if (splits > 1) {
        const int64_t work = M * ((N + 3) / 4);
        const int64_t blocks = std::min<int64_t>((work + 255) / 256, 8192);
        const bool vec4 = (N % 4 == 0) && (ldc % 4 == 0) && aligned_for(C, 4);
        if (vec4)
            hipLaunchKernelGGL(ff_splitk_reduce<true>, dim3((unsigned)blocks), dim3(256), 0, s, M, N, splits,
                               (const float*)ws, alpha, beta, C, ldc);
        else
            hipLaunchKernelGGL(ff_splitk_reduce<false>, dim3((unsigned)blocks), dim3(256), 0, s, M, N, splits,
                               (const float*)ws, alpha, beta, C, ldc);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "launch split-K reduction");
    }
    return FF_OK;
}

// Validation, quick returns and the choice of variant shared by every GEMM
// entry point.  Returns FF_OK with *v set when a GEMM kernel must run,
// FF_OK with *v null when the call is complete (nothing to do, or C was
// only scaled), or an error.  `v` in: the explicit variant, or null for
// dispatch through the set of `form`.
int gemm_prepare(const Variant*& v, std::shared_ptr<Variant>& hold, int form, int64_t M, int64_t N, int64_t K,
                 float alpha, const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                 int64_t ldc, hipStream_t s)
{
    int rc = validate(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    if (rc != FF_OK) return rc;
    if (M == 0 || N == 0) {
        v = nullptr;
        return FF_OK;
    }
    if (alpha == 0.0f || K == 0) {
        v = nullptr;
        return beta == 1.0f ? FF_OK : launch_scale(M, N, beta, C, ldc, s);
    }
    if (v == nullptr) {
        int id = variant_select_form(form, M, N, K);
        if (id < 0) return id;
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_variants.find(id);
        if (it == g_variants.end()) return fail(FF_ERR_VARIANT, "variant %d not loaded", id);
        hold = it->second;
        v = hold.get();
    }
    return FF_OK;
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// Shared body of sgemm(), sgemm_form() and sgemm_variant(); `v` may be null
// for the dispatch path, in which case the set picks it.  A call that uses
// the device's shared buffers (K-split slices, FP16 exponents, pieces) on
// another stream than the previous such call is ordered after it: an event
// is recorded on that previous stream at this moment (behind everything
// enqueued there so far) and this call's stream waits for it.  Calls on the
// stream of the previous user need no ordering and cost nothing extra.  If
// the previous stream is no longer valid (destroyed by its owner), the call
// waits for the whole device instead.  Calls made while their stream is
// captured into a graph neither wait nor become the previous user (an event
// recorded outside a capture cannot be waited on inside it, and the library
// cannot see when the graph is launched).
int gemm_common(const Variant* v, int form, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc, void* stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::shared_ptr<Variant> hold;
    int rc = gemm_prepare(v, hold, form, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
    if (rc != FF_OK || v == nullptr) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FF_ERR_ARG, "device %d beyond the supported %d", dev, kMaxDevices);
    Workspace& w = g_ws[dev];
    Buffers buf{w.ws, kWsBytes, w.scale, w.pieces, kPieceBytes};
    const bool shared = v->scaled() || v->presplit() || split_count(*v, M, N, K, buf.ws != nullptr) > 1;
    if (!shared) return launch_variant(*v, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, buf, s);
    std::lock_guard<std::mutex> lk(w.mu);
    const bool capturing = stream_capturing(s);
    if (!capturing && w.last_valid && w.last_stream != s && w.last != nullptr) {
        e = hipEventRecord(w.last, w.last_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, w.last, 0);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "order the workspace after the previous call");
        }
    }
    rc = launch_variant(*v, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, buf, s);
    if (rc == FF_OK && !capturing) {
        w.last_stream = s;
        w.last_valid = true;
    }
    return rc;
}

std::shared_ptr<Variant> find_variant(int id)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_variants.find(id);
    return it == g_variants.end() ? nullptr : it->second;
}

// ---------------------------------------------------------------------------
// Correctness screen kernels: a plain FP64 reference, one thread per element.

constexpr double kU32 = 1.0 / 16777216.0;  // 2^-24

__global__ void ff_screen_ref(int64_t M, int64_t N, int64_t K, double alpha, const float* A, int64_t lda,
                              const float* B, int64_t ldb, double beta, const float* C0, int64_t ldc0,
                              double* ref, double* tol, int epi)
{
    const int64_t total = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / N, j = idx - i * N;
        double s = 0.0, t = 0.0;
        if (alpha != 0.0) {
            for (int64_t k = 0; k < K; ++k) {
                const double a = A[i * lda + k], b = B[k * ldb + j];
                s += a * b;
                t += fabs(a) * fabs(b);
            }
        }
        double r = (alpha != 0.0 && K > 0) ? alpha * s : 0.0;
        double c0 = 0.0;
        if (beta != 0.0) {
            c0 = beta * (double)C0[i * ldc0 + j];
            r += c0;
        }
        double tl = 4.0 * (double)K * kU32 * fabs(alpha) * t;
        if (epi) tl += 2.0 * kU32 * (fabs(alpha * s) + fabs(c0));
        ref[idx] = r;
        tol[idx] = tl;
    }
}

constexpr int kCmpThreads = 256, kCmpBlocks = 1024;

// Per block: count of |C - ref| > scale*tol or non-finite C, the largest
// |C - ref| / (scale*tol), and the sums of (C - ref)^2 and ref^2 (for the
// normwise relative error).
__global__ void __launch_bounds__(kCmpThreads)
ff_screen_cmp(int64_t M, int64_t N, const float* C, int64_t ldc, const double* ref, const double* tol, double scale,
              long long* bad_out, double* ratio_out, double* err2_out, double* ref2_out)
{
    __shared__ long long sb[kCmpThreads];
    __shared__ double sr[kCmpThreads], se[kCmpThreads], sf[kCmpThreads];
    long long bad = 0;
    double mr = 0.0, e2 = 0.0, r2 = 0.0;
    const int64_t total = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / N, j = idx - i * N;
        const double c = C[i * ldc + j];
        const double d = fabs(c - ref[idx]);
        const double tl = scale * tol[idx];
        double ratio;
        if (!isfinite(c)) ratio = INFINITY;
        else if (tl > 0.0) ratio = d / tl;
        else ratio = (d == 0.0) ? 0.0 : INFINITY;
        if (!(d <= tl) || !isfinite(c)) ++bad;
        mr = fmax(mr, ratio);
        e2 += d * d;
        r2 += ref[idx] * ref[idx];
    }
    sb[threadIdx.x] = bad;
    sr[threadIdx.x] = mr;
    se[threadIdx.x] = e2;
    sf[threadIdx.x] = r2;
    __syncthreads();
    for (int w = kCmpThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sb[threadIdx.x] += sb[threadIdx.x + w];
            sr[threadIdx.x] = fmax(sr[threadIdx.x], sr[threadIdx.x + w]);
            se[threadIdx.x] += se[threadIdx.x + w];
            sf[threadIdx.x] += sf[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bad_out[blockIdx.x] = sb[0];
        ratio_out[blockIdx.x] = sr[0];
        err2_out[blockIdx.x] = se[0];
        ref2_out[blockIdx.x] = sf[0];
    }
}

}  // namespace

// ===========================================================================
// Internal entry points for the allocation-free path (noalloc.hip)

namespace fewfit_internal {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int gemm_scratch(int form, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                 const float* B, int64_t ldb, float beta, float* C, int64_t ldc, void* stream, void* scratch,
                 size_t bytes)
{
    if (form < 0 || form >= kForms) return fail(FF_ERR_ARG, "sgemm_form_noalloc: unknown form %d", form);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Variant* v = nullptr;
    std::shared_ptr<Variant> hold;
    int rc = gemm_prepare(v, hold, form, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
    if (rc != FF_OK || v == nullptr) return rc;
    // [0, kScaleRegion): maxima and exponents; then the pieces; then the
    // K-split slices, each region starting on a 256-byte boundary.
    constexpr size_t kScaleRegion = 16 << 10;
    static_assert(kScaleBytes <= kScaleRegion, "scale region");
    auto up256 = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t pieces = v->presplit() ? up256(presplit_bytes(*v, M, N, K)) : 0;
    const int splits = split_count(*v, M, N, K, true);
    const size_t slices = splits > 1 ? (size_t)splits * (size_t)(M * N) * sizeof(float) : 0;
    if (scratch == nullptr || kScaleRegion + pieces + slices > bytes)
        return fail(FF_ERR_TOO_LARGE,
                    "sgemm_form_noalloc: the call needs %zu bytes of scratch (%zu of pieces, %d K-split slices of "
                    "%zu) beyond the %zu-byte array", kScaleRegion + pieces + slices, pieces, splits,
                    slices / std::max(splits, 1), bytes);
    char* base = static_cast<char*>(scratch);
    Buffers buf{reinterpret_cast<float*>(base + kScaleRegion + pieces), bytes - kScaleRegion - pieces,
                reinterpret_cast<float*>(base), reinterpret_cast<short*>(base + kScaleRegion), pieces};
    return launch_variant(*v, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, buf, s);
}

}  // namespace fewfit_internal

// ===========================================================================
// Exported C ABI

FF_EXPORT const char* fewfit_last_error(void) { return g_err.c_str(); }

FF_EXPORT int variant_manifest_load(const char* dir)
{
    if (dir == nullptr) return fail(FF_ERR_ARG, "variant_manifest_load: dir is NULL");
    std::vector<FfDesc> list;
    std::string err;
    int rc = ff_read_manifest(dir, list, err);
    if (rc != FF_OK) return fail(rc, "%s", err.c_str());
    std::lock_guard<std::mutex> lk(g_mu);
    for (const FfDesc& d : list) {
        rc = register_variant(Variant(d), dir);
        if (rc != FF_OK) return rc;
    }
    return (int)list.size();
}

FF_EXPORT int variant_count(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return (int)g_variants.size();
}

FF_EXPORT int variant_info(int id, char* buf, size_t len)
{
    auto v = find_variant(id);
    if (!v) return fail(FF_ERR_VARIANT, "variant %d not registered", id);
    char tmp[512];
    int n = snprintf(tmp, sizeof tmp, "%d %s %d %d %d %d %d %d %d %d %d %d %d %d %d", v->id, v->name.c_str(),
                     v->mwg, v->nwg, v->kwg, v->mi, v->wm, v->wn, v->sk, v->vw, v->lds, v->gm, v->sg, v->prec, v->pd);
    if (buf && len > 0) {
        size_t c = std::min(len - 1, (size_t)n);
        memcpy(buf, tmp, c);
        buf[c] = '\0';
    }
    return n;
}

// Current device and its compute-unit count (queried once per device: the
// attribute query costs more than the rest of a dispatch).
static std::atomic<int> g_cus[kMaxDevices];

static int device_cus(int& dev, int& cus)
{
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(FF_ERR_ARG, "device %d beyond the supported %d", dev, kMaxDevices);
    cus = g_cus[dev].load(std::memory_order_relaxed);
    if (cus > 0) return FF_OK;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "query compute units");
    if (cus < 1) return fail(FF_ERR_HIP, "device reports %d compute units", cus);
    g_cus[dev].store(cus, std::memory_order_relaxed);
    return FF_OK;
}

// Log wave efficiency of every member on every training shape, for the
// current device (its compute units and whether it holds a workspace).
static int wave_table(VarSet& set)
{
    int rc = device_cus(set.dev, set.cus);
    if (rc != FF_OK) return rc;
    const bool ws = current_workspace() != nullptr;
    const size_t k = set.members.size();
    set.lw_train.assign(set.shapes.size() * k, 0.0);
    set.train_lg.clear();
    for (int64_t x : set.flat) set.train_lg.push_back(ptune_log2_size(x));
    for (size_t i = 0; i < set.shapes.size(); ++i)
        for (size_t j = 0; j < k; ++j) {
            const auto& s = set.shapes[i];
            set.lw_train[i * k + j] =
                ptune_log_wave_efficiency(launch_groups(set.members[j], s[0], s[1], s[2], ws), set.cus);
        }
    return FF_OK;
}

// Load a set file (format and checks in setfile.cpp).
FF_EXPORT int variant_set_load(const char* path)
{
    if (path == nullptr) return fail(FF_ERR_ARG, "variant_set_load: path is NULL");
    FfSetFile file;
    std::string err;
    int rc = ff_read_set_file(path, file, err);
    if (rc != FF_OK) return fail(rc, "%s", err.c_str());
    std::string dev;
    rc = device_arch(dev);
    if (rc != FF_OK) return rc;
    if (dev != file.arch) return fail(FF_ERR_ARCH, "set built for %s, device is %s", file.arch.c_str(), dev.c_str());

    auto set = std::make_shared<VarSet>();
    for (const FfDesc& d : file.members) {
        set->ids.push_back(d.id);
        set->members.emplace_back(d);
    }
    set->shapes = file.shapes;
    for (const auto& sh : file.shapes) set->flat.insert(set->flat.end(), {sh[0], sh[1], sh[2]});
    set->winners = file.winners;
    set->cost = file.cost;
    const std::string& codedir = file.codedir;
    const std::string dir = codedir[0] == '/' ? codedir : dirname_of(path) + "/" + codedir;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const Variant& v : set->members) {
        rc = register_variant(v, dir);
        if (rc != FF_OK) return rc;
    }
    rc = wave_table(*set);
    if (rc != FF_OK) return rc;
    g_set[file.form] = set;
    return (int)set->ids.size();
}

FF_EXPORT int variant_select_form(int form, int64_t M, int64_t N, int64_t K)
{
    if (form < 0 || form >= kForms) return fail(FF_ERR_ARG, "variant_select_form: unknown form %d", form);
    if (M < 0) return fail(FF_ERR_M, "variant_select: M < 0");
    if (N < 0) return fail(FF_ERR_N, "variant_select: N < 0");
    if (K < 0) return fail(FF_ERR_K, "variant_select: K < 0");
    std::shared_ptr<const VarSet> set;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        set = g_set[form];
    }
    if (!set) return fail(FF_ERR_NO_SET, "no variant set loaded for form %d", form);
    // Wave correction with the training-shape table of the device the set
    // was loaded on; on another device both sides are computed afresh.
    int dev = 0, cus = 0;
    int rc = device_cus(dev, cus);
    if (rc != FF_OK) return rc;
    const bool ws = current_workspace() != nullptr;
    const size_t k = set->members.size();
    double lq[kMaxMembers];
    std::vector<double> lt_other;
    const double* lt = set->lw_train.data();
    for (size_t j = 0; j < k; ++j) lq[j] = ptune_log_wave_efficiency(launch_groups(set->members[j], M, N, K, ws), cus);
    if (dev != set->dev || cus != set->cus) {
        lt_other.resize(set->shapes.size() * k);
        for (size_t i = 0; i < set->shapes.size(); ++i)
            for (size_t j = 0; j < k; ++j) {
                const auto& s = set->shapes[i];
                lt_other[i * k + j] =
                    ptune_log_wave_efficiency(launch_groups(set->members[j], s[0], s[1], s[2], ws), cus);
            }
        lt = lt_other.data();
    }
    const int id = ptune_dispatch_lw((int)set->shapes.size(), set->flat.data(), set->train_lg.data(), (int)k,
                                     set->ids.data(), set->cost.data(), lt, lq, M, N, K);
    if (id < 0) return fail(FF_ERR_NO_SET, "variant set has no training shapes");
    return id;
}

FF_EXPORT int variant_select(int64_t M, int64_t N, int64_t K) { return variant_select_form(0, M, N, K); }

FF_EXPORT int sgemm(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda, const float* B,
                    int64_t ldb, float beta, float* C, int64_t ldc, void* stream)
{
    return gemm_common(nullptr, 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream);
}

FF_EXPORT int sgemm_form(int form, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                         const float* B, int64_t ldb, float beta, float* C, int64_t ldc, void* stream)
{
    if (form < 0 || form >= kForms) return fail(FF_ERR_ARG, "sgemm_form: unknown form %d", form);
    return gemm_common(nullptr, form, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream);
}

FF_EXPORT int sgemm_variant(int id, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                            const float* B, int64_t ldb, float beta, float* C, int64_t ldc, void* stream)
{
    int rc = validate(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    if (rc != FF_OK) return rc;
    auto v = find_variant(id);
    if (!v) return fail(FF_ERR_VARIANT, "variant %d not registered", id);
    return gemm_common(v.get(), 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream);
}

FF_EXPORT int variant_work_groups(int id, int64_t M, int64_t N, int64_t K, int64_t* groups)
{
    if (groups == nullptr) return fail(FF_ERR_ARG, "variant_work_groups: groups is NULL");
    if (M < 0) return fail(FF_ERR_M, "variant_work_groups: M < 0");
    if (N < 0) return fail(FF_ERR_N, "variant_work_groups: N < 0");
    if (K < 0) return fail(FF_ERR_K, "variant_work_groups: K < 0");
    auto v = find_variant(id);
    if (!v) return fail(FF_ERR_VARIANT, "variant %d not registered", id);
    *groups = launch_groups(*v, M, N, K, current_workspace() != nullptr);
    return FF_OK;
}

FF_EXPORT int sgemm_time(int id, int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                         const float* B, int64_t ldb, float beta, float* C, int64_t ldc, void* stream, int warmup,
                         int reps, int trials, float* trial_ms)
{
    if (warmup < 0 || reps < 1 || trials < 1 || trial_ms == nullptr)
        return fail(FF_ERR_ARG, "sgemm_time: need warmup >= 0, reps >= 1, trials >= 1, trial_ms");
    int rc = validate(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    if (rc != FF_OK) return rc;
    auto v = find_variant(id);
    if (!v) return fail(FF_ERR_VARIANT, "variant %d not registered", id);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < warmup; ++i) {
        rc = gemm_common(v.get(), 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream);
        if (rc != FF_OK) return rc;
    }
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    rc = FF_OK;
    for (int t = 0; t < trials && rc == FF_OK; ++t) {
        e = hipEventRecord(e0, s);
        if (e != hipSuccess) { rc = hip_fail(e, "hipEventRecord"); break; }
        for (int r = 0; r < reps && rc == FF_OK; ++r)
            rc = gemm_common(v.get(), 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream);
        if (rc != FF_OK) break;
        e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { rc = hip_fail(e, "timing events"); break; }
        trial_ms[t] = ms / (float)reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

FF_EXPORT int screen_reference(int64_t M, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
                               const float* B, int64_t ldb, float beta, const float* C0, int64_t ldc0,
                               double* ref, double* tol, void* stream)
{
    if (M < 0 || N < 0 || K < 0 || lda < std::max<int64_t>(1, K) || ldb < std::max<int64_t>(1, N) ||
        (beta != 0.0f && (C0 == nullptr || ldc0 < std::max<int64_t>(1, N))) ||
        (alpha != 0.0f && K > 0 && M > 0 && N > 0 && (A == nullptr || B == nullptr)) ||
        (M * N > 0 && (ref == nullptr || tol == nullptr)))
        return fail(FF_ERR_ARG, "screen_reference: invalid arguments");
    if (M == 0 || N == 0) return FF_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t blocks = std::min<int64_t>((M * N + 255) / 256, 1 << 20);
    const int epi = (alpha != 1.0f || beta != 0.0f) ? 1 : 0;
    hipLaunchKernelGGL(ff_screen_ref, dim3((unsigned)blocks), dim3(256), 0, s, M, N, K, (double)alpha, A, lda, B,
                       ldb, (double)beta, C0, ldc0, ref, tol, epi);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? FF_OK : hip_fail(e, "screen_reference");
}

FF_EXPORT int screen_compare(int64_t M, int64_t N, const float* C, int64_t ldc, const double* ref,
                             const double* tol, double tol_scale, int64_t* nbad, double* max_ratio, double* err2,
                             double* ref2, void* stream)
{
    if (M < 0 || N < 0 || ldc < std::max<int64_t>(1, N) || nbad == nullptr || max_ratio == nullptr ||
        !(tol_scale > 0.0) || (M * N > 0 && (C == nullptr || ref == nullptr || tol == nullptr)))
        return fail(FF_ERR_ARG, "screen_compare: invalid arguments");
    *nbad = 0;
    *max_ratio = 0.0;
    if (err2) *err2 = 0.0;
    if (ref2) *ref2 = 0.0;
    if (M == 0 || N == 0) return FF_OK;
    static long long* d_bad = nullptr;
    static double* d_dbl = nullptr;  // ratio, err2, ref2 per block
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    hipError_t e = hipSuccess;
    if (d_bad == nullptr) {
        e = hipMalloc(&d_bad, kCmpBlocks * sizeof(long long));
        if (e == hipSuccess) e = hipMalloc(&d_dbl, 3 * kCmpBlocks * sizeof(double));
        if (e != hipSuccess) return hip_fail(e, "screen_compare alloc");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(ff_screen_cmp, dim3(kCmpBlocks), dim3(kCmpThreads), 0, s, M, N, C, ldc, ref, tol, tol_scale,
                       d_bad, d_dbl, d_dbl + kCmpBlocks, d_dbl + 2 * kCmpBlocks);
    std::vector<long long> hb(kCmpBlocks);
    std::vector<double> hd(3 * kCmpBlocks);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hb.data(), d_bad, kCmpBlocks * sizeof(long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hd.data(), d_dbl, 3 * kCmpBlocks * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "screen_compare");
    long long b = 0;
    double r = 0.0, e2 = 0.0, r2 = 0.0;
    for (int i = 0; i < kCmpBlocks; ++i) {
        b += hb[i];
        r = std::max(r, hd[i]);
        e2 += hd[kCmpBlocks + i];
        r2 += hd[2 * kCmpBlocks + i];
    }
    *nbad = b;
    *max_ratio = r;
    if (err2) *err2 = e2;
    if (ref2) *ref2 = r2;
    return FF_OK;
}

// ---------------------------------------------------------------------------
// Grouped persistent launches (many independent problems in one launch)

static_assert(sizeof(ff_gemm_desc) == 64, "descriptor layout shared with the kernels");

FF_EXPORT int sgemm_grouped_plan(int id, int count, ff_gemm_desc* descs, int32_t* prefix, int* vec_ok)
{
    if (count < 1 || descs == nullptr || prefix == nullptr)
        return fail(FF_ERR_ARG, "sgemm_grouped_plan: need count >= 1, descs and prefix");
    auto v = find_variant(id);
    if (!v) return fail(FF_ERR_VARIANT, "variant %d not registered", id);
    if (v->prec != 0) return fail(FF_ERR_ARG, "variant %d has no grouped form", id);
    bool vec = v->vw > 1;
    int64_t total = 0;
    for (int g = 0; g < count; ++g) {
        ff_gemm_desc& d = descs[g];
        if (d.M < 1 || d.N < 1 || d.K < 1 || d.A == nullptr || d.B == nullptr || d.C == nullptr || d.lda < d.K ||
            d.ldb < d.N || d.ldc < d.N)
            return fail(FF_ERR_ARG, "sgemm_grouped_plan: problem %d invalid (sizes >= 1, lda >= K, ldb >= N, "
                        "ldc >= N, non-null matrices)", g);
        const int64_t tiles = (int64_t)((d.M + v->mwg - 1) / v->mwg) * ((d.N + v->nwg - 1) / v->nwg);
        if (total + tiles > INT32_MAX) return fail(FF_ERR_TOO_LARGE, "sgemm_grouped_plan: too many tiles");
        d.tiles = (int32_t)tiles;
        prefix[g] = (int32_t)total;
        total += tiles;
        vec = vec && fp32_vector_ok(*v, d.N, d.K, d.lda, d.ldb, d.A, d.B);
    }
    if (vec_ok) *vec_ok = vec ? 1 : 0;
    return (int)total;
}

FF_EXPORT int sgemm_grouped(int id, int count, const ff_gemm_desc* descs, const int32_t* prefix, int total,
                            float alpha, float beta, int vec, void* stream)
{
    if (count < 1 || descs == nullptr || prefix == nullptr || total < 0)
        return fail(FF_ERR_ARG, "sgemm_grouped: need count >= 1, device descs and prefix, total >= 0");
    auto v = find_variant(id);
    if (!v) return fail(FF_ERR_VARIANT, "variant %d not registered", id);
    if (v->fgrp == nullptr) return fail(FF_ERR_ARG, "variant %d has no grouped form", id);
    if (total == 0) return FF_OK;
    const int blocks = std::min(total, v->grp_blocks);
    hipFunction_t f = vec ? v->fgrp : v->fgrp1;
    void* args[] = {(void*)&descs, (void*)&prefix, &count, &total, &alpha, &beta};
    hipError_t e = hipModuleLaunchKernel(f, (unsigned)blocks, 1, 1, (unsigned)v->threads(), 1, 1, 0,
                                         static_cast<hipStream_t>(stream), args, nullptr);
    return e == hipSuccess ? FF_OK : hip_fail(e, ("launch grouped " + v->name).c_str());
}
