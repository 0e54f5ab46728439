// SDF network with reflectiveness head (Sec. "Opaque density representation",
// "Signal representation"; App. C) on the MI355X matrix cores.
//
// Points are the GEMM's long dimension.  Every dense layer runs as an MFMA
// GEMM (v_mfma_f32_16x16x4_f32, or one of the 16-bit operand forms below) with
// the elementwise work of its neighbours fused into the operand loads
// (softplus, its derivative times a tangent or an adjoint, relu) and the bias /
// relu-mask / accumulate into its epilogue.
//
// Forward call: primal layers, then grad_x f by one reverse sweep
//   G^(8) = w_out, G^(l) = (softplus'(Z^(l)) . G^(l+1)) W_l, grad = J_PE^T G^(0).
// Backward call: J = sum g_f f + g_grad . grad_x f + g_a a.  Since
// g_grad . grad_x f is the directional derivative of f along g_grad, the
// parameter gradient is reverse mode over a primal + tangent forward pass
// (Z, H, Hdot = sp'(Z) Zdot per layer), giving per layer
//   Zdot_bar = sp'(Z) Hdot_bar,  Z_bar = sp'(Z) H_bar + sp''(Z) Zdot Hdot_bar,
//   W_bar = Z_bar^T H + Zdot_bar^T Hdot,  H_bar = Z_bar W,  Hdot_bar = Zdot_bar W,
// where sp''(Z) Zdot = beta sigma(-beta Z) Hdot, so Zdot itself is never stored.
// The training pair of calls keeps the forward's (Z, H) of every layer and the
// sweep's adjoint S = sp'(Z) G^(l+1) to every pre-activation in a caller-owned
// reserve; the backward then runs only the tangent GEMM per layer, and takes
// the tangent pass's adjoints from S (Zdot_bar = half_size S), so one adjoint
// GEMM per layer remains.
// Weight gradients reduce over points in fixed splits (no atomics).
#include <mutex>

#include "rfvr_impl.hpp"

namespace rfvr {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Eight FP32 operand values (two float4 along k) rounded to BF16 (RNE) for one
// v_mfma_f32_16x16x32_bf16.  A and B fragments use the same slot <-> k
// assignment, so the instruction's sum over its 32 slots is the sum over k.
__device__ __forceinline__ bf16x8 to_bf16x8(floatx4 lo, floatx4 hi) {
    bf16x8 r;
    r[0] = (__bf16)lo[0]; r[1] = (__bf16)lo[1]; r[2] = (__bf16)lo[2]; r[3] = (__bf16)lo[3];
    r[4] = (__bf16)hi[0]; r[5] = (__bf16)hi[1]; r[6] = (__bf16)hi[2]; r[7] = (__bf16)hi[3];
    return r;
}

// the same for one v_mfma_f32_16x16x32_f16 (FP16, RNE)
__device__ __forceinline__ f16x8 to_f16x8(floatx4 lo, floatx4 hi) {
    f16x8 r;
    r[0] = (_Float16)lo[0]; r[1] = (_Float16)lo[1]; r[2] = (_Float16)lo[2]; r[3] = (_Float16)lo[3];
    r[4] = (_Float16)hi[0]; r[5] = (_Float16)hi[1]; r[6] = (_Float16)hi[2]; r[7] = (_Float16)hi[3];
    return r;
}

// x = big + small with big = f16(x), small = f16(x - big): 22 significant bits
__device__ __forceinline__ void split_f16x8(floatx4 lo, floatx4 hi, f16x8& big, f16x8& small) {
    big = to_f16x8(lo, hi);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        small[e] = (_Float16)(lo[e] - (float)big[e]);
        small[4 + e] = (_Float16)(hi[e] - (float)big[4 + e]);
    }
}

// x = big + small with big = bf16(x), small = bf16(x - big): 16 significant bits
__device__ __forceinline__ void split_bf16x8(floatx4 lo, floatx4 hi, bf16x8& big, bf16x8& small) {
    big = to_bf16x8(lo, hi);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        small[e] = (__bf16)(lo[e] - (float)big[e]);
        small[4 + e] = (__bf16)(hi[e] - (float)big[4 + e]);
    }
}

// BF16 storage of the single-rounded BF16 backward's arrays (tangents Hdot and
// adjoints Zbar): the BF16 products that read them round them to BF16 (RNE)
// anyway, so they are stored rounded, as raw 16-bit words in buffers sized for
// FP32 (the few FP32 readers, the adjoint epilogue's Hdot and the encoding
// layer's FP32 weight-gradient product, see the rounded values), and widened
// where they are used (a main loop keeps the raw words of its prefetch and
// widens them at the LDS store, so the prefetch stays in flight)
__device__ __forceinline__ uint2 ld_raw_bf16x4(const float* base, long i) {
    return *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(base) + i);
}
__device__ __forceinline__ float4 widen_bf16x4(uint2 r) {
    return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                       __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
}
__device__ __forceinline__ float4 ld_bf16x4(const float* base, long i) { return widen_bf16x4(ld_raw_bf16x4(base, i)); }
__device__ __forceinline__ float ld_bf16(const float* base, long i) {
    return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(base)[i] << 16);
}
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ void st_bf16x4(float* base, long i, floatx4 v) {
    uint2 r;
    r.x = bf16_bits(v[0]) | (bf16_bits(v[1]) << 16);
    r.y = bf16_bits(v[2]) | (bf16_bits(v[3]) << 16);
    *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(base) + i) = r;
}
__device__ __forceinline__ void st_bf16(float* base, long i, float v) {
    reinterpret_cast<uint16_t*>(base)[i] = (uint16_t)bf16_bits(v);
}
// which operands of a GEMM are held in BF16 storage
enum { ST_A = 1, ST_B = 2, ST_C2 = 4, ST_Y = 8 };

// operand precision of a network GEMM: FP32 MFMA, BF16 MFMA, BF16 MFMA on split
// operands (a b ~ a_big b_big + a_big b_small + a_small b_big), or FP16 MFMA
// with the weights rounded once and the per-point operand split in two
// (a b ~ a_big b + a_small b, two products).  The per-point operand's rounding
// differs from point to point, and the opacity of neighbouring samples takes
// differences of their SDF values, which magnify it; the weights' rounding is
// a fixed, smooth change of the network.  FP16 serves the forward products only
// (its 5-bit exponent cannot hold the backward's adjoints, which scale with the
// upstream gradients); in the dual forward GEMM, MM_F16 means this form for
// the primal and BF16 for the tangent.
enum { MM_FP32 = 0, MM_BF16 = 1, MM_F16 = 2, MM_BF16X3 = 3 };

// operand prologues: identity, relu, or SEED: A[p][k] = H -> sp'(Z) colv[k] (the
// normal sweep's seed from the top layer's activation, formed while the tile is
// staged); the softplus activations themselves are written by the producing
// GEMM's epilogue, so no operand is transformed twice
enum { PRO_ID = 0, PRO_SEED = 1, PRO_RELU = 3 };
// epilogues (C = H = sp(Z) of a layer: sp'(Z) = 1 - e^(-beta H), e^(-beta Z) =
// 1 / (e^(beta H) - 1), so Z itself is never stored):
//            BIAS      Y = acc + bias
//            RELUMASK  Y = acc where C > 0, else 0
//            BIAS_SP   Y = softplus(acc + bias)                        (layer activation)
//            DSPMUL    Y = acc * sp'(Z)                                (normal sweep, tangent)
//            TOPADJ    Hbar = acc + scale rowv[p] colv[m], Hdotbar = scale colv[m] with
//                      C = H, C2 = Hdot of the top layer: Y = Zbar, Y2 = Zdotbar
//                      (the top trunk layer's adjoints)
//            ADJ1      Hbar = acc, Hdotbar = scale C3 / sp'(Z) with C = H, C2 = Hdot and
//                      C3 = the normal sweep's adjoint to Z of the layer below:
//                      Y = Zbar = sp'(Z) Hbar + beta sigma(-beta Z) Hdot Hdotbar
//                        = sp'(Z) Hbar + beta exp(-beta Z) Hdot scale C3
//                      (exp(-beta Z) capped at 1e30, where Hdot C3 is below 1e-60)
enum { EPI_BIAS = 0, EPI_RELUMASK = 2, EPI_BIAS_SP = 3, EPI_DSPMUL = 4, EPI_TOPADJ = 6, EPI_ADJ1 = 8 };

// Activation math of the network on the hardware exp2 / log2 / rcp units
// (v_exp_f32, v_log_f32, v_rcp_f32; ~1 ulp each): these run once per element
// in the GEMM epilogues and elementwise kernels, where the correctly rounded
// library forms would add several times their VALU work.
__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ float flog1p_pos(float e) {           // log(1 + e), e in [0, 1]
    return __builtin_amdgcn_logf(1.0f + e) * 0.6931471805599453f;
}
__device__ __forceinline__ float fsig(float x) { return __builtin_amdgcn_rcpf(1.0f + fexp(-x)); }
__device__ __forceinline__ float sp_f(float z, float beta) {
    const float bz = beta * z;
    return fmaxf(z, 0.0f) + flog1p_pos(fexp(-fabsf(bz))) * __builtin_amdgcn_rcpf(beta);
}
__device__ __forceinline__ float sp_d1(float z, float beta) { return fsig(beta * z); }
// sp'(Z) from H = sp(Z): e^(beta H) = 1 + e^(beta Z), so sp'(Z) = 1 - e^(-beta H)
// (absolute error ~1e-7, the rounding of the exponential near 1)
__device__ __forceinline__ float sp_d1_h(float h, float beta) { return 1.0f - fexp(-beta * h); }
__device__ __forceinline__ float sp_d2(float z, float beta) {
    const float s = fsig(beta * z);
    return beta * s * (1.0f - s);
}


// ----------------------------------------------------------------------------
// Y[P x M] = pro(A)[P x K] * B[M x K]^T  (+ epilogue).  K multiple of 32; A and
// B rows hold K valid or zero-padded columns; lda/ldb multiples of 4.
// Block 128 points x BM outputs, 4 waves, 16x16x4 MFMA tiles, K chunks of 32
// staged through LDS with the next chunk's global loads in flight during the
// current chunk's MFMAs.  The k index of a lane's MFMA operand is permuted so
// each lane reads 4 consecutive k (one float4) per 16-wide k group.
// ----------------------------------------------------------------------------
struct GemmArgs {
    const float* A; long lda;
    const float* B; long ldb;
    const float* bias;            // EPI_BIAS*: [M] or null
    const float* C;               // EPI_RELUMASK / DSPMUL / TOPADJ: [P][ldc]
    const float* C2;              // EPI_TOPADJ, ADJ1: [P][ldc]
    const float* C3;              // EPI_ADJ1: [P][ldc]
    long ldc;
    float* Y; long ldy;
    float* Y2;                    // EPI_TOPADJ: second output, row stride ldy
    const float* rowv;            // EPI_TOPADJ: [P] or null
    const float* colv;            // EPI_TOPADJ: [M]; PRO_SEED: [K]
    float scale;                  // EPI_TOPADJ, ADJ1
    float* cpart;                 // EPI_TOPADJ: [point tiles][M] column partials of
                                  // rowv[p] scale C + scale C2 (one row per tile), or null
    long P; int M; int K;
    float beta;
};

template <int PRO, int EPI, int BM, int MM, int ST = 0>
__global__ __launch_bounds__(256) void k_gemm_nt(GemmArgs g) {
    // padded LDS rows (BK + 4 floats): the MFMA fragment reads (16 rows, one
    // float4 column) are free of bank conflicts.  Variants measured slower on
    // this shape: an XOR-swizzled unpadded layout, two LDS buffers with one
    // barrier per chunk, 64-deep chunks (all at two waves per SIMD, against
    // three here).
    constexpr int BP = 128, BK = 32, LW = BK + 4, RPF = BK / 4;
    constexpr int WP = (BM == 128) ? 2 : 4;
    constexpr int WM = 4 / WP;
    constexpr int TP = BP / WP / 16;
    constexpr int TM = BM / WM / 16;
    constexpr int NA = BP * BK / 4 / 256;       // float4 per thread, A
    constexpr int NB = BM * BK / 4 / 256;       // float4 per thread, B
    __shared__ float sA[BP * LW];
    __shared__ float sB[BM * LW];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int wp = wv % WP, wm = wv / WP;
    const int li = lane & 15, lg = lane >> 4;
    // Work-groups are dispatched round-robin over the 8 XCDs (id % 8).  The
    // column blocks of one point tile read the same A rows, so they are given
    // ids b, b+8, ... : same XCD (same L2), consecutive in dispatch order.
    const int nmb = (g.M + BM - 1) / BM;
    const long bid = blockIdx.x;
    const long grp = bid / (8L * nmb);
    const int within = (int)(bid % (8L * nmb));
    const int mb = within / 8;
    const long pt = grp * 8 + (within % 8);
    const long p0 = pt * BP;
    const int m0 = mb * BM;
    if (p0 >= g.P) return;                       // padding work-groups of the last group
    floatx4 acc[TP][TM];
#pragma unroll
    for (int a = 0; a < TP; ++a)
#pragma unroll
        for (int b = 0; b < TM; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    float4 ra[(ST & ST_A) ? 1 : NA], rb[NB];
    uint2 ra16[(ST & ST_A) ? NA : 1];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int e = tid + i * 256;
            const int row = e / RPF, c4 = (e % RPF) * 4;
            const long p = p0 + row;
            if constexpr ((ST & ST_A) != 0) {
                ra16[i] = make_uint2(0u, 0u);
                if (p < g.P) ra16[i] = ld_raw_bf16x4(g.A, p * g.lda + k0 + c4);
            } else {
                ra[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (p < g.P) ra[i] = *reinterpret_cast<const float4*>(g.A + p * g.lda + k0 + c4);
            }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + i * 256;
            const int row = e / RPF, c4 = (e % RPF) * 4;
            const int m = m0 + row;
            rb[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (m < g.M) rb[i] = *reinterpret_cast<const float4*>(g.B + (long)m * g.ldb + k0 + c4);
        }
    };
    auto off = [](int row, int q) { return row * LW + 4 * q; };
    auto store = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int e = tid + i * 256;
            float4 v;
            if constexpr ((ST & ST_A) != 0) v = widen_bf16x4(ra16[i]);
            else v = ra[i];
            if constexpr (PRO == PRO_RELU) {
                v.x = fmaxf(v.x, 0.0f); v.y = fmaxf(v.y, 0.0f); v.z = fmaxf(v.z, 0.0f); v.w = fmaxf(v.w, 0.0f);
            }
            if constexpr (PRO == PRO_SEED) {
                const float* w = g.colv + k0 + (e % RPF) * 4;
                v.x = sp_d1_h(v.x, g.beta) * w[0]; v.y = sp_d1_h(v.y, g.beta) * w[1];
                v.z = sp_d1_h(v.z, g.beta) * w[2]; v.w = sp_d1_h(v.w, g.beta) * w[3];
            }
            *reinterpret_cast<float4*>(&sA[off(e / RPF, e % RPF)]) = v;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + i * 256;
            *reinterpret_cast<float4*>(&sB[off(e / RPF, e % RPF)]) = rb[i];
        }
    };
    auto compute = [&]() {
        const float* A_ = sA;
        const float* B_ = sB;
        if constexpr (MM == MM_BF16) {
            // the chunk's two 16-wide k groups feed one 16x16x32 BF16 MFMA
            bf16x8 af[TP], bf[TM];
#pragma unroll
            for (int a = 0; a < TP; ++a) {
                const int row = wp * (BP / WP) + a * 16 + li;
                af[a] = to_bf16x8(*reinterpret_cast<const floatx4*>(&A_[off(row, lg)]),
                                  *reinterpret_cast<const floatx4*>(&A_[off(row, lg + 4)]));
            }
#pragma unroll
            for (int b = 0; b < TM; ++b) {
                const int row = wm * (BM / WM) + b * 16 + li;
                bf[b] = to_bf16x8(*reinterpret_cast<const floatx4*>(&B_[off(row, lg)]),
                                  *reinterpret_cast<const floatx4*>(&B_[off(row, lg + 4)]));
            }
#pragma unroll
            for (int a = 0; a < TP; ++a)
#pragma unroll
                for (int b = 0; b < TM; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[b], af[a], acc[a][b], 0, 0, 0);
        } else if constexpr (MM == MM_F16) {
            // one point row's split at a time (fewer live registers)
            f16x8 bf[TM];
#pragma unroll
            for (int b = 0; b < TM; ++b) {
                const int row = wm * (BM / WM) + b * 16 + li;
                bf[b] = to_f16x8(*reinterpret_cast<const floatx4*>(&B_[off(row, lg)]),
                                 *reinterpret_cast<const floatx4*>(&B_[off(row, lg + 4)]));
            }
#pragma unroll
            for (int a = 0; a < TP; ++a) {
                const int row = wp * (BP / WP) + a * 16 + li;
                f16x8 ab, as;
                split_f16x8(*reinterpret_cast<const floatx4*>(&A_[off(row, lg)]),
                            *reinterpret_cast<const floatx4*>(&A_[off(row, lg + 4)]), ab, as);
#pragma unroll
                for (int b = 0; b < TM; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bf[b], as, acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bf[b], ab, acc[a][b], 0, 0, 0);
                }
            }
        } else if constexpr (MM == MM_BF16X3) {
            bf16x8 ab[TP], as[TP], bb[TM], bs[TM];
#pragma unroll
            for (int a = 0; a < TP; ++a) {
                const int row = wp * (BP / WP) + a * 16 + li;
                split_bf16x8(*reinterpret_cast<const floatx4*>(&A_[off(row, lg)]),
                             *reinterpret_cast<const floatx4*>(&A_[off(row, lg + 4)]), ab[a], as[a]);
            }
#pragma unroll
            for (int b = 0; b < TM; ++b) {
                const int row = wm * (BM / WM) + b * 16 + li;
                split_bf16x8(*reinterpret_cast<const floatx4*>(&B_[off(row, lg)]),
                             *reinterpret_cast<const floatx4*>(&B_[off(row, lg + 4)]), bb[b], bs[b]);
            }
#pragma unroll
            for (int a = 0; a < TP; ++a)
#pragma unroll
                for (int b = 0; b < TM; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bb[b], as[a], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bs[b], ab[a], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bb[b], ab[a], acc[a][b], 0, 0, 0);
                }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 16) {
                floatx4 af[TP], bf[TM];
#pragma unroll
                for (int a = 0; a < TP; ++a)
                    af[a] = *reinterpret_cast<const floatx4*>(&A_[off(wp * (BP / WP) + a * 16 + li, kk / 4 + lg)]);
#pragma unroll
                for (int b = 0; b < TM; ++b)
                    bf[b] = *reinterpret_cast<const floatx4*>(&B_[off(wm * (BM / WM) + b * 16 + li, kk / 4 + lg)]);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int a = 0; a < TP; ++a)
#pragma unroll
                        for (int b = 0; b < TM; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[b][s], af[a][s], acc[a][b], 0, 0, 0);
            }
        }
    };
    // one LDS buffer: store, barrier, next chunk's global loads in flight
    // during this chunk's MFMAs, barrier
    load(0);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        store(k0);
        __syncthreads();
        if (k0 + BK < g.K) load(k0 + BK);
        compute();
        __syncthreads();
    }
    // Epilogue.  The weights are the MFMA's first operand, so a lane's four
    // accumulator values acc[a][b][0..3] are four consecutive outputs
    // m = m0 + wm (BM/WM) + 16 b + 4 lg + v of one point p = p0 + wp (BP/WP)
    // + 16 a + li: one float4 of a row-major [P][ld] array.  Tiles wholly inside
    // the output (with 16-byte aligned rows) load and store float4s without
    // guards; the others clamp their loads into the arrays and guard each
    // store.  A 16-point group's loads are all issued before the first is used.
    constexpr int NC = (EPI == EPI_ADJ1) ? 3 : (EPI == EPI_TOPADJ) ? 2 : (EPI == EPI_DSPMUL || EPI == EPI_RELUMASK) ? 1 : 0;
    auto epilogue = [&](auto guarded) {
        constexpr bool GUARD = decltype(guarded)::value;
        // per-output vector (bias, or the top adjoint's column vector): the same
        // 16 values for every point group of the lane, loaded once
        constexpr bool VEC = (EPI == EPI_BIAS || EPI == EPI_BIAS_SP || EPI == EPI_TOPADJ);
        const float* vsrc = (EPI == EPI_TOPADJ) ? g.colv : g.bias;
        floatx4 vv[VEC ? TM : 1];
        if constexpr (VEC) {
#pragma unroll
            for (int b = 0; b < TM; ++b) {
                const int mb = m0 + wm * (BM / WM) + b * 16 + lg * 4;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    vv[b][v] = vsrc ? vsrc[GUARD ? min(mb + v, g.M - 1) : mb + v] : 0.0f;
            }
        }
#pragma unroll
        for (int a = 0; a < TP; ++a) {
            const long p = p0 + wp * (BP / WP) + a * 16 + li;
            const bool pin = !GUARD || p < g.P;
            const long pr = pin ? p : g.P - 1;
            floatx4 cl[NC ? NC : 1][TM];
            const float* src[3] = {g.C, g.C2, g.C3};
            if constexpr (NC > 0 && !GUARD) {
#pragma unroll
                for (int b = 0; b < TM; ++b) {
                    const int mb = m0 + wm * (BM / WM) + b * 16 + lg * 4;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        if ((ST & ST_C2) != 0 && c == 1) {
                            const float4 t = ld_bf16x4(src[c], pr * g.ldc + mb);
                            cl[c][b] = floatx4{t.x, t.y, t.z, t.w};
                        } else {
                            cl[c][b] = *reinterpret_cast<const floatx4*>(src[c] + pr * g.ldc + mb);
                        }
                    }
                }
            }
            float rv = 0.0f;
            if constexpr (EPI == EPI_TOPADJ) rv = g.rowv ? g.scale * g.rowv[pr] : 0.0f;
#pragma unroll
            for (int b = 0; b < TM; ++b) {
                const int mb = m0 + wm * (BM / WM) + b * 16 + lg * 4;
                if constexpr (NC > 0 && GUARD) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const long ci = pr * g.ldc + min(mb + v, g.M - 1);
                            cl[c][b][v] = ((ST & ST_C2) != 0 && c == 1) ? ld_bf16(src[c], ci) : src[c][ci];
                        }
                }
                floatx4 y = acc[a][b], y2 = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if constexpr (EPI == EPI_BIAS || EPI == EPI_BIAS_SP) y[v] += vv[b][v];
                    if constexpr (EPI == EPI_BIAS_SP) y[v] = sp_f(y[v], g.beta);
                    if constexpr (EPI == EPI_RELUMASK) y[v] = cl[0][b][v] > 0.0f ? y[v] : 0.0f;
                    if constexpr (EPI == EPI_DSPMUL) y[v] *= sp_d1_h(cl[0][b][v], g.beta);
                    if constexpr (EPI == EPI_TOPADJ) {
                        const float cv = vv[b][v];
                        const float hb = __builtin_fmaf(rv, cv, y[v]);
                        const float hdb = g.scale * cv;
                        const float em = fexp(-g.beta * cl[0][b][v]);   // 1 - sp'(Z)
                        const float sg = 1.0f - em;
                        y[v] = sg * hb + g.beta * em * cl[1][b][v] * hdb;
                        y2[v] = sg * hdb;
                    }
                    if constexpr (EPI == EPI_ADJ1) {
                        // the sweep kept S = sp'(Z) G, so sigma(-beta Z) G = exp(-beta Z) S,
                        // with exp(-beta Z) = 1 / (e^(beta H) - 1)
                        const float bh = g.beta * cl[0][b][v];
                        const float ex = __builtin_amdgcn_rcpf(fexp(bh) - 1.0f);
                        const float sg = 1.0f - fexp(-bh);
                        y[v] = sg * y[v] + g.beta * fminf(ex, 1e30f) * cl[1][b][v] * (g.scale * cl[2][b][v]);
                    }
                }
                constexpr bool TWO = (EPI == EPI_TOPADJ);
                constexpr bool YB = (ST & ST_Y) != 0;
                if constexpr (!GUARD) {
                    if constexpr (YB) st_bf16x4(g.Y, p * g.ldy + mb, y);
                    else *reinterpret_cast<floatx4*>(g.Y + p * g.ldy + mb) = y;
                    if constexpr (TWO) *reinterpret_cast<floatx4*>(g.Y2 + p * g.ldy + mb) = y2;
                } else if (pin) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (mb + v >= g.M) continue;
                        if constexpr (YB) st_bf16(g.Y, p * g.ldy + mb + v, y[v]);
                        else g.Y[p * g.ldy + mb + v] = y[v];
                        if constexpr (TWO) g.Y2[p * g.ldy + mb + v] = y2[v];
                    }
                }
                if constexpr (GUARD && NC >= 2) __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (EPI == EPI_TOPADJ) {
                if (g.cpart) {
                    // the group's share of the output layer's weight gradient,
                    // sum_p (rowv[p] scale H + scale Hdot) per column: a fixed-order
                    // sum over the 16 lanes of the same columns (lane bits 0-3:
                    // the points), one row per (group, wave) into LDS
#pragma unroll
                    for (int b = 0; b < TM; ++b) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            float c = pin ? __builtin_fmaf(rv, cl[0][b][v], g.scale * cl[1][b][v]) : 0.0f;
#pragma unroll
                            for (int o = 1; o < 16; o <<= 1) c += __shfl_xor(c, o);
                            if (li == 0) sA[(a * 4 + wv) * (BM / WM) + b * 16 + lg * 4 + v] = c;
                        }
                    }
                }
            }
            // the next group's loads stay behind this group's stores
            if constexpr (NC >= 2) __builtin_amdgcn_sched_barrier(0);
        }
    };
    const bool aligned = (((g.ldy | g.ldc) & 3) == 0) &&
                         (((uintptr_t)g.Y | (uintptr_t)g.Y2 | (uintptr_t)g.C | (uintptr_t)g.C2 | (uintptr_t)g.C3) & 15) == 0;
    if (aligned && p0 + BP <= g.P && m0 + BM <= g.M) epilogue(std::false_type{});
    else epilogue(std::true_type{});
    if constexpr (EPI == EPI_TOPADJ) {
        if (g.cpart) {
            // the tile's column sums: one thread per column adds the rows of
            // its waves along points and their groups in a fixed order (the LDS
            // tiles were last read before the main loop's final barrier; the
            // rows above were written after it); one partial row per tile
            __syncthreads();
            if (tid < BM) {
                const int wmc = tid / (BM / WM), col = tid % (BM / WM);
                float t = 0.0f;
                for (int q = 0; q < WP; ++q)
                    for (int a = 0; a < TP; ++a) t += sA[(a * 4 + (wmc * WP + q)) * (BM / WM) + col];
                if (m0 + tid < g.M) g.cpart[(p0 / BP) * (long)g.M + m0 + tid] = t;
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Two products with one B operand, Y = A B^T and Yd = A2 B^T (a layer's primal
// and tangent, or the two adjoints of its input), the layer's elementwise work
// in the epilogue:
//   EPI2_FWD: Z = acc + bias, H = sp(Z), Hdot = sp'(Z) acc2     -> Y, Y2, Y3
//   EPI2_ADJ: Hbar = acc, Hdotbar = acc2 with C = Z, C2 = Hdot of the layer below:
//             Zbar = sp'(Z) Hbar + beta sigma(-beta Z) Hdot Hdotbar,
//             Zdotbar = sp'(Z) Hdotbar                         -> Y, Y2
// Tiling as k_gemm_nt with BM = 128; the B tile is staged once for both.
// ----------------------------------------------------------------------------
enum { EPI2_FWD = 0, EPI2_ADJ = 1 };

struct DualArgs {
    const float* A; const float* A2; long lda;
    const float* B; long ldb;
    const float* bias;
    const float* C; const float* C2;        // EPI2_ADJ: [P][ldy]
    float* Y; float* Y2; float* Y3; long ldy;
    long P; int M; int K;
    float beta;
};

template <int EPI2, int MM, int NW>
__global__ __launch_bounds__(NW * 64, NW == 4 ? 2 : 1) void k_gemm_dual(DualArgs g) {
    // NW = 8: 4 waves along points x 2 along outputs, 128 x 128 block; NW = 4:
    // 2 x 2 waves, 64 x 128 block.  2 x 4 tiles of 16 x 16 per wave and two
    // accumulator sets (64 registers) either way.
    constexpr int NT = NW * 64;
    constexpr int BP = NW == 8 ? 128 : 64, BM = 128, BK = 32, LW = BK + 4;
    constexpr int WP = NW / 2, TP = BP / WP / 16, TM = BM / 2 / 16;
    constexpr int NA = BP * BK / 4 / NT, NB = BM * BK / 4 / NT;
    __shared__ float sA[BP * LW];
    __shared__ float sA2[BP * LW];
    __shared__ float sB[BM * LW];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int wp = wv % WP, wm = wv / WP;
    const int li = lane & 15, lg = lane >> 4;
    const int nmb = (g.M + BM - 1) / BM;
    const long bid = blockIdx.x;
    const long grp = bid / (8L * nmb);
    const int within = (int)(bid % (8L * nmb));
    const int mb = within / 8;
    const long pt = grp * 8 + (within % 8);
    const long p0 = pt * BP;
    const int m0 = mb * BM;
    if (p0 >= g.P) return;                       // padding work-groups of the last group
    floatx4 acc[TP][TM], acd[TP][TM];
#pragma unroll
    for (int a = 0; a < TP; ++a)
#pragma unroll
        for (int b = 0; b < TM; ++b) {
            acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            acd[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    // the adjoint epilogue's operands (Z and Hdot of the layer below) do not
    // depend on the products: fetch them before the main loop
    float cz[TP][TM][4], chd[TP][TM][4];
    if constexpr (EPI2 == EPI2_ADJ) {
#pragma unroll
        for (int a = 0; a < TP; ++a)
#pragma unroll
            for (int b = 0; b < TM; ++b) {
                const int m = m0 + wm * (BM / 2) + b * 16 + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const long p = p0 + wp * (BP / WP) + a * 16 + lg * 4 + v;
                    const bool in = m < g.M && p < g.P;
                    cz[a][b][v] = in ? g.C[p * g.ldy + m] : 0.0f;
                    chd[a][b][v] = in ? g.C2[p * g.ldy + m] : 0.0f;
                }
            }
    }
    float4 ra[NA], ra2[NA], rb[NB];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int e = tid + i * NT;
            const int row = e >> 3, c4 = (e & 7) * 4;
            const long p = p0 + row;
            ra[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            ra2[i] = ra[i];
            if (p < g.P) {
                const long off = p * g.lda + k0 + c4;
                ra[i] = *reinterpret_cast<const float4*>(g.A + off);
                ra2[i] = *reinterpret_cast<const float4*>(g.A2 + off);
            }
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + i * NT;
            const int row = e >> 3, c4 = (e & 7) * 4;
            const int m = m0 + row;
            rb[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (m < g.M) rb[i] = *reinterpret_cast<const float4*>(g.B + (long)m * g.ldb + k0 + c4);
        }
    };
    load(0);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int e = tid + i * NT;
            const int row = e >> 3, c4 = (e & 7) * 4;
            *reinterpret_cast<float4*>(&sA[row * LW + c4]) = ra[i];
            *reinterpret_cast<float4*>(&sA2[row * LW + c4]) = ra2[i];
        }
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int e = tid + i * NT;
            const int row = e >> 3, c4 = (e & 7) * 4;
            *reinterpret_cast<float4*>(&sB[row * LW + c4]) = rb[i];
        }
        __syncthreads();
        if (k0 + BK < g.K) load(k0 + BK);
        if constexpr (MM == MM_FP32) {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 16) {
                floatx4 af[TP], af2[TP], bf[TM];
#pragma unroll
                for (int a = 0; a < TP; ++a) {
                    const int r = (wp * (BP / WP) + a * 16 + li) * LW + kk + lg * 4;
                    af[a] = *reinterpret_cast<const floatx4*>(&sA[r]);
                    af2[a] = *reinterpret_cast<const floatx4*>(&sA2[r]);
                }
#pragma unroll
                for (int b = 0; b < TM; ++b)
                    bf[b] = *reinterpret_cast<const floatx4*>(&sB[(wm * (BM / 2) + b * 16 + li) * LW + kk + lg * 4]);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int a = 0; a < TP; ++a)
#pragma unroll
                        for (int b = 0; b < TM; ++b) {
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a][s], bf[b][s], acc[a][b], 0, 0, 0);
                            acd[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af2[a][s], bf[b][s], acd[a][b], 0, 0, 0);
                        }
            }
        } else if constexpr (MM == MM_F16) {
            // primal on FP16 operands (split per-point operand), tangent on BF16
            // (the tangent scales with the upstream gradient): the staged
            // weights are rounded both ways
            f16x8 bh[TM];
            bf16x8 bb[TM];
#pragma unroll
            for (int b = 0; b < TM; ++b) {
                const float* r = &sB[(wm * (BM / 2) + b * 16 + li) * LW + lg * 4];
                const floatx4 lo = *reinterpret_cast<const floatx4*>(r), hi = *reinterpret_cast<const floatx4*>(r + 16);
                bh[b] = to_f16x8(lo, hi);
                bb[b] = to_bf16x8(lo, hi);
            }
#pragma unroll
            for (int a = 0; a < TP; ++a) {
                const int off = (wp * (BP / WP) + a * 16 + li) * LW + lg * 4;
                f16x8 ah, al;
                split_f16x8(*reinterpret_cast<const floatx4*>(&sA[off]),
                            *reinterpret_cast<const floatx4*>(&sA[off + 16]), ah, al);
                const bf16x8 ad = to_bf16x8(*reinterpret_cast<const floatx4*>(&sA2[off]),
                                            *reinterpret_cast<const floatx4*>(&sA2[off + 16]));
#pragma unroll
                for (int b = 0; b < TM; ++b) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[b], acc[a][b], 0, 0, 0);
                    acd[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ad, bb[b], acd[a][b], 0, 0, 0);
                }
            }
        } else {
            bf16x8 bb[TM], bs[TM];
#pragma unroll
            for (int b = 0; b < TM; ++b) {
                const float* r = &sB[(wm * (BM / 2) + b * 16 + li) * LW + lg * 4];
                if constexpr (MM == MM_BF16)
                    bb[b] = to_bf16x8(*reinterpret_cast<const floatx4*>(r), *reinterpret_cast<const floatx4*>(r + 16));
                else
                    split_bf16x8(*reinterpret_cast<const floatx4*>(r), *reinterpret_cast<const floatx4*>(r + 16), bb[b], bs[b]);
            }
#pragma unroll
            for (int a = 0; a < TP; ++a) {
                const int off = (wp * (BP / WP) + a * 16 + li) * LW + lg * 4;
#pragma unroll
                for (int which = 0; which < 2; ++which) {
                    const float* r = which ? &sA2[off] : &sA[off];
                    floatx4* dst = which ? acd[a] : acc[a];
                    if constexpr (MM == MM_BF16) {
                        const bf16x8 ab = to_bf16x8(*reinterpret_cast<const floatx4*>(r), *reinterpret_cast<const floatx4*>(r + 16));
#pragma unroll
                        for (int b = 0; b < TM; ++b)
                            dst[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb[b], dst[b], 0, 0, 0);
                    } else {
                        bf16x8 ab, as;
                        split_bf16x8(*reinterpret_cast<const floatx4*>(r), *reinterpret_cast<const floatx4*>(r + 16), ab, as);
#pragma unroll
                        for (int b = 0; b < TM; ++b) {
                            dst[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as, bb[b], dst[b], 0, 0, 0);
                            dst[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bs[b], dst[b], 0, 0, 0);
                            dst[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb[b], dst[b], 0, 0, 0);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < TP; ++a)
#pragma unroll
        for (int b = 0; b < TM; ++b) {
            const int m = m0 + wm * (BM / 2) + b * 16 + li;
            if (m >= g.M) continue;
            const float bias = (EPI2 == EPI2_FWD && g.bias) ? g.bias[m] : 0.0f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long p = p0 + wp * (BP / WP) + a * 16 + lg * 4 + v;
                if (p >= g.P) continue;
                const long o = p * g.ldy + m;
                if constexpr (EPI2 == EPI2_FWD) {
                    const float z = acc[a][b][v] + bias;
                    g.Y[o] = z;
                    g.Y2[o] = sp_f(z, g.beta);
                    g.Y3[o] = sp_d1(z, g.beta) * acd[a][b][v];
                } else {
                    const float z = cz[a][b][v], hd = chd[a][b][v];
                    const float sg = fsig(g.beta * z);
                    const float hb = acc[a][b][v], hdb = acd[a][b][v];
                    g.Y[o] = sg * hb + g.beta * (1.0f - sg) * hd * hdb;
                    g.Y2[o] = sg * hdb;
                }
            }
        }
}

// ----------------------------------------------------------------------------
// Weight gradient partials: part[split][M][Kout] = sum over the split's points
// of A[p][m] * pro(B)[p][k], and with BIAS also bpart[split][m] = sum_p A[p][m].
// Block 128 (m) x 128 (k), chunks of 32 points kept point-major in LDS (float4
// stores, scalar MFMA operand reads along the point index), next chunk's loads
// in flight during the current chunk's MFMAs.
// ----------------------------------------------------------------------------
struct WgArgs {
    const float* A; long lda;                  // [P][lda], columns 0..M-1
    const float* B; const float* B2; long ldb; // [P][ldb], columns 0..Kout-1
    float* part;                               // [n_split][M][Kout]
    float* bpart;                              // [n_split][M] (BIAS)
    long P; int M; int Kout; long per_split;
    int n_split;
    float beta;
};

template <int PRO, bool BIAS, int MM, int ST = 0>
__global__ __launch_bounds__(256, MM == MM_BF16 ? 3 : 1) void k_gemm_wg(WgArgs g) {
    constexpr int BM = 128, BN = 128, BK = 32, LW = 128 + 4;
    __shared__ float sA[BK * LW];
    __shared__ float sB[BK * LW];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int wp = wv % 2, wn = wv / 2;
    const int li = lane & 15, lg = lane >> 4;
    // the (m, n) blocks of one point split share operand rows: ids 8 apart,
    // same XCD, consecutive in dispatch order
    const int nmb = (g.M + BM - 1) / BM, nnb = (g.Kout + BN - 1) / BN;
    const long bid = blockIdx.x;
    const long grp = bid / (8L * nmb * nnb);
    const int within = (int)(bid % (8L * nmb * nnb));
    const int tile = within / 8;
    const long split = grp * 8 + (within % 8);
    if (split >= g.n_split) return;              // padding work-groups of the last group
    const int m0 = (tile % nmb) * BM, n0 = (tile / nmb) * BN;
    const bool first_n = (tile / nmb) == 0;
    const long pb = split * g.per_split;
    long pe = pb + g.per_split;
    if (pe > g.P) pe = g.P;
    floatx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;                         // column sum of A (thread tid < 128 -> column tid)

    // raw 16-bit words of a BF16-stored operand's prefetch, widened at the LDS store
    float4 ra[(ST & ST_A) ? 1 : 4], rb[(ST & ST_B) ? 1 : 4];
    uint2 ra16[(ST & ST_A) ? 4 : 1], rb16[(ST & ST_B) ? 4 : 1];
    auto load = [&](long q0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * 256;
            const int row = e >> 5, c4 = (e & 31) * 4;
            const long p = q0 + row;
            if constexpr (ST == 0) {
                ra[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                rb[i] = ra[i];
                if (p < pe) {
                    if (m0 + c4 < g.M) ra[i] = *reinterpret_cast<const float4*>(g.A + p * g.lda + m0 + c4);
                    if (n0 + c4 < g.Kout) {
                        const long off = p * g.ldb + n0 + c4;
                        rb[i] = *reinterpret_cast<const float4*>(g.B + off);
                    }
                }
            } else {
                const bool la = p < pe && m0 + c4 < g.M, lb = p < pe && n0 + c4 < g.Kout;
                if constexpr ((ST & ST_A) != 0) ra16[i] = la ? ld_raw_bf16x4(g.A, p * g.lda + m0 + c4) : make_uint2(0u, 0u);
                else ra[i] = la ? *reinterpret_cast<const float4*>(g.A + p * g.lda + m0 + c4) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if constexpr ((ST & ST_B) != 0) rb16[i] = lb ? ld_raw_bf16x4(g.B, p * g.ldb + n0 + c4) : make_uint2(0u, 0u);
                else rb[i] = lb ? *reinterpret_cast<const float4*>(g.B + p * g.ldb + n0 + c4) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
    };
    if (pb < pe) load(pb);
    for (long q0 = pb; q0 < pe; q0 += BK) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = tid + i * 256;
            const int row = e >> 5, c4 = (e & 31) * 4;
            const bool live = q0 + row < pe;
            float4 v, u;
            if constexpr ((ST & ST_B) != 0) v = widen_bf16x4(rb16[i]);
            else v = rb[i];
            if constexpr ((ST & ST_A) != 0) u = widen_bf16x4(ra16[i]);
            else u = ra[i];
            if constexpr (PRO == PRO_RELU) {
                v.x = fmaxf(v.x, 0.0f); v.y = fmaxf(v.y, 0.0f); v.z = fmaxf(v.z, 0.0f); v.w = fmaxf(v.w, 0.0f);
            }
            if (!live) v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            *reinterpret_cast<float4*>(&sA[row * LW + c4]) = u;
            *reinterpret_cast<float4*>(&sB[row * LW + c4]) = v;
        }
        __syncthreads();
        if (q0 + BK < pe) load(q0 + BK);
        if constexpr (BIAS) {
            if (first_n && tid < BM) {
#pragma unroll 8
                for (int r = 0; r < BK; ++r) bsum += sA[r * LW + tid];
            }
        }
        if constexpr (MM == MM_BF16) {
            // points lg*4 + s and 16 + lg*4 + s (s < 4) fill the 8 k slots of a
            // lane; the B fragments are converted first and each A fragment
            // just before its products (scheduling barriers keep the order), so
            // that three waves fit on a SIMD
            bf16x8 bf[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                floatx4 b0, b1;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int r = lg * 4 + s;
                    b0[s] = sB[r * LW + wn * 64 + b * 16 + li];
                    b1[s] = sB[(r + 16) * LW + wn * 64 + b * 16 + li];
                }
                bf[b] = to_bf16x8(b0, b1);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                __builtin_amdgcn_sched_barrier(0);
                floatx4 a0, a1;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int r = lg * 4 + s;
                    a0[s] = sA[r * LW + wp * 64 + a * 16 + li];
                    a1[s] = sA[(r + 16) * LW + wp * 64 + a * 16 + li];
                }
                const bf16x8 af = to_bf16x8(a0, a1);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[b], acc[a][b], 0, 0, 0);
            }
        } else if constexpr (MM != MM_FP32) {
            // points lg*4 + s and 16 + lg*4 + s (s < 4) fill the 8 k slots of a lane
            floatx4 a0[4], a1[4], b0[4], b1[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int r = lg * 4 + s;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    a0[a][s] = sA[r * LW + wp * 64 + a * 16 + li];
                    a1[a][s] = sA[(r + 16) * LW + wp * 64 + a * 16 + li];
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    b0[b][s] = sB[r * LW + wn * 64 + b * 16 + li];
                    b1[b][s] = sB[(r + 16) * LW + wn * 64 + b * 16 + li];
                }
            }
            {
                bf16x8 ab[4], as[4], bb[4], bs[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) split_bf16x8(a0[a], a1[a], ab[a], as[a]);
#pragma unroll
                for (int b = 0; b < 4; ++b) split_bf16x8(b0[b], b1[b], bb[b], bs[b]);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as[a], bb[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab[a], bs[b], acc[a][b], 0, 0, 0);
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab[a], bb[b], acc[a][b], 0, 0, 0);
                    }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 16) {
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int r = kk + lg * 4 + s;
                    float af[4], bf[4];
#pragma unroll
                    for (int a = 0; a < 4; ++a) af[a] = sA[r * LW + wp * 64 + a * 16 + li];
#pragma unroll
                    for (int b = 0; b < 4; ++b) bf[b] = sB[r * LW + wn * 64 + b * 16 + li];
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b], acc[a][b], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    float* out = g.part + split * (long)g.M * g.Kout;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = n0 + wn * 64 + b * 16 + li;
            if (k >= g.Kout) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wp * 64 + a * 16 + lg * 4 + v;
                if (m < g.M) out[(long)m * g.Kout + k] = acc[a][b][v];
            }
        }
    if constexpr (BIAS) {
        if (first_n && tid < BM && m0 + tid < g.M) g.bpart[split * (long)g.M + m0 + tid] = bsum;
    }
}

// dst[m][k] (row stride k_real, k < k_real) (+)= sum_s part[s][m][k]
// fixed-order sum of partials t0 <= t < t1 with eight interleaved chains
// (t mod 8), which keep eight loads in flight
__device__ __forceinline__ float wg_chain_sum(const float* __restrict__ q, long stride, int t0, int t1) {
    float c[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    int t = t0;
    for (; t + 8 <= t1; t += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) c[u] += q[(long)(t + u) * stride];
    }
    for (; t < t1; ++t) c[(t - t0) & 7] += q[(long)t * stride];
    return ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
}

// dst (+)= sum_{t < n1} part[t] + scale2 sum_{n1 <= t < n_split} part[t]
__global__ void k_wg_reduce(const float* __restrict__ part, int n_split, int n1, float scale2, int M, int Kout,
                            int k_real, float* __restrict__ dst, int accumulate) {
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)M * k_real) return;
    const int m = (int)(o / k_real), k = (int)(o % k_real);
    const long stride = (long)M * Kout;
    const float* q = part + (long)m * Kout + k;
    float s = wg_chain_sum(q, stride, 0, n1);
    if (n1 < n_split) s = __builtin_fmaf(scale2, wg_chain_sum(q, stride, n1, n_split), s);
    dst[o] = accumulate ? dst[o] + s : s;
}

// ----------------------------------------------------------------------------
// column sums with fused element functions, two fixed-order stages
//   mode 0: X[p][m]      mode 1: s[p] relu(X[p][m])
//   mode 3: s[p] X[p][m] + X2[p][m]   (s may be NULL)
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_colsum_partial(const float* __restrict__ X,
                                                        const float* __restrict__ X2,
                                                        const float* __restrict__ s, long ldx,
                                                        long P, int M, long rows_per, int mode,
                                                        float beta, float* __restrict__ part) {
    const int m = threadIdx.x;
    if (m >= M) return;
    const long rb = (long)blockIdx.x * rows_per;
    long re = rb + rows_per;
    if (re > P) re = P;
    float acc = 0.0f;
#pragma unroll 8
    for (long p = rb; p < re; ++p) {
        const float x = X[p * ldx + m];
        float d;
        if (mode == 0) d = x;
        else if (mode == 1) d = s[p] * fmaxf(x, 0.0f);
        else d = (s ? s[p] * x : 0.0f) + X2[p * ldx + m];
        acc += d;
    }
    part[(long)blockIdx.x * M + m] = acc;
}

// dst[m] (+)= scale * sum_b part[b][m]: one work-group per column, thread t
// sums rows t, t + 256, ..., then a fixed-order tree over the 256 threads
__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ part, int nb, int M,
                                                      float scale, float* __restrict__ dst, int accumulate) {
    __shared__ float sh[256];
    const int m = blockIdx.x;
    float s = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[(long)b * M + m];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    s = sh[0] * scale;
    dst[m] = accumulate ? dst[m] + s : s;
}

// ----------------------------------------------------------------------------
// positional encoding (and its tangent along v / half_size), zero padded to ld
// ----------------------------------------------------------------------------
// one thread per (point, column): consecutive threads write consecutive
// columns of a row (coalesced); column e < 3: x_hat_e; e = 3 + 6k + j: sin
// (j < 3) or cos (j >= 3) of 2^k pi x_hat_{j mod 3}; zero padding up to ld
__global__ void k_pe(long n, const float* __restrict__ xyz, float cx, float cy, float cz,
                     float inv_half, int L, int ld, float* __restrict__ X,
                     const float* __restrict__ v, float* __restrict__ Xd) {
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n * ld) return;
    const long p = o / ld;
    const int e = (int)(o % ld);
    float val = 0.0f, dval = 0.0f;
    if (e < 3 + 6 * L) {
        const int d = e < 3 ? e : (e - 3) % 3;
        const float c = d == 0 ? cx : (d == 1 ? cy : cz);
        const float xh = (xyz[3 * p + d] - c) * inv_half;
        const float vd = v ? v[3 * p + d] * inv_half : 0.0f;
        if (e < 3) {
            val = xh;
            dval = vd;
        } else {
            const int k = (e - 3) / 6;
            const bool is_cos = ((e - 3) % 6) >= 3;
            const float scale = (float)(1 << k);
            float sn, cs;
            sincospif(scale * xh, &sn, &cs);
            const float w = 3.14159265358979f * scale * vd;
            val = is_cos ? cs : sn;
            dval = is_cos ? -sn * w : cs * w;
        }
    }
    X[o] = val;
    if (Xd) Xd[o] = dval;
}

// grad_x f = J_PE^T G0 (G0 = dF/dgamma, row stride ld, a multiple of 4): 16
// lanes per point, each taking every 16th float4 of the row (column e < 3:
// x_hat_e, e = 3 + 6k + j: sin (j < 3) or cos (j >= 3) of 2^k pi x_hat_{j mod 3},
// whose derivative is pi 2^k cos or -pi 2^k sin), then a fixed-order sum over
// the 16 lanes per dimension
__global__ void k_pe_grad(long n, const float* __restrict__ xyz, float cx, float cy, float cz,
                          float inv_half, int L, const float* __restrict__ G0, int ld,
                          float* __restrict__ grad) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long p = gid / 16;                  // the 16 lanes of a point exit together
    const int l = (int)(gid % 16);
    if (p >= n) return;
    const float xh[3] = {(xyz[3 * p] - cx) * inv_half, (xyz[3 * p + 1] - cy) * inv_half,
                         (xyz[3 * p + 2] - cz) * inv_half};
    const int ne = 3 + 6 * L;
    float acc[3] = {0.0f, 0.0f, 0.0f};
    for (int m = 4 * l; m < ld && m < ne; m += 64) {
        const float4 g4 = *reinterpret_cast<const float4*>(G0 + p * ld + m);
        const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = m + q;
            if (e >= ne) break;
            if (e < 3) {
                acc[e] += gv[q];
            } else {
                const int k = (e - 3) / 6, j = (e - 3) % 6, d = j % 3;
                const float scale = (float)(1 << k);
                const float t = scale * xh[d], w = 3.14159265358979f * scale;
                acc[d] += j < 3 ? w * cospif(t) * gv[q] : -w * sinpif(t) * gv[q];
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int o = 8; o >= 1; o >>= 1) acc[d] += __shfl_xor(acc[d], o, 16);
    if (l == 0) {
        grad[3 * p] = acc[0];   // d/dx = (d/dx_hat) / half, times f's half_size
        grad[3 * p + 1] = acc[1];
        grad[3 * p + 2] = acc[2];
    }
}

// Row kernels: 16 lanes per row (four rows per wave), each lane taking every
// 16th float4 of the row (widths are multiples of 64, rows 16-byte aligned),
// then a fixed-order sum over the 16 lanes.
constexpr int kRowLanes = 16;
__device__ __forceinline__ float row_sum16(float acc) {
#pragma unroll
    for (int d = kRowLanes / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, kRowLanes);
    return acc;
}

// out[p] = post(scale * (sum_m w[m] act(Y[p][m]) + b))
//   act: 0 identity, 3 relu ; post: 0 identity, 1 sigmoid
__global__ __launch_bounds__(256) void k_rowdot(long n, const float* __restrict__ Y, long ldy,
                                                int M, int act, int post, const float* __restrict__ w,
                                                const float* __restrict__ b, float scale, float beta,
                                                float* __restrict__ out) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long p = gid / kRowLanes;          // the 16 lanes of a row exit together
    const int l = (int)(gid % kRowLanes);
    if (p >= n) return;
    float acc = 0.0f;
    for (int m = 4 * l; m < M; m += 4 * kRowLanes) {
        const float4 y = *reinterpret_cast<const float4*>(Y + p * ldy + m);
        const bool r = act != PRO_ID;
        acc = __builtin_fmaf(w[m], r ? fmaxf(y.x, 0.0f) : y.x, acc);
        acc = __builtin_fmaf(w[m + 1], r ? fmaxf(y.y, 0.0f) : y.y, acc);
        acc = __builtin_fmaf(w[m + 2], r ? fmaxf(y.z, 0.0f) : y.z, acc);
        acc = __builtin_fmaf(w[m + 3], r ? fmaxf(y.w, 0.0f) : y.w, acc);
    }
    acc = row_sum16(acc);
    if (l == 0) {
        const float v = scale * (acc + b[0]);
        out[p] = post ? sigmoidf_(v) : v;
    }
}

// head output adjoint: ybar3 = g_a a (1-a) with a recomputed; Ybar2 = ybar3 w relu'(Y2)
__global__ __launch_bounds__(256) void k_head_out_bwd(long n, const float* __restrict__ Y2, long ld,
                                                      int M, const float* __restrict__ w,
                                                      const float* __restrict__ b,
                                                      const float* __restrict__ g_a,
                                                      float* __restrict__ ybar3,
                                                      float* __restrict__ Ybar2) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long p = gid / kRowLanes;          // the 16 lanes of a row exit together
    const int l = (int)(gid % kRowLanes);
    if (p >= n) return;
    float acc = 0.0f;
    for (int m = 4 * l; m < M; m += 4 * kRowLanes) {
        const float4 y = *reinterpret_cast<const float4*>(Y2 + p * ld + m);
        acc = __builtin_fmaf(w[m], fmaxf(y.x, 0.0f), acc);
        acc = __builtin_fmaf(w[m + 1], fmaxf(y.y, 0.0f), acc);
        acc = __builtin_fmaf(w[m + 2], fmaxf(y.z, 0.0f), acc);
        acc = __builtin_fmaf(w[m + 3], fmaxf(y.w, 0.0f), acc);
    }
    acc = row_sum16(acc);
    const float a = sigmoidf_(acc + b[0]);
    const float yb = g_a ? g_a[p] * a * (1.0f - a) : 0.0f;
    if (l == 0) ybar3[p] = yb;
    for (int m = 4 * l; m < M; m += 4 * kRowLanes) {
        const float4 y = *reinterpret_cast<const float4*>(Y2 + p * ld + m);
        float4 o;
        o.x = y.x > 0.0f ? yb * w[m] : 0.0f;
        o.y = y.y > 0.0f ? yb * w[m + 1] : 0.0f;
        o.z = y.z > 0.0f ? yb * w[m + 2] : 0.0f;
        o.w = y.w > 0.0f ? yb * w[m + 3] : 0.0f;
        *reinterpret_cast<float4*>(Ybar2 + p * ld + m) = o;
    }
}

__global__ void k_fill(float* __restrict__ p, long n, float v) {
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n) p[o] = v;
}

// out[c][r] = in[r][c] for r < R, c < C, zero in the padding; out is [Cpad][Rpad]
__global__ void k_transpose_pad(const float* __restrict__ in, int R, int C, int Rpad, int Cpad,
                                float* __restrict__ out) {
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)Rpad * Cpad) return;
    const int c = (int)(o / Rpad), r = (int)(o % Rpad);
    out[o] = (r < R && c < C) ? in[(long)r * C + c] : 0.0f;
}

// out[r][c] = in[r][c] zero padded to [R][Cpad]
__global__ void k_pad_cols(const float* __restrict__ in, int R, int C, int Cpad, float* __restrict__ out) {
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)R * Cpad) return;
    const int r = (int)(o / Cpad), c = (int)(o % Cpad);
    out[o] = c < C ? in[(long)r * C + c] : 0.0f;
}

// All of a call's weight copies in one launch: job k writes elements
// [begin[k], begin[k+1]) of the concatenated outputs, either in[R][C] zero
// padded to [R][Cpad] or its transpose zero padded to [Cpad][Rpad].
constexpr int kPrepJobs = 40;
struct PrepJob {
    const float* in;
    float* out;
    int R, C, Rpad, Cpad, transpose, pad;
};
struct PrepTable {
    PrepJob job[kPrepJobs];
    long begin[kPrepJobs + 1];
    int n;
};
__global__ void k_prep_weights(PrepTable t) {
    for (long o = (long)blockIdx.x * blockDim.x + threadIdx.x; o < t.begin[t.n];
         o += (long)gridDim.x * blockDim.x) {
        int k = 0;
        while (k + 1 < t.n && o >= t.begin[k + 1]) ++k;
        const PrepJob& j = t.job[k];
        const long q = o - t.begin[k];
        int r, c;
        if (j.transpose) { c = (int)(q / j.Rpad); r = (int)(q % j.Rpad); }
        else { r = (int)(q / j.Cpad); c = (int)(q % j.Cpad); }
        j.out[q] = (r < j.R && c < j.C) ? j.in[(long)r * j.C + c] : 0.0f;
    }
}

// ============================================================================
// host orchestration
// ============================================================================
namespace {

constexpr long kChunk = 1 << 20;          // points per pass (bounds the workspace)
#ifndef RFVR_WG_SPLITS
#define RFVR_WG_SPLITS 384
#endif
constexpr int kWgSplits = RFVR_WG_SPLITS; // weight-gradient point splits per pass
constexpr int kColBlocks = 2048;          // column-sum partial blocks

struct Layout {
    int L, W, in0, in0p, HL, HW;
    long oW[16], ob[16], o_wout, o_bout, oWh[4], obh[4], o_whout, o_bhout, total;
};

int check_net(const rfvr_mlp* n) {
    if (!n) { set_error("mlp descriptor is NULL"); return RFVR_E_INVALID; }
    if (n->n_layers < 1 || n->n_layers > 16 || n->width < 64 || n->width > 256 || n->width % 64 ||
        n->pe_octaves < 0 || n->pe_octaves > 12 || n->head_layers < 1 || n->head_layers > 4 ||
        n->head_width < 64 || n->head_width > 256 || n->head_width % 64) {
        set_error("unsupported network shape (layers 1..16, width 64..256 step 64, octaves 0..12, "
                  "head 1..4 x 64..256 step 64)");
        return RFVR_E_INVALID;
    }
    if ((3 + 6 * n->pe_octaves + 31) / 32 * 32 > n->width) {
        set_error("encoding width (3 + 6 * pe_octaves, padded to 32) must not exceed the layer width");
        return RFVR_E_INVALID;
    }
    if (!(n->softplus_beta > 0.0f) || !(n->half_size > 0.0f) || n->softplus_beta != n->softplus_beta) {
        set_error("softplus_beta and half_size must be > 0");
        return RFVR_E_INVALID;
    }
    if (n->precision != RFVR_PREC_FP32 && n->precision != RFVR_PREC_BF16 && n->precision != RFVR_PREC_BF16X3 &&
        n->precision != RFVR_PREC_F16) {
        set_error("unknown precision %d", n->precision);
        return RFVR_E_INVALID;
    }
    return RFVR_OK;
}

Layout layout(const rfvr_mlp* n) {
    Layout l;
    l.L = n->n_layers; l.W = n->width; l.HL = n->head_layers; l.HW = n->head_width;
    l.in0 = 3 + 6 * n->pe_octaves;
    l.in0p = (l.in0 + 31) / 32 * 32;
    long off = 0;
    for (int i = 0; i < l.L; ++i) {
        const int fin = i == 0 ? l.in0 : l.W;
        l.oW[i] = off; off += (long)l.W * fin;
        l.ob[i] = off; off += l.W;
    }
    l.o_wout = off; off += l.W;
    l.o_bout = off; off += 1;
    for (int h = 0; h < l.HL; ++h) {
        const int fin = h == 0 ? l.W : l.HW;
        l.oWh[h] = off; off += (long)l.HW * fin;
        l.obh[h] = off; off += l.HW;
    }
    l.o_whout = off; off += l.HW;
    l.o_bhout = off; off += 1;
    l.total = off;
    return l;
}

inline unsigned blocks(long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// device copies of the weights in the layouts the GEMMs read, 256-byte
// aligned (the flat parameter vector has matrices at odd offsets)
struct Weights {
    float* Wp[16];         // W_l [W][fin_pad], zero padded
    float* WT[16];         // W_l^T [fin_pad][W]
    float* Whp[4];         // Wh_h [HW][fin]
    float* WhT[4];         // Wh_h^T [fin][HW]
};

size_t weights_bytes(const Layout& l) {
    size_t b = 0;
    for (int i = 0; i < l.L; ++i) b += 2 * align256(sizeof(float) * (i == 0 ? l.in0p : l.W) * l.W);
    for (int h = 0; h < l.HL; ++h) b += 2 * align256(sizeof(float) * (h == 0 ? l.W : l.HW) * l.HW);
    return b;
}

Weights take_weights(WsCursor& cur, const Layout& l) {
    Weights w;
    for (int i = 0; i < l.L; ++i) {
        w.Wp[i] = cur.take<float>((size_t)(i == 0 ? l.in0p : l.W) * l.W);
        w.WT[i] = cur.take<float>((size_t)(i == 0 ? l.in0p : l.W) * l.W);
    }
    for (int h = 0; h < l.HL; ++h) {
        w.Whp[h] = cur.take<float>((size_t)(h == 0 ? l.W : l.HW) * l.HW);
        w.WhT[h] = cur.take<float>((size_t)(h == 0 ? l.W : l.HW) * l.HW);
    }
    return w;
}

hipError_t prep_weights(const Layout& l, const float* P, const Weights& w, hipStream_t st) {
    PrepTable t = {};
    long total = 0;
    auto add = [&](const float* in, float* out, int R, int C, int Rpad, int Cpad, int transpose) {
        PrepJob& j = t.job[t.n];
        j.in = in; j.out = out; j.R = R; j.C = C; j.Rpad = Rpad; j.Cpad = Cpad; j.transpose = transpose;
        t.begin[t.n] = total;
        total += (long)Rpad * Cpad;
        ++t.n;
    };
    for (int i = 0; i < l.L; ++i) {          // at most 16 layers and 4 head layers: <= 40 jobs
        const int fin = i == 0 ? l.in0 : l.W, finp = i == 0 ? l.in0p : l.W;
        add(P + l.oW[i], w.Wp[i], l.W, fin, l.W, finp, 0);
        add(P + l.oW[i], w.WT[i], l.W, fin, l.W, finp, 1);
    }
    for (int h = 0; h < l.HL; ++h) {
        const int fin = h == 0 ? l.W : l.HW;
        add(P + l.oWh[h], w.Whp[h], l.HW, fin, l.HW, fin, 0);
        add(P + l.oWh[h], w.WhT[h], l.HW, fin, l.HW, fin, 1);
    }
    t.begin[t.n] = total;
    long nb = (total + 255) / 256;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_prep_weights, dim3((unsigned)nb), dim3(256), 0, st, t);
    return hipGetLastError();
}

// operand form of the forward products (layers, head, the grad_x f sweep) and
// of the backward's products (tangent, adjoints, weight gradients)
int mm_fwd(int precision) {
    switch (precision) {
    case RFVR_PREC_BF16: return MM_BF16;
    case RFVR_PREC_BF16X3: return MM_BF16X3;
    case RFVR_PREC_F16: return MM_F16;
    default: return MM_FP32;
    }
}
int mm_bwd(int precision) { return precision == RFVR_PREC_F16 ? MM_BF16 : mm_fwd(precision); }

// launch context of the network passes: stream and matrix-operand precision
// (16-bit operands, FP32 accumulation; layers reading the encoding stay FP32)
struct Cx {
    hipStream_t st;
    int mm;        // MM_*
};

template <int PRO, int EPI, int MM, int ST = 0>
void gemm_launch(const GemmArgs& a, hipStream_t st) {
    const long tiles = (a.P + 127) / 128;
    const long groups = (tiles + 7) / 8;                 // 8 point tiles per XCD group
    if (a.M <= 64) {
        hipLaunchKernelGGL((k_gemm_nt<PRO, EPI, 64, MM, ST>), dim3((unsigned)(groups * 8)), dim3(256), 0, st, a);
    } else {
        const long nmb = (a.M + 127) / 128;
        hipLaunchKernelGGL((k_gemm_nt<PRO, EPI, 128, MM, ST>), dim3((unsigned)(groups * 8 * nmb)), dim3(256), 0,
                           st, a);
    }
}

template <int PRO, int EPI>
void gemm(const GemmArgs& a, const Cx& cx) {
    // the FP16 form exists for the forward products' epilogues only (a
    // backward context never carries MM_F16: mm_bwd maps it to BF16)
    constexpr bool FWD_EPI = EPI == EPI_BIAS || EPI == EPI_BIAS_SP || EPI == EPI_DSPMUL;
    if (cx.mm == MM_BF16) gemm_launch<PRO, EPI, MM_BF16>(a, cx.st);
    else if (cx.mm == MM_BF16X3) gemm_launch<PRO, EPI, MM_BF16X3>(a, cx.st);
    else if (cx.mm == MM_F16) {
        if constexpr (FWD_EPI) gemm_launch<PRO, EPI, MM_F16>(a, cx.st);
        else gemm_launch<PRO, EPI, MM_BF16>(a, cx.st);
    } else gemm_launch<PRO, EPI, MM_FP32>(a, cx.st);
}

// FP32 GEMM whatever the context (first layer: its operand is the encoding)
template <int PRO, int EPI, int ST = 0>
void gemm32(const GemmArgs& a, const Cx& cx) {
    gemm_launch<PRO, EPI, MM_FP32, ST>(a, cx.st);
}

// BF16 GEMM of the single-rounded BF16 backward with the ST_* operands in BF16
// storage
template <int PRO, int EPI, int ST>
void gemm_b16(const GemmArgs& a, const Cx& cx) {
    gemm_launch<PRO, EPI, MM_BF16, ST>(a, cx.st);
}

#ifndef RFVR_DUAL_NW
#define RFVR_DUAL_NW 4
#endif
template <int EPI2>
void gemm_dual(const DualArgs& a, int mm, hipStream_t st) {
    constexpr int NW = RFVR_DUAL_NW, BP = NW == 8 ? 128 : 64, BM = 128;
    const long tiles = (a.P + BP - 1) / BP;
    const long groups = (tiles + 7) / 8;
    const long nmb = (a.M + BM - 1) / BM;
    const dim3 grid((unsigned)(groups * 8 * nmb));
    if (mm == MM_BF16) hipLaunchKernelGGL((k_gemm_dual<EPI2, MM_BF16, NW>), grid, dim3(NW * 64), 0, st, a);
    else if (mm == MM_BF16X3) hipLaunchKernelGGL((k_gemm_dual<EPI2, MM_BF16X3, NW>), grid, dim3(NW * 64), 0, st, a);
    else if constexpr (EPI2 == EPI2_FWD) {
        if (mm == MM_F16) hipLaunchKernelGGL((k_gemm_dual<EPI2, MM_F16, NW>), grid, dim3(NW * 64), 0, st, a);
        else hipLaunchKernelGGL((k_gemm_dual<EPI2, MM_FP32, NW>), grid, dim3(NW * 64), 0, st, a);
    } else hipLaunchKernelGGL((k_gemm_dual<EPI2, MM_FP32, NW>), grid, dim3(NW * 64), 0, st, a);
}

DualArgs da(const float* A, const float* A2, long lda, const float* B, long ldb, const float* bias,
            const float* C, const float* C2, float* Y, float* Y2, float* Y3, long ldy,
            long P, int M, int K, float beta) {
    DualArgs g;
    g.A = A; g.A2 = A2; g.lda = lda; g.B = B; g.ldb = ldb; g.bias = bias; g.C = C; g.C2 = C2;
    g.Y = Y; g.Y2 = Y2; g.Y3 = Y3; g.ldy = ldy; g.P = P; g.M = M; g.K = K; g.beta = beta;
    return g;
}

GemmArgs ga(const float* A, long lda, const float* B, long ldb, const float* bias,
            float* Y, long ldy, long P, int M, int K, float beta, const float* C = nullptr,
            long ldc = 0, float* Y2 = nullptr) {
    GemmArgs g = {};
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.bias = bias; g.C = C; g.ldc = ldc;
    g.Y = Y; g.ldy = ldy; g.Y2 = Y2; g.P = P; g.M = M; g.K = K; g.beta = beta;
    return g;
}

// ST != 0 (BF16 storage of operands): the FP32 and single-rounded BF16 forms
template <int PRO, int ST = 0>
void wgrad(const float* A, long lda, int M, const float* B, const float* B2, long ldb, int Kout,
           long P, float beta, float* part, const Cx& cx, float* bpart = nullptr) {
    hipStream_t st = cx.st;
    WgArgs g;
    g.A = A; g.lda = lda; g.B = B; g.B2 = B2; g.ldb = ldb; g.part = part; g.bpart = bpart; g.P = P;
    g.M = M; g.Kout = Kout; g.per_split = ((P + kWgSplits - 1) / kWgSplits + 31) / 32 * 32;
    g.n_split = kWgSplits;
    g.beta = beta;
    const long tiles = (long)((M + 127) / 128) * ((Kout + 127) / 128);
    const long groups = (kWgSplits + 7) / 8;
    const dim3 grid((unsigned)(groups * 8 * tiles));
    if constexpr (ST != 0) {
        if (cx.mm == MM_BF16) {
            if (bpart) hipLaunchKernelGGL((k_gemm_wg<PRO, true, MM_BF16, ST>), grid, dim3(256), 0, st, g);
            else hipLaunchKernelGGL((k_gemm_wg<PRO, false, MM_BF16, ST>), grid, dim3(256), 0, st, g);
        } else {
            if (bpart) hipLaunchKernelGGL((k_gemm_wg<PRO, true, MM_FP32, ST>), grid, dim3(256), 0, st, g);
            else hipLaunchKernelGGL((k_gemm_wg<PRO, false, MM_FP32, ST>), grid, dim3(256), 0, st, g);
        }
    } else if (cx.mm == MM_BF16) {
        if (bpart) hipLaunchKernelGGL((k_gemm_wg<PRO, true, MM_BF16>), grid, dim3(256), 0, st, g);
        else hipLaunchKernelGGL((k_gemm_wg<PRO, false, MM_BF16>), grid, dim3(256), 0, st, g);
    } else if (cx.mm == MM_BF16X3) {
        if (bpart) hipLaunchKernelGGL((k_gemm_wg<PRO, true, MM_BF16X3>), grid, dim3(256), 0, st, g);
        else hipLaunchKernelGGL((k_gemm_wg<PRO, false, MM_BF16X3>), grid, dim3(256), 0, st, g);
    } else {
        if (bpart) hipLaunchKernelGGL((k_gemm_wg<PRO, true, MM_FP32>), grid, dim3(256), 0, st, g);
        else hipLaunchKernelGGL((k_gemm_wg<PRO, false, MM_FP32>), grid, dim3(256), 0, st, g);
    }
}

void wg_reduce(const float* part, int n_split, int M, int Kout, int k_real, float* dst, int acc,
               hipStream_t st, int n1 = -1, float scale2 = 1.0f) {
    hipLaunchKernelGGL(k_wg_reduce, dim3(blocks((long)M * k_real)), dim3(256), 0, st, part, n_split,
                       n1 < 0 ? n_split : n1, scale2, M, Kout, k_real, dst, acc);
}

void colsum(const float* X, const float* X2, const float* s, long ldx, long P, int M, int mode,
            float beta, float scale, float* part, float* dst, int acc, hipStream_t st) {
    const long per = (P + kColBlocks - 1) / kColBlocks;
    hipLaunchKernelGGL(k_colsum_partial, dim3(kColBlocks), dim3(256), 0, st, X, X2, s, ldx, P, M, per,
                       mode, beta, part);
    hipLaunchKernelGGL(k_colsum_final, dim3(M), dim3(256), 0, st, part, kColBlocks, M, scale,
                       dst, acc);
}

// --- forward workspace -------------------------------------------------------
// keep: the layers' (Z, H) go to the caller's reserve instead of the workspace
size_t fwd_bytes(const Layout& l, long n, bool keep) {
    const long c = n < kChunk ? n : kChunk;
    return weights_bytes(l) + align256(sizeof(float) * c * l.in0p) +
           (keep ? 0 : (size_t)l.L * align256(sizeof(float) * c * l.W)) + 2 * align256(sizeof(float) * c * l.W) +
           (keep ? 0 : (size_t)l.HL * align256(sizeof(float) * c * l.HW));   // head Y (else in the reserve)
}

// --- backward workspace ------------------------------------------------------
// rows of the top-adjoint GEMM's column partials: one per 128-point tile
long top_rows(long n) { return (n + 127) / 128; }

size_t bwd_bytes(const Layout& l, long n, bool keep) {
    const long c = n < kChunk ? n : kChunk;
    const long wmax = l.W > l.in0p ? l.W : l.in0p;
    return weights_bytes(l) + 2 * align256(sizeof(float) * c * l.in0p) +
           (keep ? 1 : 3) * (size_t)l.L * align256(sizeof(float) * c * l.W) +  // Hdot (and Z, H)
           4 * align256(sizeof(float) * c * l.W) +                  // Hbar, Hdotbar, Zbar, Zdotbar
           (keep ? 1 : 2) * (size_t)l.HL * align256(sizeof(float) * c * l.HW) +  // head Ybar (and Y)
           align256(sizeof(float) * c) +                            // ybar3
           align256(sizeof(float) * 2 * kWgSplits * (size_t)l.W * wmax) +
           align256(sizeof(float) * kWgSplits * (size_t)l.W) +
           align256(sizeof(float) * (size_t)kColBlocks * (l.W > l.HW ? l.W : l.HW)) +
           align256(sizeof(float) * (size_t)top_rows(c) * l.W);   // output layer column partials
}

// --- reserve of the training pair, [n][W] per trunk layer: H_i = sp(Z_i) and
// the normal sweep's adjoint S_i = df/dZ_i; then [n][HW] per head layer: its
// output before the relu ----------------------------------------------------------
size_t reserve_layer_bytes(const Layout& l, long n) { return align256(sizeof(float) * (size_t)n * l.W); }
size_t reserve_head_bytes(const Layout& l, long n) { return align256(sizeof(float) * (size_t)n * l.HW); }
size_t reserve_bytes(const Layout& l, long n) {
    return 2 * (size_t)l.L * reserve_layer_bytes(l, n) + (size_t)l.HL * reserve_head_bytes(l, n);
}
float* reserve_h(void* r, const Layout& l, long n, int i) {
    return reinterpret_cast<float*>(static_cast<char*>(r) + (size_t)i * reserve_layer_bytes(l, n));
}
float* reserve_s(void* r, const Layout& l, long n, int i) { return reserve_h(r, l, n, l.L + i); }
float* reserve_y(void* r, const Layout& l, long n, int h) {
    return reinterpret_cast<float*>(static_cast<char*>(r) + 2 * (size_t)l.L * reserve_layer_bytes(l, n) +
                                    (size_t)h * reserve_head_bytes(l, n));
}

int check_buffers(void* ws, size_t ws_bytes, size_t need, void* reserve, size_t reserve_bytes_, size_t rneed) {
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("workspace too small or misaligned: need %zu bytes", need);
        return RFVR_E_WORKSPACE;
    }
    if (rneed && (!reserve || reserve_bytes_ < rneed || (reinterpret_cast<uintptr_t>(reserve) & 255u))) {
        set_error("reserve too small or misaligned: need %zu bytes", rneed);
        return RFVR_E_WORKSPACE;
    }
    return RFVR_OK;
}

int mlp_forward(const rfvr_mlp* net, const float* xyz, long n, float* sdf, float* grad, float* refl,
                void* reserve, size_t reserve_bytes_, void* ws, size_t ws_bytes, hipStream_t st) {
    int rc;
    if ((rc = check_net(net))) return rc;
    if (n < 1 || n > RFVR_MAX_POINTS || !xyz || !net->params) {
        set_error("n in [1, RFVR_MAX_POINTS], xyz and params are required");
        return RFVR_E_INVALID;
    }
    const Layout l = layout(net);
    const bool keep = reserve_bytes_ != 0 || reserve != nullptr;
    if ((rc = check_buffers(ws, ws_bytes, fwd_bytes(l, n, keep), reserve, reserve_bytes_,
                            keep ? reserve_bytes(l, n) : 0)))
        return rc;
    const Cx cx{st, mm_fwd(net->precision)};
    const float* P = net->params;
    const float beta = net->softplus_beta, half = net->half_size, inv_half = 1.0f / net->half_size;
    const long chunk = n < kChunk ? n : kChunk;
    WsCursor cur{reinterpret_cast<char*>(ws), 0};
    const Weights w = take_weights(cur, l);
    float* X0 = cur.take<float>((size_t)chunk * l.in0p);
    float* Hw[16];
    for (int i = 0; i < l.L && !keep; ++i) Hw[i] = cur.take<float>((size_t)chunk * l.W);
    float* G[2] = {cur.take<float>((size_t)chunk * l.W), cur.take<float>((size_t)chunk * l.W)};
    float* Yw[4];
    for (int h = 0; h < l.HL && !keep; ++h) Yw[h] = cur.take<float>((size_t)chunk * l.HW);
    if ((rc = hip_status(prep_weights(l, P, w, st), "mlp weight prep"))) return rc;

    for (long c0 = 0; c0 < n; c0 += chunk) {
        const long m = (n - c0) < chunk ? (n - c0) : chunk;
        const float* x = xyz + 3 * c0;
        hipLaunchKernelGGL(k_pe, dim3(blocks(m * l.in0p)), dim3(256), 0, st, m, x, net->centre[0], net->centre[1],
                           net->centre[2], inv_half, net->pe_octaves, l.in0p, X0, nullptr, nullptr);
        // H_i = sp(H_{i-1} W_i^T + b_i) from the epilogue (the reserve's, or
        // the workspace's until the sweep has used them)
        float* H[16];
        for (int i = 0; i < l.L; ++i) H[i] = keep ? reserve_h(reserve, l, n, i) + c0 * l.W : Hw[i];
        gemm32<PRO_ID, EPI_BIAS_SP>(ga(X0, l.in0p, w.Wp[0], l.in0p, P + l.ob[0], H[0], l.W, m, l.W, l.in0p, beta),
                                    cx);
        for (int i = 1; i < l.L; ++i)
            gemm<PRO_ID, EPI_BIAS_SP>(ga(H[i - 1], l.W, w.Wp[i], l.W, P + l.ob[i], H[i], l.W, m, l.W, l.W, beta),
                                      cx);
        float* Ht = H[l.L - 1];
        if (sdf)
            hipLaunchKernelGGL(k_rowdot, dim3(blocks(m * kRowLanes)), dim3(256), 0, st, m, Ht, (long)l.W, l.W,
                               (int)PRO_ID, 0, P + l.o_wout, P + l.o_bout, half, beta, sdf + c0);
        if (refl || keep) {
            // head layers (the training forward keeps their outputs in the reserve)
            float* Yh[4];
            for (int h = 0; h < l.HL; ++h) Yh[h] = keep ? reserve_y(reserve, l, n, h) + c0 * l.HW : Yw[h];
            gemm<PRO_ID, EPI_BIAS>(ga(Ht, l.W, w.Whp[0], l.W, P + l.obh[0], Yh[0], l.HW, m, l.HW, l.W, beta), cx);
            for (int h = 1; h < l.HL; ++h)
                gemm<PRO_RELU, EPI_BIAS>(ga(Yh[h - 1], l.HW, w.Whp[h], l.HW, P + l.obh[h], Yh[h], l.HW, m, l.HW, l.HW, beta), cx);
            if (refl)
                hipLaunchKernelGGL(k_rowdot, dim3(blocks(m * kRowLanes)), dim3(256), 0, st, m, Yh[l.HL - 1], (long)l.HW,
                                   l.HW, (int)PRO_RELU, 1, P + l.o_whout, P + l.o_bhout, 1.0f, beta, refl + c0);
        }
        if (grad || keep) {
            // adjoint of f w.r.t. Z_{L-1}: S_{L-1} = sp'(Z_{L-1}) w_out, formed from
            // H_{L-1} as the first product's operand (PRO_SEED); then
            // S_{i-1} = (S_i W_i) . sp'(Z_{i-1})
            // (epilogue), and dgamma = S_0 W_0.  The training forward keeps S_i
            // (i < L-1) in the reserve: scaled by half_size, S_i and S_i / sp'(Z_i)
            // are the backward's adjoints of the tangent pass to Zdot_i and Hdot_i,
            // so the backward does not recompute them.
            int cur_g = 0;
            for (int i = l.L - 1; i >= 0; --i) {
                const int mout = i == 0 ? l.in0p : l.W;
                const bool top = i == l.L - 1;
                const float* src = top ? Ht : (keep ? reserve_s(reserve, l, n, i) + c0 * l.W : G[cur_g]);
                float* dst = (keep && i > 0) ? reserve_s(reserve, l, n, i - 1) + c0 * l.W : G[cur_g ^ 1];
                GemmArgs a = ga(src, l.W, w.WT[i], l.W, nullptr, dst, mout, m, mout, l.W, beta,
                                i > 0 ? H[i - 1] : nullptr, l.W);
                a.colv = P + l.o_wout;
                if (i > 0) {
                    if (top) gemm<PRO_SEED, EPI_DSPMUL>(a, cx);
                    else gemm<PRO_ID, EPI_DSPMUL>(a, cx);
                } else {    // the product with W_0 stays FP32
                    if (top) gemm32<PRO_SEED, EPI_BIAS>(a, cx);
                    else gemm32<PRO_ID, EPI_BIAS>(a, cx);
                }
                cur_g ^= 1;
            }
            if (grad)
                hipLaunchKernelGGL(k_pe_grad, dim3(blocks(m * 16)), dim3(256), 0, st, m, x, net->centre[0],
                                   net->centre[1], net->centre[2], inv_half, net->pe_octaves, G[cur_g],
                                   l.in0p, grad + 3 * c0);
        }
        if ((rc = hip_status(hipGetLastError(), "mlp forward"))) return rc;
    }
    return RFVR_OK;
}

// Side stream of the training backward.  A trunk layer's two weight-gradient
// products read its Zbar and arrays that stay fixed during the sweep (the
// reserve's H and S, the tangents, the encoding), and write only their own
// partials and gradient rows; so they run on a second stream beside the chain
// of adjoint products, ordered by events: they start once Zbar is written, and
// the adjoint product that next overwrites that Zbar buffer waits for them.
// One side stream per device, default priority, created on first use and held
// until the process ends; a backward call holds its mutex while it enqueues,
// so calls from several host threads on one device take turns.
struct SideStream {
    hipStream_t ss = nullptr;
    hipEvent_t ready[16] = {}, done[16] = {};
    std::mutex mu;
};
std::mutex g_side_mu;
SideStream* g_side[64] = {};

int side_stream(SideStream** out) {
    int dev = -1;
    int rc;
    if ((rc = hip_status(hipGetDevice(&dev), "hipGetDevice"))) return rc;
    if (dev < 0 || dev >= 64) { set_error("device index %d beyond 64", dev); return RFVR_E_UNSUPPORTED; }
    std::lock_guard<std::mutex> lock(g_side_mu);
    if (!g_side[dev]) {
        SideStream* s = new SideStream();
        if ((rc = hip_status(hipStreamCreateWithFlags(&s->ss, hipStreamNonBlocking), "side stream"))) {
            delete s;
            return rc;
        }
        for (int k = 0; k < 16; ++k) {
            if ((rc = hip_status(hipEventCreateWithFlags(&s->ready[k], hipEventDisableTiming), "side event")) ||
                (rc = hip_status(hipEventCreateWithFlags(&s->done[k], hipEventDisableTiming), "side event")))
                return rc;          // the partly built context is kept out of g_side (leaked, error path)
        }
        g_side[dev] = s;
    }
    *out = g_side[dev];
    return RFVR_OK;
}

int mlp_backward(const rfvr_mlp* net, const float* xyz, long n, const float* g_sdf, const float* g_grad,
                 const float* g_refl, uint32_t flags, float* g_params, void* reserve, size_t reserve_bytes_,
                 void* ws, size_t ws_bytes, hipStream_t st) {
    int rc;
    if ((rc = check_net(net))) return rc;
    if (n < 1 || n > RFVR_MAX_POINTS || !xyz || !net->params || !g_params) {
        set_error("n in [1, RFVR_MAX_POINTS], xyz, params and g_params are required");
        return RFVR_E_INVALID;
    }
    if (flags & ~(uint32_t)RFVR_ACCUMULATE) { set_error("only RFVR_ACCUMULATE is meaningful here"); return RFVR_E_INVALID; }
    const Layout l = layout(net);
    const bool keep = reserve_bytes_ != 0 || reserve != nullptr;
    if ((rc = check_buffers(ws, ws_bytes, bwd_bytes(l, n, keep), reserve, reserve_bytes_,
                            keep ? reserve_bytes(l, n) : 0)))
        return rc;
    // cxf: the plain backward's recompute of the forward products, in the
    // forward's operand form; cx: the backward's own products
    const Cx cx{st, mm_bwd(net->precision)}, cxf{st, mm_fwd(net->precision)}, cx32{st, MM_FP32};
    // the training pair's weight gradients run on the side stream when the
    // products are bound by the matrix cores (FP32); the BF16 forms are bound by
    // HBM and gain nothing measurable from it
    SideStream* side = nullptr;
    std::unique_lock<std::mutex> side_lock;
    if (keep && cx.mm == MM_FP32) {
        if ((rc = side_stream(&side))) return rc;
        side_lock = std::unique_lock<std::mutex>(side->mu);
    }
    const hipStream_t wst = side ? side->ss : st;
    const Cx cxw{wst, cx.mm}, cx32w{wst, MM_FP32};
    // single-rounded BF16 products in the training backward: the tangents Hdot
    // and the adjoints Zbar are stored in BF16 (every product reading them rounds
    // them so), which cuts the HBM bytes of these HBM-bound products by ~30 %
    const bool b16 = keep && cx.mm == MM_BF16;
    const float* P = net->params;
    float* GP = g_params;
    const float beta = net->softplus_beta, half = net->half_size, inv_half = 1.0f / net->half_size;
    const long chunk = n < kChunk ? n : kChunk;
    const long wmax = l.W > l.in0p ? l.W : l.in0p;
    WsCursor cur{reinterpret_cast<char*>(ws), 0};
    const Weights w = take_weights(cur, l);
    float* X0 = cur.take<float>((size_t)chunk * l.in0p);
    float* X0d = cur.take<float>((size_t)chunk * l.in0p);
    float *Zw[16], *Hw[16], *Hd[16];
    for (int i = 0; i < l.L && !keep; ++i) Zw[i] = cur.take<float>((size_t)chunk * l.W);
    for (int i = 0; i < l.L && !keep; ++i) Hw[i] = cur.take<float>((size_t)chunk * l.W);
    for (int i = 0; i < l.L; ++i) Hd[i] = cur.take<float>((size_t)chunk * l.W);
    float* Hb = cur.take<float>((size_t)chunk * l.W);
    float* Hdb = cur.take<float>((size_t)chunk * l.W);
    float* Zb = cur.take<float>((size_t)chunk * l.W);
    float* Zdb = cur.take<float>((size_t)chunk * l.W);
    float *Yw[4], *Ybh[4];
    for (int h = 0; h < l.HL && !keep; ++h) Yw[h] = cur.take<float>((size_t)chunk * l.HW);
    for (int h = 0; h < l.HL; ++h) Ybh[h] = cur.take<float>((size_t)chunk * l.HW);
    float* yb3 = cur.take<float>((size_t)chunk);
    float* part = cur.take<float>((size_t)2 * kWgSplits * l.W * wmax);
    float* bpart = cur.take<float>((size_t)kWgSplits * l.W);
    float* cpart = cur.take<float>((size_t)kColBlocks * (l.W > l.HW ? l.W : l.HW));
    float* tpart = cur.take<float>((size_t)top_rows(chunk) * l.W);
    if ((rc = hip_status(prep_weights(l, P, w, st), "mlp weight prep"))) return rc;

    for (long c0 = 0; c0 < n; c0 += chunk) {
        const long m = (n - c0) < chunk ? (n - c0) : chunk;
        const int acc = (c0 > 0 || (flags & RFVR_ACCUMULATE)) ? 1 : 0;
        const float* x = xyz + 3 * c0;
        const float* gf = g_sdf ? g_sdf + c0 : nullptr;
        const float* ga_ = g_refl ? g_refl + c0 : nullptr;
        float *Z[16], *H[16];   // Z: the plain backward's recomputed pre-activations only
        for (int i = 0; i < l.L; ++i) {
            Z[i] = keep ? nullptr : Zw[i];
            H[i] = keep ? reserve_h(reserve, l, n, i) + c0 * l.W : Hw[i];
        }
        // encoding and its tangent along g_grad
        hipLaunchKernelGGL(k_pe, dim3(blocks(m * l.in0p)), dim3(256), 0, st, m, x, net->centre[0], net->centre[1],
                           net->centre[2], inv_half, net->pe_octaves, l.in0p, X0,
                           g_grad ? g_grad + 3 * c0 : nullptr, X0d);
        if (keep) {
            // tangent only: Hdot_i = sp'(Z_i) (Hdot_{i-1} W_i^T), sp'(Z_i) from the
            // reserve's H_i
            const GemmArgs a0 = ga(X0d, l.in0p, w.Wp[0], l.in0p, nullptr, Hd[0], l.W, m, l.W, l.in0p, beta, H[0], l.W);
            if (b16) gemm32<PRO_ID, EPI_DSPMUL, ST_Y>(a0, cx);
            else gemm32<PRO_ID, EPI_DSPMUL>(a0, cx);
            for (int i = 1; i < l.L; ++i) {
                const GemmArgs a = ga(Hd[i - 1], l.W, w.Wp[i], l.W, nullptr, Hd[i], l.W, m, l.W, l.W, beta, H[i], l.W);
                if (b16) gemm_b16<PRO_ID, EPI_DSPMUL, ST_A | ST_Y>(a, cx);
                else gemm<PRO_ID, EPI_DSPMUL>(a, cx);
            }
        } else {
            // one dual GEMM per layer: (Z_i, H_i) and Hdot_i share W_i
            gemm_dual<EPI2_FWD>(da(X0, X0d, l.in0p, w.Wp[0], l.in0p, P + l.ob[0], nullptr, nullptr, Z[0], H[0], Hd[0],
                                   l.W, m, l.W, l.in0p, beta), MM_FP32, st);
            for (int i = 1; i < l.L; ++i)
                gemm_dual<EPI2_FWD>(da(H[i - 1], Hd[i - 1], l.W, w.Wp[i], l.W, P + l.ob[i], nullptr, nullptr, Z[i],
                                       H[i], Hd[i], l.W, m, l.W, l.W, beta), cxf.mm, st);
        }
        float* Ht = H[l.L - 1];
        // head forward (the training backward reads it from the reserve)
        float* Yh[4];
        for (int h = 0; h < l.HL; ++h) Yh[h] = keep ? reserve_y(reserve, l, n, h) + c0 * l.HW : Yw[h];
        if (!keep) {
            gemm<PRO_ID, EPI_BIAS>(ga(Ht, l.W, w.Whp[0], l.W, P + l.obh[0], Yh[0], l.HW, m, l.HW, l.W, beta), cxf);
            for (int h = 1; h < l.HL; ++h)
                gemm<PRO_RELU, EPI_BIAS>(ga(Yh[h - 1], l.HW, w.Whp[h], l.HW, P + l.obh[h], Yh[h], l.HW, m, l.HW,
                                           l.HW, beta), cxf);
        }
        // head output: ybar3, Ybar_{HL-1}
        hipLaunchKernelGGL(k_head_out_bwd, dim3(blocks(m * kRowLanes)), dim3(256), 0, st, m, Yh[l.HL - 1], (long)l.HW,
                           l.HW, P + l.o_whout, P + l.o_bhout, ga_, yb3, Ybh[l.HL - 1]);
        colsum(Yh[l.HL - 1], nullptr, yb3, l.HW, m, l.HW, 1, beta, 1.0f, cpart, GP + l.o_whout, acc, st);
        colsum(yb3, nullptr, nullptr, 1, m, 1, 0, beta, 1.0f, cpart, GP + l.o_bhout, acc, st);
        // head hidden layers, top down
        for (int h = l.HL - 1; h >= 0; --h) {
            float* Yb = Ybh[h];
            if (h > 0) {
                wgrad<PRO_RELU>(Yb, l.HW, l.HW, Yh[h - 1], nullptr, l.HW, l.HW, m, beta, part, cx, bpart);
                wg_reduce(part, kWgSplits, l.HW, l.HW, l.HW, GP + l.oWh[h], acc, st);
                hipLaunchKernelGGL(k_colsum_final, dim3(l.HW), dim3(256), 0, st, bpart, kWgSplits, l.HW, 1.0f,
                               GP + l.obh[h], acc);
                // Ybar_{h-1} = (Ybar_h Wh_h) . relu'(Y_{h-1})
                gemm<PRO_ID, EPI_RELUMASK>(ga(Yb, l.HW, w.WhT[h], l.HW, nullptr, Ybh[h - 1], l.HW, m, l.HW, l.HW, beta, Yh[h - 1], l.HW), cx);
            } else {
                wgrad<PRO_ID>(Yb, l.HW, l.HW, Ht, nullptr, l.W, l.W, m, beta, part, cx, bpart);
                wg_reduce(part, kWgSplits, l.HW, l.W, l.W, GP + l.oWh[0], acc, st);
                hipLaunchKernelGGL(k_colsum_final, dim3(l.HW), dim3(256), 0, st, bpart, kWgSplits, l.HW, 1.0f,
                               GP + l.obh[0], acc);
            }
        }
        // top of the trunk: H_bar = half g_f w_out + Ybar_0 Wh_0 and Hdot_bar =
        // half w_out, turned into the top layer's (Zbar, Zdotbar) in the
        // epilogue, which also forms the column partials of the output layer's
        // weight gradient w_out_bar = half sum_p (g_f H + Hdot) from the same
        // operands
        {
            GemmArgs a = ga(Ybh[0], l.HW, w.WhT[0], l.HW, nullptr, Zb, l.W, m, l.W, l.HW, beta, H[l.L - 1], l.W, Zdb);
            a.C2 = Hd[l.L - 1];
            a.rowv = gf;
            a.colv = P + l.o_wout;
            a.scale = half;
            a.cpart = tpart;
            if (b16) gemm_b16<PRO_ID, EPI_TOPADJ, ST_C2 | ST_Y>(a, cx);      // Zbar (Y) in BF16, Zdotbar (Y2) in FP32
            else gemm<PRO_ID, EPI_TOPADJ>(a, cx);
        }
        // sdf output layer: w_out_bar from the partials, b_out_bar = half sum g_f
        hipLaunchKernelGGL(k_colsum_final, dim3(l.W), dim3(256), 0, st, tpart, (int)top_rows(m), l.W, 1.0f,
                           GP + l.o_wout, acc);
        if (gf) colsum(gf, nullptr, nullptr, 1, m, 1, 0, beta, half, cpart, GP + l.o_bout, acc, st);
        else if (!acc) hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, GP + l.o_bout, 1L, 0.0f);
        // trunk layers, top down: the others' (Zbar, Zdotbar) from the dual
        // adjoint GEMM of the layer above
        float *Zb_c = Zb, *Zdb_c = Zdb, *Zb_n = Hb, *Zdb_n = Hdb;
        for (int i = l.L - 1; i >= 0; --i) {
            float* Zb = Zb_c;
            // Zdot_bar_i: from the dual adjoint (plain), or half S_i kept by the
            // training forward (the top layer's from the top-adjoint epilogue)
            const bool kept = keep && i < l.L - 1;
            const float* Zdb = kept ? reserve_s(reserve, l, n, i) + c0 * l.W : Zdb_c;
            const int fin = i == 0 ? l.in0 : l.W, finp = i == 0 ? l.in0p : l.W;
            if (side) {
                // everything up to Zbar_i is enqueued on st
                if ((rc = hip_status(hipEventRecord(side->ready[i], st), "side event record")) ||
                    (rc = hip_status(hipStreamWaitEvent(wst, side->ready[i], 0), "side event wait")))
                    return rc;
            }
            float* part2 = part + (size_t)kWgSplits * l.W * finp;
            if (i == 0) {
                if (b16) wgrad<PRO_ID, ST_A>(Zb, l.W, l.W, X0, nullptr, l.in0p, finp, m, beta, part, cx32w, bpart);
                else wgrad<PRO_ID>(Zb, l.W, l.W, X0, nullptr, l.in0p, finp, m, beta, part, cx32w, bpart);
                wgrad<PRO_ID>(Zdb, l.W, l.W, X0d, nullptr, l.in0p, finp, m, beta, part2, cx32w);
            } else if (b16) {
                wgrad<PRO_ID, ST_A>(Zb, l.W, l.W, H[i - 1], nullptr, l.W, finp, m, beta, part, cxw, bpart);
                wgrad<PRO_ID, ST_B>(Zdb, l.W, l.W, Hd[i - 1], nullptr, l.W, finp, m, beta, part2, cxw);
            } else {
                wgrad<PRO_ID>(Zb, l.W, l.W, H[i - 1], nullptr, l.W, finp, m, beta, part, cxw, bpart);
                wgrad<PRO_ID>(Zdb, l.W, l.W, Hd[i - 1], nullptr, l.W, finp, m, beta, part2, cxw);
            }
            wg_reduce(part, 2 * kWgSplits, l.W, finp, fin, GP + l.oW[i], acc, wst, kWgSplits, kept ? half : 1.0f);
            hipLaunchKernelGGL(k_colsum_final, dim3(l.W), dim3(256), 0, wst, bpart, kWgSplits, l.W, 1.0f,
                               GP + l.ob[i], acc);
            if (side && (rc = hip_status(hipEventRecord(side->done[i], wst), "side event record"))) return rc;
            if (i > 0 && keep) {
                // the buffer this writes held Zbar_{i+1}, read by that layer's weight gradients
                if (side && i + 1 < l.L && (rc = hip_status(hipStreamWaitEvent(st, side->done[i + 1], 0),
                                                            "side event wait")))
                    return rc;
                // Zbar_{i-1} from Hbar_{i-1} = Zbar_i W_i and Hdotbar_{i-1} = half S_{i-1} / sp'(Z_{i-1})
                GemmArgs a = ga(Zb, l.W, w.WT[i], l.W, nullptr, Zb_n, l.W, m, l.W, l.W, beta, H[i - 1], l.W);
                a.C2 = Hd[i - 1];
                a.C3 = reserve_s(reserve, l, n, i - 1) + c0 * l.W;
                a.scale = half;
                if (b16) gemm_b16<PRO_ID, EPI_ADJ1, ST_A | ST_C2 | ST_Y>(a, cx);
                else gemm<PRO_ID, EPI_ADJ1>(a, cx);
                float* t = Zb_c; Zb_c = Zb_n; Zb_n = t;
            } else if (i > 0) {
                gemm_dual<EPI2_ADJ>(da(Zb, Zdb, l.W, w.WT[i], l.W, nullptr, Z[i - 1], Hd[i - 1], Zb_n, Zdb_n, nullptr,
                                       l.W, m, l.W, l.W, beta), cx.mm, st);
                float* t = Zb_c; Zb_c = Zb_n; Zb_n = t;
                t = Zdb_c; Zdb_c = Zdb_n; Zdb_n = t;
            }
        }
        // join: the next pass reuses the encoding, tangents and partials, and the
        // caller reads the gradient on st
        if (side && (rc = hip_status(hipStreamWaitEvent(st, side->done[0], 0), "side event wait"))) return rc;
        if ((rc = hip_status(hipGetLastError(), "mlp backward"))) return rc;
    }
    return RFVR_OK;
}

}  // namespace
}  // namespace rfvr

using namespace rfvr;

extern "C" {

int64_t rfvr_mlp_param_count(const rfvr_mlp* net) {
    if (check_net(net)) return -1;
    return layout(net).total;
}

size_t rfvr_mlp_forward_ws_bytes(const rfvr_mlp* net, int64_t n) {
    if (check_net(net) || n < 1 || n > RFVR_MAX_POINTS) return 0;
    return fwd_bytes(layout(net), (long)n, false);
}

size_t rfvr_mlp_backward_ws_bytes(const rfvr_mlp* net, int64_t n) {
    if (check_net(net) || n < 1 || n > RFVR_MAX_POINTS) return 0;
    return bwd_bytes(layout(net), (long)n, false);
}

int rfvr_mlp_forward(const rfvr_mlp* net, const float* xyz, int64_t n, float* sdf, float* grad,
                     float* refl, void* ws, size_t ws_bytes, void* stream) {
    return mlp_forward(net, xyz, (long)n, sdf, grad, refl, nullptr, 0, ws, ws_bytes,
                       reinterpret_cast<hipStream_t>(stream));
}

int rfvr_mlp_backward(const rfvr_mlp* net, const float* xyz, int64_t n, const float* g_sdf,
                      const float* g_grad, const float* g_refl, uint32_t flags, float* g_params,
                      void* ws, size_t ws_bytes, void* stream) {
    return mlp_backward(net, xyz, (long)n, g_sdf, g_grad, g_refl, flags, g_params, nullptr, 0, ws, ws_bytes,
                        reinterpret_cast<hipStream_t>(stream));
}

size_t rfvr_mlp_reserve_bytes(const rfvr_mlp* net, int64_t n) {
    if (check_net(net) || n < 1 || n > RFVR_MAX_POINTS) return 0;
    return reserve_bytes(layout(net), (long)n);
}

size_t rfvr_mlp_forward_train_ws_bytes(const rfvr_mlp* net, int64_t n) {
    if (check_net(net) || n < 1 || n > RFVR_MAX_POINTS) return 0;
    return fwd_bytes(layout(net), (long)n, true);
}

size_t rfvr_mlp_backward_train_ws_bytes(const rfvr_mlp* net, int64_t n) {
    if (check_net(net) || n < 1 || n > RFVR_MAX_POINTS) return 0;
    return bwd_bytes(layout(net), (long)n, true);
}

int rfvr_mlp_forward_train(const rfvr_mlp* net, const float* xyz, int64_t n, float* sdf, float* grad,
                           float* refl, void* reserve, size_t reserve_bytes_, void* ws, size_t ws_bytes,
                           void* stream) {
    if (!reserve || !reserve_bytes_) { set_error("the training forward needs a reserve"); return RFVR_E_INVALID; }
    return mlp_forward(net, xyz, (long)n, sdf, grad, refl, reserve, reserve_bytes_, ws, ws_bytes,
                       reinterpret_cast<hipStream_t>(stream));
}

int rfvr_mlp_backward_train(const rfvr_mlp* net, const float* xyz, int64_t n, const float* g_sdf,
                            const float* g_grad, const float* g_refl, uint32_t flags, float* g_params,
                            const void* reserve, size_t reserve_bytes_, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!reserve || !reserve_bytes_) { set_error("the training backward needs a reserve"); return RFVR_E_INVALID; }
    return mlp_backward(net, xyz, (long)n, g_sdf, g_grad, g_refl, flags, g_params, const_cast<void*>(reserve),
                        reserve_bytes_, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

// ============================================================================
// proposal network: gamma_L -> [Linear(width) -> relu] x layers -> Linear(1)
// ============================================================================
namespace rfvr {
namespace {

struct PLayout {
    int L, W, in0, in0p, layers;
    long oW[4], ob[4], o_wout, o_bout, total;
};

int check_prop(const rfvr_proposal* n) {
    if (!n) { set_error("proposal descriptor is NULL"); return RFVR_E_INVALID; }
    if (n->width != 64 || n->layers < 1 || n->layers > 4 || n->pe_octaves < 0 || n->pe_octaves > 5) {
        set_error("unsupported proposal network (width 64, layers 1..4, pe_octaves 0..5)");
        return RFVR_E_INVALID;
    }
    if (!(n->half_size > 0.0f)) { set_error("half_size must be > 0"); return RFVR_E_INVALID; }
    return RFVR_OK;
}

PLayout playout(const rfvr_proposal* n) {
    PLayout l;
    l.L = n->pe_octaves; l.W = n->width; l.layers = n->layers;
    l.in0 = 3 + 6 * l.L;
    l.in0p = (l.in0 + 31) / 32 * 32;
    long off = 0;
    for (int i = 0; i < l.layers; ++i) {
        const int fin = i == 0 ? l.in0 : l.W;
        l.oW[i] = off; off += (long)l.W * fin;
        l.ob[i] = off; off += l.W;
    }
    l.o_wout = off; off += l.W;
    l.o_bout = off; off += 1;
    l.total = off;
    return l;
}

size_t pweights_bytes(const PLayout& l) {
    size_t b = 0;
    for (int i = 0; i < l.layers; ++i) b += 2 * align256(sizeof(float) * (i == 0 ? l.in0p : l.W) * l.W);
    return b;
}

size_t pbytes(const PLayout& l, long n, bool bwd) {
    const long c = n < kChunk ? n : kChunk;
    size_t b = pweights_bytes(l) + align256(sizeof(float) * c * l.in0p) +
               (size_t)l.layers * align256(sizeof(float) * c * l.W);
    if (bwd)
        b += 2 * align256(sizeof(float) * c * l.W) + align256(sizeof(float) * kWgSplits * (size_t)l.W * l.W) +
             align256(sizeof(float) * kWgSplits * (size_t)l.W) + align256(sizeof(float) * (size_t)kColBlocks * l.W);
    return b;
}

// Abar[p][m] = g[p] w[m] relu'(A[p][m])
__global__ void k_relu_out_bwd(long n, int M, const float* __restrict__ A, long ld, const float* __restrict__ w,
                               const float* __restrict__ g, float* __restrict__ Ab) {
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n * M) return;
    const long p = o / M;
    const int m = (int)(o % M);
    Ab[p * ld + m] = A[p * ld + m] > 0.0f ? g[p] * w[m] : 0.0f;
}

}  // namespace
}  // namespace rfvr

extern "C" {

int64_t rfvr_proposal_param_count(const rfvr_proposal* net) {
    if (check_prop(net)) return -1;
    return playout(net).total;
}

// one pass over all points, two threads per point in its matrix products
constexpr int64_t kPropMaxPoints = (int64_t)1 << 30;

size_t rfvr_proposal_ws_bytes(const rfvr_proposal* net, int64_t n) {
    if (check_prop(net) || n < 1 || n > kPropMaxPoints) return 0;
    return pbytes(playout(net), (long)n, true);
}

static int proposal_pass(const rfvr_proposal* net, const float* xyz, int64_t n, float* logits,
                         const float* g_logits, uint32_t flags, float* g_params, void* ws,
                         size_t ws_bytes, void* stream) {
    int rc;
    if ((rc = check_prop(net))) return rc;
    if (n < 1 || n > kPropMaxPoints || !xyz || !net->params) {
        set_error("n in [1, 2^30], xyz and params are required");
        return RFVR_E_INVALID;
    }
    const bool bwd = g_params != nullptr;
    if (bwd && !g_logits) { set_error("g_logits is required"); return RFVR_E_INVALID; }
    if (flags & ~(uint32_t)RFVR_ACCUMULATE) { set_error("only RFVR_ACCUMULATE is meaningful here"); return RFVR_E_INVALID; }
    const PLayout l = playout(net);
    const size_t need = pbytes(l, (long)n, bwd);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255u)) {
        set_error("workspace too small or misaligned: need %zu bytes", need);
        return RFVR_E_WORKSPACE;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Cx cx{st, MM_FP32};
    const float* P = net->params;
    const long chunk = n < kChunk ? (long)n : kChunk;
    WsCursor cur{reinterpret_cast<char*>(ws), 0};
    float *Wp[4], *WT[4];
    for (int i = 0; i < l.layers; ++i) {
        Wp[i] = cur.take<float>((size_t)(i == 0 ? l.in0p : l.W) * l.W);
        WT[i] = cur.take<float>((size_t)(i == 0 ? l.in0p : l.W) * l.W);
    }
    float* X0 = cur.take<float>((size_t)chunk * l.in0p);
    float* A[4];
    for (int i = 0; i < l.layers; ++i) A[i] = cur.take<float>((size_t)chunk * l.W);
    float *Ab = nullptr, *Ab2 = nullptr, *part = nullptr, *bpart = nullptr, *cpart = nullptr;
    if (bwd) {
        Ab = cur.take<float>((size_t)chunk * l.W);
        Ab2 = cur.take<float>((size_t)chunk * l.W);
        part = cur.take<float>((size_t)kWgSplits * l.W * l.W);
        bpart = cur.take<float>((size_t)kWgSplits * l.W);
        cpart = cur.take<float>((size_t)kColBlocks * l.W);
    }
    for (int i = 0; i < l.layers; ++i) {
        const int fin = i == 0 ? l.in0 : l.W, finp = i == 0 ? l.in0p : l.W;
        hipLaunchKernelGGL(k_pad_cols, dim3(blocks((long)l.W * finp)), dim3(256), 0, st, P + l.oW[i], l.W,
                           fin, finp, Wp[i]);
        hipLaunchKernelGGL(k_transpose_pad, dim3(blocks((long)l.W * finp)), dim3(256), 0, st, P + l.oW[i],
                           l.W, fin, l.W, finp, WT[i]);
    }
    const float beta = 1.0f, inv_half = 1.0f / net->half_size;
    for (long c0 = 0; c0 < n; c0 += chunk) {
        const long m = (n - c0) < chunk ? (n - c0) : chunk;
        const int acc = (c0 > 0 || (flags & RFVR_ACCUMULATE)) ? 1 : 0;
        hipLaunchKernelGGL(k_pe, dim3(blocks(m * l.in0p)), dim3(256), 0, st, m, xyz + 3 * c0, net->centre[0],
                           net->centre[1], net->centre[2], inv_half, l.L, l.in0p, X0, nullptr, nullptr);
        gemm<PRO_ID, EPI_BIAS>(ga(X0, l.in0p, Wp[0], l.in0p, P + l.ob[0], A[0], l.W, m, l.W, l.in0p, beta), cx);
        for (int i = 1; i < l.layers; ++i)
            gemm<PRO_RELU, EPI_BIAS>(ga(A[i - 1], l.W, Wp[i], l.W, P + l.ob[i], A[i], l.W, m, l.W, l.W, beta), cx);
        float* At = A[l.layers - 1];
        if (!bwd) {
            hipLaunchKernelGGL(k_rowdot, dim3(blocks(m * kRowLanes)), dim3(256), 0, st, m, At, (long)l.W, l.W,
                               (int)PRO_RELU, 0, P + l.o_wout, P + l.o_bout, 1.0f, beta, logits + c0);
        } else {
            const float* g = g_logits + c0;
            colsum(At, nullptr, g, l.W, m, l.W, 1, beta, 1.0f, cpart, g_params + l.o_wout, acc, st);
            colsum(g, nullptr, nullptr, 1, m, 1, 0, beta, 1.0f, cpart, g_params + l.o_bout, acc, st);
            hipLaunchKernelGGL(k_relu_out_bwd, dim3(blocks(m * l.W)), dim3(256), 0, st, m, l.W, At, (long)l.W,
                               P + l.o_wout, g, Ab);
            for (int i = l.layers - 1; i >= 0; --i) {
                const int fin = i == 0 ? l.in0 : l.W, finp = i == 0 ? l.in0p : l.W;
                if (i == 0)
                    wgrad<PRO_ID>(Ab, l.W, l.W, X0, nullptr, l.in0p, finp, m, beta, part, cx, bpart);
                else
                    wgrad<PRO_RELU>(Ab, l.W, l.W, A[i - 1], nullptr, l.W, finp, m, beta, part, cx, bpart);
                wg_reduce(part, kWgSplits, l.W, finp, fin, g_params + l.oW[i], acc, st);
                hipLaunchKernelGGL(k_colsum_final, dim3(l.W), dim3(256), 0, st, bpart, kWgSplits, l.W, 1.0f,
                               g_params + l.ob[i], acc);
                if (i > 0) {
                    gemm<PRO_ID, EPI_RELUMASK>(ga(Ab, l.W, WT[i], l.W, nullptr, Ab2, l.W, m, l.W, l.W,
                                                  beta, A[i - 1], l.W), cx);
                    float* t = Ab; Ab = Ab2; Ab2 = t;
                }
            }
        }
        if ((rc = hip_status(hipGetLastError(), "proposal network"))) return rc;
    }
    return RFVR_OK;
}

int rfvr_proposal_forward(const rfvr_proposal* net, const float* xyz, int64_t n, float* logits,
                          void* ws, size_t ws_bytes, void* stream) {
    if (!logits) { set_error("logits output is NULL"); return RFVR_E_INVALID; }
    return proposal_pass(net, xyz, n, logits, nullptr, 0, nullptr, ws, ws_bytes, stream);
}

int rfvr_proposal_backward(const rfvr_proposal* net, const float* xyz, int64_t n,
                           const float* g_logits, uint32_t flags, float* g_params,
                           void* ws, size_t ws_bytes, void* stream) {
    if (!g_params) { set_error("g_params output is NULL"); return RFVR_E_INVALID; }
    return proposal_pass(net, xyz, n, nullptr, g_logits, flags, g_params, ws, ws_bytes, stream);
}

}  // extern "C"
