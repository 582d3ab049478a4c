// Learned surrogate of the refinement filter (a project addition; the
// paper has no learned component).  For every (instance row, column):
//   h_j = (T^j X) for j = 0..3 (h_0 = X), m_c / s_c = mean / std of h_3 over
//   movable rows, r_c = root mean square of h_0 - h_3 over movable rows,
//   f = [(h0 - h3)/r_c, (h1 - h3)/r_c, (h2 - h3)/r_c, (h3 - m_c)/s_c,
//        log1p(d), hsum/d, log(s_c / r_c)],
//   o = w3 . relu(W2 relu(W1 f + b1) + b2) + b3,
//   y = beta_0 h0 + beta_1 h1 + beta_2 h2 + beta_3 h3 + r_c o   (fixed rows keep their input).
// r_c, the displacement of three hops, is a length of the graph's local
// neighbourhoods while s_c grows with the die, so the scaled differences and
// the output correction keep their size on netlists of any size.
//
// Inference runs the three layers on the matrix cores: 16 samples per
// wavefront, bfloat16 operands, float32 accumulation.  Every layer is
// computed transposed (hidden x samples): the accumulator of one 16-row
// output tile leaves lane l with rows 4(l/16)..4(l/16)+3 of sample l%16.
// Layer 1 (7 features padded to K = 16) uses v_mfma_f32_16x16x16_bf16, whose
// B operand has exactly that layout.  Layers 2 and 3 contract over the 64
// hidden units with gfx950's v_mfma_f32_16x16x32_bf16, whose B operand gives
// lane l eight K slots 8(l/16)..8(l/16)+7: the lane's rows of two output
// tiles fill them (slots 8g..8g+3 hold hidden units 32p+4g..+3, slots
// 8g+4..8g+7 hold 32p+16+4g..+3), and the weights are loaded into the A
// operand with the same permutation of K, so no data moves between lanes.  Training runs forward and
// backward in float32 with the same bfloat16 rounding points (weights,
// features and hidden activations), gradients straight through the
// rounding, accumulated per workgroup in a fixed order and reduced in a
// fixed order.
#include <algorithm>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;
constexpr int kH = AHR_MLP_HIDDEN;      // 64
constexpr int kFP = 8;                  // padded feature count
constexpr int kNP = AHR_MLP_NPARAM;     // 4801
constexpr int oW1 = 0, oB1 = kH * kFP, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kH;
static_assert(oB3 + 1 == kNP, "parameter layout");

typedef short v2s __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Hidden unit of K slot q (0..31) of chunk p in the layers contracting over
// the hidden units (see above).
__device__ __forceinline__ int hid(int p, int q) { return 32 * p + ((q & 4) ? 16 : 0) + 4 * (q >> 3) + (q & 3); }

__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0,
                                                  0);
}

// float32 -> bfloat16, round to nearest even (v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ short bf16_bits(float x) { return __builtin_bit_cast(short, static_cast<__bf16>(x)); }
__device__ __forceinline__ float bf16_round(float x) { return static_cast<float>(static_cast<__bf16>(x)); }

// ---------------------------------------------------------------- inference

// relu then bfloat16 of two values, as relu of the bfloat16 values (rounding
// keeps the sign): one packed conversion, then one packed signed 16-bit max
// with 0, since a negative bfloat16 has its sign bit set.
typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v2s relu_bf16x2(float a, float b) {
    const v2bf t = __builtin_convertvector((v2f{a, b}), v2bf);
    return __builtin_elementwise_max(__builtin_bit_cast(v2s, t), v2s{0, 0});
}

__device__ __forceinline__ v4s relu_bf16x4(v4f acc) {
    const v2s lo = relu_bf16x2(acc[0], acc[1]), hi = relu_bf16x2(acc[2], acc[3]);
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3);
}

struct MlpRegs {
    v4s w1[4];        // A tiles of W1 (hidden 16m.., features 0..15)
    v8s w2[8];        // A tiles of W2 (out 16n.., in chunk p of 32, K permuted), index 2n + p
    v8s w3[2];        // A tiles with w3 in row 0 (chunk p, K permuted)
    float b1[16], b2[16];
    float b3;
};

__device__ __forceinline__ void load_mlp(const float* __restrict__ P, MlpRegs& R) {
    const int l = lane_id(), i = l & 15, g = l >> 4;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int k = 4 * g + j;
            R.w1[m][j] = k < kFP ? bf16_bits(P[oW1 + (16 * m + i) * kFP + k]) : static_cast<short>(0);
            R.b1[4 * m + j] = P[oB1 + 16 * m + k];
            R.b2[4 * m + j] = P[oB2 + 16 * m + k];
        }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int h = hid(p, 8 * g + j);
            R.w3[p][j] = i == 0 ? bf16_bits(P[oW3 + h]) : static_cast<short>(0);
#pragma unroll
            for (int n = 0; n < 4; ++n) R.w2[2 * n + p][j] = bf16_bits(P[oW2 + (16 * n + i) * kH + h]);
        }
    R.b3 = P[oB3];
}

// One tile of 16 samples.  f holds features 4(l/16)..4(l/16)+3 of sample
// l%16; the result is valid in lanes 0..15 (sample = lane).
__device__ __forceinline__ float mlp_tile(const MlpRegs& R, const float f[4]) {
    const v2bf x01 = __builtin_convertvector((v2f{f[0], f[1]}), v2bf);
    const v2bf x23 = __builtin_convertvector((v2f{f[2], f[3]}), v2bf);
    const v4s x = __builtin_shufflevector(__builtin_bit_cast(v2s, x01), __builtin_bit_cast(v2s, x23), 0, 1, 2, 3);
    v4s a1[4], a2[4];
    // each layer's accumulator starts at its bias (float32)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        v4f acc = {R.b1[4 * m], R.b1[4 * m + 1], R.b1[4 * m + 2], R.b1[4 * m + 3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(R.w1[m], x, acc, 0, 0, 0);
        a1[m] = relu_bf16x4(acc);
    }
    // the lane's rows of output tiles 2p and 2p+1: the B operand of chunk p
    v8s b1[2], b2[2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b1[p][j] = a1[2 * p][j];
            b1[p][4 + j] = a1[2 * p + 1][j];
        }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        v4f acc = {R.b2[4 * n], R.b2[4 * n + 1], R.b2[4 * n + 2], R.b2[4 * n + 3]};
#pragma unroll
        for (int p = 0; p < 2; ++p) acc = mfma32(R.w2[2 * n + p], b1[p], acc);
        a2[n] = relu_bf16x4(acc);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b2[p][j] = a2[2 * p][j];
            b2[p][4 + j] = a2[2 * p + 1][j];
        }
    v4f acc = {R.b3, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < 2; ++p) acc = mfma32(R.w3[p], b2[p], acc);
    return acc[0];
}

// o[s] for a flat list of feature rows feats[n][8].
__global__ void __launch_bounds__(kBT) k_mlp_forward(const float* __restrict__ P, const float* __restrict__ feats,
                                                     int64_t n, float* __restrict__ o) {
    MlpRegs R;
    load_mlp(P, R);
    const int l = lane_id(), g = l >> 4;
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBT / kWave);
    const int64_t ntiles = (n + 15) / 16;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * (kBT / kWave) + wave_id(); t < ntiles; t += waves) {
        const int64_t smp = t * 16 + (l & 15);
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        if (smp < n && g < 2) {
            float4 v = reinterpret_cast<const float4*>(feats + smp * kFP)[g];
            f[0] = v.x, f[1] = v.y, f[2] = v.z, f[3] = v.w;
        }
        float r = mlp_tile(R, f);
        if (l < 16 && smp < n) o[smp] = r;
    }
}

// Signal value h of (execution row, column) from the scaled chain z
// (inv_s = 1 / s of the row; 0 for an isolated row, whose value is its input).
__device__ __forceinline__ float unscale(const float* z, int C, int r, int c, float inv_s, const float* in,
                                         const int32_t* perm) {
    return inv_s > 0.f ? z[static_cast<int64_t>(r) * C + c] * inv_s : in[static_cast<int64_t>(perm[r]) * C + c];
}

struct LearnArgs {
    const float* z0;        // the expanded input, scaled like the hops
    const float* z1;
    const float* z2;
    const float* z3;
    const float* scale;
    const double* deg;
    const float* hsum;
    const float* stats;     // [3][C]: mean and std of h3, rms of h0 - h3
    const float4* rowf;     // [n_inst] per execution row: 1/s, log1p(d), hsum/d, row code (bits)
    const float* in;
    float* out;
    float* feats;           // optional [n_inst * C][8], instance order
    float* hops;            // optional [4][n_inst][C], instance order
    const uint8_t* flags;
    const int32_t* perm;
    const float* params;
    float beta[4];
    int32_t n_inst;
    int write_out;
};

// Per-row inputs of the features, once per row instead of once per column:
// 1/s, log1p(d), hsum/d (the last two in float64, then rounded), and the
// row's instance with its fixed flag in the sign bit (the bits of w), so the
// network's epilogue needs no dependent load to find where its result goes.
__device__ __forceinline__ int row_inst(int code) { return code & 0x7fffffff; }
__device__ __forceinline__ bool row_fixed(int code) { return code < 0; }

__global__ void k_row_feat(int32_t n, const float* __restrict__ scale, const double* __restrict__ deg,
                           const float* __restrict__ hsum, const int32_t* __restrict__ perm,
                           const uint8_t* __restrict__ flags, float4* __restrict__ rowf) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float s = scale[r];
    const double d = deg[r];
    const int inst = perm[r];
    const int code = inst | ((flags[inst] & AHR_NODE_FIXED) ? static_cast<int>(0x80000000u) : 0);
    rowf[r] = make_float4(s > 0.f ? 1.f / s : 0.f, static_cast<float>(log1p(d)),
                          d > 0 ? static_cast<float>(static_cast<double>(hsum[r]) / d) : 0.f, __int_as_float(code));
}

// One sample's inputs: the scaled hops z_j (h = z_j / s once the row's 1/s
// is known) and the row inputs, none depending on another, so the next
// group's loads are in flight while the current one runs through the
// network.
struct SampleIn {
    float h[4];
    float4 rf;
};

template <int C>
__device__ __forceinline__ SampleIn sample_load(const LearnArgs& a, int64_t smp) {
    SampleIn t;
    const int64_t r = smp / C;
    t.h[0] = t.h[1] = t.h[2] = t.h[3] = 0.f;
    t.rf = make_float4(0.f, 0.f, 0.f, 0.f);
    if (r < a.n_inst) {
        t.rf = a.rowf[r];
        t.h[0] = a.z0[smp];
        t.h[1] = a.z1[smp];
        t.h[2] = a.z2[smp];
        t.h[3] = a.z3[smp];
    }
    return t;
}

// The hops' values from the loaded z: h = z / s, or the input for a row
// with s = 0 (isolated: every power of the operator keeps its value), which
// is rare, so its dependent load sits in a branch of its own.
template <int C>
__device__ __forceinline__ void sample_unscale(const LearnArgs& a, SampleIn& t, int64_t smp) {
    const float inv_s = t.rf.x;
    if (inv_s > 0.f) {
#pragma unroll
        for (int j = 0; j < 4; ++j) t.h[j] *= inv_s;
    } else if (smp / C < a.n_inst) {
        const float v = a.in[static_cast<int64_t>(row_inst(__float_as_int(t.rf.w))) * C + smp % C];
#pragma unroll
        for (int j = 0; j < 4; ++j) t.h[j] = v;
    }
}

// The learned filter over the instance rows, 64 samples (64/C rows x C
// columns) per wavefront and step: each lane loads and featurises its own
// sample (its column is the same at every step, as 64 % C == 0, so its
// column statistics are loaded once), then the network runs the four
// 16-sample matrix-core tiles in turn, each fed by shuffles (features 0..3
// to lanes 0..15, features 4..7 to lanes 16..31), and every lane takes its
// sample's result back and writes it.  The next step's loads are in flight
// meanwhile.  A sample's result does not depend on its tile's other samples.
template <int C>
__global__ void __launch_bounds__(kBT) k_mlp_learned(LearnArgs a) {
    MlpRegs R;
    load_mlp(a.params, R);
    const int l = lane_id(), g = l >> 4, i = l & 15;
    const int c = l % C;
    const float mc = a.stats[c], sc = a.stats[C + c], rc = a.stats[2 * C + c];
    const float inv_sc = 1.f / sc, inv_rc = 1.f / rc;
    const float lsr = static_cast<float>(log(static_cast<double>(sc) / static_cast<double>(rc)));
    const int64_t waves = static_cast<int64_t>(gridDim.x) * (kBT / kWave);
    const int64_t nsteps = (static_cast<int64_t>(a.n_inst) * C + kWave - 1) / kWave;
    int64_t t = static_cast<int64_t>(blockIdx.x) * (kBT / kWave) + wave_id();
    SampleIn cur = sample_load<C>(a, t * kWave + l);
    for (; t < nsteps; t += waves) {
        const SampleIn nxt = sample_load<C>(a, (t + waves) * kWave + l);
        const int64_t smp = t * kWave + l;
        sample_unscale<C>(a, cur, smp);
        float F[8];
        F[0] = (cur.h[0] - cur.h[3]) * inv_rc;
        F[1] = (cur.h[1] - cur.h[3]) * inv_rc;
        F[2] = (cur.h[2] - cur.h[3]) * inv_rc;
        F[3] = (cur.h[3] - mc) * inv_sc;
        F[4] = cur.rf.y;
        F[5] = cur.rf.z;
        F[6] = lsr;
        F[7] = 0.f;
        float mine = 0.f;
#pragma unroll
        for (int j = 0; j < kWave / 16; ++j) {
            const int src = 16 * j + i;
            float f[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float lo = __shfl(F[k], src), hi = __shfl(F[4 + k], src);
                f[k] = g == 0 ? lo : (g == 1 ? hi : 0.f);
            }
            const float o = __shfl(mlp_tile(R, f), i);     // tile j's result for sample 16 j + i
            if (g == j) mine = o;
        }
        const int64_t r = smp / C;
        if (r < a.n_inst) {
            const int code = __float_as_int(cur.rf.w), inst = row_inst(code);
            const int64_t oc = static_cast<int64_t>(inst) * C + c;
            if (a.feats) {
                float* fp = a.feats + oc * kFP;
                fp[0] = F[0], fp[1] = F[1], fp[2] = F[2], fp[3] = F[3];
            }
            if (a.hops) {
                const int64_t nc = static_cast<int64_t>(a.n_inst) * C;
#pragma unroll
                for (int j = 0; j < 4; ++j) a.hops[j * nc + oc] = cur.h[j];
            }
            if (a.write_out) {
                float y = a.beta[0] * cur.h[0] + a.beta[1] * cur.h[1] + a.beta[2] * cur.h[2] + a.beta[3] * cur.h[3] +
                          rc * mine;
                a.out[oc] = row_fixed(code) ? a.in[oc] : y;
            }
        }
        cur = nxt;
    }
}

// Features 4..7 of every sample (the row values, the column's log(s/r) and
// the padding), for the exported feature rows.
template <int C>
__global__ void k_feature_row(LearnArgs a) {
    int64_t smp = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (smp >= static_cast<int64_t>(a.n_inst) * C) return;
    const int r = static_cast<int>(smp / C), c = static_cast<int>(smp % C);
    const float4 rf = a.rowf[r];
    const double lsr = log(static_cast<double>(a.stats[C + c]) / static_cast<double>(a.stats[2 * C + c]));
    *reinterpret_cast<float4*>(a.feats + (static_cast<int64_t>(a.perm[r]) * C + c) * kFP + 4) =
        make_float4(rf.y, rf.z, static_cast<float>(lsr), 0.f);
}

// Column statistics over movable instance rows in one pass (fixed grid,
// float64 partials added in a fixed order): per column the sums of h3 - c
// and (h3 - c)^2, with c the column's value at execution row 0 (a shift that
// lies inside the data, so the variance E[(h3-c)^2] - E[h3-c]^2 loses few
// digits), and of (h0 - h3)^2.
constexpr int kStatGrid = 512;

template <int C>
__global__ void __launch_bounds__(kBT) k_colstat(LearnArgs a, double* __restrict__ part) {
    __shared__ double red[kBT / kWave];
    constexpr int W = 3 * C + 1;
    double shift[C];
#pragma unroll
    for (int c = 0; c < C; ++c) shift[c] = 0;
    if (a.n_inst > 0) {
        const float inv_s0 = a.rowf[0].x;
#pragma unroll
        for (int c = 0; c < C; ++c) shift[c] = unscale(a.z3, C, 0, c, inv_s0, a.in, a.perm);
    }
    double acc[W];
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = 0;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x; r < a.n_inst;
         r += static_cast<int64_t>(kStatGrid) * kBT) {
        const float4 rf = a.rowf[r];
        if (row_fixed(__float_as_int(rf.w))) continue;
        const float inv_s = rf.x;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double h = unscale(a.z3, C, static_cast<int>(r), c, inv_s, a.in, a.perm);
            const double d = h - shift[c];
            const double d0 = unscale(a.z0, C, static_cast<int>(r), c, inv_s, a.in, a.perm) - h;
            acc[c] += d;
            acc[C + c] += d * d;
            acc[2 * C + c] += d0 * d0;
        }
        acc[3 * C] += 1.0;
    }
#pragma unroll
    for (int c = 0; c < W; ++c) {
        double v = block_sum_f64<kBT>(acc[c], red);
        if (threadIdx.x == 0) part[static_cast<int64_t>(blockIdx.x) * W + c] = v;
    }
}

// stats [3][C]: mean and standard deviation of h3, rms of h0 - h3 (a zero
// deviation or rms becomes 1).  One workgroup: each thread adds a fixed
// stride of the partials in order, then a fixed block reduction.
template <int C>
__global__ void __launch_bounds__(kBT) k_colstat_final(LearnArgs a, const double* __restrict__ part,
                                                       float* __restrict__ stats) {
    __shared__ double red[kBT / kWave];
    constexpr int W = 3 * C + 1;
    double tot[W];
#pragma unroll
    for (int c = 0; c < W; ++c) tot[c] = 0;
    for (int b = threadIdx.x; b < kStatGrid; b += kBT)
#pragma unroll
        for (int c = 0; c < W; ++c) tot[c] += part[static_cast<int64_t>(b) * W + c];
#pragma unroll
    for (int c = 0; c < W; ++c) tot[c] = block_sum_f64<kBT>(tot[c], red);
    if (threadIdx.x != 0) return;
    const double n = tot[3 * C];
    const float inv_s0 = a.n_inst > 0 ? a.rowf[0].x : 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const double shift = a.n_inst > 0 ? unscale(a.z3, C, 0, c, inv_s0, a.in, a.perm) : 0.0;
        const double m1 = n > 0 ? tot[c] / n : 0.0;
        const double var = n > 0 ? tot[C + c] / n - m1 * m1 : 0.0;
        const double sd = var > 0 ? sqrt(var) : 0.0;
        const double rms = n > 0 ? sqrt(tot[2 * C + c] / n) : 0.0;
        stats[c] = n > 0 ? static_cast<float>(shift + m1) : 0.f;
        stats[C + c] = sd > 0 ? static_cast<float>(sd) : 1.f;
        stats[2 * C + c] = rms > 0 ? static_cast<float>(rms) : 1.f;
    }
}

// ---------------------------------------------------------------- training

constexpr int kTS = 32;           // samples per tile
constexpr int kGradGrid = 240;    // workgroups (fixed: fixes the summation order)

// Q: the inference's bfloat16 rounding points (weights, features, hidden
// activations); without, float32 operands throughout.
template <bool Q>
__device__ __forceinline__ float qround(float x) {
    if constexpr (Q) return bf16_round(x);
    else return x;
}

template <bool Q>
__global__ void __launch_bounds__(kBT) k_mlp_grad(const float* __restrict__ P, const float* __restrict__ feats,
                                                  const float* __restrict__ target, int64_t n, float inv_n,
                                                  float* __restrict__ part, double* __restrict__ loss_part) {
    __shared__ float W1q[kH * kFP], W2q[kH * kH], w3q[kH], b1[kH], b2[kH];
    __shared__ float X[kTS][kFP];
    __shared__ float Z1[kTS][kH], A1[kTS][kH], Z2[kTS][kH], D2[kTS][kH];
    __shared__ float dO[kTS];
    __shared__ double red[kBT / kWave];
    const int t = threadIdx.x;
    for (int e = t; e < kH * kFP; e += kBT) W1q[e] = qround<Q>(P[oW1 + e]);
    for (int e = t; e < kH * kH; e += kBT) W2q[e] = qround<Q>(P[oW2 + e]);
    if (t < kH) {
        w3q[t] = qround<Q>(P[oW3 + t]);
        b1[t] = P[oB1 + t];
        b2[t] = P[oB2 + t];
    }
    const float b3 = P[oB3];
    float gW2[16], gW1[2], gv = 0.f;     // gv: gb1 / gb2 / gw3 / gb3 entry of this thread
    for (int q = 0; q < 16; ++q) gW2[q] = 0.f;
    gW1[0] = gW1[1] = 0.f;
    double loss = 0;
    __syncthreads();
    const int64_t ntiles = (n + kTS - 1) / kTS;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += kGradGrid) {
        const int64_t s0 = tile * kTS;
        {
            int s = t / kFP, f = t % kFP;
            int64_t smp = s0 + s;
            X[s][f] = smp < n ? qround<Q>(feats[smp * kFP + f]) : 0.f;
        }
        __syncthreads();
        for (int q = 0; q < 8; ++q) {
            int e = t + kBT * q, s = e / kH, h = e % kH;
            float z = b1[h];
            for (int f = 0; f < kFP; ++f) z = __fmaf_rn(X[s][f], W1q[h * kFP + f], z);
            Z1[s][h] = z;
            A1[s][h] = qround<Q>(z > 0.f ? z : 0.f);
        }
        __syncthreads();
        for (int q = 0; q < 8; ++q) {
            int e = t + kBT * q, s = e / kH, h = e % kH;
            float z = b2[h];
            for (int k = 0; k < kH; ++k) z = __fmaf_rn(A1[s][k], W2q[h * kH + k], z);
            Z2[s][h] = z;
        }
        __syncthreads();
        if (t < kTS) {
            int64_t smp = s0 + t;
            float o = b3;
            for (int h = 0; h < kH; ++h) {
                float z = Z2[t][h];
                o = __fmaf_rn(qround<Q>(z > 0.f ? z : 0.f), w3q[h], o);
            }
            if (smp < n) {
                float e = o - target[smp];
                loss += static_cast<double>(e) * e;
                dO[t] = 2.f * e * inv_n;
            } else {
                dO[t] = 0.f;
            }
        }
        __syncthreads();
        for (int q = 0; q < 8; ++q) {
            int e = t + kBT * q, s = e / kH, h = e % kH;
            D2[s][h] = Z2[s][h] > 0.f ? dO[s] * w3q[h] : 0.f;
        }
        __syncthreads();
        for (int q = 0; q < 16; ++q) {
            int e = t + kBT * q, h = e / kH, k = e % kH;
            float a = gW2[q];
            for (int s = 0; s < kTS; ++s) a = __fmaf_rn(D2[s][h], A1[s][k], a);
            gW2[q] = a;
        }
        if (t >= kH && t < 2 * kH) {
            for (int s = 0; s < kTS; ++s) gv += D2[s][t - kH];
        } else if (t >= 2 * kH && t < 3 * kH) {
            int h = t - 2 * kH;
            for (int s = 0; s < kTS; ++s) {
                float z = Z2[s][h];
                gv = __fmaf_rn(dO[s], qround<Q>(z > 0.f ? z : 0.f), gv);
            }
        } else if (t == 3 * kH) {
            for (int s = 0; s < kTS; ++s) gv += dO[s];
        }
        __syncthreads();
        // dz1 = (W2^T dz2) masked by z1 > 0, into Z2 (no longer needed)
        for (int q = 0; q < 8; ++q) {
            int e = t + kBT * q, s = e / kH, k = e % kH;
            float a = 0.f;
            for (int h = 0; h < kH; ++h) a = __fmaf_rn(D2[s][h], W2q[h * kH + k], a);
            Z2[s][k] = Z1[s][k] > 0.f ? a : 0.f;
        }
        __syncthreads();
        for (int q = 0; q < 2; ++q) {
            int e = t + kBT * q, h = e / kFP, f = e % kFP;
            float a = gW1[q];
            for (int s = 0; s < kTS; ++s) a = __fmaf_rn(Z2[s][h], X[s][f], a);
            gW1[q] = a;
        }
        if (t < kH)
            for (int s = 0; s < kTS; ++s) gv += Z2[s][t];
        __syncthreads();
    }
    float* pb = part + static_cast<int64_t>(blockIdx.x) * kNP;
    for (int q = 0; q < 16; ++q) pb[oW2 + t + kBT * q] = gW2[q];
    for (int q = 0; q < 2; ++q) pb[oW1 + t + kBT * q] = gW1[q];
    if (t < kH) pb[oB1 + t] = gv;
    else if (t < 2 * kH) pb[oB2 + t - kH] = gv;
    else if (t < 3 * kH) pb[oW3 + t - 2 * kH] = gv;
    else if (t == 3 * kH) pb[oB3] = gv;
    double ls = block_sum_f64<kBT>(loss, red);
    if (t == 0) loss_part[blockIdx.x] = ls;
}

__global__ void k_mlp_grad_final(const float* __restrict__ part, const double* __restrict__ loss_part, double inv_n,
                                 float* __restrict__ grad, double* __restrict__ loss) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNP) {
        float a = 0.f;
        for (int b = 0; b < kGradGrid; ++b) a += part[static_cast<int64_t>(b) * kNP + p];
        grad[p] = a;
    }
    if (p == 0 && loss) {
        double s = 0;
        for (int b = 0; b < kGradGrid; ++b) s += loss_part[b];
        *loss = s * inv_n;
    }
}

__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    float gp = g[p];
    float mp = b1 * m[p] + (1.f - b1) * gp;
    float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

template <int C>
void learned_c(Graph& g, const ahr_filter_spec& spec, const float* params, const float beta[4], const float* in,
               float* out, float* feats, float* hops, float* stats_out, hipStream_t s) {
    run_hops(g, spec, in, C, s);
    LearnArgs a;
    a.z0 = g.z0.p;
    a.z1 = g.zh[0].p;
    a.z2 = g.zh[1].p;
    a.z3 = g.zh[2].p;
    a.scale = g.scale.p;
    a.deg = g.deg.p;
    a.hsum = g.hsum.p;
    a.in = in;
    a.out = out;
    a.feats = feats;
    a.hops = hops;
    a.flags = g.nl.node_flags;
    a.perm = g.perm.p;
    a.params = params;
    for (int j = 0; j < 4; ++j) a.beta[j] = beta[j];
    a.n_inst = g.n_inst;
    a.write_out = out != nullptr;
    DevBuf<double> part;
    DevBuf<float> stats;
    DevBuf<float4> rowf;
    part.ensure(static_cast<size_t>(kStatGrid) * (3 * C + 1), s);
    stats.ensure(3 * C, s);
    rowf.ensure(static_cast<size_t>(g.n_inst) + 1, s);
    a.stats = stats.p;
    a.rowf = rowf.p;
    hipLaunchKernelGGL(k_row_feat, dim3(grid_for(g.n_inst, kBT)), dim3(kBT), 0, s, g.n_inst, g.scale.p, g.deg.p,
                       g.hsum.p, g.perm.p, g.nl.node_flags, rowf.p);
    AHR_LAUNCHED("k_row_feat");
    hipLaunchKernelGGL((k_colstat<C>), dim3(kStatGrid), dim3(kBT), 0, s, a, part.p);
    AHR_LAUNCHED("k_colstat");
    hipLaunchKernelGGL((k_colstat_final<C>), dim3(1), dim3(kBT), 0, s, a, part.p, stats.p);
    AHR_LAUNCHED("k_colstat_final");
    if (stats_out) AHR_HIP(hipMemcpyAsync(stats_out, stats.p, 3 * C * sizeof(float), hipMemcpyDeviceToDevice, s));
    {
        ProfScope ps(kStageMlp, s);
        // one resident set of workgroups, each wave walking its tiles with
        // the prefetch running: workgroups per CU at this kernel's occupancy
        // times the CUs
        const int64_t ntiles = (static_cast<int64_t>(g.n_inst) * C + 15) / 16;
        int dev = 0, cus = 0, per_cu = 0;
        AHR_HIP(hipGetDevice(&dev));
        AHR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        AHR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_learned<C>, kBT, 0));
        const int64_t resident = static_cast<int64_t>(cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
        const int64_t blocks = std::min<int64_t>((ntiles + 3) / 4, resident);
        hipLaunchKernelGGL((k_mlp_learned<C>), dim3(static_cast<unsigned>(blocks < 1 ? 1 : blocks)), dim3(kBT), 0, s,
                           a);
        AHR_LAUNCHED("k_mlp_learned");
    }
    if (feats) {
        const int64_t ns = static_cast<int64_t>(g.n_inst) * C;
        hipLaunchKernelGGL((k_feature_row<C>), dim3(grid_for(ns, kBT)), dim3(kBT), 0, s, a);
        AHR_LAUNCHED("k_feature_row");
    }
    part.release(s);
    stats.release(s);
    rowf.release(s);
}

}  // namespace

void run_learned(Graph& g, const ahr_filter_spec& spec, const float* params, const float beta[4], const float* in,
                 float* out, int32_t ncols, float* feats, float* hops, float* stats, hipStream_t s) {
    switch (ncols) {
        case 1: learned_c<1>(g, spec, params, beta, in, out, feats, hops, stats, s); break;
        case 2: learned_c<2>(g, spec, params, beta, in, out, feats, hops, stats, s); break;
        case 4: learned_c<4>(g, spec, params, beta, in, out, feats, hops, stats, s); break;
        case 8: learned_c<8>(g, spec, params, beta, in, out, feats, hops, stats, s); break;
        default: throw Error{AHR_EUNSUPPORTED, "ncols must be 1, 2, 4 or 8"};
    }
}

void mlp_forward(const float* params, const float* feats, int64_t n, float* o, hipStream_t s) {
    if (n <= 0) return;
    const int64_t ntiles = (n + 15) / 16;
    const int64_t blocks = std::min<int64_t>((ntiles + 3) / 4, 256 * 16);
    hipLaunchKernelGGL(k_mlp_forward, dim3(static_cast<unsigned>(blocks)), dim3(kBT), 0, s, params, feats, n, o);
    AHR_LAUNCHED("k_mlp_forward");
}

void mlp_loss_grad(const float* params, const float* feats, const float* target, int64_t n, float* grad,
                   double* loss, bool rounding, hipStream_t s) {
    DevBuf<float> part;
    DevBuf<double> lpart;
    part.ensure(static_cast<size_t>(kGradGrid) * kNP, s);
    lpart.ensure(kGradGrid, s);
    const float inv_n = n > 0 ? 1.f / static_cast<float>(n) : 0.f;
    if (rounding)
        hipLaunchKernelGGL(k_mlp_grad<true>, dim3(kGradGrid), dim3(kBT), 0, s, params, feats, target, n, inv_n,
                           part.p, lpart.p);
    else
        hipLaunchKernelGGL(k_mlp_grad<false>, dim3(kGradGrid), dim3(kBT), 0, s, params, feats, target, n, inv_n,
                           part.p, lpart.p);
    AHR_LAUNCHED("k_mlp_grad");
    hipLaunchKernelGGL(k_mlp_grad_final, dim3(grid_for(kNP, kBT)), dim3(kBT), 0, s, part.p, lpart.p,
                       n > 0 ? 1.0 / static_cast<double>(n) : 0.0, grad, loss);
    AHR_LAUNCHED("k_mlp_grad_final");
    part.release(s);
    lpart.release(s);
}

void mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step, float lr, float b1, float b2,
              float eps, hipStream_t s) {
    const float c1 = 1.f - powf(b1, static_cast<float>(step));
    const float c2 = 1.f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(kNP, kBT)), dim3(kBT), 0, s, params, m, v, grad, lr, b1, b2, eps, c1, c2);
    AHR_LAUNCHED("k_adam");
}

}  // namespace ahr
