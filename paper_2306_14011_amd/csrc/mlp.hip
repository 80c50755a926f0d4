// FP32 kernels of the launch-parameter autotuner's regression network:
// training (forward, backward and Adam over minibatches, one workgroup),
// loss/gradient, prediction, and the exhaustive sweep of the launch space
// with a top-k selection of the lowest predicted runtimes.
//
// Network IN -> 64 -> 64 -> 64 -> 1 with ReLU hidden layers; parameters are
// one flat array W1[64][IN], b1, W2[64][64], b2, W3[64][64], b3, W4[64], b4.
// IN is 14 (the launch features) or 16 (the launch features followed by two
// problem-size features); every kernel is instantiated for both widths.
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "../../include/fv.h"
#include "fv_device.h"

namespace mlp {

constexpr int H = FV_MLP_HID;

// Offsets of the flat parameter array of the network with IN inputs.
template <int IN>
struct Lay {
    static constexpr int oW1 = 0;
    static constexpr int oB1 = oW1 + H * IN;
    static constexpr int oW2 = oB1 + H;
    static constexpr int oB2 = oW2 + H * H;
    static constexpr int oW3 = oB2 + H;
    static constexpr int oB3 = oW3 + H * H;
    static constexpr int oW4 = oB3 + H;
    static constexpr int oB4 = oW4 + H;
    static constexpr int NP = oB4 + 1;
};
static_assert(Lay<FV_MLP_IN>::NP == FV_MLP_NPARAM, "parameter count");
static_assert(Lay<FV_MLP_IN_SIZED>::NP == FV_MLP_NPARAM_SIZED, "parameter count");
static_assert(FV_MLP_IN_SIZED == FV_MLP_IN + FV_MLP_MAX_EXTRA, "input widths");
constexpr int NP_MAX = Lay<FV_MLP_IN_SIZED>::NP;
constexpr int MAXN = 65536;
constexpr int TB = 1024;  // threads of the single-workgroup kernels

// Scratch of the training / gradient kernels for n rows.
struct Scratch {
    float* Z1;    // [n][H] pre-activations
    float* Z2;
    float* Z3;
    float* Da;    // [n][H] deltas
    float* Db;
    float* out;   // [n]
    float* dout;  // [n]
    float* grad;  // [NP_MAX]
};

inline size_t scratch_bytes(int n) { return ((size_t)5 * n * H + 2 * (size_t)n + NP_MAX) * sizeof(float) + 256; }

inline Scratch carve(void* ws, int n) {
    float* p = (float*)ws;
    Scratch s;
    s.Z1 = p;
    p += (size_t)n * H;
    s.Z2 = p;
    p += (size_t)n * H;
    s.Z3 = p;
    p += (size_t)n * H;
    s.Da = p;
    p += (size_t)n * H;
    s.Db = p;
    p += (size_t)n * H;
    s.out = p;
    p += n;
    s.dout = p;
    p += n;
    s.grad = p;
    return s;
}

__device__ __forceinline__ float relu(float z) { return z > 0.f ? z : 0.f; }

// Block-wide sum; every thread gets the result. sm holds TB/64 floats.
__device__ float block_sum(float v, float* sm) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sm[w] = v;
    __syncthreads();
    float t = 0.f;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) t += sm[i];
    __syncthreads();
    return t;
}

// Row r of the minibatch -> row of X.
__device__ __forceinline__ int row_of(const int32_t* rows, int r) { return rows ? rows[r] : r; }

// Dense layer over a minibatch: Z[r][o] = b[o] + sum_i W[o][i] act(A[r][i]).
// act is identity for the input layer (A = X rows) and ReLU otherwise.
template <int IN, int NIN, bool INPUT>
__device__ void layer_fwd(const float* __restrict__ P, int oW, int oB, const float* A, const float* __restrict__ X,
                          const int32_t* rows, int sz, float* Z) {
    for (int e = threadIdx.x; e < sz * H; e += blockDim.x) {
        const int r = e / H, o = e - r * H;
        float a = P[oB + o];
        if (INPUT) {
            const float* x = X + (size_t)row_of(rows, r) * IN;
            for (int i = 0; i < NIN; ++i) a = fmaf(P[oW + o * NIN + i], x[i], a);
        } else {
            const float* h = A + (size_t)r * H;
            for (int i = 0; i < NIN; ++i) a = fmaf(P[oW + o * NIN + i], relu(h[i]), a);
        }
        Z[e] = a;
    }
}

// Forward + loss + backward over sz rows; gradient into s.grad, returns the loss.
template <int IN>
__device__ float forward_backward(const float* __restrict__ P, const float* __restrict__ X,
                                  const float* __restrict__ Y, const int32_t* rows, int sz, float alpha,
                                  const Scratch& s, float* sm) {
    using L = Lay<IN>;
    constexpr int oW1 = L::oW1, oB1 = L::oB1, oW2 = L::oW2, oB2 = L::oB2, oW3 = L::oW3, oB3 = L::oB3,
                  oW4 = L::oW4, oB4 = L::oB4, NP = L::NP;
    layer_fwd<IN, IN, true>(P, oW1, oB1, nullptr, X, rows, sz, s.Z1);
    __syncthreads();
    layer_fwd<IN, H, false>(P, oW2, oB2, s.Z1, X, rows, sz, s.Z2);
    __syncthreads();
    layer_fwd<IN, H, false>(P, oW3, oB3, s.Z2, X, rows, sz, s.Z3);
    __syncthreads();
    float sq = 0.f;
    const float inv = 1.0f / (float)sz;
    for (int r = threadIdx.x; r < sz; r += blockDim.x) {
        float a = P[oB4];
        const float* h = s.Z3 + (size_t)r * H;
        for (int i = 0; i < H; ++i) a = fmaf(P[oW4 + i], relu(h[i]), a);
        s.out[r] = a;
        const float d = a - Y[row_of(rows, r)];
        s.dout[r] = d * inv;
        sq += d * d;
    }
    float w2 = 0.f;
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
        const bool bias = (p >= oB1 && p < oW2) || (p >= oB2 && p < oW3) || (p >= oB3 && p < oW4) || p == oB4;
        if (!bias) w2 += P[p] * P[p];
    }
    sq = block_sum(sq, sm);
    w2 = block_sum(w2, sm);
    const float loss = 0.5f * sq * inv + 0.5f * alpha * w2 * inv;
    const float lam = alpha * inv;

    // output layer: gW4[i] = sum_r dout_r relu(Z3[r][i]) + lam W4[i]; gb4 = sum_r dout_r
    for (int i = threadIdx.x; i < H + 1; i += blockDim.x) {
        float g = 0.f;
        if (i < H) {
            for (int r = 0; r < sz; ++r) g = fmaf(s.dout[r], relu(s.Z3[(size_t)r * H + i]), g);
            s.grad[oW4 + i] = g + lam * P[oW4 + i];
        } else {
            for (int r = 0; r < sz; ++r) g += s.dout[r];
            s.grad[oB4] = g;
        }
    }
    // D3[r][i] = dout_r W4[i] [Z3 > 0]
    for (int e = threadIdx.x; e < sz * H; e += blockDim.x) {
        const int r = e / H, i = e - r * H;
        s.Da[e] = s.Z3[e] > 0.f ? s.dout[r] * P[oW4 + i] : 0.f;
    }
    __syncthreads();
    // hidden layers 3 and 2: weight gradients from the delta, then the delta below
    const float* Zin[2] = {s.Z2, s.Z1};
    const int oWs[2] = {oW3, oW2};
    const int oBs[2] = {oB3, oB2};
    float* Dcur = s.Da;
    float* Dnext = s.Db;
    for (int L = 0; L < 2; ++L) {
        const float* Zi = Zin[L];
        const int oW = oWs[L], oB = oBs[L];
        for (int e = threadIdx.x; e < H * H + H; e += blockDim.x) {
            float g = 0.f;
            if (e < H * H) {
                const int o = e / H, i = e - o * H;
                for (int r = 0; r < sz; ++r) g = fmaf(Dcur[(size_t)r * H + o], relu(Zi[(size_t)r * H + i]), g);
                s.grad[oW + e] = g + lam * P[oW + e];
            } else {
                const int o = e - H * H;
                for (int r = 0; r < sz; ++r) g += Dcur[(size_t)r * H + o];
                s.grad[oB + o] = g;
            }
        }
        for (int e = threadIdx.x; e < sz * H; e += blockDim.x) {
            const int r = e / H, i = e - r * H;
            float a = 0.f;
            for (int o = 0; o < H; ++o) a = fmaf(Dcur[(size_t)r * H + o], P[oW + o * H + i], a);
            Dnext[e] = Zi[e] > 0.f ? a : 0.f;
        }
        __syncthreads();
        float* t = Dcur;
        Dcur = Dnext;
        Dnext = t;
    }
    // input layer: gW1[o][i] = sum_r D1[r][o] x_r[i] + lam W1; gb1
    for (int e = threadIdx.x; e < H * IN + H; e += blockDim.x) {
        float g = 0.f;
        if (e < H * IN) {
            const int o = e / IN, i = e - o * IN;
            for (int r = 0; r < sz; ++r) g = fmaf(Dcur[(size_t)r * H + o], X[(size_t)row_of(rows, r) * IN + i], g);
            s.grad[oW1 + e] = g + lam * P[oW1 + e];
        } else {
            const int o = e - H * IN;
            for (int r = 0; r < sz; ++r) g += Dcur[(size_t)r * H + o];
            s.grad[oB1 + o] = g;
        }
    }
    __syncthreads();
    return loss;
}

template <int IN>
__global__ void __launch_bounds__(TB) k_loss_grad(const float* __restrict__ P, const float* __restrict__ X,
                                                  const float* __restrict__ Y, int n, float alpha, float* grad,
                                                  float* loss, Scratch s) {
    __shared__ float sm[TB / 64];
    const float l = forward_backward<IN>(P, X, Y, nullptr, n, alpha, s, sm);
    for (int p = threadIdx.x; p < Lay<IN>::NP; p += blockDim.x) grad[p] = s.grad[p];
    if (threadIdx.x == 0) *loss = l;
}

template <int IN>
__global__ void __launch_bounds__(TB) k_train(float* P, float* M, float* V, int32_t* tptr, const float* __restrict__ X,
                                              const float* __restrict__ Y, int n, const int32_t* __restrict__ order,
                                              fv_mlp_hparams hp, float* epoch_loss, int32_t* epochs_run, Scratch s) {
    __shared__ float sm[TB / 64];
    int t = *tptr;
    float best = FLT_MAX;
    int noimp = 0;
    int e = 0;
    for (; e < hp.max_epochs; ++e) {
        float acc = 0.f;
        for (int start = 0; start < n; start += hp.batch) {
            const int sz = min(hp.batch, n - start);
            const float lb = forward_backward<IN>(P, X, Y, order + (size_t)e * n + start, sz, hp.alpha, s, sm);
            acc += lb * (float)sz;
            ++t;
            // bias-corrected step size, scalar, in double
            const double c2 = 1.0 - pow((double)hp.beta2, (double)t);
            const double c1 = 1.0 - pow((double)hp.beta1, (double)t);
            const float lrt = (float)((double)hp.lr * sqrt(c2) / c1);
            for (int p = threadIdx.x; p < Lay<IN>::NP; p += blockDim.x) {
                const float g = s.grad[p];
                const float m = hp.beta1 * M[p] + (1.f - hp.beta1) * g;
                const float v = hp.beta2 * V[p] + (1.f - hp.beta2) * g * g;
                M[p] = m;
                V[p] = v;
                P[p] -= lrt * m / (sqrtf(v) + hp.eps);
            }
            __syncthreads();
        }
        const float el = acc / (float)n;
        if (threadIdx.x == 0) epoch_loss[e] = el;
        if (el > best - hp.tol) ++noimp;
        else noimp = 0;
        if (el < best) best = el;
        if (noimp > hp.n_iter_no_change) {
            ++e;
            break;
        }
    }
    if (threadIdx.x == 0) {
        *epochs_run = e;
        *tptr = t;
    }
}

// Forward pass of one row, weights read uniformly across the wave.
template <int IN>
__device__ __forceinline__ float forward_row(const float* __restrict__ P, const float* x) {
    using L = Lay<IN>;
    constexpr int oW1 = L::oW1, oB1 = L::oB1, oW2 = L::oW2, oB2 = L::oB2, oW3 = L::oW3, oB3 = L::oB3,
                  oW4 = L::oW4, oB4 = L::oB4;
    float h1[H], h2[H];
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float a = P[oB1 + o];
#pragma unroll
        for (int i = 0; i < IN; ++i) a = fmaf(P[oW1 + o * IN + i], x[i], a);
        h1[o] = relu(a);
    }
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float a = P[oB2 + o];
#pragma unroll
        for (int i = 0; i < H; ++i) a = fmaf(P[oW2 + o * H + i], h1[i], a);
        h2[o] = relu(a);
    }
    float out = P[oB4];
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float a = P[oB3 + o];
#pragma unroll
        for (int i = 0; i < H; ++i) a = fmaf(P[oW3 + o * H + i], h2[i], a);
        out = fmaf(P[oW4 + o], relu(a), out);
    }
    return out;
}

template <int IN>
__global__ void __launch_bounds__(256) k_predict(const float* __restrict__ P, const float* __restrict__ X, int n,
                                                 float* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    float x[IN];
#pragma unroll
    for (int i = 0; i < IN; ++i) x[i] = X[(size_t)r * IN + i];
    out[r] = forward_row<IN>(P, x);
}

// ---------------------------------------------------------------------------
// Sweep of the launch space.

constexpr int KMAX = 8;
constexpr int SWEEP_T = 256;
constexpr int SWEEP_MAXB = 4096;

struct SweepTab {
    int32_t radix[FV_NSITES];
    float f1[FV_NSITES][FV_SPACE_MAXC];
    float f2[FV_NSITES][FV_SPACE_MAXC];
    float extra[FV_MLP_MAX_EXTRA];
};

// (v, i) orders before (w, j): lower value, ties to the lower index; NaN last.
__device__ __forceinline__ bool before(float v, long long i, float w, long long j) {
    return v < w || (v == w && i < j);
}

// Thread-local ascending top-k list.
struct TopK {
    float v[KMAX];
    long long i[KMAX];
    __device__ void init() {
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {
            v[q] = FLT_MAX;
            i[q] = LLONG_MAX;
        }
    }
    __device__ void insert(float val, long long idx) {
        if (!(val == val)) val = FLT_MAX;  // NaN never wins
        if (!before(val, idx, v[KMAX - 1], i[KMAX - 1])) return;
        float cv = val;
        long long ci = idx;
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {
            if (before(cv, ci, v[q], i[q])) {
                const float tv = v[q];
                const long long ti = i[q];
                v[q] = cv;
                i[q] = ci;
                cv = tv;
                ci = ti;
            }
        }
    }
};

// k rounds of block-wide argmin over cnt (value, index) pairs in vals/idxs
// (LDS or global); selected entries are overwritten with FLT_MAX/LLONG_MAX.
// Thread 0 writes the winners to ov/oi in ascending order.
__device__ void select_topk(float* vals, long long* idxs, int cnt, int k, float* ov, long long* oi, float* smv,
                            long long* smi, int* smp) {
    for (int round = 0; round < k; ++round) {
        float bv = FLT_MAX;
        long long bi = LLONG_MAX;
        int bp = -1;
        for (int p = threadIdx.x; p < cnt; p += blockDim.x) {
            if (before(vals[p], idxs[p], bv, bi)) {
                bv = vals[p];
                bi = idxs[p];
                bp = p;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const float ov2 = __shfl_xor(bv, off, 64);
            const long long oi2 = __shfl_xor(bi, off, 64);
            const int op2 = __shfl_xor(bp, off, 64);
            if (before(ov2, oi2, bv, bi)) {
                bv = ov2;
                bi = oi2;
                bp = op2;
            }
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            smv[w] = bv;
            smi[w] = bi;
            smp[w] = bp;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int nw = blockDim.x >> 6;
            for (int q = 1; q < nw; ++q)
                if (before(smv[q], smi[q], bv, bi)) {
                    bv = smv[q];
                    bi = smi[q];
                    bp = smp[q];
                }
            ov[round] = bv;
            oi[round] = bi;
            if (bp >= 0) {
                vals[bp] = FLT_MAX;
                idxs[bp] = LLONG_MAX;
            }
        }
        __syncthreads();
    }
}

// The sweep on the matrix cores. A wave takes 32 configurations at a time and
// runs the network in transposed form, Z^T = W H^T, with
// v_mfma_f32_32x32x2f32: M = 32 neurons of a block (two blocks per 64-wide
// layer), N = the 32 configurations, K = 2 inputs per instruction. Operand
// lanes: A (32 x 2) has neuron l % 32 and input l / 32, B (2 x 32) input
// l / 32 and configuration l % 32; the 32 x 32 result holds configuration
// l % 32 in every lane and, in register v, neuron 8 (v / 4) + 4 (l / 32) +
// (v % 4). So the activations never move: the next layer takes register v of
// block b as one K pair (lanes 0-31 and 32-63 hold different neurons), and its
// weight operand is permuted to the same neuron order. Each layer's bias is
// one more K step with inputs (1, 0). The weight operands are staged once per
// workgroup in LDS, in the instruction's lane order; the sums run in another
// order than the row-per-thread forward pass (FP32 rounding apart, the same
// network).
typedef float v16f __attribute__((ext_vector_type(16)));

template <int IN>
struct MfLds {
    static constexpr int S1 = IN / 2;                  // K steps of layer 1 (IN is even)
    static constexpr int A1 = 0;                       // [block][step 0 .. S1][lane]
    static constexpr int A2 = A1 + 2 * (S1 + 1) * 64;  // [block][step 0 .. 32][lane]
    static constexpr int A3 = A2 + 2 * 33 * 64;
    static constexpr int W4 = A3 + 2 * 33 * 64;        // [block * 16 + register][lane]
    static constexpr int FLOATS = W4 + 32 * 64;
};

// Neuron of register v of block b in lane half h of a result.
__device__ __forceinline__ int mf_neuron(int b, int v, int h) { return 32 * b + 8 * (v >> 2) + 4 * h + (v & 3); }

// One layer: c[b] = sum over the NST K steps of A (block b, step st) times
// bval(st), the two blocks interleaved. The steps go in groups of four whose
// weight operands are read from LDS while the previous group's instructions
// issue; the scheduling barrier keeps the compiler from hoisting every read
// of the layer (and the registers they take) to its start.
template <int NST, int AOFF, class BF>
__device__ __forceinline__ void mf_layer(const float* A, int lane, BF bval, v16f* c) {
    constexpr int G = 4;
    c[0] = v16f{};
    c[1] = v16f{};
    float a[2][2 * G];
#pragma unroll
    for (int q = 0; q < G; ++q)
        if (q < NST)
#pragma unroll
            for (int b = 0; b < 2; ++b) a[0][2 * q + b] = A[AOFF + (b * NST + q) * 64 + lane];
#pragma unroll
    for (int g = 0; g * G < NST; ++g) {
        const int cur = g & 1;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int st = (g + 1) * G + q;
            if (st < NST)
#pragma unroll
                for (int b = 0; b < 2; ++b) a[cur ^ 1][2 * q + b] = A[AOFF + (b * NST + st) * 64 + lane];
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int st = g * G + q;
            if (st < NST) {
                const float bv = bval(st);
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    c[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[cur][2 * q + b], bv, c[b], 0, 0, 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

constexpr int MF_LDS_BYTES = MfLds<FV_MLP_IN_SIZED>::FLOATS * 4 > SWEEP_T * KMAX * 12
                                 ? MfLds<FV_MLP_IN_SIZED>::FLOATS * 4
                                 : SWEEP_T * KMAX * 12;

template <int IN>
__global__ void __launch_bounds__(SWEEP_T) k_sweep_mfma(const float* __restrict__ P, SweepTab tab, long long begin,
                                                         long long count, int k, float* __restrict__ pv,
                                                         long long* __restrict__ pi) {
    using L = Lay<IN>;
    using M = MfLds<IN>;
    static_assert(IN % 2 == 0, "layer 1 takes inputs in pairs");
    __shared__ __align__(16) unsigned char lds[MF_LDS_BYTES];
    __shared__ float smv[SWEEP_T / 64];
    __shared__ long long smi[SWEEP_T / 64];
    __shared__ int smp[SWEEP_T / 64];
    float* A = (float*)lds;
    // stage the weight operands
    for (int e = threadIdx.x; e < M::FLOATS; e += SWEEP_T) {
        const int l = e & 63, row = e >> 6, m32 = l & 31, h = l >> 5;
        float w;
        if (e < M::A2) {
            const int b = row / (M::S1 + 1), st = row % (M::S1 + 1), m = 32 * b + m32;
            w = st < M::S1 ? P[L::oW1 + m * IN + 2 * st + h] : (h == 0 ? P[L::oB1 + m] : 0.f);
        } else if (e < M::W4) {
            const bool l2 = e < M::A3;
            const int r = row - (l2 ? M::A2 : M::A3) / 64, b = r / 33, st = r % 33, m = 32 * b + m32;
            const int oW = l2 ? L::oW2 : L::oW3, oB = l2 ? L::oB2 : L::oB3;
            w = st < 32 ? P[oW + m * H + mf_neuron(st >> 4, st & 15, h)] : (h == 0 ? P[oB + m] : 0.f);
        } else {
            const int r = row - M::W4 / 64;
            w = P[L::oW4 + mf_neuron(r >> 4, r & 15, h)];
        }
        A[e] = w;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, h = lane >> 5;
    const float one = h == 0 ? 1.f : 0.f;
    const float b4 = P[L::oB4];
    TopK top;
    top.init();
    const long long tiles = (count + 31) / 32;
    const long long nw = (long long)gridDim.x * (SWEEP_T / 64);
    for (long long t = (long long)blockIdx.x * (SWEEP_T / 64) + (threadIdx.x >> 6); t < tiles; t += nw) {
        const long long r = t * 32 + (lane & 31);
        const bool valid = r < count;
        const long long idx = begin + (valid ? r : count - 1);
        unsigned long long rem = (unsigned long long)idx;
        float x[IN];
#pragma unroll
        for (int site = 0; site < FV_NSITES; ++site) {
            const unsigned rd = (unsigned)tab.radix[site];
            const unsigned c = (unsigned)(rem % rd);
            rem /= rd;
            x[2 * site] = tab.f1[site][c];
            x[2 * site + 1] = tab.f2[site][c];
        }
#pragma unroll
        for (int j = 2 * FV_NSITES; j < IN; ++j) x[j] = tab.extra[j - 2 * FV_NSITES];
        v16f c1[2], c2[2], c3[2];
        mf_layer<M::S1 + 1, M::A1>(A, lane, [&](int st) { return st < M::S1 ? (h ? x[2 * st + 1] : x[2 * st]) : one; },
                                   c1);
        mf_layer<33, M::A2>(A, lane, [&](int st) { return st < 32 ? relu(c1[st >> 4][st & 15]) : one; }, c2);
        mf_layer<33, M::A3>(A, lane, [&](int st) { return st < 32 ? relu(c2[st >> 4][st & 15]) : one; }, c3);
        float part = 0.f;
#pragma unroll
        for (int q = 0; q < 32; ++q) part = fmaf(A[M::W4 + q * 64 + lane], relu(c3[q >> 4][q & 15]), part);
        const float out = b4 + (part + __shfl_xor(part, 32, 64));
        if (valid && h == 0) top.insert(out, idx);
    }
    __syncthreads();  // the weight operands are dead: the LDS takes the per-thread lists
    float* lv = (float*)lds;
    long long* li = (long long*)(lds + SWEEP_T * KMAX * 4);
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
        lv[threadIdx.x * KMAX + q] = top.v[q];
        li[threadIdx.x * KMAX + q] = top.i[q];
    }
    __syncthreads();
    select_topk(lv, li, SWEEP_T * KMAX, k, pv + (size_t)blockIdx.x * KMAX, pi + (size_t)blockIdx.x * KMAX, smv, smi,
                smp);
    if (threadIdx.x == 0)
        for (int q = k; q < KMAX; ++q) {
            pv[(size_t)blockIdx.x * KMAX + q] = FLT_MAX;
            pi[(size_t)blockIdx.x * KMAX + q] = LLONG_MAX;
        }
}

__global__ void __launch_bounds__(1024) k_sweep_final(float* pv, long long* pi, int cnt, int k, float* top_val,
                                                      long long* top_idx) {
    __shared__ float smv[16];
    __shared__ long long smi[16];
    __shared__ int smp[16];
    __shared__ float ov[KMAX];
    __shared__ long long oi[KMAX];
    select_topk(pv, pi, cnt, k, ov, oi, smv, smi, smp);
    if (threadIdx.x < k) {
        top_val[threadIdx.x] = ov[threadIdx.x];
        top_idx[threadIdx.x] = oi[threadIdx.x];
    }
}

}  // namespace mlp

namespace mlp {

// Per-block top-k lists of the sweep: values, then (256-byte aligned) indices.
constexpr size_t sweep_scratch_bytes() {
    return (((size_t)SWEEP_MAXB * KMAX * sizeof(float) + 255) & ~(size_t)255) +
           (size_t)SWEEP_MAXB * KMAX * sizeof(long long);
}

// Device scratch of fv_mlp_sweep_static: room for the per-block lists of the
// largest sweep grid (SWEEP_MAXB blocks; larger counts are covered by the
// kernel's grid-stride loop, so no count needs more). Every device the
// library runs on holds its own copy until the process ends.
constexpr size_t STATIC_SCRATCH_BYTES = 393216;
static_assert(STATIC_SCRATCH_BYTES >= sweep_scratch_bytes(), "static sweep scratch too small");
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mu;
static void* scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device, looked up once per
// device (the host-side name of the array is not a device address).
static int static_scratch(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        fprintf(stderr, "fv_mlp_sweep_static: no usable current device\n");
        return FV_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fprintf(stderr, "fv_mlp_sweep_static: hipGetSymbolAddress failed: %s\n", hipGetErrorString(e));
            return FV_EDEVICE;
        }
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return FV_OK;
}

static int launch_status() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        fprintf(stderr, "fv_mlp: launch failed: %s\n", hipGetErrorString(e));
        return FV_EDEVICE;
    }
    return FV_OK;
}

// Validates the sweep's arguments and enqueues it with the per-block lists in
// `ws` (at least sweep_scratch_bytes(), 256-byte aligned). Every list entry
// the final selection reads is written by the block kernel of the same call,
// so `ws` needs no clearing.
static int sweep_launch(const float* params, const fv_tune_space* space, int64_t begin, int64_t count, int32_t k,
                        int64_t* top_idx, float* top_val, void* ws, hipStream_t st) {
    if (!params || !space || !top_idx || !top_val || !ws) return FV_EINVAL;
    if (k < 1 || k > KMAX || begin < 0 || count < 1) return FV_EINVAL;
    if (space->n_extra != 0 && space->n_extra != FV_MLP_MAX_EXTRA) return FV_EINVAL;
    SweepTab tab;
    int64_t total = 1;
    for (int s = 0; s < FV_NSITES; ++s) {
        const int r = space->radix[s];
        if (r < 1 || r > FV_SPACE_MAXC) return FV_EINVAL;
        tab.radix[s] = r;
        total *= r;
        for (int c = 0; c < FV_SPACE_MAXC; ++c) {
            tab.f1[s][c] = c < r ? space->f1[s][c] : 0.f;
            tab.f2[s][c] = c < r ? space->f2[s][c] : 0.f;
        }
    }
    for (int j = 0; j < FV_MLP_MAX_EXTRA; ++j) tab.extra[j] = j < space->n_extra ? space->extra[j] : 0.f;
    if (begin + count > total) return FV_EINVAL;
    // a workgroup's four waves take 32 configurations each per round
    long long blocks = (count + 4 * 32 - 1) / (4 * 32);
    if (blocks > SWEEP_MAXB) blocks = SWEEP_MAXB;
    float* pv = (float*)ws;
    long long* pi = (long long*)((char*)ws + (((size_t)SWEEP_MAXB * KMAX * sizeof(float) + 255) & ~(size_t)255));
    if (space->n_extra == 0)
        hipLaunchKernelGGL(k_sweep_mfma<FV_MLP_IN>, dim3((unsigned)blocks), dim3(SWEEP_T), 0, st, params, tab,
                           (long long)begin, (long long)count, k, pv, pi);
    else
        hipLaunchKernelGGL(k_sweep_mfma<FV_MLP_IN_SIZED>, dim3((unsigned)blocks), dim3(SWEEP_T), 0, st, params, tab,
                           (long long)begin, (long long)count, k, pv, pi);
    hipLaunchKernelGGL(k_sweep_final, dim3(1), dim3(1024), 0, st, pv, pi, (int)(blocks * KMAX), k, top_val,
                       (long long*)top_idx);
    return launch_status();
}

}  // namespace mlp

// ---------------------------------------------------------------------------
// C ABI.

static int mlp_check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        fprintf(stderr, "fv_mlp: launch failed: %s\n", hipGetErrorString(e));
        return FV_EDEVICE;
    }
    return FV_OK;
}

extern "C" {

int fv_mlp_workspace(int32_t n, size_t* bytes) {
    if (n < 1 || n > mlp::MAXN || !bytes) return FV_EINVAL;
    *bytes = mlp::scratch_bytes(n);
    return FV_OK;
}

int fv_mlp_loss_grad(const float* params, int32_t n_in, const float* X, const float* y, int32_t n, float alpha,
                     float* grad, float* loss, void* workspace, size_t ws_bytes, void* stream) {
    if (!params || !X || !y || !grad || !loss || !workspace) return FV_EINVAL;
    if (n_in != FV_MLP_IN && n_in != FV_MLP_IN_SIZED) return FV_EINVAL;
    if (n < 1 || n > mlp::MAXN || !(alpha >= 0.f)) return FV_EINVAL;
    if (ws_bytes < mlp::scratch_bytes(n)) return FV_EWORKSPACE;
    mlp::Scratch s = mlp::carve(workspace, n);
    if (n_in == FV_MLP_IN)
        hipLaunchKernelGGL(mlp::k_loss_grad<FV_MLP_IN>, dim3(1), dim3(mlp::TB), 0, (hipStream_t)stream, params, X, y,
                           n, alpha, grad, loss, s);
    else
        hipLaunchKernelGGL(mlp::k_loss_grad<FV_MLP_IN_SIZED>, dim3(1), dim3(mlp::TB), 0, (hipStream_t)stream, params,
                           X, y, n, alpha, grad, loss, s);
    return mlp_check_launch();
}

int fv_mlp_predict(const float* params, int32_t n_in, const float* X, int32_t n, float* out, void* stream) {
    if (!params || !X || !out || n < 0) return FV_EINVAL;
    if (n_in != FV_MLP_IN && n_in != FV_MLP_IN_SIZED) return FV_EINVAL;
    if (n == 0) return FV_OK;
    if (n_in == FV_MLP_IN)
        hipLaunchKernelGGL(mlp::k_predict<FV_MLP_IN>, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                           params, X, n, out);
    else
        hipLaunchKernelGGL(mlp::k_predict<FV_MLP_IN_SIZED>, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                           params, X, n, out);
    return mlp_check_launch();
}

int fv_mlp_train(float* params, int32_t n_in, float* adam_m, float* adam_v, int32_t* adam_t, const float* X,
                 const float* y, int32_t n, const int32_t* order, const fv_mlp_hparams* hp, float* epoch_loss,
                 int32_t* epochs_run, void* workspace, size_t ws_bytes, void* stream) {
    if (!params || !adam_m || !adam_v || !adam_t || !X || !y || !order || !hp || !epoch_loss || !epochs_run ||
        !workspace)
        return FV_EINVAL;
    if (n_in != FV_MLP_IN && n_in != FV_MLP_IN_SIZED) return FV_EINVAL;
    if (n < 1 || n > mlp::MAXN || hp->batch < 1 || hp->max_epochs < 0 || hp->n_iter_no_change < 0) return FV_EINVAL;
    if (!(hp->lr > 0.f) || !(hp->beta1 >= 0.f && hp->beta1 < 1.f) || !(hp->beta2 >= 0.f && hp->beta2 < 1.f) ||
        !(hp->eps > 0.f) || !(hp->alpha >= 0.f))
        return FV_EINVAL;
    const int bmax = hp->batch < n ? hp->batch : n;
    if (ws_bytes < mlp::scratch_bytes(bmax)) return FV_EWORKSPACE;
    mlp::Scratch s = mlp::carve(workspace, bmax);
    if (n_in == FV_MLP_IN)
        hipLaunchKernelGGL(mlp::k_train<FV_MLP_IN>, dim3(1), dim3(mlp::TB), 0, (hipStream_t)stream, params, adam_m,
                           adam_v, adam_t, X, y, n, order, *hp, epoch_loss, epochs_run, s);
    else
        hipLaunchKernelGGL(mlp::k_train<FV_MLP_IN_SIZED>, dim3(1), dim3(mlp::TB), 0, (hipStream_t)stream, params,
                           adam_m, adam_v, adam_t, X, y, n, order, *hp, epoch_loss, epochs_run, s);
    return mlp_check_launch();
}

int fv_mlp_sweep_workspace(size_t* bytes) {
    if (!bytes) return FV_EINVAL;
    *bytes = mlp::sweep_scratch_bytes();
    return FV_OK;
}

int fv_mlp_sweep(const float* params, const fv_tune_space* space, int64_t begin, int64_t count, int32_t k,
                 int64_t* top_idx, float* top_val, void* workspace, size_t ws_bytes, void* stream) {
    if (!workspace) return FV_EINVAL;
    if (ws_bytes < mlp::sweep_scratch_bytes()) return FV_EWORKSPACE;
    return mlp::sweep_launch(params, space, begin, count, k, top_idx, top_val, workspace, (hipStream_t)stream);
}

int fv_mlp_sweep_static(const float* params, const fv_tune_space* space, int64_t begin, int64_t count, int32_t k,
                        int64_t* top_idx, float* top_val, void* stream) {
    // Sizes: k above 8 is rejected by the argument check (FV_EINVAL); any
    // count fits, the block count being capped at the scratch's capacity.
    void* ws = nullptr;
    const int rc = mlp::static_scratch(&ws);
    if (rc != FV_OK) return rc;
    return mlp::sweep_launch(params, space, begin, count, k, top_idx, top_val, ws, (hipStream_t)stream);
}

}  // extern "C"
