// Learned part: training pairs drawn from the field, multi-candidate Adam
// training (one workgroup per (learning rate, L2) candidate, Fig. 4), and
// selection by validation code entropy (Sec. 4.3).
#include "pwrel_kernels.h"
#include "pwrel_train.h"

namespace pwrel {

// splitmix64 (Steele, Lea, Flood), used as a counter-based hash of seed ^ i
__device__ __forceinline__ unsigned long long mix64(unsigned long long s)
{
    unsigned long long z = s + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Sampling.  kind: 0 = not drawn / dropped, 1 = training pair, 2 = validation.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ int draw(const SampleArgs &a, const DevConsts &c, long long i,
                                    int (&u)[6], int &t)
{
    const double U = (double)(mix64(a.seed ^ (unsigned long long)i) >> 11) * 0x1p-53;
    if (!(U < a.rho))
        return 0;
    const long long n1 = a.n[1], n2 = a.n[2];
    const long long gx = i % n2, gy = (i / n2) % n1, gz = i / (n1 * n2);
    const int B = a.B;
    // every neighbour must exist (and lie in the block in independent mode)
    if (gx == 0 || (D >= 2 && gy == 0) || (D >= 3 && gz == 0))
        return 0;
    if (a.independent && (gx % B == 0 || (D >= 2 && gy % B == 0) || (D >= 3 && gz % B == 0)))
        return 0;
    const T *x = reinterpret_cast<const T *>(a.x);
    int err = kOk;
    int nv[8];
    constexpr int NO = (1 << D) - 1;
#pragma unroll
    for (int o = 0; o <= NO; ++o) {
        const long long j = i - (o & 1) - ((o >> 1) & 1) * n2 - ((o >> 2) & 1) * n1 * n2;
        nv[o] = grid_value((double)x[j], c, err);
    }
    int npos = 0, nneg = 0;
#pragma unroll
    for (int o = 0; o <= NO; ++o) {
        npos += (nv[o] > c.p_zero && nv[o] <= c.b_sign) ? 1 : 0;
        nneg += (nv[o] > c.b_sign) ? 1 : 0;
    }
    if (npos != NO + 1 && nneg != NO + 1)
        return 0;
    const long long tt = (long long)nv[0] - nv[1];
    if (!(tt > -kR && tt < kR))
        return 0;
    constexpr int K = (1 << D) - 2;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long uk = (long long)nv[k + 2] - nv[1];
        if (!(uk > -kR && uk < kR))
            return 0;
        u[k] = (int)uk;
    }
    t = (int)tt;
    return U < 0.2 * a.rho ? 2 : 1;
}

// pass 1: pairs per chunk of kSampleChunk points, training and validation
template <typename T, int D>
__global__ void __launch_bounds__(256) k_sample_count(SampleArgs a, uint32_t *cnt_tr,
                                                      uint32_t *cnt_va)
{
    __shared__ unsigned s_tr, s_va;
    if (threadIdx.x == 0)
        s_tr = s_va = 0;
    __syncthreads();
    const DevConsts c = *a.c;
    const long long base = (long long)blockIdx.x * kSampleChunk;
    unsigned ntr = 0, nva = 0;
    for (int q = threadIdx.x; q < kSampleChunk; q += blockDim.x) {
        const long long i = base + q;
        if (i >= a.N)
            break;
        int u[6], t;
        const int kind = draw<T, D>(a, c, i, u, t);
        ntr += kind == 1;
        nva += kind == 2;
    }
    atomicAdd(&s_tr, ntr);
    atomicAdd(&s_va, nva);
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt_tr[blockIdx.x] = s_tr;
        cnt_va[blockIdx.x] = s_va;
    }
}

// pass 2: write the pairs in ascending point order.  The chunk is walked in
// rounds of 256 points; a wave ballot and the per-wave totals in LDS give
// each kept pair its rank among the training pairs, the validation pairs and
// all pairs (the sum of the two).
template <typename T, int D>
__global__ void __launch_bounds__(256) k_sample_write(SampleArgs a, SampleOut o)
{
    __shared__ unsigned wtr[4], wva[4];
    __shared__ unsigned long long run_tr, run_va;
    constexpr int K = (1 << D) - 2;
    if (threadIdx.x == 0) {
        run_tr = o.off_tr[blockIdx.x];
        run_va = o.off_va[blockIdx.x];
    }
    __syncthreads();
    const DevConsts c = *a.c;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    const long long base = (long long)blockIdx.x * kSampleChunk;
    for (int r0 = 0; r0 < kSampleChunk; r0 += 256) {
        const long long i = base + r0 + threadIdx.x;
        int u[6] = {0, 0, 0, 0, 0, 0}, t = 0;
        const int kind = i < a.N ? draw<T, D>(a, c, i, u, t) : 0;
        const unsigned long long mtr = __ballot(kind == 1), mva = __ballot(kind == 2);
        if (lane == 0) {
            wtr[w] = (unsigned)__popcll(mtr);
            wva[w] = (unsigned)__popcll(mva);
        }
        __syncthreads();
        unsigned long long btr = run_tr, bva = run_va;
        for (int q = 0; q < w; ++q) {
            btr += wtr[q];
            bva += wva[q];
        }
        const unsigned long long rtr = btr + (unsigned)__popcll(mtr & below);
        const unsigned long long rva = bva + (unsigned)__popcll(mva & below);
        if (kind == 1 && o.u_tr && rtr < o.cap_tr) {
            for (int k = 0; k < K; ++k)
                o.u_tr[rtr * K + k] = (float)u[k];
            o.t_tr[rtr] = (float)t;
        } else if (kind == 2 && o.u_tr && rva < o.cap_va) {
            for (int k = 0; k < K; ++k)
                o.u_va[rva * K + k] = (float)u[k];
            o.t_va[rva] = (float)t;
        }
        const unsigned long long ra = rtr + rva;
        if (kind != 0 && o.t_all && ra < o.cap_all) {
            for (int k = 0; k < K; ++k)
                o.u_all[ra * K + k] = u[k];
            o.t_all[ra] = t;
            o.isval[ra] = kind == 2 ? 1 : 0;
            o.idx_all[ra] = (unsigned long long)i;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int q = 0; q < 4; ++q) {
                run_tr += wtr[q];
                run_va += wva[q];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// sigma = max(1, RMS of the training targets): per-workgroup FP64 partial
// sums, then one workgroup adds them in index order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_sumsq(const float *t, long long n, double *part)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        s += (double)t[i] * (double)t[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < d)
            sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = sh[0];
}

__global__ void k_sigma(const double *part, int nparts, long long n, double *sigma)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i)
        s += part[i];
    double sg = n > 0 ? sqrt(s / (double)n) : 1.0;
    *sigma = sg < 1.0 ? 1.0 : sg;
}

// ---------------------------------------------------------------------------
// Forward and backward of one minibatch (shared by the trainer and the
// gradient entry point).  Thread i < nb owns pair i; parameter layout
// [w1 (H x K) | b1 (H) | v (H) | b2] in the scaled domain.
// ---------------------------------------------------------------------------
// HM: compile-time bound of the hidden width H (H <= HM)
template <int HM, int K>
__device__ __forceinline__ float forward_pair(const float *th, int H, const float *us, float ts,
                                              float alpha, float *zrow)
{
    const float *W = th, *b1 = th + H * K, *v = th + H * K + H;
    float y = th[H * K + 2 * H];
#pragma unroll
    for (int j = 0; j < HM; ++j) {
        if (j < H) {
            float a = b1[j];
#pragma unroll
            for (int k = 0; k < K; ++k)
                a = __builtin_fmaf(W[j * K + k], us[k], a);
            zrow[j] = a;
            const float h = a < 0.0f ? alpha * a : a;
            y = __builtin_fmaf(v[j], h, y);
        }
    }
    return y - ts;
}

// Minibatch rows in LDS padded to an odd number of words, so that the
// threads of a wave, one pair each, meet distinct banks
constexpr int kUsRow = 9;   // scaled inputs (K <= 6)
constexpr int kZzRow = 33;  // hidden pre-activations (H <= 32)

// data part of the gradient of parameter p over pairs i0 .. i1 - 1 of the
// minibatch held in LDS (gy = d loss / d y per pair, z = hidden
// pre-activations); the leaky-ReLU slope at 0 is 1.  The regularisation term
// is added by the caller.
template <int K>
__device__ __forceinline__ float grad_part(int p, int H, int i0, int i1, const float (*us)[kUsRow],
                                           const float *gy, const float (*zz)[kZzRow],
                                           const float *th, float alpha)
{
    float g = 0.0f;
    constexpr int KK = K > 0 ? K : 1;
    const float *v = th + H * K + H;
    if (p < H * K) {
        const int j = p / KK, k = p % KK;
#pragma unroll 4
        for (int i = i0; i < i1; ++i) {
            const float gz = gy[i] * v[j] * (zz[i][j] < 0.0f ? alpha : 1.0f);
            g = __builtin_fmaf(gz, us[i][k], g);
        }
    } else if (p < H * K + H) {
        const int j = p - H * K;
#pragma unroll 4
        for (int i = i0; i < i1; ++i)
            g += gy[i] * v[j] * (zz[i][j] < 0.0f ? alpha : 1.0f);
    } else if (p < H * K + 2 * H) {
        const int j = p - H * K - H;
#pragma unroll 4
        for (int i = i0; i < i1; ++i) {
            const float z = zz[i][j];
            g = __builtin_fmaf(gy[i], z < 0.0f ? alpha * z : z, g);
        }
    } else {
#pragma unroll 4
        for (int i = i0; i < i1; ++i)
            g += gy[i];
    }
    return g;
}

// whether parameter p carries the L2 term (first- and second-layer weights)
__device__ __forceinline__ bool regularised(int p, int H, int K)
{
    return p < H * K || (p >= H * K + H && p < H * K + 2 * H);
}

// gradient of parameter p over the whole minibatch
template <int K>
__device__ __forceinline__ float grad_param(int p, int H, int nb, const float (*us)[kUsRow],
                                            const float *gy, const float (*zz)[kZzRow],
                                            const float *th, float alpha, float lambda)
{
    float g = grad_part<K>(p, H, 0, nb, us, gy, zz, th, alpha);
    if (regularised(p, H, K))
        g = __builtin_fmaf(lambda, th[p], g);
    return g;
}

struct TrainSmem {
    float th[kMaxParams], m[kMaxParams], v[kMaxParams];
    float us[256][kUsRow];
    float gy[256];
    float zz[256][kZzRow];
    float loss[256];
};

// One workgroup of kTrainThreads per candidate: a minibatch's forward pass
// by one thread per pair, then each parameter's gradient by kGradSplit
// threads over a share of the pairs each (their partial sums added in a
// fixed order), then the Adam step.
constexpr int kTrainThreads = 1024;
constexpr int kGradSplit = 4;

template <int HM, int K>
__global__ void __launch_bounds__(kTrainThreads) k_train(TrainArgs a)
{
    __shared__ TrainSmem sm;
    const int H = a.H, P = H * K + 2 * H + 1;
    const int tid = threadIdx.x, cand = blockIdx.x;
    const int part = tid % kGradSplit, prow = tid / kGradSplit;
    constexpr int PROWS = kTrainThreads / kGradSplit;
    const float lr = (float)a.lr[cand], lam = (float)a.lambda[cand];
    const float inv_sigma = (float)(1.0 / *a.sigma);
    for (int p = tid; p < P; p += blockDim.x) {
        sm.th[p] = a.theta0[p];
        sm.m[p] = sm.v[p] = 0.0f;
    }
    __syncthreads();
    long long step = 0;
    const int batch = a.batch;
    for (int ep = 0; ep < a.epochs; ++ep) {
        for (long long s0 = 0; s0 < a.n; s0 += batch) {
            const int nb = (int)(a.n - s0 < batch ? a.n - s0 : batch);
            const float inv_nb = 1.0f / (float)nb;
            if (tid < nb) {
                const long long i = s0 + tid;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    sm.us[tid][k] = a.u[i * K + k] * inv_sigma;
                const float r = forward_pair<HM, K>(sm.th, H, sm.us[tid], a.t[i] * inv_sigma,
                                                    a.alpha, sm.zz[tid]);
                sm.gy[tid] = r * inv_nb;
            }
            __syncthreads();
            ++step;
            const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
            // pairs of this thread's share (contiguous)
            const int per = (nb + kGradSplit - 1) / kGradSplit;
            const int i0 = part * per, i1 = i0 + per < nb ? i0 + per : nb;
            float gnew[(kMaxParams + PROWS - 1) / PROWS];
#pragma unroll
            for (int q = 0; q < (kMaxParams + PROWS - 1) / PROWS; ++q) {
                const int p = prow + q * PROWS;
                float g = p < P ? grad_part<K>(p, H, i0, i1, sm.us, sm.gy, sm.zz, sm.th, a.alpha)
                                : 0.0f;
                // the kGradSplit shares sit in consecutive lanes: add them pairwise
                g += __shfl_xor(g, 1, kGradSplit);
                g += __shfl_xor(g, 2, kGradSplit);
                if (p < P && regularised(p, H, K))
                    g = __builtin_fmaf(lam, sm.th[p], g);
                gnew[q] = g;
            }
            // every gradient reads theta before any update writes it
            __syncthreads();
            if (part == 0) {
#pragma unroll
                for (int q = 0; q < (kMaxParams + PROWS - 1) / PROWS; ++q) {
                    const int p = prow + q * PROWS;
                    if (p >= P)
                        continue;
                    const float g = gnew[q];
                    const float mm = 0.9f * sm.m[p] + 0.1f * g;
                    const float vv = 0.999f * sm.v[p] + 0.001f * g * g;
                    sm.m[p] = mm;
                    sm.v[p] = vv;
                    sm.th[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
                }
            }
            __syncthreads();
        }
    }
    for (int p = tid; p < P; p += blockDim.x)
        a.theta_out[(long long)cand * P + p] = sm.th[p];
}

// loss and gradient of theta on n pairs (minibatches of 256 summed in order)
template <int HM, int K>
__global__ void __launch_bounds__(256) k_loss_grad(GradArgs a)
{
    __shared__ TrainSmem sm;
    const int H = a.H, P = H * K + 2 * H + 1;
    const int tid = threadIdx.x;
    const float inv_sigma = (float)(1.0 / a.sigma);
    const float inv_n = 1.0f / (float)a.n;
    for (int p = tid; p < P; p += blockDim.x)
        sm.th[p] = a.theta[p];
    float gacc[2] = {0.0f, 0.0f};
    float lacc = 0.0f;
    __syncthreads();
    for (long long s0 = 0; s0 < a.n; s0 += 256) {
        const int nb = (int)(a.n - s0 < 256 ? a.n - s0 : 256);
        if (tid < nb) {
            const long long i = s0 + tid;
#pragma unroll
            for (int k = 0; k < K; ++k)
                sm.us[tid][k] = a.u[i * K + k] * inv_sigma;
            const float r = forward_pair<HM, K>(sm.th, H, sm.us[tid], a.t[i] * inv_sigma,
                                                a.alpha, sm.zz[tid]);
            sm.gy[tid] = r * inv_n;
            lacc += 0.5f * r * r;
        }
        __syncthreads();
        for (int p = tid, q = 0; p < P; p += blockDim.x, ++q)
            gacc[q] += grad_param<K>(p, H, nb, sm.us, sm.gy, sm.zz, sm.th, a.alpha, 0.0f);
        __syncthreads();
    }
    const float lam = (float)a.lambda;
    for (int p = tid, q = 0; p < P; p += blockDim.x, ++q) {
        float g = gacc[q];
        if (p < H * K || (p >= H * K + H && p < H * K + 2 * H))
            g = __builtin_fmaf(lam, sm.th[p], g);
        a.grad[p] = g;
    }
    sm.loss[tid] = lacc;
    __syncthreads();
    if (tid == 0) {
        float l = 0.0f;
        for (int q = 0; q < (int)blockDim.x; ++q)
            l += sm.loss[q];
        l *= inv_n;
        float reg = 0.0f;
        for (int p = 0; p < H * K; ++p)
            reg = __builtin_fmaf(sm.th[p], sm.th[p], reg);
        for (int j = 0; j < H; ++j)
            reg = __builtin_fmaf(sm.th[H * K + H + j], sm.th[H * K + H + j], reg);
        *a.loss = l + 0.5f * lam * reg;
    }
}

// ---------------------------------------------------------------------------
// Validation: histogram of the codes each candidate gives on the validation
// pairs (the FP32 network of the compressor, raw domain), then the score
// J = sum_s c_s rint(2^32 log2 c_s) per candidate.
// ---------------------------------------------------------------------------
template <int D, int HP>
__global__ void __launch_bounds__(256) k_val_hist(ValArgs a)
{
    constexpr int K = (1 << D) - 2;
    constexpr int WIN = 4096;
    __shared__ unsigned win[WIN];
    __shared__ float4 wl[kWlds];
    const int cand = blockIdx.y;
    stage_weights<HP>(wl, a.nets[cand]);
    for (int i = threadIdx.x; i < WIN; i += blockDim.x)
        win[i] = 0u;
    __syncthreads();
    const WeightsLds wt{wl};
    unsigned long long *hist = a.hist + (long long)cand * 65536;
    const int lo = kR - WIN / 2;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (long long)gridDim.x * blockDim.x) {
        int nv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < K; ++k)
            nv[k + 2] = (int)a.u[i * K + k];
        const long long pred = predict<D, HP>(nv, (1 << D) - 1, true, wt, a.nets[cand].b2,
                                              a.nets[cand].alpha);
        const int code = make_code(pred, (int)a.t[i], true);
        const int k = code - lo;
        if (k >= 0 && k < WIN)
            atomicAdd(&win[k], 1u);
        else
            atomicAdd(&hist[code], 1ULL);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < WIN; i += blockDim.x)
        if (win[i])
            atomicAdd(&hist[lo + i], (unsigned long long)win[i]);
}

__device__ __forceinline__ long long qlog(unsigned long long c)
{
    return c ? (long long)__builtin_rint(det_log2((double)c) * 4294967296.0) : 0LL;
}

__global__ void __launch_bounds__(256) k_entropy_j(const unsigned long long *hist, long long *out)
{
    __shared__ long long sh[256];
    const unsigned long long *h = hist + (long long)blockIdx.x * 65536;
    long long s = 0;
    for (int i = threadIdx.x; i < 65536; i += blockDim.x)
        if (h[i])
            s += (long long)h[i] * qlog(h[i]);
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (threadIdx.x < (unsigned)d)
            sh[threadIdx.x] += sh[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[blockIdx.x] = sh[0];
}

// raw-domain networks: w1 / sigma, b1, v * sigma, b2 * sigma (FP64, then FP32)
__global__ void k_fold(FoldArgs a)
{
    const int c = blockIdx.x;  // 0 = initial network
    MlpW *out = a.nets + c;
    const double sg = *a.sigma;
    const int H = a.H, K = a.K, P = H * K + 2 * H + 1;
    for (int i = threadIdx.x; i < PWREL_MAX_HIDDEN * PWREL_MAX_INPUTS; i += blockDim.x) {
        const int j = i / PWREL_MAX_INPUTS, k = i % PWREL_MAX_INPUTS;
        float w = 0.0f;
        if (j < H && k < K)
            w = c == 0 ? a.init.w1[j][k] : (float)((double)a.theta[(c - 1) * P + j * K + k] / sg);
        out->w1[j][k] = w;
    }
    for (int j = threadIdx.x; j < PWREL_MAX_HIDDEN; j += blockDim.x) {
        float b = 0.0f, v = 0.0f;
        if (j < H) {
            b = c == 0 ? a.init.b1[j] : a.theta[(c - 1) * P + H * K + j];
            v = c == 0 ? a.init.v[j] : (float)((double)a.theta[(c - 1) * P + H * K + H + j] * sg);
        }
        out->b1[j] = b;
        out->v[j] = v;
    }
    if (threadIdx.x == 0) {
        out->b2 = c == 0 ? a.init.b2 : (float)((double)a.theta[(c - 1) * P + H * K + 2 * H] * sg);
        out->alpha = a.init.alpha;
    }
}

// q(c) = rint(2^32 log2 c) for the per-block judge of the compressor
__global__ void k_qtable(long long *q, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        q[i] = qlog((unsigned long long)i);
}

// ===========================================================================
// launchers
// ===========================================================================
template <typename T, int D>
static void sample_pass(bool count, const SampleArgs &a, unsigned grid, uint32_t *ct,
                        uint32_t *cv, const SampleOut *o, hipStream_t s)
{
    if (count)
        hipLaunchKernelGGL((k_sample_count<T, D>), dim3(grid), dim3(256), 0, s, a, ct, cv);
    else
        hipLaunchKernelGGL((k_sample_write<T, D>), dim3(grid), dim3(256), 0, s, a, *o);
}

hipError_t launch_sample(bool count, const SampleArgs &a, int D, int dtype, uint32_t *ct,
                         uint32_t *cv, const SampleOut *o, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.N + kSampleChunk - 1) / kSampleChunk);
#define PW_S(DD)                                                                              \
    if (D == DD) {                                                                            \
        if (dtype == PWREL_F32)                                                               \
            sample_pass<float, DD>(count, a, grid, ct, cv, o, s);                            \
        else                                                                                  \
            sample_pass<double, DD>(count, a, grid, ct, cv, o, s);                           \
    }
    PW_S(1) PW_S(2) PW_S(3)
#undef PW_S
    return hipGetLastError();
}

hipError_t launch_sigma(const float *t, long long n, double *part, double *sigma, hipStream_t s)
{
    const int grid = 256;
    hipLaunchKernelGGL(k_sumsq, dim3(grid), dim3(256), 0, s, t, n, part);
    hipLaunchKernelGGL(k_sigma, dim3(1), dim3(64), 0, s, part, grid, n, sigma);
    return hipGetLastError();
}

template <int H>
static void train_k(int K, const TrainArgs &a, int ncand, hipStream_t s)
{
    if (K == 6)
        hipLaunchKernelGGL((k_train<H, 6>), dim3(ncand), dim3(kTrainThreads), 0, s, a);
    else if (K == 2)
        hipLaunchKernelGGL((k_train<H, 2>), dim3(ncand), dim3(kTrainThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_train<H, 0>), dim3(ncand), dim3(kTrainThreads), 0, s, a);
}

hipError_t launch_train(int H, int K, const TrainArgs &a, int ncand, hipStream_t s)
{
    if (H <= 8)
        train_k<8>(K, a, ncand, s);
    else if (H <= 16)
        train_k<16>(K, a, ncand, s);
    else
        train_k<32>(K, a, ncand, s);
    return hipGetLastError();
}

template <int H>
static void grad_k(int K, const GradArgs &a, hipStream_t s)
{
    if (K == 6)
        hipLaunchKernelGGL((k_loss_grad<H, 6>), dim3(1), dim3(256), 0, s, a);
    else if (K == 2)
        hipLaunchKernelGGL((k_loss_grad<H, 2>), dim3(1), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_loss_grad<H, 0>), dim3(1), dim3(256), 0, s, a);
}

hipError_t launch_loss_grad(int H, int K, const GradArgs &a, hipStream_t s)
{
    if (H <= 8)
        grad_k<8>(K, a, s);
    else if (H <= 16)
        grad_k<16>(K, a, s);
    else
        grad_k<32>(K, a, s);
    return hipGetLastError();
}

template <int D>
static void val_k(int HP, const ValArgs &a, int ncand, hipStream_t s)
{
    const unsigned gx = (unsigned)std::max(1LL, std::min(64LL, (a.n + 4095) / 4096));
    if (HP == 8)
        hipLaunchKernelGGL((k_val_hist<D, 8>), dim3(gx, ncand), dim3(256), 0, s, a);
    else if (HP == 16)
        hipLaunchKernelGGL((k_val_hist<D, 16>), dim3(gx, ncand), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_val_hist<D, 32>), dim3(gx, ncand), dim3(256), 0, s, a);
}

hipError_t launch_validate(int D, int HP, const ValArgs &a, int ncand, long long *scores,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u64_n, dim3((unsigned)(ncand * 65536 / 256)), dim3(256), 0, s,
                       a.hist, (long long)ncand * 65536);
    if (a.n > 0) {
        if (D == 3)
            val_k<3>(HP, a, ncand, s);
        else if (D == 2)
            val_k<2>(HP, a, ncand, s);
        else
            val_k<1>(HP, a, ncand, s);
    }
    hipLaunchKernelGGL(k_entropy_j, dim3(ncand), dim3(256), 0, s, a.hist, scores);
    return hipGetLastError();
}

hipError_t launch_fold(const FoldArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_fold, dim3(a.ncand + 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_qtable(long long *q, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_qtable, dim3((n + 255) / 256), dim3(256), 0, s, q, n);
    return hipGetLastError();
}

}  // namespace pwrel

namespace pwrel {
// ---------------------------------------------------------------------------
// The trained Huffman table's input (Sec. 4.3: the code frequencies of the
// validation blocks, on which the compression is simulated): block b of the
// stream order is a validation block iff u01(splitmix64(seed ^ b)) < frac.
// One wave per block adds the block's codes (block-major) to a 4096-bin LDS
// window around the zero-error code, the rest to global bins; each
// workgroup flushes its window once.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_table_hist(const uint16_t *__restrict__ codes, GeoArgs g,
                                                    double frac, unsigned long long seed,
                                                    unsigned long long *__restrict__ hist)
{
    constexpr int WIN = 4096;
    __shared__ unsigned win[WIN];
    for (int i = threadIdx.x; i < WIN; i += blockDim.x)
        win[i] = 0u;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
    const int lo = kR - WIN / 2;
    for (long long b = wave; b < g.nblocks; b += nwaves) {
        const double U = (double)(mix64(seed ^ (unsigned long long)b) >> 11) * 0x1p-53;
        if (!(U < frac))
            continue;
        const long long bx = b % g.nb[2], by = (b / g.nb[2]) % g.nb[1],
                        bz = b / (g.nb[1] * g.nb[2]);
        const BlockGeo q = block_geo3(bz, by, bx, g.n, g.bd[0], g.bd[1], g.bd[2]);
        const long long bsize = (long long)q.ez * q.ey * q.ex;
        for (long long i = lane; i < bsize; i += 64) {
            const int code = codes[q.start + i];
            const int k = code - lo;
            if (k >= 0 && k < WIN)
                atomicAdd(&win[k], 1u);
            else
                atomicAdd(&hist[code], 1ULL);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < WIN; i += blockDim.x)
        if (win[i])
            atomicAdd(&hist[lo + i], (unsigned long long)win[i]);
}

hipError_t launch_table_hist(const uint16_t *codes, const Geom &g, double frac, uint64_t seed,
                             unsigned long long *hist, hipStream_t s)
{
    GeoArgs a{};
    for (int d = 0; d < 3; ++d) {
        a.n[d] = g.n[d];
        a.bd[d] = g.bd[d];
        a.nb[d] = g.nb[d];
    }
    a.nblocks = g.nblocks;
    hipLaunchKernelGGL(k_zero_u64_n, dim3(256), dim3(256), 0, s, hist, 65536LL);
    const long long wg = std::max<long long>(1, std::min<long long>((g.nblocks + 3) / 4, 2048));
    hipLaunchKernelGGL(k_table_hist, dim3((unsigned)wg), dim3(256), 0, s, codes, a, frac,
                       (unsigned long long)seed, hist);
    return hipGetLastError();
}

__global__ void k_zero_u64_n(unsigned long long *p, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0ULL;
}
}  // namespace pwrel
