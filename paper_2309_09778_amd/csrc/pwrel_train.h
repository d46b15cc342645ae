// Argument blocks and launchers of the learned part (training, sampling,
// validation) and of the matrix-core codec path.
#pragma once

#include "pwrel_kernels.h"

namespace pwrel {

constexpr int kSampleChunk = 16384;              // points per sampling workgroup
constexpr int kMaxParams = 32 * 6 + 2 * 32 + 1;  // H = 32, K = 6
constexpr int kMaxTrained = 16;                 // trained candidates per launch

struct SampleArgs {
    const void *x;
    long long n[3];
    long long N;
    int B;
    int independent;
    double rho;
    unsigned long long seed;
    const DevConsts *c;
};

// Pairs in ascending point order.  Split form (training): FP32 training and
// validation arrays; combined form (checking): int32 pairs with a flag.
// Either form may be absent (null u pointer).
struct SampleOut {
    const unsigned long long *off_tr, *off_va;  // exclusive prefix counts per chunk
    float *u_tr, *t_tr, *u_va, *t_va;
    unsigned long long cap_tr, cap_va;
    int *u_all, *t_all;
    unsigned char *isval;
    unsigned long long *idx_all;
    unsigned long long cap_all;
};

struct TrainArgs {
    int H;  // hidden width (the kernel is instantiated for a width >= H)
    const float *u, *t;
    long long n;
    const double *sigma;  // device scalar
    float alpha;
    int batch, epochs;
    const float *theta0;
    float *theta_out;
    double lr[kMaxTrained], lambda[kMaxTrained];
};

struct GradArgs {
    int H;
    const float *theta, *u, *t;
    long long n;
    double sigma, lambda;
    float alpha;
    float *grad, *loss;
};

struct ValArgs {
    const float *u, *t;
    long long n;
    const MlpW *nets;  // device array, one per candidate (raw domain)
    unsigned long long *hist;  // [ncand][65536]
};

// Raw-domain networks of the candidates: nets[0] = the initial network,
// nets[1 + c] = candidate c of theta [ncand][P] with the scale folded in.
struct FoldArgs {
    const float *theta;
    const double *sigma;
    int H, K, ncand;
    MlpW init;
    MlpW *nets;
};

hipError_t launch_sample(bool count, const SampleArgs &a, int D, int dtype, uint32_t *ct,
                         uint32_t *cv, const SampleOut *o, hipStream_t s);
hipError_t launch_sigma(const float *t, long long n, double *part, double *sigma, hipStream_t s);
hipError_t launch_train(int H, int K, const TrainArgs &a, int ncand, hipStream_t s);
hipError_t launch_loss_grad(int H, int K, const GradArgs &a, hipStream_t s);
hipError_t launch_validate(int D, int HP, const ValArgs &a, int ncand, long long *scores,
                           hipStream_t s);
hipError_t launch_qtable(long long *q, int n, hipStream_t s);
hipError_t launch_fold(const FoldArgs &a, hipStream_t s);

__global__ void k_zero_u64_n(unsigned long long *p, long long n);
// code counts of the trained table's validation blocks (codes block-major)
hipError_t launch_table_hist(const uint16_t *codes, const Geom &g, double frac, uint64_t seed,
                             unsigned long long *hist, hipStream_t s);

}  // namespace pwrel
