// GSP-based initialization (Section IV of the paper, eqs. "GiFt" and "GiFt
// filter"): the multi-band filter H = sum_b alpha_b Atilde_{sigma_b}^{k_b}
// on the unsigned netlist graph, Atilde_sigma = D_sigma^-1/2 (A + sigma I)
// D_sigma^-1/2, then every fixed row reset to its input (step 3).  Its output
// is Algorithm 1's g^(0).
//
// Atilde_sigma is the refinement operator T = I - L/lambda of the graph
// with self-loop weight sigma and lambda fixed at 1, so each band runs on the
// filter chain of filter.hip.  Bands that share sigma share one chain (one
// normalisation, k_max hops); the chains of distinct sigmas are added.
#include "ahr_internal.hpp"

namespace ahr {

namespace {

constexpr int kBT = 256;

__global__ void __launch_bounds__(kBT) k_add_into(float* __restrict__ acc, const float* __restrict__ x, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i < n) acc[i] += x[i];
}

}  // namespace

void run_gift(Graph& g, const ahr_gift_spec& gs, const float* in, float* out, int32_t ncols, hipStream_t s) {
    // distinct sigmas in order of first appearance
    float sig[AHR_MAX_BANDS];
    int nsig = 0;
    for (int b = 0; b < gs.nbands; ++b) {
        bool seen = false;
        for (int t = 0; t < nsig; ++t) seen = seen || sig[t] == gs.sigma[b];
        if (!seen) sig[nsig++] = gs.sigma[b];
    }
    const int64_t n = static_cast<int64_t>(g.n_inst) * ncols;
    DevBuf<float> tmp;
    if (nsig > 1) tmp.ensure(static_cast<size_t>(n), s);
    for (int t = 0; t < nsig; ++t) {
        ahr_filter_spec fs{};
        fs.nbands = 0;
        for (int b = 0; b < gs.nbands; ++b) {
            if (gs.sigma[b] != sig[t]) continue;
            fs.k[fs.nbands] = gs.k[b];
            fs.alpha[fs.nbands] = gs.alpha[b];
            ++fs.nbands;
        }
        fs.sigma = sig[t];
        fs.lambda_mode = AHR_LAMBDA_FIXED;
        fs.lambda_fixed = 1.f;
        run_filter(g, fs, in, t == 0 ? out : tmp.p, ncols, s);
        if (t > 0) {
            hipLaunchKernelGGL(k_add_into, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, out, tmp.p, n);
            AHR_LAUNCHED("k_add_into");
        }
    }
    // each chain reset the fixed rows to the input: after adding several, once more
    if (nsig > 1) relax(g, in, out, out, ncols, 1.f, s);
    tmp.release(s);
}

}  // namespace ahr
