// Diagnostics on gfx950: the Pauli-string density D_t(x) of Appendix D, a
// histogram of the coefficients rescaled by the largest one.
#include "orqa_device.h"

namespace orqa {

// Counts of v = c (signed) or |c| over bins [t_k, t_(k+1)), the last one
// closed, with t_k = M * edge_k (M = max |c| of the lane).  counts[nb] takes
// values below t_0, counts[nb + 1] values above t_nb.  Strings that the
// pending truncation of the operator drops are skipped (the max is that of
// the untruncated operator, which truncation never lowers: the largest
// string survives any eps0 < 1, and with eps0 >= 1 nothing is counted).
template <typename CT, int LP>
__global__ __launch_bounds__(kThreads) void k_histogram(HistArgs A) {
    __shared__ double sT[kHistMaxBins + 1];
    __shared__ uint32_t sC[kHistMaxBins + 2];
    __shared__ double sThr[LP];
    const CT* __restrict__ C = static_cast<const CT*>(A.C);
    const int nb = A.nbins;
    const double M = bits_to_d(A.ctrl->maxbits[A.mx][A.lane]);
    for (int k = threadIdx.x; k <= nb; k += kThreads) sT[k] = M * A.edges[k];
    for (int k = threadIdx.x; k < nb + 2; k += kThreads) sC[k] = 0;
    const bool filt = A.eps_pend > 0.0;
    if (threadIdx.x < LP) sThr[threadIdx.x] = filt ? A.eps_pend * bits_to_d(A.ctrl->maxbits[A.mx][threadIdx.x]) : -1.0;
    __syncthreads();
    const uint64_t nf = A.ctrl->nf[A.buf];
    const uint64_t n = nf + A.ctrl->nb[A.buf];
    for (uint64_t i = blockIdx.x * uint64_t(kThreads) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kThreads) {
        const CT* row = C + vphys(i, nf, A.cap) * LP;
        if (filt) {
            bool keep = false;
#pragma unroll
            for (int a = 0; a < LP; ++a) keep |= absd(row[a]) > sThr[a];
            if (!keep) continue;
        }
        const double c = static_cast<double>(row[A.lane]);
        const double v = A.is_signed ? c : absd(c);
        int slot;
        if (v < sT[0]) {
            slot = nb;
        } else if (v > sT[nb]) {
            slot = nb + 1;
        } else {  // largest k with t_k <= v, at most nb - 1
            int lo = 0, hi = nb;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sT[mid] <= v) lo = mid;
                else hi = mid;
            }
            slot = lo;
        }
        atomicAdd(&sC[slot], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb + 2; k += kThreads)
        if (sC[k]) atomicAdd(reinterpret_cast<unsigned long long*>(&A.counts[k]), static_cast<unsigned long long>(sC[k]));
}

hipError_t launch_histogram(const HistArgs& a, int dtype, int lp, hipStream_t s, int grid) {
#define L_H(T, L) k_histogram<T, L><<<dim3(grid), dim3(kThreads), 0, s>>>(a)
    ORQA_DISPATCH(dtype, lp, L_H);
#undef L_H
    return hipGetLastError();
}

}  // namespace orqa
