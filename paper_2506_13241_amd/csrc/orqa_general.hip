// General Pauli rotations on gfx950: any generator sigma_J (several qubits,
// X, Y and Z letters, any angle), for gates outside the streaming RX merge and
// the fused Z-only Clifford pass.  Eq. update_rule: a string sigma_P that
// commutes with sigma_J is unchanged; one that anticommutes keeps cos(theta)
// times its coefficient and sends +-sin(theta) times it to the child
// sigma_C = sigma_(P xor J).  Every key receives at most two contributions (its
// own parent part and the child of its partner), so after the branch pass and
// a full sort by (x, z) a merge of adjacent equal keys completes the gate.
#include "orqa_device.h"

namespace orqa {

// Child sign: sigma_C sigma_J = i^e sigma_P with
// e = |x_C & z_C| + |x_J & z_J| + 2 |z_C & x_J| - |x_P & z_P| (mod 4)
// (sigma(x, z) = i^|x&z| X^x Z^z and Z^a X^b = (-1)^(a.b) X^b Z^a); the child's
// coefficient is -sin(theta) c_P for e = 1 and +sin(theta) c_P for e = 3.  For
// x_J = 0 this is the Z-only rule of the Clifford pass, for sigma_J = X_q the
// rule of the RX merge.
__device__ __forceinline__ bool gen_child_negative(const ulonglong2& xp, const ulonglong2& zp, const ulonglong2& xc,
                                                   const ulonglong2& zc, const ulonglong2& xj, const ulonglong2& zj) {
    const int e = k_popc_and(xc, zc) + k_popc_and(xj, zj) + 2 * k_popc_and(zc, xj) - k_popc_and(xp, zp);
    return (e & 3) == 1;
}

// Run of a child: the parent's bits at the generator's key positions.  Parents
// of one class keep their relative order under the xor with J (the first bit
// where two of them differ is not one that J flips), so the children of one
// class, in input order, form a sorted run.
__device__ __forceinline__ uint32_t run_class(const GenArgs& A, const ulonglong2& x, const ulonglong2& z) {
    uint32_t c = 0;
    for (int q = 0; q < A.run_bits; ++q) {
        const ulonglong2& v = A.run_isz[q] ? z : x;
        const int pos = A.run_pos[q];
        c |= uint32_t(((pos < 64 ? v.x : v.y) >> (pos & 63)) & 1u) << q;
    }
    return c;
}

template <typename CT, int LP>
__device__ __forceinline__ bool gen_keep(const CT* c, const double* thr) {
    bool keep = false;
#pragma unroll
    for (int a = 0; a < LP; ++a) keep |= absd(c[a]) > thr[a];
    return keep;
}

// Element k of thread tid in a tile is input t0 + k * 256 + tid (striped, so
// loads and stores of a wave cover contiguous memory).  Its output offset in
// input order: the outputs of every element with a smaller k, then those of
// threads before tid at the same k.  Counts per element are at most 2, so the
// four per-k scans fit in two packed 16-bit scans.
static_assert(kGenIPT == 4, "scan_striped4 packs four counts");
__device__ __forceinline__ void scan_striped4(const uint32_t (&c)[4], uint32_t* s_wave, uint32_t (&off)[4],
                                              uint32_t& total) {
    uint32_t t01, t23;
    const uint32_t o01 = block_excl_scan(c[0] | (c[1] << 16), s_wave, t01);
    const uint32_t o23 = block_excl_scan(c[2] | (c[3] << 16), s_wave, t23);
    const uint32_t T0 = t01 & 0xFFFFu, T1 = t01 >> 16, T2 = t23 & 0xFFFFu, T3 = t23 >> 16;
    off[0] = o01 & 0xFFFFu;
    off[1] = T0 + (o01 >> 16);
    off[2] = T0 + T1 + (o23 & 0xFFFFu);
    off[3] = T0 + T1 + T2 + (o23 >> 16);
    total = T0 + T1 + T2 + T3;
}

// Branch: reads the (virtual, x-rotated) input, applies the pending truncation,
// writes parents and children compacted to the front of the output, in input
// order (each parent before its child), with x in the stored frame (the sign
// algebra runs on the true x).  For x_J = 0 every output stays in its
// parent's x-group and the groups keep their order.  Output offsets by a
// two-level decoupled look-back over tiles.
template <typename CT, int LP>
__global__ __launch_bounds__(kThreads) void k_gen_branch(GenArgs A, GateTrig g) {
    __shared__ uint32_t sWave[4];
    __shared__ uint32_t sTile;
    __shared__ uint64_t sBase;
    __shared__ double sThr[LP];
    Ctrl* ctrl = A.ctrl;
    const CT* __restrict__ Cin = static_cast<const CT*>(A.Cin);
    CT* __restrict__ Cout = static_cast<CT*>(A.Cout);
    const int tid = threadIdx.x, wave = tid >> 6;
    const bool skip = ctrl->err != 0u;
    const uint64_t nf = ctrl->nf[A.in_buf];
    const uint64_t n = nf + ctrl->nb[A.in_buf];
    const uint64_t ntiles = skip ? 0 : (n + kGenTile - 1) / kGenTile;
    const uint32_t ep = ctrl->epoch;
    const bool filt = A.eps_in > 0.0;
    if (tid < LP) sThr[tid] = filt ? A.eps_in * bits_to_d(ctrl->maxbits[A.mx_in][tid]) : -1.0;
    __syncthreads();
    const ulonglong2 xj = make_ulonglong2(A.xj0, A.xj1), zj = make_ulonglong2(A.zj0, A.zj1);
    // the generator's x in the stored frame (stored x = true x rotated right by xrot)
    const ulonglong2 xjs = rotl_n(xj, (A.nq - A.xrot) % A.nq, A.nq);

    for (;;) {
        const uint32_t tile = acquire_tile(ctrl, &sTile);
        if (tile >= ntiles) break;
        const uint64_t t0 = uint64_t(tile) * kGenTile;
        ulonglong2 xs[kGenIPT], zs[kGenIPT];
        uint32_t nout[kGenIPT];
#pragma unroll
        for (int k = 0; k < kGenIPT; ++k) {
            const uint64_t i = t0 + uint64_t(k) * kThreads + tid;
            nout[k] = 0;
            xs[k] = make_ulonglong2(0, 0);
            zs[k] = make_ulonglong2(0, 0);
            if (i >= n) continue;
            const uint64_t p = vphys(i, nf, A.cap);
            xs[k] = A.Xin[p];  // as stored; the true x for the algebra below
            zs[k] = A.Zin[p];
            if (filt && !gen_keep<CT, LP>(Cin + p * LP, sThr)) continue;
            const ulonglong2 xt = rotl_n(xs[k], A.xrot, A.nq);
            const bool anti = ((k_popc_and(xt, zj) + k_popc_and(zs[k], xj)) & 1) != 0;
            nout[k] = anti ? uint32_t(g.any_c != 0) + uint32_t(g.any_s != 0) : 1u;
        }
        uint32_t tot, off[kGenIPT];
        scan_striped4(nout, sWave, off, tot);
        if (wave == 0) {
            const uint64_t b = lookback_wave2(A.status, A.status + 2 * A.max_tiles, tile, ep, tot, &ctrl->err);
            if (lane_id() == 0) sBase = b;
        }
        __syncthreads();
        const uint64_t base = sBase;
        if (tile == ntiles - 1 && tid == 0) {
            const uint64_t total = base + tot;
            if (total > A.cap) {
                atomicOr(&ctrl->err, kErrCapacity);
                atomicMax(reinterpret_cast<unsigned long long*>(&ctrl->need), static_cast<unsigned long long>(total));
            } else {
                ctrl->nf[A.out_buf] = total;
                ctrl->nb[A.out_buf] = 0;
            }
        }
#pragma unroll
        for (int k = 0; k < kGenIPT; ++k) {
            if (nout[k] == 0) continue;
            uint64_t o = base + off[k];
            const uint64_t i = t0 + uint64_t(k) * kThreads + tid;
            const CT* ce = Cin + vphys(i, nf, A.cap) * LP;
            const ulonglong2 xt = rotl_n(xs[k], A.xrot, A.nq);
            const ulonglong2 xw = xs[k];  // x as stored: outputs keep the stored frame
            const bool anti = ((k_popc_and(xt, zj) + k_popc_and(zs[k], xj)) & 1) != 0;
            if (!anti) {  // commutes: unchanged
                if (o < A.cap) {
                    A.Xout[o] = xw;
                    A.Zout[o] = zs[k];
#pragma unroll
                    for (int a = 0; a < LP; ++a) Cout[o * LP + a] = ce[a];
                    if (A.Lout) {
#pragma unroll
                        for (int a = 0; a < LP; ++a) A.Lout[o * LP + a] = 0.0f;
                    }
                    if (A.Tout) A.Tout[o] = 0u;
                }
                ++o;
                continue;
            }
            if (g.any_c) {
                if (o < A.cap) {
                    A.Xout[o] = xw;
                    A.Zout[o] = zs[k];
                    if constexpr (sizeof(CT) == 4) {
                        if (A.Lout) {
#pragma unroll
                            for (int a = 0; a < LP; ++a) {
                                const F32x2 p = mul_split(ce[a], g.cs_hi[a], g.cs_lo[a]);
                                Cout[o * LP + a] = p.hi;
                                A.Lout[o * LP + a] = p.lo;
                            }
                        }
                    }
                    if (sizeof(CT) != 4 || !A.Lout) {
#pragma unroll
                        for (int a = 0; a < LP; ++a) Cout[o * LP + a] = Arith<CT>::scale_c(g, a, ce[a]);
                    }
                    if (A.Tout) A.Tout[o] = 0u;
                }
                ++o;
            }
            if (g.any_s) {
                const ulonglong2 xc = make_ulonglong2(xt.x ^ xj.x, xt.y ^ xj.y);
                const ulonglong2 zc = make_ulonglong2(zs[k].x ^ zj.x, zs[k].y ^ zj.y);
                const bool neg = gen_child_negative(xt, zs[k], xc, zc, xj, zj);
                if (o < A.cap) {
                    A.Xout[o] = make_ulonglong2(xw.x ^ xjs.x, xw.y ^ xjs.y);
                    A.Zout[o] = zc;
                    if constexpr (sizeof(CT) == 4) {
                        if (A.Lout) {
#pragma unroll
                            for (int a = 0; a < LP; ++a) {
                                const float h = neg ? -g.sn_hi[a] : g.sn_hi[a];
                                const float l = neg ? -g.sn_lo[a] : g.sn_lo[a];
                                const F32x2 p = mul_split(ce[a], h, l);
                                Cout[o * LP + a] = p.hi;
                                A.Lout[o * LP + a] = p.lo;
                            }
                        }
                    }
                    if (sizeof(CT) != 4 || !A.Lout) {
#pragma unroll
                        for (int a = 0; a < LP; ++a) Cout[o * LP + a] = Arith<CT>::scale_s(g, a, ce[a], neg);
                    }
                    if (A.Tout) A.Tout[o] = 1u + run_class(A, xw, zs[k]);
                }
                ++o;
            }
        }
        __syncthreads();
    }
    if (finish_launch(ctrl)) {
        if (__hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            for (int a = 0; a < kMaxLanes; ++a) ctrl->maxbits[A.mx_in][a] = 0ull;
            if (ntiles == 0) {
                ctrl->nf[A.out_buf] = 0;
                ctrl->nb[A.out_buf] = 0;
            }
            ctrl->stages_done += 1;
            ctrl->cnt_updates += n;
        }
    }
}

// Merge: the input is sorted by (x, z) (front run only); each key appears at
// most twice (a parent part and a child part) and its entries are summed.
// Writes the unique keys compacted and the per-lane max of the results.
template <typename CT, int LP>
__global__ __launch_bounds__(kThreads) void k_gen_reduce(GenArgs A) {
    __shared__ uint32_t sWave[4];
    __shared__ uint32_t sTile;
    __shared__ uint64_t sBase;
    Ctrl* ctrl = A.ctrl;
    const CT* __restrict__ Cin = static_cast<const CT*>(A.Cin);
    CT* __restrict__ Cout = static_cast<CT*>(A.Cout);
    const int tid = threadIdx.x, wave = tid >> 6;
    const bool skip = ctrl->err != 0u;
    const uint64_t n = ctrl->nf[A.in_buf];
    const uint64_t ntiles = skip ? 0 : (n + kGenTile - 1) / kGenTile;
    const uint32_t ep = ctrl->epoch;
    double vmax[LP];
#pragma unroll
    for (int a = 0; a < LP; ++a) vmax[a] = 0.0;

    for (;;) {
        const uint32_t tile = acquire_tile(ctrl, &sTile);
        if (tile >= ntiles) break;
        const uint64_t t0 = uint64_t(tile) * kGenTile;
        uint32_t first[kGenIPT];
#pragma unroll
        for (int k = 0; k < kGenIPT; ++k) {
            const uint64_t i = t0 + uint64_t(k) * kThreads + tid;  // striped, scanned in input order
            first[k] = 0;
            if (i >= n) continue;
            const ulonglong2 x = A.Xin[i], z = A.Zin[i];
            const bool f = i == 0 || !k_eq(x, A.Xin[i - 1]) || !k_eq(z, A.Zin[i - 1]);
            if (f && i + 2 < n && k_eq(x, A.Xin[i + 2]) && k_eq(z, A.Zin[i + 2]))
                atomicOr(&ctrl->err, kErrInternal);  // three entries of one key cannot occur
            first[k] = f;
        }
        uint32_t tot, off[kGenIPT];
        scan_striped4(first, sWave, off, tot);
        if (wave == 0) {
            const uint64_t b = lookback_wave2(A.status, A.status + 2 * A.max_tiles, tile, ep, tot, &ctrl->err);
            if (lane_id() == 0) sBase = b;
        }
        __syncthreads();
        const uint64_t base = sBase;
        if (tile == ntiles - 1 && tid == 0) {
            ctrl->nf[A.out_buf] = base + tot;
            ctrl->nb[A.out_buf] = 0;
        }
#pragma unroll
        for (int k = 0; k < kGenIPT; ++k) {
            if (!first[k]) continue;
            const uint64_t o = base + off[k];
            const uint64_t i = t0 + uint64_t(k) * kThreads + tid;
            const ulonglong2 x = A.Xin[i], z = A.Zin[i];
            const bool two = i + 1 < n && k_eq(x, A.Xin[i + 1]) && k_eq(z, A.Zin[i + 1]);
            A.Xout[o] = x;
            A.Zout[o] = z;
#pragma unroll
            for (int a = 0; a < LP; ++a) {
                CT v = Cin[i * LP + a];
                bool done = false;
                if constexpr (sizeof(CT) == 4) {
                    if (A.Lin) {  // unevaluated pairs: two-sum of the heads, one rounding
                        const float l1 = A.Lin[i * LP + a];
                        if (two) {
                            const F32x2 s = two_sum(v, Cin[(i + 1) * LP + a]);
                            v = s.hi + (s.lo + (l1 + A.Lin[(i + 1) * LP + a]));
                        } else {
                            v = v + l1;
                        }
                        done = true;
                    }
                }
                if (!done && two) v = v + Cin[(i + 1) * LP + a];
                Cout[o * LP + a] = v;
                vmax[a] = fmax(vmax[a], absd(v));
            }
        }
        __syncthreads();
    }
    // the waves' maxima combined in LDS, one device atomic per lane and
    // workgroup (all workgroups leave together; atomics on one word queue)
    __shared__ unsigned long long sWmax[LP];
    if (tid < LP) sWmax[tid] = 0ull;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < LP; ++a) {
        const double mx = wave_max_d(vmax[a]);
        if (lane_id() == 0 && mx > 0.0) atomicMax(&sWmax[a], static_cast<unsigned long long>(d_to_bits(mx)));
    }
    __syncthreads();
    if (tid < LP && sWmax[tid] != 0ull)
        atomicMax(reinterpret_cast<unsigned long long*>(&ctrl->maxbits[A.mx_out][tid]), sWmax[tid]);
    if (finish_launch(ctrl)) {
        if (ntiles == 0 && __hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            ctrl->nf[A.out_buf] = 0;
            ctrl->nb[A.out_buf] = 0;
        }
    }
}

// ================================================================ merge of sorted runs
// (x, z) order, x major, as the radix sort produces it.
__device__ __forceinline__ bool key_le(const ulonglong2& xa, const ulonglong2& za, const ulonglong2& xb,
                                       const ulonglong2& zb) {
    return k_eq(xa, xb) ? k_le(za, zb) : k_lt(xa, xb);
}

__device__ __forceinline__ int merge_pair_of(const MergeArgs& A, uint64_t tile) {
    int p = 0;
    while (p + 1 < A.npairs && A.pairs[p + 1].tile0 <= tile) ++p;
    return p;
}

// Merge path: the number of A elements among the first d outputs of the
// merge of A and B, A first on equal keys.
__global__ __launch_bounds__(kThreads) void k_merge_split(MergeArgs A) {
    const uint64_t t = blockIdx.x * uint64_t(kThreads) + threadIdx.x;
    if (t == 0) {
        A.ctrl->nf[A.dst_buf] = A.n;
        A.ctrl->nb[A.dst_buf] = 0;
    }
    if (t >= A.ntiles) return;
    const MergePair P = A.pairs[merge_pair_of(A, t)];
    const uint64_t d = (t - P.tile0) * kMergeTile;
    const uint64_t b0 = P.a0 + P.na;
    uint64_t lo = d > P.nb ? d - P.nb : 0, hi = d < P.na ? d : P.na;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const uint64_t j = b0 + d - 1 - mid;
        if (key_le(A.Xs[P.a0 + mid], A.Zs[P.a0 + mid], A.Xs[j], A.Zs[j])) lo = mid + 1;
        else hi = mid;
    }
    A.split[t] = lo;
}

// One output tile per workgroup: its A and B ranges staged in LDS, each thread
// finds the sources of kMergeIPT consecutive outputs from its own merge-path
// split, and the tile is then written in striped order (coalesced stores).
template <typename CT, int LP>
__global__ __launch_bounds__(kThreads) void k_merge_pairs(MergeArgs A) {
    __shared__ ulonglong2 sX[kMergeTile];
    __shared__ ulonglong2 sZ[kMergeTile];
    __shared__ uint16_t sSrc[kMergeTile];
    const uint64_t t = blockIdx.x;
    const MergePair P = A.pairs[merge_pair_of(A, t)];
    const uint64_t total = P.na + P.nb;
    const uint64_t d0 = (t - P.tile0) * kMergeTile;
    const uint64_t d1 = d0 + kMergeTile < total ? d0 + kMergeTile : total;
    const uint64_t a_lo = A.split[t];
    const uint64_t a_hi = d1 == total ? P.na : A.split[t + 1];
    const uint64_t b_lo = d0 - a_lo;
    const int cntA = int(a_hi - a_lo), cnt = int(d1 - d0), cntB = cnt - cntA;
    const uint64_t gA = P.a0 + a_lo, gB = P.a0 + P.na + b_lo;
    for (int i = threadIdx.x; i < cnt; i += kThreads) {
        const uint64_t g = i < cntA ? gA + i : gB + (i - cntA);
        sX[i] = A.Xs[g];
        sZ[i] = A.Zs[g];
    }
    __syncthreads();
    const int dd = threadIdx.x * kMergeIPT;
    if (dd < cnt) {
        int lo = dd > cntB ? dd - cntB : 0, hi = dd < cntA ? dd : cntA;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int j = cntA + dd - 1 - mid;
            if (key_le(sX[mid], sZ[mid], sX[j], sZ[j])) lo = mid + 1;
            else hi = mid;
        }
        int ai = lo, bi = dd - lo;
#pragma unroll
        for (int k = 0; k < kMergeIPT; ++k) {
            const int oo = dd + k;
            if (oo >= cnt) break;
            const bool takeA = ai < cntA && (bi >= cntB || key_le(sX[ai], sZ[ai], sX[cntA + bi], sZ[cntA + bi]));
            sSrc[oo] = uint16_t(takeA ? ai : cntA + bi);
            if (takeA) ++ai;
            else ++bi;
        }
    }
    __syncthreads();
    const CT* __restrict__ Cs = static_cast<const CT*>(A.Cs);
    CT* __restrict__ Cd = static_cast<CT*>(A.Cd);
    for (int oo = threadIdx.x; oo < cnt; oo += kThreads) {
        const int l = sSrc[oo];
        const uint64_t src = l < cntA ? gA + l : gB + (l - cntA);
        const uint64_t out = P.a0 + d0 + oo;
        A.Xd[out] = sX[l];
        A.Zd[out] = sZ[l];
#pragma unroll
        for (int a = 0; a < LP; ++a) Cd[out * LP + a] = Cs[src * LP + a];
        if (A.Ls) {
#pragma unroll
            for (int a = 0; a < LP; ++a) A.Ld[out * LP + a] = A.Ls[src * LP + a];
        }
    }
}

hipError_t launch_merge_pairs(const MergeArgs& a, int dtype, int lp, hipStream_t s) {
    if (a.npairs < 1 || a.npairs > kMergeMaxPairs || a.ntiles == 0) return hipErrorInvalidValue;
    const unsigned sgrid = unsigned((a.ntiles + kThreads - 1) / kThreads);
    k_merge_split<<<dim3(sgrid), dim3(kThreads), 0, s>>>(a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define L_MP(T, L) k_merge_pairs<T, L><<<dim3(unsigned(a.ntiles)), dim3(kThreads), 0, s>>>(a)
    ORQA_DISPATCH(dtype, lp, L_MP);
#undef L_MP
    return hipGetLastError();
}

hipError_t launch_gen_branch(const GenArgs& a, const GateTrig& g, int dtype, int lp, hipStream_t s, int grid) {
#define L_GB(T, L) k_gen_branch<T, L><<<dim3(grid), dim3(kThreads), 0, s>>>(a, g)
    ORQA_DISPATCH(dtype, lp, L_GB);
#undef L_GB
    return hipGetLastError();
}

hipError_t launch_gen_reduce(const GenArgs& a, int dtype, int lp, hipStream_t s, int grid) {
#define L_GR(T, L) k_gen_reduce<T, L><<<dim3(grid), dim3(kThreads), 0, s>>>(a)
    ORQA_DISPATCH(dtype, lp, L_GR);
#undef L_GR
    return hipGetLastError();
}

}  // namespace orqa
