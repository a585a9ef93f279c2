// Int3.4 Lottery BP for codes with at most 64*16 checks: one wavefront per
// shot, check-centric.
//
// Per shot the wave keeps
//   * beta (C2V, int8) of every edge in VGPRs: lane L owns checks L + 64*s,
//     s < SLOTS, and holds their 8 padded slots packed in one u64 per check;
//   * lambda of every column twice in its LDS slice (current / next), as
//     biased 16-bit values packed in pairs (|lambda| <= 5*127 fits).
// Int3.4 arithmetic is exact, so lambda^(i) = mu + sum of beta^(i) is built
// with integer LDS atomic adds into `next` (order-independent): one fused pass
// per check gathers lambda^(i-1) from `current`, forms
// alpha = sat(lambda - beta_old) (== mu + the other C2V messages), runs
// min1/min2/argmin/sign parity, stores the new beta in VGPRs and adds it to
// `next`.  A second pass over columns takes the hard decision (ballot into the
// correction words), forms the syndrome estimate by LDS atomic XOR (only
// columns with e = 1) and resets `current` to mu for the next iteration.
// There is no variable-node gather.  Padding slots point at column n, whose
// `current` value is reset to 254 each iteration: it always yields
// alpha = +127, the sentinel that never wins a minimum.
//
// The lottery (Algorithm 3) runs after the column pass with U from the
// previous syndrome estimate and lambda^(i) read from LDS; the flip acts on
// the next iteration's alpha (message flip) or on lambda_v* (LLR flip).
#include "lbp_internal.h"

namespace lbp {
namespace {

constexpr int BIAS = 32768;
constexpr int PAD_LAMBDA = 254;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ int wave_incl_scan(int x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Philox4x64-10 (Salmon et al., SC'11), word 0 for counter (c0, c1, 0, 0), key (k0, 0).
__device__ uint64_t philox_w0(uint64_t k0, uint64_t c0, uint64_t c1) {
    uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0, ka = k0, kb = 0;
#pragma unroll 1
    for (int r = 0; r < 10; ++r) {
        uint64_t h0 = __umul64hi(0xD2E7470EE14C6C93ULL, x0), l0 = 0xD2E7470EE14C6C93ULL * x0;
        uint64_t h1 = __umul64hi(0xCA5A826395121157ULL, x2), l1 = 0xCA5A826395121157ULL * x2;
        uint64_t y0 = h1 ^ x1 ^ ka, y2 = h0 ^ x3 ^ kb;
        x0 = y0; x1 = l1; x2 = y2; x3 = l0;
        ka += 0x9E3779B97F4A7C15ULL;
        kb += 0xBB67AE8584CAA73BULL;
    }
    return x0;
}

__device__ __forceinline__ int sbyte(uint64_t w, int k) { return (int)(int8_t)(uint8_t)(w >> (8 * k)); }

__device__ __forceinline__ int med3i(int a, int b, int c) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int t = hi < c ? hi : c;
    return lo > t ? lo : t;
}

__device__ __forceinline__ int sat127(int x) { return x > 127 ? 127 : (x < -127 ? -127 : x); }

__device__ __forceinline__ int scale_q(const BpParams &P, int i, int mag) {
    if (P.scale_mode == 1) return (P.scale_k * mag) >> 3;
    int sh = i + 1 > 30 ? 30 : i + 1;
    return mag - (mag >> sh);
}

// Lottery selection (Algorithm 3), U from the previous syndrome estimate SHp.
__device__ int lottery_pick_q(const DevCode &C, uint64_t seed, uint64_t shot_id, int i, const uint16_t *L,
                              const uint32_t *S, const uint32_t *SHp, int lane) {
    int N = 0;
    for (int w0 = 0; w0 < C.mw; w0 += 64) {
        int w = w0 + lane;
        N += wave_sum(__popc(w < C.mw ? (SHp[w] ^ S[w]) : 0u));
    }
    if (N == 0) return -1;
    const uint64_t x = philox_w0(seed, shot_id, (uint64_t)i);
    uint32_t k = (uint32_t)(((x >> 32) * (uint64_t)N) >> 32);
    int cstar = 0;
    for (int w0 = 0; w0 < C.mw; w0 += 64) {
        int w = w0 + lane;
        uint32_t u = w < C.mw ? (SHp[w] ^ S[w]) : 0u;
        int cnt = __popc(u);
        int incl = wave_incl_scan(cnt, lane);
        int tot = __shfl(incl, 63, 64);
        if ((int)k < tot) {
            int excl = incl - cnt;
            bool here = (int)k >= excl && (int)k < incl;
            int pos = 0;
            if (here) {
                uint32_t t = u;
                for (int q = (int)k - excl; q > 0; --q) t &= t - 1;
                pos = w * 32 + __ffs(t) - 1;
            }
            cstar = __shfl(pos, __ffsll((unsigned long long)__ballot(here)) - 1, 64);
            break;
        }
        k -= (uint32_t)tot;
    }
    int cnt = -1, v = 0x7FFFFFFF, q = 0;
    if (lane < DEG) {
        uint32_t vv = C.cn_cols[cstar * DEG + lane];
        if (vv != NOPOS) {
            v = (int)vv;
            const uint64_t tab = C.vn_tab[v];
            cnt = 0;
#pragma unroll
            for (int j = 0; j < CDEG; ++j) {
                uint32_t p = (uint32_t)(tab >> (16 * j)) & 0xFFFFu;
                if (p != NOPOS) {
                    uint32_t c = p / DEG;
                    cnt += ((SHp[c >> 5] ^ S[c >> 5]) >> (c & 31)) & 1u;
                }
            }
            int l = (int)L[v] - BIAS;
            q = l < 0 ? -l : l;
        }
    }
    int bc = -1, bq = 0, bv = -1;
#pragma unroll
    for (int kk = 0; kk < DEG; ++kk) {
        int ck = __shfl(cnt, kk, 64), vk = __shfl(v, kk, 64), qk = __shfl(q, kk, 64);
        if (ck < 0) continue;
        if (bv < 0 || ck > bc || (ck == bc && (qk < bq || (qk == bq && vk < bv)))) {
            bc = ck;
            bq = qk;
            bv = vk;
        }
    }
    return bv;
}

template <int SLOTS, bool LLR_FLIP>
__global__ __launch_bounds__(1024) void bp_int8_kernel(BpArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DevCode &C = a.code;
    const BpParams &P = a.prm;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = C.n, m = C.m;
    // block-shared column index of every padded slot: cidx[(s*64 + lane)*DEG + k],
    // read as one 16-byte vector per check
    uint16_t *cidx = (uint16_t *)smem;
    for (int t = threadIdx.x; t < SLOTS * DEG * 64; t += blockDim.x) {
        const int c = t / DEG, k = t % DEG;
        uint32_t v = c < m ? C.cn_cols[c * DEG + k] : NOPOS;
        cidx[t] = (uint16_t)(v == NOPOS ? n : v);
    }
    __syncthreads();
    unsigned char *base = smem + (((size_t)SLOTS * DEG * 64 * 2 + 15) & ~(size_t)15) + (size_t)wv * a.wave_bytes;
    const size_t lwords = (size_t)(n + 3) / 2;  // (n + 2) biased 16-bit lambda values, padded to pairs
    uint32_t *LA = (uint32_t *)base;
    uint32_t *LB = LA + lwords;
    uint32_t *S = (uint32_t *)(base + ((2 * lwords * 4 + 15) & ~(size_t)15));
    uint32_t *SH0 = S + C.mw, *SH1 = SH0 + C.mw, *EH = SH1 + C.mw;
    const int gwave = blockIdx.x * (blockDim.x >> 6) + wv;
    float *stage = a.stage + (size_t)gwave * 2 * n;
    const uint32_t last_mask = (m & 31) ? ((1u << (m & 31)) - 1u) : ~0u;
    const int nvs = (n + 63) >> 6;

    for (;;) {
        int64_t item = 0;
        if (a.ring) {
            if (lane == 0) item = serve_claim(*a.ring);
            item = uniform64(item);
            if (item < 0) break;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the host's writes of this ring slot
        } else {
            uint32_t it0 = 0;
            if (lane == 0) it0 = atomicAdd(&a.counters[0], 1u);
            item = (int64_t)__builtin_amdgcn_readfirstlane(it0);
            if (item >= a.n_work) break;
        }
        // a ring item lives in slot item & mask; a batch item names its shot
        const int64_t shot = a.ring ? (item & a.ring->mask) : a.work_list ? (int64_t)a.work_list[item] : item;
        const uint64_t *keys = a.ring ? a.ring->keys : a.shot_keys;
        const uint64_t seed = keys ? keys[2 * shot] : P.seed;
        const uint64_t shot_id = keys ? keys[2 * shot + 1] : a.first_shot_id + (uint64_t)shot;
        float *llr_row = a.llr_out ? a.llr_out + shot * n : nullptr;
        const uint32_t *syn_row = (a.ring ? a.ring->syn : a.synd) + shot * C.mw;

        for (int w = lane; w < C.mw; w += 64) {
            uint32_t x = syn_row[w];
            S[w] = w == C.mw - 1 ? (x & last_mask) : x;
        }
        // lambda^(-1) = mu in both buffers (Algorithm 1 initialisation: alpha^(0) = mu)
        for (int v = lane; v < n; v += 64) {
            const uint16_t mb = (uint16_t)(C.mu_q[v] + BIAS);
            ((uint16_t *)LA)[v] = mb;
            ((uint16_t *)LB)[v] = mb;
        }
        if (lane < 2) ((uint16_t *)LA)[n + lane] = (uint16_t)(PAD_LAMBDA + BIAS);
        wave_sync();
        uint64_t bq[SLOTS];  // beta of the previous iteration, packed int8
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) bq[s] = 0;
        // bit s: measured syndrome of check lane + 64 s (S is zero beyond m)
        uint32_t srow = 0;
#pragma unroll 1
        for (int s = 0; s < (m + 63) / 64; ++s) {
            const int w = 2 * s + (lane >> 5);
            if (w < C.mw) srow |= ((S[w] >> (lane & 31)) & 1u) << s;
        }

        int it = 0, fv = -1;
        bool converged = false;
        uint32_t *Lc = LA, *Ln = LB;
        for (int i = 0; i < P.max_iter; ++i) {
            uint32_t *SHc = (i & 1) ? SH1 : SH0;
            uint32_t *SHp = (i & 1) ? SH0 : SH1;
            const uint16_t *Lc16 = (const uint16_t *)Lc;
            // ---- check-node pass: alpha from lambda^(i-1), beta^(i), lambda^(i) += beta^(i)
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                int al[DEG], vv[DEG], lr[DEG];
                int m1 = 1 << 20, m2 = 1 << 20, px = -(int)((srow >> s) & 1);
                const uint4 cw = ((const uint4 *)cidx)[s * 64 + lane];
                const uint32_t cws[4] = {cw.x, cw.y, cw.z, cw.w};
#pragma unroll
                for (int k = 0; k < DEG; ++k) vv[k] = (int)((cws[k >> 1] >> (16 * (k & 1))) & 0xFFFFu);
#pragma unroll
                for (int k = 0; k < DEG; ++k) lr[k] = Lc16[vv[k]];
#pragma unroll
                for (int k = 0; k < DEG; ++k) {
                    const int v = vv[k];
                    const int lam = lr[k] - BIAS;
                    const int b0 = sbyte(bq[s], k);
                    int x = sat127(lam - b0);
                    // flip (fv = -1 matches nothing): negated alpha, or alpha from -lambda
                    const int xf = LLR_FLIP ? sat127(-lam - b0) : -x;
                    x = v == fv ? xf : x;
                    al[k] = x;
                    const int key = ((x < 0 ? -x : x) << 3) | k;  // |alpha|, first index on ties
                    m2 = med3i(key, m1, m2);  // second smallest (m1 <= m2)
                    m1 = key < m1 ? key : m1;
                    px ^= x;  // sign bit: parity of the syndrome bit and the negative alphas
                }
                const int par = px < 0;
                const int arg = m1 & 7;
                const int s1 = scale_q(P, i, m1 >> 3), s2 = scale_q(P, i, m2 >> 3);
                uint64_t packed = 0;
#pragma unroll
                for (int k = 0; k < DEG; ++k) {
                    const int mag = k == arg ? s2 : s1;
                    const int b = (par ^ (al[k] < 0)) ? -mag : mag;
                    const int v = vv[k];
                    // biased 16-bit halves: the sum never leaves [0, 65535], so no carry crosses halves
                    atomicAdd(&Ln[v >> 1], (uint32_t)(b << ((v & 1) * 16)));
                    packed |= (uint64_t)(uint8_t)b << (8 * k);
                }
                // opaque to the optimiser: otherwise it forwards the 8 unpacked
                // values to the next iteration and keeps 8 registers per check
                asm volatile("" : "+v"(packed));
                bq[s] = packed;
            }
            for (int w = lane; w < C.mw; w += 64) SHc[w] = 0u;
            wave_sync();
            // ---- column pass: hard decision, corrections, syndrome estimate, reset
            const bool last = i == P.max_iter - 1;
            const uint16_t *Ln16 = (const uint16_t *)Ln;
            uint16_t *Lc16w = (uint16_t *)Lc;
            for (int vs = 0; vs < nvs; ++vs) {
                const int v = vs * 64 + lane;
                const bool valid = v < n;
                const int l = valid ? (int)Ln16[v] - BIAS : 1;
                const bool e = valid && l <= 0;
                const uint64_t bal = __ballot(e);
                if (lane == 0) {
                    EH[2 * vs] = (uint32_t)bal;
                    EH[2 * vs + 1] = (uint32_t)(bal >> 32);
                }
                if (e) {
                    const uint64_t tab = C.vn_tab[v];
#pragma unroll
                    for (int j = 0; j < CDEG; ++j) {
                        uint32_t p = (uint32_t)(tab >> (16 * j)) & 0xFFFFu;
                        if (p != NOPOS) {
                            uint32_t c = p / DEG;
                            atomicXor(&SHc[c >> 5], 1u << (c & 31));
                        }
                    }
                }
                if (valid) {
                    Lc16w[v] = (uint16_t)(C.mu_q[v] + BIAS);  // accumulation base of iteration i+1
                    if (llr_row) llr_row[v] = (float)l;
                    if (last) {
                        stage[v] = (float)l;
                        stage[n + v] = 0.f;
                    }
                }
            }
            if (lane < 2) ((uint16_t *)Ln)[n + lane] = (uint16_t)(PAD_LAMBDA + BIAS);
            wave_sync();
            bool mism = false;
            for (int w = lane; w < C.mw; w += 64) mism |= SHc[w] != S[w];
            it = i + 1;
            if (__ballot(mism) == 0ull) {
                converged = true;
                break;
            }
            fv = -1;
            if (P.lottery && i >= P.skip && i <= P.max_iter - 2)
                fv = lottery_pick_q(C, seed, shot_id, i, Ln16, S, SHp, lane);
            uint32_t *t = Lc;
            Lc = Ln;
            Ln = t;
            wave_sync();
        }

        if (a.ring) {
            const ServeRing &R = *a.ring;
            uint32_t *corr_row = R.corr + shot * C.nw;
            for (int w = lane; w < C.nw; w += 64) corr_row[w] = EH[w];
            const bool osd = !converged && P.osd != OSD_NONE;
            if (osd) {
                float *dst = R.llr + shot * 2 * n;
                for (int v = lane; v < 2 * n; v += 64) dst[v] = stage[v];
            }
            if (lane == 0) {
                R.flags[shot] = converged ? (uint8_t)FLAG_CONVERGED : osd ? (uint8_t)(FLAG_OSD | FLAG_OSD_PENDING) : 0;
                R.iters[shot] = it;
            }
            serve_publish(R, item, lane);
            wave_sync();
            continue;
        }
        for (int w = lane; w < C.nw; w += 64) a.corr[shot * C.nw + w] = EH[w];
        const uint8_t fl = converged ? (uint8_t)FLAG_CONVERGED : (uint8_t)(P.osd != OSD_NONE ? FLAG_OSD : 0);
        if (lane == 0) {
            a.flags[shot] = fl;
            if (a.iters) a.iters[shot] = it;
        }
        if (!converged && P.osd != OSD_NONE) {
            uint32_t q = 0;
            if (lane == 0) q = atomicAdd(&a.counters[1], 1u);
            q = __builtin_amdgcn_readfirstlane(q);
            if (lane == 0) a.fail_list[q] = (int32_t)shot;
            if ((int64_t)q < a.fail_cap) {
                float *dst = a.fail_llr + (size_t)q * 2 * n;
                for (int v = lane; v < 2 * n; v += 64) dst[v] = stage[v];
            }
        }
        wave_sync();
    }
}

}  // namespace

int bp_int8_slots(int m) {
    const int need = (m + 63) / 64;
    for (int s : {1, 2, 4, 8, 14, 16})
        if (need <= s) return s;
    return 0;
}

int bp_int8_table_bytes(int slots) { return (int)(((size_t)slots * DEG * 64 * 2 + 15) & ~(size_t)15); }

int bp_int8_wave_bytes(int m, int n) {
    size_t mw = (size_t)(m + 31) / 32;
    size_t eh = 2 * (size_t)((n + 63) / 64);
    size_t lwords = (size_t)(n + 3) / 2;
    size_t tot = ((2 * lwords * 4 + 15) & ~(size_t)15) + 4 * (3 * mw + eh);
    return (int)((tot + 15) & ~(size_t)15);
}

template <int SLOTS, bool LLR_FLIP>
static hipError_t launch_q(const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    size_t lds = (size_t)bp_int8_table_bytes(SLOTS) + (size_t)a.wave_bytes * wpb;
    hipError_t e = hipFuncSetAttribute((const void *)bp_int8_kernel<SLOTS, LLR_FLIP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bp_int8_kernel<SLOTS, LLR_FLIP>), dim3(blocks), dim3(64 * wpb), lds, s, a);
    return hipGetLastError();
}

template <int SLOTS>
static hipError_t launch_s(const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    return a.prm.flip == FLIP_LLR ? launch_q<SLOTS, true>(a, blocks, wpb, s) : launch_q<SLOTS, false>(a, blocks, wpb, s);
}

template <int SLOTS>
static hipError_t occ_q(int wpb, int lds, int *out) {
    // both flip variants use the same registers to within the allocation granule;
    // the message-flip variant is the one queried
    hipError_t e = hipFuncSetAttribute((const void *)bp_int8_kernel<SLOTS, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bp_int8_kernel<SLOTS, false>, 64 * wpb, (size_t)lds);
}

hipError_t launch_bp_int8(int slots, const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    switch (slots) {
    case 1: return launch_s<1>(a, blocks, wpb, s);
    case 2: return launch_s<2>(a, blocks, wpb, s);
    case 4: return launch_s<4>(a, blocks, wpb, s);
    case 8: return launch_s<8>(a, blocks, wpb, s);
    case 14: return launch_s<14>(a, blocks, wpb, s);
    default: return launch_s<16>(a, blocks, wpb, s);
    }
}

hipError_t bp_int8_max_blocks_per_cu(int slots, int wpb, int lds, int *out) {
    switch (slots) {
    case 1: return occ_q<1>(wpb, lds, out);
    case 2: return occ_q<2>(wpb, lds, out);
    case 4: return occ_q<4>(wpb, lds, out);
    case 8: return occ_q<8>(wpb, lds, out);
    case 14: return occ_q<14>(wpb, lds, out);
    default: return occ_q<16>(wpb, lds, out);
    }
}

}  // namespace lbp
