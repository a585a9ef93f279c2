// Plain global-memory Lottery BP: the comparison path for the fused kernels.
//
// The same decoding as lbp_decode for FP32 / FP16 message storage, written the
// way a straightforward GPU port is: every message lives in HBM
// ([shots][m][DEG] alpha and beta, [shots][2][n] lambda), one thread per check
// or per column, and one kernel launch per half-iteration:
//   cn    (shot, check):  alpha -> beta           (Algorithm 1, CN update)
//   col   (shot, column): beta -> lambda, e_hat, next alpha (LLR update, hard
//                          decision, VN update of the next iteration)
//   check (wave per shot): syndrome estimate, termination, lottery
//                          (Algorithm 3), failure list for OSD
// All arithmetic is fp32.  Column sums run in ascending check order as exact
// TwoSum pairs (lambda is stored as hi and lo), and each stored message is the
// exact value rounded once to the storage format (fp16 through fp32, which
// rounds like one step: 24 >= 2 * 11 + 2), so the messages follow the method's
// reading without any fp64 on the device; nothing is kept on chip between
// launches.
#include <hip/hip_fp16.h>

#include "device_util.h"
#include "lbp_internal.h"

namespace lbp {
namespace {

// Round an fp32 value to the message storage format, saturating at the
// format's largest finite value.
__device__ __forceinline__ float store_msg(int msg, float x) {
    if (msg == MSG_FP16) {
        __half h = __float2half_rn(x);
        if (__hisinf(h)) return x > 0.f ? 65504.0f : -65504.0f;
        return __half2float(h);
    }
    if (__builtin_isinf(x)) return x > 0.f ? 3.402823466e38f : -3.402823466e38f;
    return x;
}

__device__ __forceinline__ float mu_of(const DevCode &C, int msg, int v) {
    return msg == MSG_FP16 ? C.mu_f16[v] : C.mu_f32[v];
}

// mu + sum of the terms b[j] selected by mask, in ascending check order, as an
// exact pair (hi, lo) with hi the sum rounded once to fp32.
__device__ __forceinline__ void exact_sum(float mu, const float (&b)[CDEG], uint32_t mask, float &hi, float &lo) {
    hi = mu;
    lo = 0.f;
    for (int j = 0; j < CDEG; ++j)
        if ((mask >> j) & 1u) {
            float s, e;
            two_sum(hi, b[j], s, e);
            hi = s;
            lo += e;
        }
    if (__builtin_isinf(hi)) {
        lo = 0.f;
        return;
    }
    float s, e;
    two_sum(hi, lo, s, e);
    hi = s;
    lo = e;
}

// alpha^(0) = mu on every real slot, +inf (never a minimum) on padding slots.
__global__ void bl_init(BlArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t slots = (int64_t)a.code.m * DEG;
    if (t >= a.shots * slots) return;
    const int64_t shot = t / slots;
    const int e = (int)(t - shot * slots);
    const uint32_t v = a.code.cn_cols[e];
    a.alpha[t] = v == NOPOS ? __builtin_inff() : store_msg(a.msg, mu_of(a.code, a.msg, (int)v));
    if (e == 0) {
        a.active[shot] = 1;
        a.flipv[shot] = -1;
    }
    if (e < 2 * a.code.mw) a.shat[shot * 2 * a.code.mw + e] = 0u;
}

// Check-node update of iteration i for every active shot.
__global__ void bl_cn(BlArgs a, int i) {
    const int64_t shot = blockIdx.x;
    const int c = blockIdx.y * blockDim.x + threadIdx.x;
    const DevCode &C = a.code;
    if (c >= C.m || !a.active[shot]) return;
    const int64_t base = (shot * C.m + c) * DEG;
    const int deg = C.cn_deg[c];
    const int fv = a.flipv[shot];
    const bool llr = a.prm.flip == FLIP_LLR && i > 0;
    const float *lhi = a.lam + shot * 2 * C.n, *llo = lhi + C.n;
    float x[DEG];
    float m1 = __builtin_inff(), m2 = __builtin_inff();
    int arg = -1, par = (a.synd[shot * C.mw + (c >> 5)] >> (c & 31)) & 1u;
    for (int k = 0; k < DEG; ++k) {
        const uint32_t v = C.cn_cols[c * DEG + k];
        if (k >= deg) break;
        float al;
        if (llr) {
            // lambda - beta from the exact pair, rounded once (LLR flip: lambda may be negated)
            float s1, e1, s2, e2;
            two_sum(lhi[v], -a.beta[base + k], s1, e1);
            two_sum(s1, e1 + llo[v], s2, e2);
            al = store_msg(a.msg, __builtin_isinf(s1) ? s1 : s2);
        } else {
            al = a.alpha[base + k];
        }
        if (!llr && (int)v == fv) al = -al;  // message flip (Algorithm 3)
        x[k] = al;
        const float mag = __builtin_fabsf(al);
        if (mag < m1) {
            m2 = m1;
            m1 = mag;
            arg = k;
        } else if (mag < m2) {
            m2 = mag;
        }
        par ^= al < 0.f;
    }
    if (deg == 1) m2 = CAP_FLOAT;
    const float s1 = scale_float(a.prm.scale_mode, a.prm.scale_f, i, m1);
    const float s2 = scale_float(a.prm.scale_mode, a.prm.scale_f, i, m2);
    for (int k = 0; k < deg; ++k) {
        const float b = k == arg ? s2 : s1;
        const int neg = par ^ (x[k] < 0.f);
        a.beta[base + k] = store_msg(a.msg, neg ? -b : b);
    }
}

// lambda^(i), e_hat^(i) and (message-flip mode) alpha^(i+1) of every column.
__global__ void bl_col(BlArgs a) {
    const int64_t shot = blockIdx.x;
    const int v = blockIdx.y * blockDim.x + threadIdx.x;
    const DevCode &C = a.code;
    if (!a.active[shot]) return;  // uniform per block
    const bool valid = v < C.n;
    float b[CDEG];
    uint32_t pos[CDEG];
    uint32_t mask = 0;
    float hi = 1.f, lo = 0.f;
    if (valid) {
        const u32x4 tab = col_positions(C, v);
        const float mu = mu_of(C, a.msg, v);
        for (int j = 0; j < CDEG; ++j) {
            pos[j] = tab[j];
            b[j] = pos[j] != NOPOS32 ? a.beta[shot * C.m * DEG + pos[j]] : 0.f;
            if (pos[j] != NOPOS32) mask |= 1u << j;
        }
        exact_sum(mu, b, mask, hi, lo);
        a.lam[shot * 2 * C.n + v] = hi;
        a.lam[shot * 2 * C.n + C.n + v] = lo;
        if (a.prm.flip == FLIP_MSG) {
            for (int j = 0; j < CDEG; ++j) {
                if (pos[j] == NOPOS32) continue;
                float xh, xl;
                exact_sum(mu, b, mask & ~(1u << j), xh, xl);  // extrinsic sum, rounded once
                a.alpha[shot * C.m * DEG + pos[j]] = store_msg(a.msg, xh);
            }
        }
    }
    const uint64_t bal = __ballot(valid && hard_pair(hi, lo));
    if ((threadIdx.x & 63) == 0 && v < C.n) {
        const int w = v >> 5;
        a.ehat[shot * C.nw + w] = (uint32_t)bal;
        if (w + 1 < C.nw) a.ehat[shot * C.nw + w + 1] = (uint32_t)(bal >> 32);
    }
}

// Syndrome estimate, termination and lottery of iteration i: one wave per shot.
__global__ void bl_check(BlArgs a, int i) {
    const DevCode &C = a.code;
    const BpParams &P = a.prm;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const uint32_t last_mask = (C.m & 31) ? ((1u << (C.m & 31)) - 1u) : ~0u;
    for (int64_t shot = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); shot < a.shots;
         shot += waves) {
        if (!a.active[shot]) continue;
        const uint32_t *S = a.synd + shot * C.mw;
        uint32_t *SHc = a.shat + (shot * 2 + (i & 1)) * C.mw;
        const uint32_t *SHp = a.shat + (shot * 2 + ((i + 1) & 1)) * C.mw;
        const uint32_t *EH = a.ehat + shot * C.nw;
        bool mism = false;
        for (int w = lane; w < C.mw; w += 64) {
            uint32_t x = 0;
            for (int bit = 0; bit < 32; ++bit) {
                const int c = w * 32 + bit;
                if (c >= C.m) break;
                uint32_t p = 0;
                for (int k = 0; k < C.cn_deg[c]; ++k) {
                    const uint32_t v = C.cn_cols[c * DEG + k];
                    p ^= (EH[v >> 5] >> (v & 31)) & 1u;
                }
                x |= p << bit;
            }
            SHc[w] = x;
            const uint32_t s = w == C.mw - 1 ? (S[w] & last_mask) : S[w];
            mism |= x != s;
        }
        const bool conv = __ballot(mism) == 0ull;
        if (conv || i == P.max_iter - 1) {
            for (int w = lane; w < C.nw; w += 64) a.corr[shot * C.nw + w] = EH[w];
            if (lane == 0) {
                a.active[shot] = 0;
                a.flags[shot] = conv ? (uint8_t)FLAG_CONVERGED : (uint8_t)(P.osd != OSD_NONE ? FLAG_OSD : 0);
                if (a.iters) a.iters[shot] = i + 1;
                if (!conv && P.osd != OSD_NONE) {
                    const uint32_t q = atomicAdd(&a.counters[1], 1u);
                    a.fail_list[q] = (int32_t)shot;
                }
            }
            continue;
        }
        if (lane == 0) atomicAdd(&a.counters[0], 1u);
        int fv = -1;
        if (P.lottery && i >= P.skip && i <= P.max_iter - 2) {
            // U = checks whose previous estimate differs from s, ascending
            int N = 0;
            for (int w = lane; w < C.mw; w += 64) {
                const uint32_t s = w == C.mw - 1 ? (S[w] & last_mask) : S[w];
                N += __popc(SHp[w] ^ s);
            }
            for (int o = 32; o > 0; o >>= 1) N += __shfl_xor(N, o, 64);
            if (N > 0) {
                const uint64_t seed = a.shot_keys ? a.shot_keys[2 * shot] : P.seed;
                const uint64_t sid = a.shot_keys ? a.shot_keys[2 * shot + 1] : a.first_shot_id + (uint64_t)shot;
                uint64_t x1;
                const uint64_t x = philox_word01(seed, sid, (uint64_t)i, x1);
                const int cn_rule = P.rule & 3, vn_rule = (P.rule >> 4) & 3;
                int cstar = -1;
                if (cn_rule == LOT_CN_WORST) {
                    // the check of U with the most neighbours in the hard decision, first of equals
                    int best = -1;
                    for (int c = 0; c < C.m; ++c) {  // uniform scan: clarity over speed
                        const uint32_t s = (S[c >> 5] >> (c & 31)) & 1u;
                        if (!(((SHp[c >> 5] >> (c & 31)) & 1u) ^ s)) continue;
                        int cnt = 0;
                        for (int k = 0; k < C.cn_deg[c]; ++k) {
                            const uint32_t v = C.cn_cols[c * DEG + k];
                            cnt += (int)((EH[v >> 5] >> (v & 31)) & 1u);
                        }
                        if (cnt > best) {
                            best = cnt;
                            cstar = c;
                        }
                    }
                } else {
                    int k = (int)(((x >> 32) * (uint64_t)N) >> 32);
                    for (int w = 0; w < C.mw && cstar < 0; ++w) {  // uniform scan: clarity over speed
                        const uint32_t s = w == C.mw - 1 ? (S[w] & last_mask) : S[w];
                        uint32_t u = SHp[w] ^ s;
                        const int cnt = __popc(u);
                        if (k < cnt) {
                            for (int q = 0; q < k; ++q) u &= u - 1;
                            cstar = w * 32 + __ffs(u) - 1;
                        }
                        k -= cnt;
                    }
                }
                int best_v = -1, best_cnt = -1;
                long long best_q = 0;
                for (int e = 0; e < C.cn_deg[cstar]; ++e) {
                    const int v = C.cn_cols[cstar * DEG + e];
                    const u32x4 tab = col_positions(C, v);
                    int cnt = 0;
                    for (int j = 0; j < CDEG; ++j) {
                        const uint32_t p = tab[j];
                        if (p == NOPOS32) continue;
                        const int c = (int)(p / DEG);
                        const uint32_t s = (S[c >> 5] >> (c & 31)) & 1u;
                        cnt += (int)(((SHp[c >> 5] >> (c & 31)) & 1u) ^ s);
                    }
                    const long long q = (long long)quantized_abs_pair(a.lam[shot * 2 * C.n + v],
                                                                      a.lam[shot * 2 * C.n + C.n + v]);
                    if (best_v < 0 || lottery_key_less(vn_rule, cnt, q, v, best_cnt, best_q, best_v)) {
                        best_v = v;
                        best_cnt = cnt;
                        best_q = q;
                    }
                }
                fv = best_v;
                if (vn_rule == LOT_VN_RANDOM)
                    fv = C.cn_cols[cstar * DEG + (int)(((x1 >> 32) * (uint64_t)C.cn_deg[cstar]) >> 32)];
            }
        }
        if (lane == 0) {
            if (P.flip == FLIP_LLR) {
                if (fv >= 0) {
                    a.lam[shot * 2 * C.n + fv] = -a.lam[shot * 2 * C.n + fv];
                    a.lam[shot * 2 * C.n + C.n + fv] = -a.lam[shot * 2 * C.n + C.n + fv];
                }
                a.flipv[shot] = -1;
            } else {
                a.flipv[shot] = fv;
            }
        }
    }
}

// lambda of failed shots [from, from + count) into the OSD staging format (hi[n], lo[n]).
__global__ void bl_stage(BlArgs a, int64_t from, int64_t count, float *dst, uint32_t *ocounters) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = a.code.n;
    if (t == 0) ocounters[1] = (uint32_t)count;
    if (t >= count * 2 * n) return;
    const int64_t q = t / (2 * n);
    const int64_t r = t - q * 2 * n;
    dst[q * 2 * n + r] = a.lam[(int64_t)a.fail_list[from + q] * 2 * n + r];
}

}  // namespace

hipError_t baseline_init(const BlArgs &a, hipStream_t s) {
    const int64_t total = a.shots * a.code.m * DEG;
    hipLaunchKernelGGL(bl_init, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t baseline_iteration(const BlArgs &a, int i, hipStream_t s) {
    hipLaunchKernelGGL(bl_cn, dim3((unsigned)a.shots, (unsigned)((a.code.m + 255) / 256)), dim3(256), 0, s, a, i);
    hipLaunchKernelGGL(bl_col, dim3((unsigned)a.shots, (unsigned)((a.code.n + 255) / 256)), dim3(256), 0, s, a);
    const int64_t blocks = std::min<int64_t>((a.shots + 3) / 4, 65536);
    hipLaunchKernelGGL(bl_check, dim3((unsigned)blocks), dim3(256), 0, s, a, i);
    return hipGetLastError();
}

hipError_t baseline_stage(const BlArgs &a, int64_t from, int64_t count, float *dst, uint32_t *ocounters,
                          hipStream_t s) {
    const int64_t total = std::max<int64_t>(1, count * 2 * a.code.n);
    hipLaunchKernelGGL(bl_stage, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, from, count, dst,
                       ocounters);
    return hipGetLastError();
}

}  // namespace lbp
