// Batched Lottery BP on gfx950: one wavefront decodes one shot at a time, or,
// for codes whose per-shot state leaves room for few shots per CU, one
// workgroup decodes one shot (the GRP variant of bp_kernel).
//
// Normalized min-sum BP (Algorithm 1) with the lottery policy (Algorithm 3)
// and the delayed-syndrome trick of Sec. IV-B: the unsatisfied set of
// iteration i is taken from the syndrome estimate of iteration i-1, so the
// lottery can be decided between the check-node and variable-node halves of
// iteration i without waiting for iteration i's syndrome.
//
// Work distribution: the grid is persistent; each wave pulls the next shot from
// a global counter, runs it to convergence (or I iterations) and writes its
// outputs.  A wave never waits for another wave, so early-terminating shots do
// not idle the SIMD behind a slow one.
//
// Per-wave (per-workgroup in GRP) LDS, the shot's whole state:
//   E  [m][DEG] messages, in place: alpha (V2C) before the check-node half,
//               beta (C2V) after it; padding slots hold a sentinel that never
//               wins a minimum and is never read by a column.
//   S  [mw]     measured syndrome
//   SH [2][mw]  syndrome estimate of the current / previous iteration
//   EH [2*ceil(n/64)] hard decision of the current iteration (ballot words)
//
// Check-node half: lane L owns checks L, L+64, ...; it reads its padded row
// with one vector LDS load, runs min1/min2/argmin/sign-parity sequentially over
// the row in registers and writes the row back.  A sequential pass costs ~3
// VALU ops per edge against ~9 for a cross-lane segmented butterfly, which is
// why rows are not spread across lanes.
// Variable-node half: lane L owns columns L, L+64, ...; it gathers its <= CDEG
// C2V messages through the column table, forms lambda (fixed ascending-check
// order, so float results are deterministic), the hard decision, the syndrome
// estimate (LDS atomic XOR, order-independent) and the next V2C messages.
#include "device_util.h"
#include "lbp_internal.h"

#include <hip/hip_fp16.h>

namespace lbp {
namespace {

// ---------------------------------------------------------------- formats

template <int MSG> struct Fmt;

template <> struct Fmt<MSG_INT8> {
    using T = int8_t;
    using A = int32_t;
    static __device__ __forceinline__ A load(T x) { return (A)x; }
    static __device__ __forceinline__ T sat(A x) { return (T)(x > 127 ? 127 : (x < -127 ? -127 : x)); }
    static __device__ __forceinline__ T pad() { return (T)127; }
    static __device__ __forceinline__ A mu(const DevCode &C, int v) { return C.mu_q[v]; }
    static __device__ __forceinline__ bool hard(A l) { return l <= 0; }
};

template <> struct Fmt<MSG_FP16> {
    using T = __half;
    using A = float;
    static __device__ __forceinline__ A load(T x) { return __half2float(x); }
    static __device__ __forceinline__ T sat(A x) {
        __half h = __float2half_rn(x);
        if (__hisinf(h)) h = __float2half_rn(x > 0.f ? 65504.f : -65504.f);
        return h;
    }
    static __device__ __forceinline__ T pad() { return __ushort_as_half((unsigned short)0x7C00u); }
    static __device__ __forceinline__ A mu(const DevCode &C, int v) { return C.mu_f16[v]; }
    static __device__ __forceinline__ bool hard(A l) { return l <= TAU_FLOAT; }
};

template <> struct Fmt<MSG_FP32> {
    using T = float;
    using A = float;
    static __device__ __forceinline__ A load(T x) { return x; }
    static __device__ __forceinline__ T sat(A x) {
        if (__builtin_isinf(x)) return x > 0.f ? 3.402823466e38f : -3.402823466e38f;
        return x;
    }
    static __device__ __forceinline__ T pad() { return __builtin_inff(); }
    static __device__ __forceinline__ A mu(const DevCode &C, int v) { return C.mu_f32[v]; }
    static __device__ __forceinline__ bool hard(A l) { return l <= TAU_FLOAT; }
};

// Check-node scale applied to a magnitude.
__device__ __forceinline__ int scale_int8(const BpParams &P, int i, int mag) {
    if (P.scale_mode == 1) return (P.scale_k * mag) >> 3;
    int sh = i + 1 > 30 ? 30 : i + 1;
    return mag - (mag >> sh);
}

// A column sum carried as an unevaluated pair hi + lo.  Int x.y sums are exact
// integers (lo = 0); FP32 and FP16 sums use TwoSum so that the pair equals the
// exact sum (fp16 terms span about 40 binades, more than an fp32 significand
// holds), hi is that sum rounded once to fp32, and every decision taken on
// lambda sees the exact value.
template <typename A> struct Lam {
    A hi;
    float lo;
};

// mu plus the C2V messages b[j] selected by `mask`, in ascending check order.
template <int MSG>
__device__ __forceinline__ Lam<typename Fmt<MSG>::A> sum_terms(typename Fmt<MSG>::A mu,
                                                               const typename Fmt<MSG>::A b[CDEG], uint32_t mask) {
    using A = typename Fmt<MSG>::A;
    if constexpr (MSG != MSG_INT8) {
        float hi = mu, lo = 0.f;
#pragma unroll
        for (int j = 0; j < CDEG; ++j)
            if ((mask >> j) & 1u) {
                float s, e;
                two_sum(hi, b[j], s, e);
                hi = s;
                lo += e;
            }
        if (__builtin_isinf(hi)) return {hi, 0.f};
        float s, e;
        two_sum(hi, lo, s, e);
        return {s, e};
    } else {
        A acc = mu;
#pragma unroll
        for (int j = 0; j < CDEG; ++j)
            if ((mask >> j) & 1u) acc += b[j];
        return {acc, 0.f};
    }
}

// Loads the column's C2V messages; returns the slot mask and lambda = mu + sum.
template <int MSG, class TB>
__device__ __forceinline__ Lam<typename Fmt<MSG>::A> column_lambda(const DevCode &C, int v, typename TB::T tab,
                                                                   const typename Fmt<MSG>::T *E,
                                                                   typename Fmt<MSG>::A b[CDEG], uint32_t &mask) {
    using F = Fmt<MSG>;
    mask = 0;
#pragma unroll
    for (int j = 0; j < CDEG; ++j) {
        uint32_t p = TB::pos(tab, j);
        b[j] = p != TB::NONE ? F::load(E[p]) : (typename F::A)0;
        if (p != TB::NONE) mask |= 1u << j;
    }
    return sum_terms<MSG>(F::mu(C, v), b, mask);
}

// Hard decision e = [lambda <= threshold] on the exact value hi + lo.
template <int MSG>
__device__ __forceinline__ bool hard_decision(const Lam<typename Fmt<MSG>::A> &l) {
    if constexpr (MSG == MSG_INT8) return l.hi <= 0;
    else return l.hi < TAU_FLOAT || (l.hi == TAU_FLOAT && l.lo <= 0.f);
}

// Q(|lambda|): |lambda| for Int x.y, floor(|lambda| * 2^12) for float (exact).
template <int MSG>
__device__ __forceinline__ uint64_t quantized_abs(const Lam<typename Fmt<MSG>::A> &l) {
    if constexpr (MSG == MSG_INT8) return (uint64_t)(l.hi < 0 ? -l.hi : l.hi);
    else return quantized_abs_pair(l.hi, l.lo);
}

// ------------------------------------------------------------ check-node half

template <int MSG>
__device__ void cn_half(const DevCode &C, const BpParams &P, int i, typename Fmt<MSG>::T *E,
                        const uint32_t *S, int t0, int tn) {
    using F = Fmt<MSG>;
    using T = typename F::T;
    for (int c = t0; c < C.m; c += tn) {
        T a[DEG];
        T *row = E + c * DEG;
#pragma unroll
        for (int k = 0; k < DEG; ++k) a[k] = row[k];
        const int deg = C.cn_deg[c];
        int par = (S[c >> 5] >> (c & 31)) & 1;  // (-1)^{s_c}
        T out[DEG];
        if constexpr (MSG == MSG_INT8) {
            int m1 = 1 << 20, m2 = 1 << 20, arg = 0;
#pragma unroll
            for (int k = 0; k < DEG; ++k) {
                int x = a[k];
                int mag = x < 0 ? -x : x;
                if (mag < m1) { m2 = m1; m1 = mag; arg = k; }
                else if (mag < m2) m2 = mag;
                par ^= (x < 0);
            }
            // padding slots hold 127: a degree-1 check sends the format's maximum
            m1 = m1 < P.qmax ? m1 : P.qmax;
            m2 = m2 < P.qmax ? m2 : P.qmax;
            const int s1 = scale_int8(P, i, m1), s2 = scale_int8(P, i, m2);
#pragma unroll
            for (int k = 0; k < DEG; ++k) {
                int mag = k == arg ? s2 : s1;
                int neg = par ^ ((int)a[k] < 0);
                out[k] = k < deg ? (T)(neg ? -mag : mag) : F::pad();
            }
        } else {
            float m1 = __builtin_inff(), m2 = __builtin_inff();
            int arg = 0;
            float x[DEG];
#pragma unroll
            for (int k = 0; k < DEG; ++k) {
                x[k] = F::load(a[k]);
                float mag = __builtin_fabsf(x[k]);
                if (mag < m1) { m2 = m1; m1 = mag; arg = k; }
                else if (mag < m2) m2 = mag;
                par ^= (x[k] < 0.f);
            }
            if (deg == 1) m2 = CAP_FLOAT;
            const float s1 = scale_float(P.scale_mode, P.scale_f, i, m1), s2 = scale_float(P.scale_mode, P.scale_f, i, m2);
#pragma unroll
            for (int k = 0; k < DEG; ++k) {
                float mag = k == arg ? s2 : s1;
                int neg = par ^ (x[k] < 0.f);
                out[k] = k < deg ? F::sat(neg ? -mag : mag) : F::pad();
            }
        }
#pragma unroll
        for (int k = 0; k < DEG; ++k) row[k] = out[k];
    }
}

// ------------------------------------------------------------ lottery selection

// Worst check of U (Sec. III-B): the most neighbours whose hard decision on
// lambda^(i) (rebuilt from E) is 1, the smallest index among equals.
template <int MSG, class TB>
__device__ int worst_check(const DevCode &C, const typename Fmt<MSG>::T *E, const uint32_t *S, const uint32_t *SHp,
                           int lane) {
    unsigned long long best = 0;
    for (int c0 = 0; c0 < C.m; c0 += 64) {
        const int c = c0 + lane;
        if (c < C.m && (((SHp[c >> 5] ^ S[c >> 5]) >> (c & 31)) & 1u)) {
            int cnt = 0;
            const int deg = C.cn_deg[c];
            for (int k = 0; k < deg; ++k) {
                const int v = C.cn_cols[c * DEG + k];
                typename Fmt<MSG>::A b[CDEG];
                uint32_t mask;
                cnt += hard_decision<MSG>(column_lambda<MSG, TB>(C, v, TB::load(C, v), E, b, mask)) ? 1 : 0;
            }
            const unsigned long long key = ((unsigned long long)(cnt + 1) << 32) | (0xFFFFFFFFu - (uint32_t)c);
            best = key > best ? key : best;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(best, o, 64);
        best = y > best ? y : best;
    }
    return (int)(0xFFFFFFFFu - (uint32_t)best);
}

// Algorithm 3 with U taken from the previous iteration's syndrome estimate
// SHp; lambda^(i) of the candidates is rebuilt from the C2V messages of
// iteration i still held in E, with the same arithmetic as the VN half.
// P.rule picks the design-space variant (Sec. III-B): random or worst check;
// proposed key (count, Q, column), Q-first, unreliable (Q, column) or a
// random neighbour drawn from word 1 of the same Philox block.
template <int MSG, class TB>
__device__ int lottery_select(const DevCode &C, const BpParams &P, uint64_t seed, uint64_t shot_id, int i,
                              const typename Fmt<MSG>::T *E, const uint32_t *S, const uint32_t *SHp, int lane) {
    using F = Fmt<MSG>;
    int N = 0;
    for (int w0 = 0; w0 < C.mw; w0 += 64) {
        int w = w0 + lane;
        uint32_t u = w < C.mw ? (SHp[w] ^ S[w]) : 0u;
        N += wave_sum(__popc(u));
    }
    if (N == 0) return -1;
    const int cn_rule = P.rule & 3, vn_rule = (P.rule >> 4) & 3;
    uint64_t x1;
    const uint64_t x = philox_word01(seed, shot_id, (uint64_t)i, x1);
    int cstar = -1;
    if (cn_rule == LOT_CN_WORST) {
        cstar = __builtin_amdgcn_readfirstlane(worst_check<MSG, TB>(C, E, S, SHp, lane));
    } else {
        uint32_t k = (uint32_t)(((x >> 32) * (uint64_t)N) >> 32);  // floor(r * N)
        for (int w0 = 0; w0 < C.mw; w0 += 64) {
            int w = w0 + lane;
            uint32_t u = w < C.mw ? (SHp[w] ^ S[w]) : 0u;
            int cnt = __popc(u);
            int incl = wave_incl_scan(cnt, lane);
            int tot = __builtin_amdgcn_readlane(incl, 63);
            if ((int)k < tot) {
                int excl = incl - cnt;
                bool here = (int)k >= excl && (int)k < incl;
                int pos = 0;
                if (here) {
                    uint32_t t = u;
                    for (int q = (int)k - excl; q > 0; --q) t &= t - 1;
                    pos = w * 32 + __ffs(t) - 1;
                }
                uint64_t b = __ballot(here);
                cstar = __builtin_amdgcn_readlane(pos, __ffsll((unsigned long long)b) - 1);
                break;
            }
            k -= (uint32_t)tot;
        }
    }
    if (vn_rule == LOT_VN_RANDOM) {
        const uint32_t k = (uint32_t)(((x1 >> 32) * (uint64_t)C.cn_deg[cstar]) >> 32);
        return C.cn_cols[cstar * DEG + (int)k];
    }
    // candidates v in V(c*), ordered by the neighbour rule
    int cnt = -1, v = 0x7FFFFFFF;
    uint64_t q = 0;
    if (lane < DEG) {
        uint32_t vv = C.cn_cols[cstar * DEG + lane];
        if (vv != NOPOS) {
            v = (int)vv;
            const typename TB::T tab = TB::load(C, v);
            typename F::A b[CDEG];
            uint32_t mask;
            Lam<typename F::A> lam = column_lambda<MSG, TB>(C, v, tab, E, b, mask);
            cnt = 0;
#pragma unroll
            for (int j = 0; j < CDEG; ++j) {
                uint32_t p = TB::pos(tab, j);
                if (p != TB::NONE) {
                    uint32_t c = p / DEG;
                    cnt += ((SHp[c >> 5] ^ S[c >> 5]) >> (c & 31)) & 1u;
                }
            }
            q = quantized_abs<MSG>(lam);
        }
    }
    int bc = -1, bv = -1;
    uint64_t bq = 0;
#pragma unroll
    for (int k = 0; k < DEG; ++k) {
        int ck = __builtin_amdgcn_readlane(cnt, k), vk = __builtin_amdgcn_readlane(v, k);
        uint64_t qk = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(q >> 32), k) << 32) |
                      __builtin_amdgcn_readlane((uint32_t)q, k);
        if (ck < 0) continue;
        if (bv < 0 || lottery_key_less(vn_rule, ck, qk, vk, bc, bq, bv)) {
            bc = ck;
            bq = qk;
            bv = vk;
        }
    }
    return bv;
}

// ------------------------------------------------------------ variable-node half

template <int MSG, class TB>
__device__ void vn_half(const DevCode &C, const BpParams &P, int fv, bool last, typename Fmt<MSG>::T *E,
                        uint32_t *SH, uint32_t *EH, int lane, int w0, int wn, float *llr_row, float *stage) {
    using F = Fmt<MSG>;
    using A = typename F::A;
    const int nvs = (C.n + 63) >> 6;
    for (int vs = w0; vs < nvs; vs += wn) {
        const int v = vs * 64 + lane;
        const bool valid = v < C.n;
        const typename TB::T tab = valid ? TB::load(C, v) : TB::empty();
        A b[CDEG];
        uint32_t mask = 0;
        Lam<A> lam{(A)1, 0.f};
        if (valid) lam = column_lambda<MSG, TB>(C, v, tab, E, b, mask);
        const bool e = valid && hard_decision<MSG>(lam);
        const uint64_t bal = __ballot(e);
        if (lane == 0) {
            EH[2 * vs] = (uint32_t)bal;
            EH[2 * vs + 1] = (uint32_t)(bal >> 32);
        }
        if (e) {
#pragma unroll
            for (int j = 0; j < CDEG; ++j) {
                uint32_t p = TB::pos(tab, j);
                if (p != TB::NONE) {
                    uint32_t c = p / DEG;
                    atomicXor(&SH[c >> 5], 1u << (c & 31));
                }
            }
        }
        if (!valid) continue;
        if (llr_row) llr_row[v] = (float)lam.hi;
        if (last) {
            stage[v] = (float)lam.hi;
            stage[C.n + v] = lam.lo;
            continue;
        }
        const bool flipv = v == fv;
        if constexpr (MSG == MSG_INT8) {
            const int l2 = (P.flip == FLIP_LLR && flipv) ? -lam.hi : lam.hi;
#pragma unroll
            for (int j = 0; j < CDEG; ++j) {
                uint32_t p = TB::pos(tab, j);
                if (p != TB::NONE) {
                    int a = l2 - b[j];  // == mu + sum of the other C2V messages
                    a = a > P.qmax ? P.qmax : (a < -P.qmax ? -P.qmax : a);
                    if (P.flip == FLIP_MSG && flipv) a = -a;
                    E[p] = (int8_t)a;
                }
            }
        } else if (P.flip == FLIP_MSG) {
            const A mu = F::mu(C, v);
#pragma unroll
            for (int j = 0; j < CDEG; ++j) {
                uint32_t p = TB::pos(tab, j);
                if (p != TB::NONE) {
                    // extrinsic sum in ascending check order, rounded once to the format
                    A a = sum_terms<MSG>(mu, b, mask & ~(1u << j)).hi;
                    E[p] = F::sat(flipv ? -a : a);
                }
            }
        } else {
            const float sg = flipv ? -1.f : 1.f;
#pragma unroll
            for (int j = 0; j < CDEG; ++j) {
                uint32_t p = TB::pos(tab, j);
                if (p != TB::NONE) {
                    // (+-lambda) - beta_j from the exact pair, rounded once
                    float s1, e1, s2, e2;
                    two_sum(sg * (float)lam.hi, -(float)b[j], s1, e1);
                    two_sum(s1, e1 + sg * lam.lo, s2, e2);
                    E[p] = F::sat(__builtin_isinf(s1) ? s1 : s2);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ one shot

// Sync of the threads that decode one shot: the wave, or the block in GRP.
template <bool GRP>
__device__ __forceinline__ void shot_sync() {
    if constexpr (GRP) __syncthreads();
    else wave_sync();
}

// Decode one shot (Algorithm 1 with Algorithm 3) in the LDS state E, S, SH0,
// SH1, EH; returns whether BP converged and sets *it to the iterations run.
// Thread t0 of tn works on checks and words, wave w0 of wn on 64-column groups;
// in GRP, wave 0 runs the lottery and passes v* through *grp_fv (LDS).  The
// lambda of the last iteration is written to stage (hi[n], lo[n]) when the run
// reaches the iteration limit, and to llr_row when it is not null.
template <int MSG, class TB, bool GRP>
__device__ bool decode_shot(const DevCode &C, const BpParams &P, uint64_t seed, uint64_t shot_id,
                            const uint32_t *syn_row, typename Fmt<MSG>::T *E, uint32_t *S, uint32_t *SH0,
                            uint32_t *SH1, uint32_t *EH, float *llr_row, float *stage, int lane, int wv, int t0,
                            int tn, int w0, int wn, int32_t *grp_fv, int &it) {
    using F = Fmt<MSG>;
    using T = typename F::T;
    // padding bits of the last word are ignored (they could otherwise name checks >= m)
    const uint32_t last_mask = (C.m & 31) ? ((1u << (C.m & 31)) - 1u) : ~0u;
    // SH1 is the estimate "before iteration 0" that the lottery of iteration 0
    // reads when K = 0: the hard decision of the prior, H * 0 = 0
    for (int w = t0; w < C.mw; w += tn) {
        uint32_t x = syn_row[w];
        S[w] = w == C.mw - 1 ? (x & last_mask) : x;
        SH1[w] = 0u;
    }
    // alpha^(0) = mu (Algorithm 1 initialisation); padding slots get the sentinel.
    for (int c = t0; c < C.m; c += tn) {
        const int deg = C.cn_deg[c];
#pragma unroll
        for (int k = 0; k < DEG; ++k)
            if (k >= deg) E[c * DEG + k] = F::pad();
    }
    for (int v = t0; v < C.n; v += tn) {
        const typename TB::T tab = TB::load(C, v);
        const T mu = F::sat(F::mu(C, v));
#pragma unroll
        for (int j = 0; j < CDEG; ++j) {
            uint32_t p = TB::pos(tab, j);
            if (p != TB::NONE) E[p] = mu;
        }
    }
    shot_sync<GRP>();

    it = 0;
    for (int i = 0; i < P.max_iter; ++i) {
        uint32_t *SHc = (i & 1) ? SH1 : SH0;
        uint32_t *SHp = (i & 1) ? SH0 : SH1;
        cn_half<MSG>(C, P, i, E, S, t0, tn);
        shot_sync<GRP>();
        int fv = -1;
        const bool lot = P.lottery && i >= P.skip && i <= P.max_iter - 2;
        if constexpr (GRP) {
            if (lot && wv == 0) {
                const int f = lottery_select<MSG, TB>(C, P, seed, shot_id, i, E, S, SHp, lane);
                if (lane == 0) *grp_fv = f;
            }
        } else if (lot) {
            fv = lottery_select<MSG, TB>(C, P, seed, shot_id, i, E, S, SHp, lane);
        }
        for (int w = t0; w < C.mw; w += tn) SHc[w] = 0u;
        shot_sync<GRP>();
        if constexpr (GRP) {
            if (lot) fv = *grp_fv;
        }
        const bool last = i == P.max_iter - 1;
        vn_half<MSG, TB>(C, P, fv, last, E, SHc, EH, lane, w0, wn, llr_row, stage);
        shot_sync<GRP>();
        bool mism = false;
        for (int w = t0; w < C.mw; w += tn) mism |= SHc[w] != S[w];
        it = i + 1;
        bool differs;
        if constexpr (GRP) differs = __syncthreads_or(mism) != 0;
        else differs = __ballot(mism) != 0ull;
        if (!differs) return true;
    }
    return false;
}

// Outputs of a batch shot: corrections, flags, iterations, and for a failed
// shot with OSD its failure-list entry and staged lambda (when it fits).
template <bool GRP>
__device__ void batch_outputs(const DevCode &C, const BpParams &P, int64_t shot, bool converged, int it,
                              const uint32_t *EH, const float *stage, uint32_t *corr, uint8_t *flags, int32_t *iters,
                              uint32_t *counters, int32_t *fail_list, float *fail_llr, int64_t fail_cap, int lane,
                              int t0, int tn, uint32_t *grp_q) {
    for (int w = t0; w < C.nw; w += tn) corr[shot * C.nw + w] = EH[w];
    const uint8_t fl = converged ? (uint8_t)FLAG_CONVERGED : (uint8_t)(P.osd != OSD_NONE ? FLAG_OSD : 0);
    if (t0 == 0) {
        flags[shot] = fl;
        if (iters) iters[shot] = it;
    }
    if (!converged && P.osd != OSD_NONE) {
        uint32_t q = 0;
        if constexpr (GRP) {
            if (threadIdx.x == 0) {
                *grp_q = atomicAdd(&counters[1], 1u);
                fail_list[*grp_q] = (int32_t)shot;
            }
            __syncthreads();
            q = *grp_q;
        } else {
            if (lane == 0) q = atomicAdd(&counters[1], 1u);
            q = __builtin_amdgcn_readfirstlane(q);
            if (lane == 0) fail_list[q] = (int32_t)shot;
        }
        if ((int64_t)q < fail_cap) {
            float *dst = fail_llr + (size_t)q * 2 * C.n;
            for (int v = t0; v < 2 * C.n; v += tn) dst[v] = stage[v];
        }
    }
}

// ------------------------------------------------------------------ kernel

// GRP = false: each wave of the block decodes its own shot (per-wave LDS state).
// GRP = true: the whole block decodes one shot.  The check-node half splits the
// checks over the block's threads, the variable-node half the 64-column groups
// over its waves, block barriers separate the halves, and wave 0 runs the
// lottery and takes work items.  This is for large codes, whose per-shot state
// leaves room for only a few shots per CU: one wave per shot would leave the CU
// with too few waves to hide LDS and memory latency.
template <int MSG, class TB, bool GRP>
__global__ __launch_bounds__(1024) void bp_kernel(BpArgs a) {
    using F = Fmt<MSG>;
    using T = typename F::T;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ ClaimLds claim;  // serving, a shot per wave: the block's ring lock and its waves' claimed items
    __shared__ int64_t grp_item;     // GRP: the block's current work item, -1 when there is none
    __shared__ int32_t grp_fv;       // GRP: the lottery's column of this iteration
    __shared__ uint32_t grp_q;       // GRP: the shot's failure-list position
    const DevCode &C = a.code;
    const BpParams &P = a.prm;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int nwv = (int)(blockDim.x >> 6);
    // work split: thread t0 of tn over checks and words, wave w0 of wn over 64-column groups
    const int t0 = GRP ? (int)threadIdx.x : lane, tn = GRP ? (int)blockDim.x : 64;
    const int w0 = GRP ? wv : 0, wn = GRP ? nwv : 1;
    claim.clear(threadIdx.x);
    __syncthreads();
    unsigned char *base = smem + (GRP ? (size_t)0 : (size_t)wv * a.wave_bytes);
    T *E = (T *)base;
    size_t off = ((size_t)C.m * DEG * sizeof(T) + 15) & ~(size_t)15;
    uint32_t *S = (uint32_t *)(base + off);
    uint32_t *SH0 = S + C.mw;
    uint32_t *SH1 = SH0 + C.mw;
    uint32_t *EH = SH1 + C.mw;
    const int slot = GRP ? (int)blockIdx.x : (int)blockIdx.x * nwv + wv;  // shot slot: its staging row
    float *stage = a.stage + (size_t)slot * 2 * C.n;

    int64_t ring_next = 0, ring_end = 0;  // serving, a workgroup per shot: thread 0's claimed range
    for (;;) {
        int64_t item = 0;
        if constexpr (GRP) {
            if (threadIdx.x == 0) {
                if (a.ring) {
                    // thread 0 keeps the block's claimed range in ring_next / ring_end
                    if (ring_next >= ring_end) {
                        uint32_t cnt = 1;
                        const int64_t first = serve_claim(*a.ring, a.ring->claim_max, &cnt);
                        ring_next = first;
                        ring_end = first < 0 ? first : first + (int64_t)cnt;
                    }
                    grp_item = ring_next < 0 ? -1 : ring_next++;
                } else {
                    const uint32_t it0 = atomicAdd(&a.counters[0], 1u);
                    grp_item = (int64_t)it0 < a.n_work ? (int64_t)it0 : -1;
                }
            }
            __syncthreads();
            item = grp_item;
            if (item < 0) break;
            if (a.ring) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the host's writes of this ring slot
        } else if (a.ring) {
            item = serve_claim_block(*a.ring, &claim, wv, lane);
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
        // wave-uniform: the lottery's Philox rounds then run on the scalar unit
        const uint64_t seed = (uint64_t)uniform64((int64_t)(keys ? keys[2 * shot] : P.seed));
        const uint64_t shot_id =
            (uint64_t)uniform64((int64_t)(keys ? keys[2 * shot + 1] : a.first_shot_id + (uint64_t)shot));
        float *llr_row = a.llr_out ? a.llr_out + shot * C.n : nullptr;
        const uint32_t *syn_row = (a.ring ? a.ring->syn : a.synd) + shot * C.mw;

        int it = 0;
        const bool converged = decode_shot<MSG, TB, GRP>(C, P, seed, shot_id, syn_row, E, S, SH0, SH1, EH, llr_row,
                                                         stage, lane, wv, t0, tn, w0, wn, &grp_fv, it);

        if (a.ring) {
            const ServeRing &R = *a.ring;
            uint32_t *corr_row = R.corr + shot * C.nw;
            for (int w = t0; w < C.nw; w += tn) corr_row[w] = EH[w];
            const bool osd = !converged && P.osd != OSD_NONE;
            if (osd) {
                float *dst = R.llr + shot * 2 * C.n;
                for (int v = t0; v < 2 * C.n; v += tn) dst[v] = stage[v];
            }
            if (t0 == 0) {
                R.flags[shot] = converged ? (uint8_t)FLAG_CONVERGED : osd ? (uint8_t)(FLAG_OSD | FLAG_OSD_PENDING) : 0;
                R.iters[shot] = it;
            }
            if constexpr (GRP) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // every thread's stores, before the entry
                __syncthreads();
                if (wv == 0) serve_publish(R, item, lane);
            } else {
                serve_publish(R, item, lane);
            }
            shot_sync<GRP>();
            continue;
        }
        batch_outputs<GRP>(C, P, shot, converged, it, EH, stage, a.corr, a.flags, a.iters, a.counters, a.fail_list,
                           a.fail_llr, a.fail_cap, lane, t0, tn, &grp_q);
        shot_sync<GRP>();
    }
}

// One persistent launch over several groups of shots (uneven codes, formats and
// parameters): every wave claims the next work item, finds its group in the
// descriptor table (groups hold consecutive item ranges) and decodes that shot
// with the group's code, format and parameters in its LDS slice, which is sized
// for the largest group.  Results are those of lbp_decode of each group alone.
template <int MSG, class TB>
__device__ void multi_shot(const GroupDesc &G, int64_t shot, unsigned char *base, float *stage, int lane) {
    using T = typename Fmt<MSG>::T;
    const DevCode &C = G.code;
    T *E = (T *)base;
    uint32_t *S = (uint32_t *)(base + (((size_t)C.m * DEG * sizeof(T) + 15) & ~(size_t)15));
    uint32_t *SH0 = S + C.mw, *SH1 = SH0 + C.mw, *EH = SH1 + C.mw;
    int it = 0;
    const bool conv = decode_shot<MSG, TB, false>(C, G.prm, G.prm.seed, G.first_shot_id + (uint64_t)shot,
                                                  G.synd + shot * C.mw, E, S, SH0, SH1, EH, nullptr, stage, lane, 0,
                                                  lane, 64, 0, 1, nullptr, it);
    batch_outputs<false>(C, G.prm, shot, conv, it, EH, stage, G.corr, G.flags, G.iters, G.counters, G.fail_list,
                         G.fail_llr, G.n_shots, lane, lane, 64, nullptr);
    wave_sync();
}

template <class TB>
__global__ __launch_bounds__(1024) void bp_multi_kernel(MultiArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned char *base = smem + (size_t)wv * a.wave_bytes;
    float *stage = a.stage + (size_t)(blockIdx.x * (blockDim.x >> 6) + wv) * (size_t)a.stage_stride;
    for (;;) {
        uint32_t it0 = 0;
        if (lane == 0) it0 = atomicAdd(a.counter, 1u);
        const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane(it0);
        if (item >= a.n_work) break;
        int g = 0;
        while (g + 1 < a.n_groups && item >= a.groups[g + 1].first_item) ++g;
        const GroupDesc &G = a.groups[g];
        const int64_t shot = item - G.first_item;
        switch (G.msg) {
        case MSG_INT8: multi_shot<MSG_INT8, TB>(G, shot, base, stage, lane); break;
        case MSG_FP16: multi_shot<MSG_FP16, TB>(G, shot, base, stage, lane); break;
        default: multi_shot<MSG_FP32, TB>(G, shot, base, stage, lane); break;
        }
    }
}

__global__ void reset_kernel(uint32_t *c, int count) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) c[i] = 0u;
}

__global__ void fill_i32_kernel(int32_t *b, int32_t v, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) b[i] = v;
}

__global__ void gather_list_kernel(const uint32_t *counters, const int32_t *fail_list, int64_t from, int32_t *out,
                                   int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = fail_list[from + i];
    (void)counters;
}

}  // namespace

int bp_wave_bytes(int msg, int m, int n) {
    size_t esz = msg == MSG_INT8 ? 1 : (msg == MSG_FP16 ? 2 : 4);
    size_t off = ((size_t)m * DEG * esz + 15) & ~(size_t)15;
    size_t mw = (size_t)(m + 31) / 32;
    size_t eh = 2 * (size_t)((n + 63) / 64);
    size_t tot = off + 4 * (3 * mw + eh);
    return (int)((tot + 15) & ~(size_t)15);
}

hipError_t launch_reset(uint32_t *counters, int count, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3((count + 255) / 256), dim3(256), 0, s, counters, count);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *buf, int32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, buf, value, count);
    return hipGetLastError();
}

hipError_t launch_gather_list(const uint32_t *counters, const int32_t *fail_list, int64_t from, int32_t *out,
                              int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_list_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, counters,
                       fail_list, from, out, count);
    return hipGetLastError();
}

template <int MSG, class TB, bool GRP>
static hipError_t launch_t(const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    size_t lds = GRP ? (size_t)a.wave_bytes : (size_t)a.wave_bytes * wpb;
    hipError_t e = hipFuncSetAttribute((const void *)bp_kernel<MSG, TB, GRP>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bp_kernel<MSG, TB, GRP>), dim3(blocks), dim3(64 * wpb), lds, s, a);
    return hipGetLastError();
}

template <class TB, bool GRP>
static hipError_t launch_tb(int msg, const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    switch (msg) {
    case MSG_INT8: return launch_t<MSG_INT8, TB, GRP>(a, blocks, wpb, s);
    case MSG_FP16: return launch_t<MSG_FP16, TB, GRP>(a, blocks, wpb, s);
    default: return launch_t<MSG_FP32, TB, GRP>(a, blocks, wpb, s);
    }
}

hipError_t launch_bp(int msg, const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    if (a.group)
        return a.code.vn_tab4 ? launch_tb<ColTab32, true>(msg, a, blocks, wpb, s)
                              : launch_tb<ColTab16, true>(msg, a, blocks, wpb, s);
    return a.code.vn_tab4 ? launch_tb<ColTab32, false>(msg, a, blocks, wpb, s)
                          : launch_tb<ColTab16, false>(msg, a, blocks, wpb, s);
}

hipError_t launch_bp_multi(const MultiArgs &a, int blocks, int wpb, hipStream_t s) {
    const size_t lds = (size_t)a.wave_bytes * wpb;
    hipLaunchKernelGGL(bp_multi_kernel<ColTab16>, dim3(blocks), dim3(64 * wpb), lds, s, a);
    return hipGetLastError();
}

hipError_t bp_multi_prepare(int lds_bytes) {
    return hipFuncSetAttribute((const void *)bp_multi_kernel<ColTab16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               lds_bytes);
}

hipError_t bp_multi_max_blocks_per_cu(int wpb, int lds, int *out) {
    hipError_t e = bp_multi_prepare(lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bp_multi_kernel<ColTab16>, 64 * wpb, (size_t)lds);
}

template <int MSG, class TB, bool GRP>
static hipError_t occ_t(int wpb, int lds, int *out) {
    hipError_t e =
        hipFuncSetAttribute((const void *)bp_kernel<MSG, TB, GRP>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bp_kernel<MSG, TB, GRP>, 64 * wpb, (size_t)lds);
}

template <class TB, bool GRP>
static hipError_t occ_tb(int msg, int wpb, int lds, int *out) {
    switch (msg) {
    case MSG_INT8: return occ_t<MSG_INT8, TB, GRP>(wpb, lds, out);
    case MSG_FP16: return occ_t<MSG_FP16, TB, GRP>(wpb, lds, out);
    default: return occ_t<MSG_FP32, TB, GRP>(wpb, lds, out);
    }
}

hipError_t bp_max_blocks_per_cu(int msg, bool wide, bool group, int wpb, int lds, int *out) {
    if (group) return wide ? occ_tb<ColTab32, true>(msg, wpb, lds, out) : occ_tb<ColTab16, true>(msg, wpb, lds, out);
    return wide ? occ_tb<ColTab32, false>(msg, wpb, lds, out) : occ_tb<ColTab16, false>(msg, wpb, lds, out);
}

}  // namespace lbp
