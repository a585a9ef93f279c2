// Int3.4 Lottery BP for codes with at most 64*16 checks: one wavefront per
// shot, check-centric, two edges per VALU instruction.
//
// Per shot the wave keeps
//   * beta (C2V, int8) of every edge in VGPRs: lane L owns checks L + 64*s,
//     s < SLOTS, and holds their 8 padded slots packed in two u32 per check;
//   * lambda of every column in its LDS slice as one u32 per column holding
//     two biased 16-bit values (value + 2^15): the lambda of the previous
//     iteration ("current") and the sum being built for this one ("next").
//     The halves swap roles every iteration.  |lambda| <= 5*127 keeps every
//     partial sum inside its half, so halves never carry into each other.
// Int3.4 arithmetic is exact, so lambda^(i) = mu + sum of beta^(i) is built
// with integer LDS atomic adds into the next half (order-independent): one
// fused pass per check gathers lambda^(i-1) from the current halves, forms
// alpha = lambda - beta_old (== mu + the other C2V messages), runs
// min1/min2/argmin/sign parity, keeps the new beta in VGPRs and adds it to
// the next halves.  A second pass over columns takes the hard decision (ballot
// into the correction words), forms the syndrome estimate by LDS atomic XOR
// (only columns with e = 1) and resets the consumed half to mu.  There is no
// variable-node gather.
//
// The check pass works on pairs of edges in packed 16-bit registers (the
// v_pk_* integer instructions): the two lambda values of a pair are gathered
// into the two halves of a register, and the int8 beta of four edges is
// unpacked into two pairs with one byte-permute each, whose selectors also
// sign-extend.  Each check's slots are paired (1,3), (0,2), (5,7), (4,6).
//
// Padding slots point at pad columns (after column n-1) whose current half is
// reset to 254 each iteration: alpha >= +127 there, saturated to the format's
// maximum, a key that never wins a minimum (and the magnitude a degree-1 check
// sends).  Pads are spread over PAD_COLS columns so that their sums cannot
// leave a 16-bit half either.
//
// The lottery (Algorithm 3) runs after the column pass with U from the
// previous syndrome estimate and lambda^(i) read from LDS; the flip acts on
// the next iteration's alpha (message flip) or on lambda_v* (LLR flip), inside
// a wave-uniform branch taken only by the slots that hold a check of v*.
#include <climits>
#include <vector>

#include "device_util.h"
#include "lbp_internal.h"

namespace lbp {
namespace {

constexpr int BIAS = 32768;
constexpr int PAD_LAMBDA = 254;
constexpr int PAD_COLS = 48;

// LDS bytes of the column-offset table ahead of the waves' slices (see row_offsets).
__host__ __device__ inline int bp_int8_table_bytes_t(int table, int slots, int m0) {
    return table == 0 ? slots * 64 * 16 : table == 1 ? (2 * m0 + 1) * 32 : 0;
}

typedef short v2i16 __attribute__((ext_vector_type(2)));
typedef unsigned short v2u16 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v2i16 as_i16(uint32_t x) { return __builtin_bit_cast(v2i16, x); }
__device__ __forceinline__ v2u16 as_u16(uint32_t x) { return __builtin_bit_cast(v2u16, x); }
__device__ __forceinline__ uint32_t as_u32(v2i16 x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t as_u32(v2u16 x) { return __builtin_bit_cast(uint32_t, x); }

// lambda^(i) of column v: the half that received this iteration's sum.
__device__ __forceinline__ int lambda_next(const uint32_t *L, int v, int nxt_hi) {
    const uint32_t w = L[v];
    return (int)(nxt_hi ? (w >> 16) : (w & 0xFFFFu)) - BIAS;
}

// Worst check of U (Sec. III-B): the most neighbours in the current hard
// decision (lambda^(i) <= 0, read from the half nxt_hi), the smallest index
// among equals.  One check per lane, wave-wide maximum.
__device__ int worst_check(const DevCode &C, const uint32_t *S, const uint32_t *SHp, const uint32_t *L, int nxt_hi,
                           int lane) {
    unsigned long long best = 0;
    for (int c0 = 0; c0 < C.m; c0 += 64) {
        const int c = c0 + lane;
        if (c < C.m && (((SHp[c >> 5] ^ S[c >> 5]) >> (c & 31)) & 1u)) {
            int cnt = 0;
            const int deg = C.cn_deg[c];
            for (int k = 0; k < deg; ++k) {
                const uint32_t v = C.cn_cols[c * DEG + k];
                cnt += lambda_next(L, (int)v, nxt_hi) <= 0;
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

// Lottery selection (Algorithm 3), U from the previous syndrome estimate SHp,
// under the design-space rule `rule` (CN rule | VN rule << 4, Sec. III-B):
// random or worst check; proposed key (count, Q, column), Q-first (Q, count,
// column), unreliable (Q, column) or a random neighbour.  Q = |lambda|.
__device__ int lottery_pick_q(const DevCode &C, int rule, uint64_t seed, uint64_t shot_id, int i, const uint32_t *L,
                              int nxt_hi, const uint32_t *S, const uint32_t *SHp, int lane) {
    int N = 0;
    for (int w0 = 0; w0 < C.mw; w0 += 64) {
        int w = w0 + lane;
        N += wave_sum(__popc(w < C.mw ? (SHp[w] ^ S[w]) : 0u));
    }
    if (N == 0) return -1;
    const int cn_rule = rule & 3, vn_rule = (rule >> 4) & 3;
    uint64_t x1;
    const uint64_t x = philox_word01(seed, shot_id, (uint64_t)i, x1);
    int cstar = 0;
    if (cn_rule == LOT_CN_WORST) {
        cstar = __builtin_amdgcn_readfirstlane(worst_check(C, S, SHp, L, nxt_hi, lane));
    } else {
        uint32_t k = (uint32_t)(((x >> 32) * (uint64_t)N) >> 32);
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
                cstar = __builtin_amdgcn_readlane(pos, __ffsll((unsigned long long)__ballot(here)) - 1);
                break;
            }
            k -= (uint32_t)tot;
        }
    }
    if (vn_rule == LOT_VN_RANDOM) {
        const uint32_t k = (uint32_t)(((x1 >> 32) * (uint64_t)C.cn_deg[cstar]) >> 32);
        return C.cn_cols[cstar * DEG + (int)k];
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
            int l = lambda_next(L, v, nxt_hi);
            q = l < 0 ? -l : l;
        }
    }
    int bc = -1, bq = 0, bv = -1;
#pragma unroll
    for (int kk = 0; kk < DEG; ++kk) {
        int ck = __builtin_amdgcn_readlane(cnt, kk), vk = __builtin_amdgcn_readlane(v, kk),
            qk = __builtin_amdgcn_readlane(q, kk);
        if (ck < 0) continue;
        if (bv < 0 || lottery_key_less(vn_rule, ck, qk, vk, bc, bq, bv)) {
            bc = ck;
            bq = qk;
            bv = vk;
        }
    }
    return bv;
}

// Byte-permute selectors (byte i of the result = byte sel_i of {src0, src1},
// src1 the low word; 8 / 10 = sign of byte 1 of src1 / src0, 9 / 11 = of byte 3):
// (b1, b3) and (b0, b2) of a word of four int8, sign-extended to int16 pairs,
// and the inverse (pairs back to four bytes).
constexpr uint32_t SEL_13 = 0x09030801u;    // src1 = w: b1, sign(b1), b3, sign(b3)
constexpr uint32_t SEL_02 = 0x0B020A00u;    // src0 = w << 8, src1 = w: b0, sign(b0), b2, sign(b2)
constexpr uint32_t SEL_PACK = 0x06020400u;  // src0 = (b1, b3), src1 = (b0, b2) -> b0 b1 b2 b3

// One check of the check pass on its four slot pairs.  PAR: which half holds
// the current lambda (0: low, 1: high); the sum for this iteration goes to the
// other half.  FLIP: the wave-uniform flip path (fo = v*'s offset in both halves).
template <int PAR, bool FLIP, bool LLR_FLIP>
__device__ __forceinline__ void check_update(const uint4 cw, uint32_t &bw0, uint32_t &bw1, uint32_t syn_bit,
                                             unsigned char *Lb, uint32_t base, v2u16 kmul, v2u16 shv, uint32_t fo,
                                             uint32_t qm2) {
    const uint32_t T[4] = {cw.x, cw.y, cw.z, cw.w};  // (off1,off3) (off0,off2) (off5,off7) (off4,off6)
    // ---- gather lambda^(i-1) of the eight columns into four pairs
    uint32_t lam[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t a0 = base + (T[p] & 0xFFFFu), a1 = base + (T[p] >> 16);
        const uint32_t l0 = *(const uint16_t *)(Lb + a0 + 2 * PAR);
        const uint32_t l1 = *(const uint16_t *)(Lb + a1 + 2 * PAR);
        lam[p] = l0 | (l1 << 16);
    }
    // ---- beta_old pairs
    const uint32_t b[4] = {__builtin_amdgcn_perm(bw0, bw0, SEL_13), __builtin_amdgcn_perm(bw0 << 8, bw0, SEL_02),
                           __builtin_amdgcn_perm(bw1, bw1, SEL_13), __builtin_amdgcn_perm(bw1 << 8, bw1, SEL_02)};
    // ---- alpha, keys, min1/min2 per half, sign parity (stage by stage over the
    // four pairs, so that dependent packed instructions are never adjacent)
    v2i16 l[4], x[4], mg[4];
    v2u16 key[4];
    const v2u16 kslot[4] = {{1, 3}, {0, 2}, {5, 7}, {4, 6}};
#pragma unroll
    for (int p = 0; p < 4; ++p) l[p] = as_i16(lam[p] ^ 0x80008000u);  // biased -> signed lambda
    if constexpr (FLIP) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            // per half: d == 0 exactly where the slot names v*; (d | -d) has its top bit clear only there
            const v2u16 d = as_u16(T[p]) - as_u16(fo);
            const v2u16 nz = (d | ((v2u16){0, 0} - d)) >> (v2u16){15, 15};
            const v2i16 fm = as_i16(as_u32(nz - (v2u16){1, 1}));  // -1 in the halves naming v*
            if constexpr (LLR_FLIP) l[p] = (l[p] ^ fm) - fm;  // lambda_v* negated
            x[p] = l[p] - as_i16(b[p]);
            if constexpr (!LLR_FLIP) x[p] = (x[p] ^ fm) - fm;  // messages of v* negated
        }
    } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) x[p] = l[p] - as_i16(b[p]);
    }
    // |alpha| saturated at qmax, both halves of qm2 (the sign of alpha is the sign of its saturated value)
#pragma unroll
    for (int p = 0; p < 4; ++p) mg[p] = (v2i16){0, 0} - x[p];
#pragma unroll
    for (int p = 0; p < 4; ++p) mg[p] = __builtin_elementwise_max(x[p], mg[p]);
#pragma unroll
    for (int p = 0; p < 4; ++p) mg[p] = __builtin_elementwise_min(mg[p], as_i16(qm2));
    // |alpha| << 3 | slot as one packed multiply-add (the factor is hidden from the
    // optimiser, which would otherwise turn it back into a shift and an or)
    v2u16 eight = {8, 8};
    asm("" : "+v"(eight));
#pragma unroll
    for (int p = 0; p < 4; ++p) key[p] = as_u16(as_u32(mg[p])) * eight + kslot[p];
    const uint32_t px = as_u32(x[0]) ^ as_u32(x[1]) ^ as_u32(x[2]) ^ as_u32(x[3]);
    v2u16 m1 = __builtin_elementwise_min(key[0], key[1]);
    v2u16 m2 = __builtin_elementwise_max(key[0], key[1]);
    const v2u16 m1b = __builtin_elementwise_min(key[2], key[3]);
    const v2u16 m2b = __builtin_elementwise_max(key[2], key[3]);
    m2 = __builtin_elementwise_min(__builtin_elementwise_max(m1, m1b), __builtin_elementwise_min(m2, m2b));
    m1 = __builtin_elementwise_min(m1, m1b);
    // merge the two halves: minimum and second minimum over all eight keys
    const uint32_t m1a = m1.x, m1c = m1.y, m2a = m2.x, m2c = m2.y;
    const uint32_t k1 = m1a < m1c ? m1a : m1c;
    const uint32_t hi1 = m1a < m1c ? m1c : m1a;
    const uint32_t m2m = m2a < m2c ? m2a : m2c;
    const uint32_t k2 = hi1 < m2m ? hi1 : m2m;
    const uint32_t par = (((px ^ (px >> 16)) >> 15) & 1u) ^ syn_bit;
    // the scale on both magnitudes g = key >> 3 at once: s = ((K g) >> 3) - (g >> SH), with
    // (K, SH) = (8, min(i+1, 15)) for sigma_i (g - (g >> (i+1)); g < 2^7, so SH = 15 covers
    // every i >= 14) and (k, 15) for a constant k/8 ((k g) >> 3)
    const v2u16 gg = (v2u16){(unsigned short)k1, (unsigned short)k2} >> (v2u16){3, 3};
    const v2u16 ss = ((gg * kmul) >> (v2u16){3, 3}) - (gg >> shv);
    const v2u16 s11 = __builtin_shufflevector(ss, ss, 0, 0), s22 = __builtin_shufflevector(ss, ss, 1, 1);
    const v2u16 k1p = {(unsigned short)(k1 + 1), (unsigned short)(k1 + 1)};
    const uint32_t s1p = as_u32(s11);
    const uint32_t dxp = as_u32(s11 ^ s22);
    const uint32_t pp = par ? 0x80008000u : 0u;
    uint32_t nb[4];
    v2i16 eq[4], sm[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) eq[p] = as_i16(as_u32(key[p] - k1p));  // per half: negative only at the argmin
#pragma unroll
    for (int p = 0; p < 4; ++p) eq[p] = eq[p] >> (v2i16){15, 15};                 // -1 at the argmin slot
#pragma unroll
    for (int p = 0; p < 4; ++p) sm[p] = as_i16(as_u32(x[p]) ^ pp) >> (v2i16){15, 15};  // -1 where beta < 0
    // opaque masks: knowing each half is 0 or -1, the optimiser would rewrite the
    // bitwise selects below as per-half compares and selects (five times the work)
#pragma unroll
    for (int p = 0; p < 4; ++p) asm("" : "+v"(eq[p]), "+v"(sm[p]));
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t mag = s1p ^ (dxp & as_u32(eq[p]));  // s2 at the argmin, s1 elsewhere
        nb[p] = as_u32((as_i16(mag) ^ sm[p]) - sm[p]);
    }
    // ---- add the new beta to the other half of each column word
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t a0 = base + (T[p] & 0xFFFFu), a1 = base + (T[p] >> 16);
        uint32_t v0, v1;
        if constexpr (PAR == 0) {  // the sum goes to the high halves
            v0 = nb[p] << 16;
            v1 = nb[p] & 0xFFFF0000u;
        } else {                   // the sum goes to the low halves (sign-extended: no borrow leaves the half)
            v0 = (uint32_t)(((int32_t)(nb[p] << 16)) >> 16);
            v1 = (uint32_t)(((int32_t)nb[p]) >> 16);
        }
        __hip_atomic_fetch_add((uint32_t *)(Lb + a0), v0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add((uint32_t *)(Lb + a1), v1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    bw0 = __builtin_amdgcn_perm(nb[0], nb[1], SEL_PACK);
    bw1 = __builtin_amdgcn_perm(nb[2], nb[3], SEL_PACK);
}

// Where the column offsets of a check come from (template TABLE):
//   0: a per-check table, cidx4[s*64 + lane] = the four offset pairs of check lane + 64 s;
//   1 / 2: the space-time structure of Eq. 1, H = [I_r (x) H0 | D (x) I_m0]: check
//      c = t m0 + s0 (t = c / m0) reads row s0 (t = 0), m0 + s0 (t >= 1) or 2 m0 (the
//      padding checks c >= m) of a compact table whose rows hold offset pairs b and
//      multiplier pairs k (4 n0 for data slots, 4 m0 for measurement slots, 0 for
//      padding); the check's offsets are b + t k, two slots per packed instruction.
//      The compact table lives in LDS (1) or is read from global memory (2).
struct StShape {
    uint32_t m0, r, magic;  // magic = floor(2^32 / m0) + 1: c / m0 = umulhi(c, magic) for c < 2^16
};

template <int TABLE>
__device__ __forceinline__ uint4 row_offsets(const uint4 *tab, int s, int lane, const StShape &st) {
    if constexpr (TABLE == 0) {
        return tab[s * 64 + lane];
    } else {
        uint32_t c = (uint32_t)(lane + 64 * s);
        // opaque: the offsets depend on the lane and slot only, and hoisted out of the
        // iteration loop all slots' offsets are held (spilled) across it
        if constexpr (TABLE != 0) asm volatile("" : "+v"(c));
        const uint32_t t = __umulhi(c, st.magic);
        const uint32_t s0 = c - t * st.m0;
        const uint32_t row = t == 0 ? s0 : (t < st.r ? st.m0 + s0 : 2 * st.m0);
        const uint4 b = tab[2 * row], k = tab[2 * row + 1];
        const v2u16 tt = {(unsigned short)t, (unsigned short)t};
        uint4 o;
        o.x = as_u32(as_u16(b.x) + as_u16(k.x) * tt);
        o.y = as_u32(as_u16(b.y) + as_u16(k.y) * tt);
        o.z = as_u32(as_u16(b.z) + as_u16(k.z) * tt);
        o.w = as_u32(as_u16(b.w) + as_u16(k.w) * tt);
        return o;
    }
}

// The check pass of one iteration over all of the lane's checks.  flipslots (bit s:
// slot s holds a check of v*) is wave-uniform, so the flip variant is a scalar branch.
// ANY_FLIP: some slot holds a check of v* this iteration (the lottery's flip acts);
// the pass without any flip, by far the common one, then has no per-slot branch.
template <int SLOTS, int PAR, bool LLR_FLIP, int TABLE, bool ANY_FLIP>
__device__ __forceinline__ void check_pass(const uint4 *tab, const StShape &st, uint32_t (&bq)[SLOTS][2],
                                           uint32_t srow, unsigned char *Lb, uint32_t base, int lane, v2u16 kmul,
                                           v2u16 shv, uint32_t flipslots, uint32_t fo, uint32_t qm2) {
    const uint32_t fs = __builtin_amdgcn_readfirstlane(flipslots);
    // opaque: otherwise the per-slot bits are hoisted out of the iteration loop and
    // held (and spilled) as SLOTS registers across it (with the global-memory table
    // the allocation without this is the better one)
    uint32_t sr = srow;
    if constexpr (TABLE != 2) asm volatile("" : "+v"(sr));
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const uint4 cw = row_offsets<TABLE>(tab, s, lane, st);
        const uint32_t sb = (sr >> s) & 1u;
        if (ANY_FLIP && (fs & (1u << s)))
            check_update<PAR, true, LLR_FLIP>(cw, bq[s][0], bq[s][1], sb, Lb, base, kmul, shv, fo, qm2);
        else
            check_update<PAR, false, LLR_FLIP>(cw, bq[s][0], bq[s][1], sb, Lb, base, kmul, shv, fo, qm2);
        // opaque to the optimiser: otherwise it forwards unpacked values to the next
        // iteration and keeps several registers per check
        asm volatile("" : "+v"(bq[s][0]), "+v"(bq[s][1]));
    }
}

// Syndrome estimate contribution of a column whose hard decision is 1: flip the
// bit of each of its checks (order-independent LDS atomics).
__device__ __forceinline__ void xor_checks(const DevCode &C, int v, uint32_t *SHc) {
    const uint64_t tab = C.vn_tab[v];
#pragma unroll
    for (int j = 0; j < CDEG; ++j) {
        const uint32_t p = (uint32_t)(tab >> (16 * j)) & 0xFFFFu;
        if (p != NOPOS) {
            const uint32_t c = p / DEG;
            atomicXor(&SHc[c >> 5], 1u << (c & 31));
        }
    }
}

// Column pass of an iteration whose sums went to half 1 - PAR: hard decision of
// lambda^(i) (e = [lambda <= 0], i.e. biased half <= BIAS), syndrome estimate by
// LDS atomic XOR of the columns with e = 1, and reset of the consumed half PAR to
// mu (the accumulation base of iteration i+1).  Corrections and lambda leave the
// wave once per shot, after the last iteration.
template <int PAR, bool MU_UNIFORM>
__device__ __forceinline__ void column_pass(const DevCode &C, uint32_t *L, uint32_t *SHc, int n, int lane,
                                            uint32_t mu_b) {
    uint16_t *Lh = (uint16_t *)L;
    const int nfull = n >> 6;
    if (nfull < 64) {
        // first the hard decisions (bit vs: column 64 vs + lane has e = 1), then the
        // column-table loads of those columns, one per lane at a time: a wave waits
        // for about one table load per iteration instead of one per group with an e = 1
        uint64_t emask = 0;
#pragma unroll 2
        for (int vs = 0; vs < nfull; ++vs) {
            const int v = vs * 64 + lane;
            const uint32_t w = L[v];
            const uint32_t h = PAR == 0 ? (w >> 16) : (w & 0xFFFFu);
            emask |= (uint64_t)(h <= (uint32_t)BIAS) << vs;
            Lh[2 * v + PAR] = (uint16_t)(MU_UNIFORM ? mu_b : (uint32_t)(C.mu_q[v] + BIAS));
        }
        const int v = nfull * 64 + lane;
        if (v < n) {
            const uint32_t w = L[v];
            const uint32_t h = PAR == 0 ? (w >> 16) : (w & 0xFFFFu);
            emask |= (uint64_t)(h <= (uint32_t)BIAS) << nfull;
            Lh[2 * v + PAR] = (uint16_t)(MU_UNIFORM ? mu_b : (uint32_t)(C.mu_q[v] + BIAS));
        }
        while (__ballot(emask != 0ull)) {
            if (emask) {
                const int vs = __ffsll((unsigned long long)emask) - 1;
                emask &= emask - 1ull;
                xor_checks(C, vs * 64 + lane, SHc);
            }
        }
        return;
    }
#pragma unroll 2
    for (int vs = 0; vs < nfull; ++vs) {
        const int v = vs * 64 + lane;
        const uint32_t w = L[v];
        const uint32_t h = PAR == 0 ? (w >> 16) : (w & 0xFFFFu);
        if (h <= (uint32_t)BIAS) xor_checks(C, v, SHc);
        Lh[2 * v + PAR] = (uint16_t)(MU_UNIFORM ? mu_b : (uint32_t)(C.mu_q[v] + BIAS));
    }
    const int v = nfull * 64 + lane;
    if (v < n) {
        const uint32_t w = L[v];
        const uint32_t h = PAR == 0 ? (w >> 16) : (w & 0xFFFFu);
        if (h <= (uint32_t)BIAS) xor_checks(C, v, SHc);
        Lh[2 * v + PAR] = (uint16_t)(MU_UNIFORM ? mu_b : (uint32_t)(C.mu_q[v] + BIAS));
    }
}

// SERVE: the serving variant (work from a ring, a.ring non-null).  Batch and
// serving decodes are separate instantiations so that the ring's claim code does
// not take part in the batch kernel's register allocation, which sits at the
// 128-VGPR limit.
template <int SLOTS, bool LLR_FLIP, int TABLE, bool SERVE>
__global__ __launch_bounds__(1024) void bp_int8_kernel(BpArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ ClaimLds claim;  // serving: the block's ring lock and its waves' claimed items
    const DevCode &C = a.code;
    const BpParams &P = a.prm;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    claim.clear(threadIdx.x);
    if (!SERVE && threadIdx.x == 0) atomicAdd(&a.counters[3], 1u);  // resident BP blocks, for OSD alongside
    const int n = C.n, m = C.m;
    // column offsets of the checks (TABLE 0: per check; 1: compact space-time rows in
    // LDS; 2: compact rows read from global memory), ahead of the waves' slices
    const int table_bytes = bp_int8_table_bytes_t(TABLE, SLOTS, C.st_m0);
    if constexpr (TABLE == 0) {
        // byte offsets (4 * column) of every padded slot, paired as
        // cidx4[s*64 + lane] = {(o1,o3), (o0,o2), (o5,o7), (o4,o6)} of check lane + 64 s
        uint32_t *cidx = (uint32_t *)smem;
        for (int t = threadIdx.x; t < SLOTS * 64 * 4; t += blockDim.x) {
            const int c = t >> 2, w = t & 3;
            const int k0 = (w & 2) * 2 + ((w & 1) ? 0 : 1);  // slot of the low half: 1, 0, 5, 4
            uint32_t off[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = k0 + 2 * h;
                uint32_t v = c < m ? C.cn_cols[c * DEG + k] : NOPOS;
                if (v == NOPOS) v = (uint32_t)n + (uint32_t)((c * DEG + k) % PAD_COLS);
                off[h] = 4u * v;
            }
            cidx[t] = off[0] | (off[1] << 16);
        }
    } else if constexpr (TABLE == 1) {
        for (int t = threadIdx.x; t < table_bytes / 4; t += blockDim.x) ((uint32_t *)smem)[t] = C.st_tab[t];
    }
    __syncthreads();
    const uint4 *tab = TABLE == 2 ? (const uint4 *)C.st_tab : (const uint4 *)smem;
    StShape st{(uint32_t)C.st_m0, (uint32_t)C.st_r, C.st_m0 ? (uint32_t)(0xFFFFFFFFull / (uint32_t)C.st_m0) + 1u : 0u};
    unsigned char *base_p = smem + (size_t)table_bytes + (size_t)wv * a.wave_bytes;
    uint32_t *L = (uint32_t *)base_p;  // [n + PAD_COLS] column words
    unsigned char *Lb = smem;
    const uint32_t base = (uint32_t)(base_p - smem);
    const int nl = n + PAD_COLS;
    uint32_t *S = (uint32_t *)(base_p + (((size_t)nl * 4 + 15) & ~(size_t)15));
    uint32_t *SH0 = S + C.mw, *SH1 = SH0 + C.mw;
    const uint32_t last_mask = (m & 31) ? ((1u << (m & 31)) - 1u) : ~0u;
    const int nvs = (n + 63) >> 6;
    const bool mu_uniform = C.mu_q_uniform != INT32_MIN;
    const uint32_t mu_b = (uint32_t)((mu_uniform ? C.mu_q_uniform : 0) + BIAS);
    const uint32_t pad_b = (uint32_t)(PAD_LAMBDA + BIAS);
    const uint32_t qm2 = (uint32_t)P.qmax | ((uint32_t)P.qmax << 16);  // Int x.y saturation, both halves
    // check-node scale: (K, SH) of check_update, both halves
    const unsigned short kscale = P.scale_mode == 1 ? (unsigned short)P.scale_k : (unsigned short)8;
    const v2u16 kmul = {kscale, kscale};

    for (;;) {
        int64_t item = 0;
        if constexpr (SERVE) {
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
        const int64_t shot = SERVE ? (item & a.ring->mask) : a.work_list ? (int64_t)a.work_list[item] : item;
        const uint64_t *keys = SERVE ? a.ring->keys : a.shot_keys;
        // wave-uniform: the lottery's Philox rounds then run on the scalar unit
        const uint64_t seed = (uint64_t)uniform64((int64_t)(keys ? keys[2 * shot] : P.seed));
        const uint64_t shot_id =
            (uint64_t)uniform64((int64_t)(keys ? keys[2 * shot + 1] : a.first_shot_id + (uint64_t)shot));
        const uint32_t *syn_row = (SERVE ? a.ring->syn : a.synd) + shot * C.mw;

        // SH1 is the estimate "before iteration 0" that the lottery of iteration 0
        // reads when K = 0: the hard decision of the prior, H * 0 = 0
        for (int w = lane; w < C.mw; w += 64) {
            uint32_t x = syn_row[w];
            S[w] = w == C.mw - 1 ? (x & last_mask) : x;
            SH1[w] = 0u;
        }
        // lambda^(-1) = mu in both halves (Algorithm 1 initialisation: alpha^(0) = mu)
        for (int v = lane; v < nl; v += 64) {
            const uint32_t mb = v < n ? (mu_uniform ? mu_b : (uint32_t)(C.mu_q[v] + BIAS)) : pad_b;
            L[v] = mb | (mb << 16);
        }
        wave_sync();
        uint32_t bq[SLOTS][2];  // beta of the previous iteration, int8, slots 0-3 and 4-7
#pragma unroll
        for (int s = 0; s < SLOTS; ++s) bq[s][0] = bq[s][1] = 0u;
        // bit s: measured syndrome of check lane + 64 s (S is zero beyond m)
        uint32_t srow = 0;
#pragma unroll 1
        for (int s = 0; s < (m + 63) / 64; ++s) {
            const int w = 2 * s + (lane >> 5);
            if (w < C.mw) srow |= ((S[w] >> (lane & 31)) & 1u) << s;
        }

        int it = 0;
        bool converged = false;
        uint32_t flipslots = 0, fo = 0;
        for (int i = 0; i < P.max_iter; ++i) {
            uint32_t *SHc = (i & 1) ? SH1 : SH0;
            uint32_t *SHp = (i & 1) ? SH0 : SH1;
            const int par = i & 1;  // half holding lambda^(i-1)
            const unsigned short sh = P.scale_mode == 1 ? (unsigned short)15 : (unsigned short)(i + 1 > 15 ? 15 : i + 1);
            const v2u16 shv = {sh, sh};
            // ---- check-node pass: alpha from lambda^(i-1), beta^(i), lambda^(i) += beta^(i)
            if (flipslots == 0) {
                if (par == 0)
                    check_pass<SLOTS, 0, LLR_FLIP, TABLE, false>(tab, st, bq, srow, Lb, base, lane, kmul, shv, 0u, fo, qm2);
                else
                    check_pass<SLOTS, 1, LLR_FLIP, TABLE, false>(tab, st, bq, srow, Lb, base, lane, kmul, shv, 0u, fo, qm2);
            } else {
                if (par == 0)
                    check_pass<SLOTS, 0, LLR_FLIP, TABLE, true>(tab, st, bq, srow, Lb, base, lane, kmul, shv, flipslots,
                                                                fo, qm2);
                else
                    check_pass<SLOTS, 1, LLR_FLIP, TABLE, true>(tab, st, bq, srow, Lb, base, lane, kmul, shv, flipslots,
                                                                fo, qm2);
            }
            for (int w = lane; w < C.mw; w += 64) SHc[w] = 0u;
            wave_sync();
            // ---- column pass: hard decision, syndrome estimate, reset of the consumed half
            if (mu_uniform) {
                if (par == 0) column_pass<0, true>(C, L, SHc, n, lane, mu_b);
                else column_pass<1, true>(C, L, SHc, n, lane, mu_b);
            } else {
                if (par == 0) column_pass<0, false>(C, L, SHc, n, lane, mu_b);
                else column_pass<1, false>(C, L, SHc, n, lane, mu_b);
            }
            // pads: re-arm the half that just collected this iteration's pad sums (it is
            // read next iteration); the other half collects the next sums from 254
            if (lane < PAD_COLS) ((uint16_t *)L)[2 * (n + lane) + (par ^ 1)] = (uint16_t)pad_b;
            wave_sync();
            bool mism = false;
            for (int w = lane; w < C.mw; w += 64) mism |= SHc[w] != S[w];
            it = i + 1;
            if (__ballot(mism) == 0ull) {
                converged = true;
                break;
            }
            flipslots = 0;
            if (P.lottery && i >= P.skip && i <= P.max_iter - 2) {
                const int nxt_hi = par == 0;
                const int fv = lottery_pick_q(C, P.rule, seed, shot_id, i, L, nxt_hi, S, SHp, lane);
                if (fv >= 0) {
                    // slots holding a check of v*: its column table names them
                    const uint64_t tab = C.vn_tab[__builtin_amdgcn_readfirstlane(fv)];
#pragma unroll
                    for (int j = 0; j < CDEG; ++j) {
                        const uint32_t p = (uint32_t)(tab >> (16 * j)) & 0xFFFFu;
                        if (p != NOPOS) flipslots |= 1u << ((p / DEG) >> 6);
                    }
                    flipslots = __builtin_amdgcn_readfirstlane(flipslots);
                    fo = 4u * (uint32_t)fv;
                    fo = fo | (fo << 16);
                }
            }
            wave_sync();
        }

        // ---- once per shot: corrections (hard decision of the last lambda), the
        // lambda outputs, and for a failed shot its lambda for OSD as int16
        const int fin_hi = ((it - 1) & 1) == 0;  // half holding lambda of the last iteration
        const bool osd = !converged && P.osd != OSD_NONE;
        uint32_t fail_q = 0;  // the failed shot's list position
        uint32_t *corr_row;
        int16_t *lam_dst = nullptr;
        if constexpr (SERVE) {
            corr_row = a.ring->corr + shot * C.nw;
            if (osd) lam_dst = a.ring->llr16 + shot * n;
        } else {
            corr_row = a.corr + shot * C.nw;
            if (osd) {
                uint32_t q = 0;
                if (lane == 0) q = atomicAdd(&a.counters[1], 1u);
                fail_q = __builtin_amdgcn_readfirstlane(q);
                if ((int64_t)fail_q < a.fail_cap) lam_dst = a.fail_q + (size_t)fail_q * n;
            }
        }
        float *llr_row = a.llr_out ? a.llr_out + shot * n : nullptr;
        for (int vs = 0; vs < nvs; ++vs) {
            const int v = vs * 64 + lane;
            const bool valid = v < n;
            const int l = valid ? lambda_next(L, v, fin_hi) : 1;
            const uint64_t bal = __ballot(l <= 0);
            if (lane < 2 && 2 * vs + lane < C.nw) corr_row[2 * vs + lane] = lane ? (uint32_t)(bal >> 32) : (uint32_t)bal;
            if (valid) {
                if (llr_row) llr_row[v] = (float)l;
                if (lam_dst) lam_dst[v] = (int16_t)l;
            }
        }
        if constexpr (SERVE) {
            const ServeRing &R = *a.ring;
            if (lane == 0) {
                R.flags[shot] = converged ? (uint8_t)FLAG_CONVERGED : osd ? (uint8_t)(FLAG_OSD | FLAG_OSD_PENDING) : 0;
                R.iters[shot] = it;
            }
            serve_publish(R, item, lane);
            wave_sync();
            continue;
        }
        const uint8_t fl = converged ? (uint8_t)FLAG_CONVERGED : (uint8_t)(P.osd != OSD_NONE ? FLAG_OSD : 0);
        if (lane == 0) {
            a.flags[shot] = fl;
            if (a.iters) a.iters[shot] = it;
        }
        if (osd) {
            // publish the list entry after the staged lambda, the correction and the
            // flags: an OSD block running alongside takes the position only then
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0)
                __hip_atomic_store(&a.fail_list[fail_q], (int32_t)shot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        wave_sync();
    }
    if constexpr (!SERVE) {
        __syncthreads();  // every wave of the block is done: count the block finished
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicAdd(&a.counters[4], 1u);
        }
    }
}

}  // namespace

int bp_int8_slots(int m, int n) {
    if ((int64_t)(n + PAD_COLS) * 4 > 65535) return 0;  // column offsets are 16-bit
    const int need = (m + 63) / 64;
    for (int s : {1, 2, 4, 8, 14, 16})
        if (need <= s) return s;
    return 0;
}

int bp_int8_table_bytes(int table, int slots, int m0) { return bp_int8_table_bytes_t(table, slots, m0); }

bool bp_int8_build_st_table(const uint16_t *cols, int m, int n, int r, int m0, int n0, std::vector<uint32_t> &out) {
    const int slots = bp_int8_slots(m, n);
    if (!slots || r < 2 || m != r * m0) return false;
    const int rows = 2 * m0 + 1;
    out.assign((size_t)rows * 8, 0u);
    // slot pairs of the four offset words, as in the per-check table
    const int pair_k[4][2] = {{1, 3}, {0, 2}, {5, 7}, {4, 6}};
    std::vector<int> pad_load(PAD_COLS, 0);
    for (int R = 0; R < rows; ++R) {
        // the check whose columns the row describes: row R < 2 m0 is check R (round 0 for
        // R < m0, round 1 after), row 2 m0 none (padding)
        const int c = R < 2 * m0 ? R : -1;
        const int t = R < m0 ? 0 : 1;
        uint32_t off[DEG], mul[DEG];
        for (int k = 0; k < DEG; ++k) {
            const uint32_t v = c >= 0 ? cols[(size_t)c * DEG + k] : NOPOS;
            if (v == NOPOS) {
                off[k] = 4u * (uint32_t)(n + (R * DEG + k) % PAD_COLS);
                mul[k] = 0;
            } else {
                mul[k] = 4u * (uint32_t)((int)v < r * n0 ? n0 : m0);
                off[k] = 4u * v - (uint32_t)t * mul[k];  // the offset at t = 0 of this row's checks
            }
            if (off[k] > 0xFFFFu || (uint64_t)off[k] + (uint64_t)(r - 1) * mul[k] > 0xFFFFu) return false;
        }
        for (int w = 0; w < 4; ++w) {
            out[(size_t)R * 8 + w] = off[pair_k[w][0]] | (off[pair_k[w][1]] << 16);
            out[(size_t)R * 8 + 4 + w] = mul[pair_k[w][0]] | (mul[pair_k[w][1]] << 16);
        }
    }
    // the padding columns' sums of one iteration must stay inside a 16-bit half:
    // count the padded slots each receives over all 64 * slots check positions
    for (int c = 0; c < 64 * slots; ++c) {
        const int t = c / m0, s0 = c - t * m0;
        const int R = t == 0 ? s0 : (t < r ? m0 + s0 : 2 * m0);
        for (int k = 0; k < DEG; ++k) {
            const uint32_t v = R < 2 * m0 ? cols[(size_t)R * DEG + k] : NOPOS;
            if (v == NOPOS) ++pad_load[(R * DEG + k) % PAD_COLS];
        }
    }
    for (int j = 0; j < PAD_COLS; ++j)
        if (PAD_LAMBDA + 127 * pad_load[j] > 32767) return false;
    return true;
}

int bp_int8_wave_bytes(int m, int n) {
    size_t mw = (size_t)(m + 31) / 32;
    size_t tot = (((size_t)(n + PAD_COLS) * 4 + 15) & ~(size_t)15) + 4 * (3 * mw);  // L, then S, SH0, SH1
    return (int)((tot + 15) & ~(size_t)15);
}

template <int SLOTS, bool LLR_FLIP, int TABLE, bool SERVE>
static hipError_t launch_v(const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    size_t lds = (size_t)bp_int8_table_bytes_t(TABLE, SLOTS, a.code.st_m0) + (size_t)a.wave_bytes * wpb;
    hipError_t e = hipFuncSetAttribute((const void *)bp_int8_kernel<SLOTS, LLR_FLIP, TABLE, SERVE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bp_int8_kernel<SLOTS, LLR_FLIP, TABLE, SERVE>), dim3(blocks), dim3(64 * wpb), lds, s, a);
    return hipGetLastError();
}

template <int SLOTS, bool LLR_FLIP, int TABLE>
static hipError_t launch_q(const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    return a.ring ? launch_v<SLOTS, LLR_FLIP, TABLE, true>(a, blocks, wpb, s)
                  : launch_v<SLOTS, LLR_FLIP, TABLE, false>(a, blocks, wpb, s);
}

template <int SLOTS, int TABLE>
static hipError_t launch_s(const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    return a.prm.flip == FLIP_LLR ? launch_q<SLOTS, true, TABLE>(a, blocks, wpb, s)
                                  : launch_q<SLOTS, false, TABLE>(a, blocks, wpb, s);
}

template <int SLOTS, int TABLE>
static hipError_t occ_q(int wpb, int lds, int *out) {
    // both flip variants use the same registers to within the allocation granule;
    // the message-flip variant is the one queried
    hipError_t e = hipFuncSetAttribute((const void *)bp_int8_kernel<SLOTS, false, TABLE, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, bp_int8_kernel<SLOTS, false, TABLE, false>, 64 * wpb,
                                                         (size_t)lds);
}

// The compact space-time tables are built for the large slot counts only, where
// the per-check table takes most of the LDS (8 to 16 KiB).
hipError_t launch_bp_int8(int slots, int table, const BpArgs &a, int blocks, int wpb, hipStream_t s) {
    if (table == 1 || table == 2) {
        switch (slots) {
        case 8: return table == 1 ? launch_s<8, 1>(a, blocks, wpb, s) : launch_s<8, 2>(a, blocks, wpb, s);
        case 14: return table == 1 ? launch_s<14, 1>(a, blocks, wpb, s) : launch_s<14, 2>(a, blocks, wpb, s);
        case 16: return table == 1 ? launch_s<16, 1>(a, blocks, wpb, s) : launch_s<16, 2>(a, blocks, wpb, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (slots) {
    case 1: return launch_s<1, 0>(a, blocks, wpb, s);
    case 2: return launch_s<2, 0>(a, blocks, wpb, s);
    case 4: return launch_s<4, 0>(a, blocks, wpb, s);
    case 8: return launch_s<8, 0>(a, blocks, wpb, s);
    case 14: return launch_s<14, 0>(a, blocks, wpb, s);
    default: return launch_s<16, 0>(a, blocks, wpb, s);
    }
}

hipError_t bp_int8_max_blocks_per_cu(int slots, int table, int wpb, int lds, int *out) {
    if (table == 1 || table == 2) {
        switch (slots) {
        case 8: return table == 1 ? occ_q<8, 1>(wpb, lds, out) : occ_q<8, 2>(wpb, lds, out);
        case 14: return table == 1 ? occ_q<14, 1>(wpb, lds, out) : occ_q<14, 2>(wpb, lds, out);
        case 16: return table == 1 ? occ_q<16, 1>(wpb, lds, out) : occ_q<16, 2>(wpb, lds, out);
        default: return hipErrorInvalidValue;
        }
    }
    switch (slots) {
    case 1: return occ_q<1, 0>(wpb, lds, out);
    case 2: return occ_q<2, 0>(wpb, lds, out);
    case 4: return occ_q<4, 0>(wpb, lds, out);
    case 8: return occ_q<8, 0>(wpb, lds, out);
    case 14: return occ_q<14, 0>(wpb, lds, out);
    default: return occ_q<16, 0>(wpb, lds, out);
    }
}

}  // namespace lbp
