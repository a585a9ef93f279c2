// OSD-0 (Algorithm 2) and OSD-CS for the shots whose BP run did not converge.
//
// One workgroup per failed shot (persistent over the failure list): 1024 or 512
// threads with G in LDS or global memory, one or two rows of G per lane with G
// in registers (m < 1024).
//  1. LLR sorting: bitonic sort of (orderable(lambda) << 32 | column) keys in
//     LDS, i.e. ascending lambda with ties broken by column (stable order).
//  2. Basis selection + LU/forward substitution as one Gauss-Jordan sweep in
//     sorted column order.  The permuted matrix is never materialised: the
//     workgroup keeps only G, the accumulated row operations (m x m bits,
//     identity at the start) and s' = G s.  The reduced form of any column j
//     of H is G h_j, and h_j has at most CDEG non-zeros, so testing column j
//     costs <= CDEG bit reads per row.  A column whose reduced form has a 1 in
//     a row that is not yet a pivot becomes a basis column: the lowest such row
//     is its pivot and the pivot row of G is XORed into every other row with a
//     1 there (packed 32-bit words).  The first rank(H) independent columns in
//     sorted order form the basis S (unique), so the result is independent of
//     the pivot-row choice.
//  3. Backward substitution is implicit (Gauss-Jordan): e_S[pivot row r] = s'_r.
//     A row never chosen as pivot must have s'_r = 0, else s is not in the
//     column space of H (flag, keep the BP hard decision).
//  4. OSD-CS: candidate t (no column, one non-basis column, or two of the
//     first `order` non-basis columns in sorted order) costs
//     |s' + G H_T t| + |t|; the first candidate of minimum cost wins.
//  5. Error vector construction / inverse mapping: bits are scattered to the
//     original column indices.
// G lives in LDS (row-major, odd word stride: conflict-free column access)
// when it fits, otherwise in a per-workgroup global buffer (word-major, so
// that a column word of all rows is one coalesced access).
#include "device_util.h"
#include "lbp_internal.h"

namespace lbp {
namespace {

constexpr int OSD_THREADS = 1024;
constexpr int OSD_WAVES = OSD_THREADS / 64;
// Smallest m whose global-G OSD keeps an occupancy mask of G: it pays from ~4096
// checks on (surface d=21 and up) and cost a few percent at d=17, where G's
// columns are short.
constexpr int OSD_OCC_MIN_M = 4096;

// Words of that mask: bit t of word (w * ceil(mw/32) + t/32) is set when some row
// of the 32-row group t may have a non-zero word w of G.
__host__ __device__ inline int osd_occ_words(int m) {
    const int mw = (m + 31) / 32;
    return mw * ((mw + 31) / 32);
}

__device__ __forceinline__ uint32_t orderable(float f) {
    uint32_t u = __float_as_uint(f);
    if (u == 0x80000000u) u = 0u;  // -0 sorts with +0
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

struct GView {
    uint32_t *g;
    int m, mws, in_lds;
    __device__ __forceinline__ uint32_t &at(int r, int w) const {
        return in_lds ? g[(size_t)r * mws + w] : g[(size_t)w * m + r];
    }
};

// Bit of row r of the reduced column with check rows rows[0..nr).
__device__ __forceinline__ uint32_t xbit(const GView &G, int r, const int *rows, int nr) {
    uint32_t x = 0;
    for (int k = 0; k < nr; ++k) x ^= (G.at(r, rows[k] >> 5) >> (rows[k] & 31)) & 1u;
    return x;
}

__device__ __forceinline__ int col_rows(const OsdArgs &a, int col, int *rows) {
    int nr = 0;
    if (a.vn_tab4) {
        const u32x4 tab = a.vn_tab4[col];
#pragma unroll
        for (int j = 0; j < CDEG; ++j)
            if (tab[j] != NOPOS32) rows[nr++] = (int)(tab[j] / DEG);
        return nr;
    }
    const uint64_t tab = a.vn_tab[col];
#pragma unroll
    for (int j = 0; j < CDEG; ++j) {
        uint32_t p = (uint32_t)(tab >> (16 * j)) & 0xFFFFu;
        if (p != NOPOS) rows[nr++] = (int)(p / DEG);
    }
    return nr;
}

// Exclusive block scan of one int per thread; *total receives the sum.
__device__ int block_excl_scan(int x, int *scr, int *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = (int)(blockDim.x >> 6);
    int incl = wave_incl_scan(x, lane);
    if (lane == 63) scr[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        int v = lane < nwv ? scr[lane] : 0;
        int vi = wave_incl_scan(v, lane);
        if (lane < nwv) scr[lane] = vi - v;
        if (lane == nwv - 1) scr[16] = vi;
    }
    __syncthreads();
    int r = scr[wid] + incl - x;
    *total = scr[16];
    __syncthreads();
    return r;
}

// Step 1 (LLR sorting): perm[j] = j-th column in ascending (lambda, column)
// order, lambda = hi + lo.  Bitonic sort of P u64 keys: without a lo part the
// key is orderable(hi) << 32 | column; with one (fp32 messages) it is
// orderable(hi) << 32 | orderable(lo), and the column rides along in `cols`
// (P u16; P < 2n, so they fit the space of n floats) as the tie-break.  With
// i16 set, lambda is int16 (the Int x.y kernel's integers) and its key
// lambda + 2^15 keeps the same order.
__device__ void sort_columns(const float *lam, int n, int P, int has_lo, int i16, unsigned long long *keys,
                             uint16_t *cols, uint16_t *perm) {
    const int tid = threadIdx.x, nth = blockDim.x;
    const int16_t *lq = (const int16_t *)lam;
    for (int j = tid; j < n; j += nth) {
        const uint32_t hk = i16 ? (uint32_t)((int32_t)lq[j] + 32768) : orderable(lam[j]);
        const unsigned long long h = (unsigned long long)hk << 32;
        keys[j] = h | (has_lo ? orderable(lam[n + j]) : (unsigned)j);
        if (has_lo) cols[j] = (uint16_t)j;
    }
    __syncthreads();
    // the ascending bitonic network of sort_columns_i16 below: the slots n .. P - 1
    // stand for an element above every (key, column) pair and are never touched
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            const int tb = (n >> 1) + jj < (P >> 1) ? (n >> 1) + jj : (P >> 1);
            for (int t = tid; t < tb; t += nth) {
                const int i = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
                const int l = jj == (k >> 1) ? i ^ (k - 1) : i + jj;
                if (l >= n) continue;
                const unsigned long long x = keys[i], y = keys[l];
                if (has_lo) {
                    const uint16_t cx = cols[i], cy = cols[l];
                    if (x > y || (x == y && cx > cy)) {
                        keys[i] = y; keys[l] = x;
                        cols[i] = cy; cols[l] = cx;
                    }
                } else if (x > y) {
                    keys[i] = y; keys[l] = x;
                }
            }
            __syncthreads();
        }
    }
    for (int j = tid; j < n; j += nth) perm[j] = has_lo ? cols[j] : (uint16_t)(keys[j] & 0xFFFFu);
    __syncthreads();
}

// Step 1 for int16 lambda: the key (lambda + 2^15) << 16 | column is 32 bits, so
// the sort moves half the bytes of the general one and its keys take P * 4
// bytes of LDS.
__device__ void sort_columns_i16(const int16_t *lq, int n, int P, uint32_t *keys, uint16_t *perm) {
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int j = tid; j < n; j += nth) keys[j] = ((uint32_t)((int32_t)lq[j] + 32768) << 16) | (uint32_t)j;
    __syncthreads();
    // Bitonic network with every block sorted ascending: each merge of blocks of size k
    // first compares element i with its mirror i ^ (k - 1), then halves as usual.  The
    // slots n .. P - 1 stand for +infinity (keys are unique and below ~0u), which never
    // moves in this form, so every pair whose upper slot is >= n is skipped and those
    // slots are never stored.
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            // pair t has i >= 2 (t - jj + 1): none from t = n / 2 + jj on reaches below n
            const int tb = (n >> 1) + jj < (P >> 1) ? (n >> 1) + jj : (P >> 1);
            for (int t = tid; t < tb; t += nth) {
                const int i = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
                const int l = jj == (k >> 1) ? i ^ (k - 1) : i + jj;
                if (l < n) {
                    const uint32_t x = keys[i], y = keys[l];
                    if (x > y) {
                        keys[i] = y;
                        keys[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int j = tid; j < n; j += nth) perm[j] = (uint16_t)(keys[j] & 0xFFFFu);
    __syncthreads();
}

// Step 1 for int16 lambda, as a stable LSD radix sort on lambda + 2^15 (four 4-bit
// digits).  The columns enter in index order, so the result is the ascending
// (lambda, column) order of the keys above.  Elements go in tiles of 64; a lane's
// rank among the equal digits of its tile comes from four ballots, the (digit,
// tile) counts are scanned digit-major, and each element lands at its count's
// offset plus its rank.  keys holds 2n words (source and destination), hist
// 16 ceil(n / 64) u16 counts, scr the block scan's 17 ints.
__device__ void sort_columns_radix16(const int16_t *lq, int n, uint32_t *keys, uint16_t *hist, int *scr,
                                     uint16_t *perm) {
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6), nwv = nth >> 6;
    const int ntl = (n + 63) >> 6, ne = 16 * ntl;
    const uint64_t below = (1ull << lane) - 1ull;  // lanes before this one
    uint32_t *src = keys, *dst = keys + n;
    for (int j = tid; j < n; j += nth) src[j] = ((uint32_t)((int32_t)lq[j] + 32768) << 16) | (uint32_t)j;
    __syncthreads();
    for (int pass = 0; pass < 4; ++pass) {
        const int sh = 16 + 4 * pass;
        // counts of digit l in tile T, written by lane l
        for (int T = wid; T < ntl; T += nwv) {
            const int i = 64 * T + lane;
            const bool valid = i < n;
            const uint32_t d = valid ? (src[i] >> sh) & 15u : 0u;
            const uint64_t vm = __ballot(valid);
            const uint64_t b0 = __ballot(d & 1u), b1 = __ballot(d & 2u), b2 = __ballot(d & 4u), b3 = __ballot(d & 8u);
            if (lane < 16) {
                const uint64_t mk = vm & ((lane & 1) ? b0 : ~b0) & ((lane & 2) ? b1 : ~b1) &
                                    ((lane & 4) ? b2 : ~b2) & ((lane & 8) ? b3 : ~b3);
                hist[lane * ntl + T] = (uint16_t)__popcll(mk);
            }
        }
        __syncthreads();
        // exclusive scan of the counts in (digit, tile) order
        const int per = (ne + nth - 1) / nth, e0 = tid * per;
        const int e1 = e0 + per < ne ? e0 + per : ne;
        int sum = 0;
        for (int e = e0; e < e1; ++e) sum += hist[e];
        int total;
        int off = block_excl_scan(sum, scr, &total);
        for (int e = e0; e < e1; ++e) {
            const int c = hist[e];
            hist[e] = (uint16_t)off;
            off += c;
        }
        __syncthreads();
        for (int T = wid; T < ntl; T += nwv) {
            const int i = 64 * T + lane;
            const bool valid = i < n;
            const uint32_t v = valid ? src[i] : 0u;
            const uint32_t d = (v >> sh) & 15u;
            const uint64_t vm = __ballot(valid);
            const uint64_t b0 = __ballot(d & 1u), b1 = __ballot(d & 2u), b2 = __ballot(d & 4u), b3 = __ballot(d & 8u);
            const uint64_t mk = vm & ((d & 1u) ? b0 : ~b0) & ((d & 2u) ? b1 : ~b1) & ((d & 4u) ? b2 : ~b2) &
                                ((d & 8u) ? b3 : ~b3);
            if (valid) dst[hist[d * ntl + T] + __popcll(mk & below)] = v;
        }
        __syncthreads();
        uint32_t *t = src;
        src = dst;
        dst = t;
    }
    for (int j = tid; j < n; j += nth) perm[j] = (uint16_t)(src[j] & 0xFFFFu);  // four passes: src is keys
    __syncthreads();
}

// Non-basis columns in sorted order -> tl[0..nt).
__device__ int list_nonbasis(const uint8_t *isb, const uint16_t *perm, int n, uint16_t *tl, int *scr) {
    const int nth = blockDim.x;
    const int chunk = (n + nth - 1) / nth;
    const int lo = threadIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    int cnt = 0;
    for (int j = lo; j < hi; ++j) cnt += !isb[j];
    int nt;
    int off = block_excl_scan(cnt, scr, &nt);
    for (int j = lo; j < hi; ++j)
        if (!isb[j]) tl[off++] = perm[j];
    __syncthreads();
    return nt;
}

// Pair index -> (a, b), a < b < w, lexicographic.
__device__ __forceinline__ void pair_of(int pi, int w, int &aa, int &bb) {
    int rem = pi;
    aa = 0;
    while (rem >= w - 1 - aa) { rem -= w - 1 - aa; ++aa; }
    bb = aa + 1 + rem;
}

// Next failure-list position for the calling block, or -1 (thread 0 calls it;
// the modes are those of OsdArgs::claim_mode 1 and 2).
__device__ int64_t osd_claim(const OsdArgs &a) {
    const uint32_t cap = a.fail_cap < (int64_t)0xFFFFFFFFu ? (uint32_t)a.fail_cap : 0xFFFFFFFFu;
    int idle = 0;
    for (;;) {
        uint32_t produced = __hip_atomic_load(&a.counters[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (produced > cap) produced = cap;
        const uint32_t c = __hip_atomic_load(a.claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (c < produced) {
            if (atomicCAS(a.claim, c, c + 1) == c) {
                // the wave that took this position publishes it right after its stores
                int32_t *fl = const_cast<int32_t *>(a.fail_list);
                while (__hip_atomic_load(fl + c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < 0)
                    __builtin_amdgcn_s_sleep(1);
                return (int64_t)c;
            }
            continue;
        }
        if (a.claim_mode != 1) return -1;
        const uint32_t done = __hip_atomic_load(&a.counters[4], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (done >= (uint32_t)a.bp_grid) {  // BP has finished: the count is final
            produced = __hip_atomic_load(&a.counters[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (produced > cap) produced = cap;
            if (c >= produced) return -1;
            continue;
        }
        // wait for more failures only while every BP block is resident (BP then
        // finishes whatever this block holds); otherwise leave them to the launch after BP
        if (__hip_atomic_load(&a.counters[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (uint32_t)a.bp_grid)
            return -1;
        if (idle < 5) ++idle;
        for (int z = 0; z < (1 << idle); ++z) __builtin_amdgcn_s_sleep(2);
    }
}

__global__ __launch_bounds__(1024, 8) void osd_lds_kernel(OsdArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int m = a.m, n = a.n, tid = threadIdx.x, lane = tid & 63;
    const int nth = (int)blockDim.x;  // 512 or 1024; a thread's rows fit one 32-bit mask (m <= 32 nth)
    const int P = a.sort_p;
    unsigned char *gblk = (unsigned char *)(a.gscratch + (size_t)blockIdx.x * a.scratch_words);
    unsigned char *q0, *c0;  // next free byte of LDS, and of the per-column arrays
    unsigned long long *keys;
    if (a.cols_global) {
        // large n: sort keys and per-column arrays after G in the block's scratch
        c0 = gblk + (((size_t)m * a.mws * 4 + 255) & ~(size_t)255);
        keys = (unsigned long long *)c0;
        c0 += ((size_t)P * 8 + 255) & ~(size_t)255;
        q0 = smem;
    } else {
        size_t gbytes = a.g_in_lds ? (size_t)m * a.mws * 4 : 0;
        size_t rbytes = gbytes > (size_t)P * 8 ? gbytes : (size_t)P * 8;
        rbytes = (rbytes + 15) & ~(size_t)15;
        keys = (unsigned long long *)smem;
        c0 = smem + rbytes;
        q0 = nullptr;
    }
    uint16_t *scol = (uint16_t *)c0;                 c0 += ((size_t)n * 4 + 15) & ~(size_t)15;
    uint16_t *perm = (uint16_t *)c0;                 c0 += ((size_t)n * 2 + 15) & ~(size_t)15;
    uint16_t *tl = (uint16_t *)c0;                   c0 += ((size_t)n * 2 + 15) & ~(size_t)15;
    uint8_t *isb = c0;                               c0 += ((size_t)n + 15) & ~(size_t)15;
    if (!a.cols_global) q0 = c0;
    uint16_t *pcol = (uint16_t *)q0;                 q0 += ((size_t)m * 2 + 15) & ~(size_t)15;
    uint8_t *piv = q0;                               q0 += ((size_t)m + 15) & ~(size_t)15;
    uint8_t *sp = q0;                                q0 += ((size_t)m + 15) & ~(size_t)15;
    uint32_t *pl_w = (uint32_t *)q0;                 q0 += ((size_t)a.mw * 4 + 15) & ~(size_t)15;
    uint32_t *pl_v = (uint32_t *)q0;                 q0 += ((size_t)a.mw * 4 + 15) & ~(size_t)15;
    unsigned long long *Yq = (unsigned long long *)q0; q0 += ((size_t)((m + 63) >> 6) * 8 + 15) & ~(size_t)15;
    // G in global memory (large m): the occupancy mask of its words lives in LDS
    const bool use_occ = !a.g_in_lds && m >= OSD_OCC_MIN_M;
    uint32_t *occ = use_occ ? (uint32_t *)q0 : nullptr;
    if (use_occ) q0 += ((size_t)osd_occ_words(m) * 4 + 15) & ~(size_t)15;
    uint32_t *cw = (uint32_t *)q0;                   q0 += ((size_t)a.nw * 4 + 15) & ~(size_t)15;
    uint32_t *red = (uint32_t *)q0;                  q0 += 16 * 4;
    int *scr = (int *)q0;                            q0 += 32 * 4;
    unsigned long long *best64 = (unsigned long long *)q0;

    // occ: a set bit (w, t) says rows 32t..32t+31 may hold a non-zero word w of G
    // (a superset, never cleared), so the column test loads only G's words that
    // can be non-zero; G stays sparse on the codes that need this.
    const int mwt = (a.mw + 31) / 32;  // mask words per G word
    const int krows = (m + nth - 1) / nth;

    GView G;
    G.g = a.g_in_lds ? (uint32_t *)smem : (uint32_t *)gblk;
    G.m = m;
    G.mws = a.mws;
    G.in_lds = a.g_in_lds;

    uint32_t nfail = a.counters[1];
    if ((int64_t)nfail > a.fail_cap) nfail = (uint32_t)a.fail_cap;

    __shared__ int32_t claimed;
    uint32_t qs = blockIdx.x;  // claim_mode 0: strided over the complete list
    for (;;) {
        uint32_t q;
        if (a.claim_mode == 0) {
            if (qs >= nfail) break;
            q = qs;
            qs += gridDim.x;
        } else {
            if (tid == 0) claimed = (int32_t)osd_claim(a);
            __syncthreads();
            const int32_t qq = claimed;
            __syncthreads();  // rewritten next round only after every thread read it
            if (qq < 0) break;
            q = (uint32_t)qq;
        }
        const int64_t shot = a.fail_list[q];
        // hi[n] then lo[n], or int16 [n]
        const size_t lrow = (size_t)(a.llr_by_shot ? shot : (int64_t)q);
        const float *lam = a.llr_i16 ? (const float *)((const int16_t *)a.fail_llr + lrow * n) : a.fail_llr + lrow * 2 * n;

        // ---- 1. sort (lambda, column) ascending
        sort_columns(lam, n, P, a.has_lo, a.llr_i16, keys, scol, perm);

        // ---- 2. G = I, s' = s
        const int mw = a.mw;
        for (size_t idx = tid; idx < (size_t)m * mw; idx += nth) {
            int r = (int)(idx / mw), w = (int)(idx % mw);
            G.at(r, w) = (w == (r >> 5)) ? (1u << (r & 31)) : 0u;
        }
        if (occ)
            for (int idx = tid; idx < mw * mwt; idx += nth) {
                const int w = idx / mwt, j = idx % mwt;  // G = I: group w holds word w
                occ[idx] = (w >> 5) == j ? 1u << (w & 31) : 0u;
            }
        const uint32_t *sw = a.synd + shot * a.mw;
        for (int r = tid; r < m; r += nth) {
            sp[r] = (uint8_t)((sw[r >> 5] >> (r & 31)) & 1u);
            piv[r] = 0;
        }
        for (int j = tid; j < n; j += nth) isb[j] = 0;
        if (tid < 3) red[tid] = 0xFFFFFFFFu;
        if (tid == 3) red[4] = red[5] = 0u;
        __syncthreads();

        // ---- 3. Gauss-Jordan in sorted column order.  G stays sparse (a row combines
        // few checks), so a pivot step first lists the pivot row's non-zero words and
        // every updated row touches only those.
        int rank = 0, step = 0;
        for (int j = 0; j < n && rank < m; ++j) {
            const int col = perm[j];
            int rows[CDEG];
            const int nr = col_rows(a, col, rows);
            const int slot = step % 3;
            if (tid == 0) red[(step + 1) % 3] = 0xFFFFFFFFu;
            uint32_t xm = 0, cand = 0xFFFFFFFFu;
            int k = 0;
            for (int r = tid; r < m; r += nth, ++k) {
                uint32_t x = 0;
                if (occ) {
                    const int t = r >> 5;
                    for (int q = 0; q < nr; ++q) {
                        const int c = rows[q];
                        if ((occ[(c >> 5) * mwt + (t >> 5)] >> (t & 31)) & 1u)
                            x ^= (G.at(r, c >> 5) >> (c & 31)) & 1u;
                    }
                } else {
                    x = xbit(G, r, rows, nr);
                }
                xm |= x << k;
                if (x && !piv[r] && (uint32_t)r < cand) cand = (uint32_t)r;
            }
            cand = wave_min_u32(cand);
            if (lane == 0 && cand != 0xFFFFFFFFu) atomicMin(&red[slot], cand);
            __syncthreads();
            const uint32_t pv = red[slot];
            ++step;
            if (pv == 0xFFFFFFFFu) continue;
            uint32_t *cnt = &red[4 + (rank & 1)];  // the other counter is reset for the next pivot step
            for (int w = tid; w < mw; w += nth) {
                const uint32_t v = G.at((int)pv, w);
                if (v) {
                    const uint32_t i = atomicAdd(cnt, 1u);
                    pl_w[i] = (uint32_t)w;
                    pl_v[i] = v;
                }
            }
            if (tid == 0) red[4 + ((rank + 1) & 1)] = 0u;
            __syncthreads();
            const int nl = (int)*cnt;
            const uint8_t spv = sp[pv];
            for (k = 0; k < krows; ++k) {
                const int r = k * nth + tid;
                const bool upd = r < m && (uint32_t)r != pv && ((xm >> k) & 1u);
                if (r < m && (uint32_t)r == pv) {
                    piv[r] = 1;
                    pcol[r] = (uint16_t)col;
                } else if (upd) {
                    for (int i = 0; i < nl; ++i) G.at(r, (int)pl_w[i]) ^= pl_v[i];
                    sp[r] ^= spv;
                    // the bit of this row's group is only ever read by this wave (its 64
                    // rows span two groups), and LDS operations of a wave stay in order
                    if (occ) {
                        const int t = r >> 5;
                        for (int i = 0; i < nl; ++i) atomicOr(&occ[(int)pl_w[i] * mwt + (t >> 5)], 1u << (t & 31));
                    }
                }
            }
            if (tid == 0) isb[j] = 1;
            ++rank;
            // No barrier here: a thread only ever updates and tests its own rows, and
            // everything shared (the pivot row, the word list, red[]) is next touched
            // after the next step's first barrier, which every thread reaches only
            // once its updates of this step are done.
        }

        // ---- consistency: a row with no pivot reduced to 0 = s'_r
        int bad = 0;
        for (int r = tid; r < m; r += nth) bad |= (!piv[r] && sp[r]);
        bad = __syncthreads_or(bad);
        if (bad) {
            if (tid == 0) a.flags[shot] = (uint8_t)(FLAG_OSD | FLAG_OSD_INCONSISTENT);
            __syncthreads();
            continue;
        }

        // ---- 4. OSD-CS candidate sweep on 64-row ballots of G's columns:
        // Bq[q*m + c] holds column c of G over rows 64q..64q+63, Yq[q] those rows of s',
        // so a candidate's cost is a popcount per 64 rows.
        int t0 = -1, t1 = -1;
        if (a.mode == OSD_CS) {
            const int nt = list_nonbasis(isb, perm, n, tl, scr);
            const int nq = (m + 63) >> 6, krows = (m + nth - 1) / nth;
            unsigned long long *Bq = (unsigned long long *)(a.gscratch + (size_t)blockIdx.x * a.scratch_words +
                                                            a.cs_offset_words);
            for (int k = 0; k < krows; ++k) {
                const int r = k * nth + tid, q = r >> 6;  // q is wave-uniform
                const uint64_t yb = __ballot(r < m && sp[r]);
                if (lane == 0 && q < nq) Yq[q] = yb;
                for (int w = 0; w < mw; ++w) {
                    const uint32_t v = r < m ? G.at(r, w) : 0u;
                    unsigned long long mine = 0;
                    for (int b = 0; b < 32; ++b) {
                        const unsigned long long bal = __ballot((v >> b) & 1u);
                        mine = lane == b ? bal : mine;
                    }
                    if (q < nq && lane < 32 && 32 * w + lane < m) Bq[(size_t)q * m + 32 * w + lane] = mine;
                }
            }
            if (tid == 0) *best64 = ~0ull;
            __syncthreads();
            uint32_t cost0 = 0;
            for (int q = 0; q < nq; ++q) cost0 += __popcll(Yq[q]);
            // OSD-0 candidate: cost |s'|, enumeration index 0
            unsigned long long best = (unsigned long long)cost0 << 32;
            for (int ai = tid; ai < nt; ai += nth) {
                int rows[CDEG];
                const int nr = col_rows(a, tl[ai], rows);
                unsigned long long cost = 1;
                for (int q = 0; q < nq; ++q) {
                    unsigned long long x = Yq[q];
                    for (int t = 0; t < nr; ++t) x ^= Bq[(size_t)q * m + rows[t]];
                    cost += __popcll(x);
                }
                unsigned long long key = (cost << 32) | (unsigned long long)(1 + ai);
                best = key < best ? key : best;
            }
            const int w = a.order < nt ? a.order : nt;
            const int npairs = w * (w - 1) / 2;
            for (int pi = tid; pi < npairs; pi += nth) {
                int aa, bb;
                pair_of(pi, w, aa, bb);
                int ra[CDEG], rb[CDEG];
                const int na = col_rows(a, tl[aa], ra), nb = col_rows(a, tl[bb], rb);
                unsigned long long cost = 2;
                for (int q = 0; q < nq; ++q) {
                    unsigned long long x = Yq[q];
                    for (int t = 0; t < na; ++t) x ^= Bq[(size_t)q * m + ra[t]];
                    for (int t = 0; t < nb; ++t) x ^= Bq[(size_t)q * m + rb[t]];
                    cost += __popcll(x);
                }
                unsigned long long key = (cost << 32) | (unsigned long long)(1 + nt + pi);
                best = key < best ? key : best;
            }
            best = wave_min_u64(best);
            if (lane == 0) atomicMin(best64, best);
            __syncthreads();
            const unsigned idx = (unsigned)(*best64 & 0xFFFFFFFFull);
            if (idx >= 1 && idx <= (unsigned)nt) {
                t0 = tl[idx - 1];
            } else if (idx > (unsigned)nt) {
                int aa, bb;
                pair_of((int)idx - 1 - nt, w, aa, bb);
                t0 = tl[aa];
                t1 = tl[bb];
            }
        }

        // ---- 5. e_S = s' + G H_T t on the basis, t on the rest; scatter to columns
        for (int ww = tid; ww < a.nw; ww += nth) cw[ww] = 0u;
        __syncthreads();
        int r0[CDEG], r1[CDEG], n0 = 0, n1 = 0;
        if (t0 >= 0) n0 = col_rows(a, t0, r0);
        if (t1 >= 0) n1 = col_rows(a, t1, r1);
        for (int r = tid; r < m; r += nth) {
            if (!piv[r]) continue;
            uint32_t e = sp[r];
            if (t0 >= 0) e ^= xbit(G, r, r0, n0);
            if (t1 >= 0) e ^= xbit(G, r, r1, n1);
            if (e) {
                int c = pcol[r];
                atomicOr(&cw[c >> 5], 1u << (c & 31));
            }
        }
        if (tid == 0) {
            if (t0 >= 0) atomicOr(&cw[t0 >> 5], 1u << (t0 & 31));
            if (t1 >= 0) atomicOr(&cw[t1 >> 5], 1u << (t1 & 31));
        }
        __syncthreads();
        for (int ww = tid; ww < a.nw; ww += nth) a.corr[shot * a.nw + ww] = cw[ww];
        if (tid == 0) a.flags[shot] = (uint8_t)FLAG_OSD;  // clears a serving ring's pending bit
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
// Register-resident variant for m < 32*NW <= 1024: a lane owns rows of G as
// NW-word vector registers, so the Gauss-Jordan XOR of a pivot row is NW VALU
// ops against a broadcast LDS copy, and the bit of the reduced column is read
// with a wave-uniform word index (indexed register move, no LDS).  One block
// barrier per column.  For OSD-CS each wave turns every column c of G into
// 64-bit ballots of its rows; the cost of a candidate is then a popcount per
// ballot.
template <int NW>
using vrow = uint32_t __attribute__((ext_vector_type(NW)));

// Byte offsets of the register kernel's LDS arrays; the host sizes the block's
// dynamic LDS with the same function.  The sort keys (P u32 for int16 lambda,
// else P u64) are dead after the sort, and the sorted columns' check lists
// (n u64) reuse their space.  vb is the byte size of one candidate row vector.
struct RegLds {
    uint32_t cols, perm, tl, isb, crow, csp, cw, wkey, scr, Y, best, total;
};

__host__ __device__ inline RegLds reg_lds_layout(int n, int P, int nw_corr, int vb, int i16) {
    auto al = [](uint32_t x) { return (x + 15u) & ~15u; };
    RegLds L{};
    uint32_t keys = (uint32_t)P * (i16 ? 4u : 8u);
    if (keys < (uint32_t)n * 8u) keys = (uint32_t)n * 8u;
    uint32_t o = al(keys);
    L.cols = o;
    if (!i16) o += al((uint32_t)n * 4);  // tie-break columns of the pair keys (P u16)
    L.perm = o;  o += al((uint32_t)n * 2);
    L.tl = o;    o += al((uint32_t)n * 2);
    L.isb = o;   o += al((uint32_t)n);
    o = (o + (uint32_t)vb - 1) & ~((uint32_t)vb - 1);  // the row loads and stores assume this alignment
    L.crow = o;  o += 32u * (uint32_t)vb;
    L.csp = o;   o += 32 * 4;
    L.cw = o;    o += al((uint32_t)nw_corr * 4);
    L.wkey = o;  o += 32 * 4;
    L.scr = o;   o += 32 * 4;
    L.Y = o;     o += 16 * 8;
    L.best = o;  o += 16;
    L.total = o;
    return L;
}

static_assert(sizeof(vrow<28>) == 128 && sizeof(vrow<32>) == 128 && sizeof(vrow<16>) == 64 && sizeof(vrow<8>) == 32,
              "osd_block_bytes assumes power-of-two vector sizes");

template <int NW>
__device__ __forceinline__ uint32_t row_bit(const vrow<NW> &g, int c) {
    return (g[c >> 5] >> (c & 31)) & 1u;  // c is wave-uniform
}

// A column's checks for the elimination, wave-uniform: its D <= CDEG check indices
// (< 2^13) in the low 16-bit fields, the fields past D naming check m (a bit that is
// zero in every row of G: its support is [0, m), and m < 32 NW), D in bits 61-63.
static_assert(CDEG == 4, "the packed check list holds four checks");

template <int NW, int R>
__device__ __forceinline__ void reduced_bits_add(const vrow<NW> (&g)[R], uint64_t chk, int j, uint32_t (&x)[R]) {
    const int c = (int)((chk >> (16 * j)) & 0x1FFFu);
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] ^= row_bit<NW>(g[k], c);
}

// Bit of each of the lane's R rows of the reduced column G h_j, from the packed
// check list of column j (one indexed register read per check and row; checks 3
// and 4 only where the column has them).
template <int NW, int R>
__device__ __forceinline__ void reduced_bits(const vrow<NW> (&g)[R], uint64_t chk, uint32_t (&x)[R]) {
    uint32_t d = (uint32_t)(chk >> 32) >> 29;
    asm volatile("" : "+s"(d));  // a 32-bit scalar: the tests below stay scalar compares
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = 0;
    reduced_bits_add<NW, R>(g, chk, 0, x);
    reduced_bits_add<NW, R>(g, chk, 1, x);
    if (d > 2u) {
        reduced_bits_add<NW, R>(g, chk, 2, x);
        if (d > 3u) reduced_bits_add<NW, R>(g, chk, 3, x);
    }
}

__device__ __forceinline__ uint64_t uniform_tab(const uint64_t *vn_tab, int col) {
    col = __builtin_amdgcn_readfirstlane(col);
    uint64_t t = vn_tab[col];
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)t), hi = __builtin_amdgcn_readfirstlane((uint32_t)(t >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// 32 x 32 bit transpose within each half of the wave: afterwards bit i of lane
// 32 h + j is bit j of lane 32 h + i's input.  Five block-swap stages (Hacker's
// Delight, transpose32), the partner lane of stage s being lane ^ s (ds_swizzle in
// bit-mask mode, within 32 lanes).
// Branch-free: the lower lane of a pair keeps x's bits in M and takes the
// partner's M bits shifted up (rotl(p, S) & ~M); the upper lane keeps ~M and takes
// rotr(p, S) & M (the bits a rotation wraps around fall outside the taken mask).
template <int S>
__device__ __forceinline__ uint32_t transpose_stage(uint32_t x, int lane) {
    constexpr uint32_t M = S == 16 ? 0x0000FFFFu : S == 8 ? 0x00FF00FFu : S == 4 ? 0x0F0F0F0Fu
                         : S == 2 ? 0x33333333u : 0x55555555u;  // bits whose index has bit S clear
    constexpr int LS = S == 16 ? 4 : S == 8 ? 3 : S == 4 ? 2 : S == 2 ? 1 : 0;
    const uint32_t p = (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (S << 10) | 0x1F);
    const uint32_t up = 0u - ((uint32_t)(lane >> LS) & 1u);  // ~0 in the upper lane of the pair
    const uint32_t keep = M ^ up;
    const uint32_t rot = (32u - S) ^ (up & ((uint32_t)S ^ (32u - S)));  // upper: S, lower: 32 - S
    const uint32_t q = __builtin_amdgcn_alignbit(p, p, rot);           // rotate right by rot
    return (x & keep) | (q & ~keep);
}

__device__ __forceinline__ uint32_t transpose32(uint32_t x, int lane) {
    x = transpose_stage<16>(x, lane);
    x = transpose_stage<8>(x, lane);
    x = transpose_stage<4>(x, lane);
    x = transpose_stage<2>(x, lane);
    return transpose_stage<1>(x, lane);
}

// Lane i's 64-row ballot of column 32 w + i (words w and w + 1 of the wave's
// rows xa and xb): each half transposes both words, then the halves trade the
// parts the other one needs.
__device__ __forceinline__ uint64_t column_ballots(uint32_t xa, uint32_t xb, int lane) {
    const uint32_t ta = transpose32(xa, lane), tb = transpose32(xb, lane);
    const bool lo = lane < 32;
    const uint32_t y = (uint32_t)__shfl_xor((int)(lo ? tb : ta), 32, 64);
    return lo ? (((uint64_t)y << 32) | ta) : (((uint64_t)tb << 32) | y);
}

// The candidate sweep's 64-row ballots of G's columns are stored column-major,
// 16 group slots per column: the ballots of check c are B[16 c .. 16 c + ngr), so
// one thread reads a check's groups as ceil(ngr / 2) 16-byte loads.  Y holds the
// groups' ballots of s'.

// popcount over the block's rows of (s' + reduced columns named by ta and tb):
// every load of a candidate is issued before the first XOR that needs it.
__device__ __forceinline__ uint32_t ballot_cost(const uint4 *B4, const uint4 *Y4, int ngr, uint64_t ta,
                                                uint64_t tb) {
    const int nq = (ngr + 1) >> 1;
    uint4 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = q < nq ? Y4[q] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int j = 0; j < 2 * CDEG; ++j) {
        const uint32_t p = (uint32_t)((j < CDEG ? ta : tb) >> (16 * (j % CDEG))) & 0xFFFFu;
        if (p != NOPOS) {
            const uint4 *col = B4 + (size_t)(p / DEG) * 8;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nq) {
                    const uint4 v = col[q];
                    acc[q].x ^= v.x;
                    acc[q].y ^= v.y;
                    acc[q].z ^= v.z;
                    acc[q].w ^= v.w;
                }
        }
    }
    uint32_t cost = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (q < nq) {
            cost += __popc(acc[q].x) + __popc(acc[q].y);
            if (2 * q + 1 < ngr) cost += __popc(acc[q].z) + __popc(acc[q].w);  // the slot after the last group is not written
        }
    return cost;
}

// Group `w`'s 64-row mask of the XOR of the reduced columns named by ta and tb.
__device__ __forceinline__ uint64_t ballot_cost_mask(const unsigned long long *B, int w, uint64_t ta, uint64_t tb) {
    unsigned long long x = 0;
#pragma unroll
    for (int j = 0; j < CDEG; ++j) {
        uint32_t p = (uint32_t)(ta >> (16 * j)) & 0xFFFFu;
        if (p != NOPOS) x ^= B[(size_t)(p / DEG) * 16 + w];
        uint32_t q = (uint32_t)(tb >> (16 * j)) & 0xFFFFu;
        if (q != NOPOS) x ^= B[(size_t)(q / DEG) * 16 + w];
    }
    return x;
}

// Each lane holds R rows of G (rows tid and nth + tid), NW words per row.  A
// column step's wave-uniform work (slot parse, loop control, candidate
// publication) is paid once per wave, so R = 2 halves it per shot against R = 1;
// the per-row VALU work is the same.  R = 1 is compiled for 8 waves per SIMD
// (<= 64 VGPRs, some registers of the non-elimination phases spill), R = 2 for 4
// (<= 128 VGPRs); either way two blocks share a CU, which hides one shot's step
// barrier and LDS latency behind the other's.
template <int NW, int R>
__global__ __launch_bounds__(1024 / R, 8 / R) void osd_reg_kernel(OsdArgs a) {
    static_assert(R == 1 || R == 2, "one or two rows per lane");
    // a published candidate row carries its s' bit in the vector's padding word, if it has one
    constexpr bool SP_IN_ROW = sizeof(vrow<NW>) > 4 * NW;
    extern __shared__ __align__(16) unsigned char smem[];
    const int m = a.m, n = a.n, tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nth = blockDim.x, nwv = nth >> 6;
    const int P = a.sort_p;
    int row[R];
    bool valid[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        row[k] = k * nth + tid;
        valid[k] = row[k] < m;
    }
    const RegLds L = reg_lds_layout(n, P, a.nw, (int)sizeof(vrow<NW>), a.llr_i16);
    uint16_t *scol = (uint16_t *)(smem + L.cols);
    uint16_t *perm = (uint16_t *)(smem + L.perm);
    uint16_t *tl = (uint16_t *)(smem + L.tl);
    uint8_t *isb = smem + L.isb;
    vrow<NW> *crow = (vrow<NW> *)(smem + L.crow);
    uint32_t *csp = (uint32_t *)(smem + L.csp);
    uint32_t *cw = (uint32_t *)(smem + L.cw);
    uint32_t *wkey = (uint32_t *)(smem + L.wkey);  // two alternating slots of the step's pivot key
    int *scr = (int *)(smem + L.scr);
    unsigned long long *Y = (unsigned long long *)(smem + L.Y);
    unsigned long long *best64 = (unsigned long long *)(smem + L.best);
    // 64-row ballots of G's columns, column-major: B[16 c + g] for group g = k * nwv + w,
    // rows k * nth + 64 w + lane (R * nwv <= 16)
    unsigned long long *B = (unsigned long long *)a.gscratch + (size_t)blockIdx.x * 16 * m;
    const int ngr = R * nwv;

    uint32_t nfail = a.counters[1];
    if ((int64_t)nfail > a.fail_cap) nfail = (uint32_t)a.fail_cap;

    __shared__ int32_t claimed;
    uint32_t qs = blockIdx.x;  // claim_mode 0: strided over the complete list
    for (;;) {
        uint32_t q;
        if (a.claim_mode == 0) {
            if (qs >= nfail) break;
            q = qs;
            qs += gridDim.x;
        } else {
            if (tid == 0) claimed = (int32_t)osd_claim(a);
            __syncthreads();
            const int32_t qq = claimed;
            __syncthreads();  // rewritten next round only after every thread read it
            if (qq < 0) break;
            q = (uint32_t)qq;
        }
        const int64_t shot = a.fail_list[q];
        const size_t lrow = (size_t)(a.llr_by_shot ? shot : (int64_t)q);
        const float *lam = a.llr_i16 ? (const float *)((const int16_t *)a.fail_llr + lrow * n) : a.fail_llr + lrow * 2 * n;

        // ---- 1. sort (lambda, column) ascending
        if (a.llr_i16) {
            // the radix sort's counts use the candidate-row buffers, idle until the elimination
            if (32 * ((n + 63) >> 6) <= 32 * (int)sizeof(vrow<NW>))
                sort_columns_radix16((const int16_t *)lam, n, (uint32_t *)smem, (uint16_t *)crow, scr, perm);
            else
                sort_columns_i16((const int16_t *)lam, n, P, (uint32_t *)smem, perm);
        } else {
            sort_columns(lam, n, P, a.has_lo, 0, (unsigned long long *)smem, scol, perm);
        }

        // check lists of the sorted columns (packed as reduced_bits reads them),
        // staged over the dead sort keys
        uint64_t *ptab = (uint64_t *)smem;
        for (int j = tid; j < n; j += nth) {
            const uint64_t t = a.vn_tab[perm[j]];
            uint64_t c = 0;
            uint32_t d = 0;
#pragma unroll
            for (int k = 0; k < CDEG; ++k) {
                const uint32_t p = (uint32_t)(t >> (16 * k)) & 0xFFFFu;
                if (p != NOPOS) {
                    c |= (uint64_t)(p / DEG) << (16 * d);
                    ++d;
                }
            }
            for (uint32_t k = d; k < (uint32_t)CDEG; ++k) c |= (uint64_t)m << (16 * k);
            ptab[j] = c | ((uint64_t)d << 61);
        }

        // ---- 2. G = I, s' = s
        vrow<NW> g[R];
        uint32_t sp[R];
        int pcol[R];
        uint64_t freem[R];  // wave-uniform: lanes whose row k is valid and not yet a pivot
        const uint32_t *sw = a.synd + shot * a.mw;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            // the identity rows depend on the lane only; kept opaque so that they are
            // rebuilt here per shot instead of being hoisted out of the shot loop
            // and held (spilled) across it
            int rk = valid[k] ? row[k] : -1;
            asm volatile("" : "+v"(rk));
#pragma unroll
            for (int w = 0; w < NW; ++w) g[k][w] = (rk >= 0 && w == (rk >> 5)) ? (1u << (rk & 31)) : 0u;
            sp[k] = valid[k] ? (sw[row[k] >> 5] >> (row[k] & 31)) & 1u : 0u;
            pcol[k] = 0;
            freem[k] = __ballot(valid[k]);
        }
        for (int j = tid; j < n; j += nth) isb[j] = 0;
        if (tid < 2) wkey[tid] = 0u;
        __syncthreads();

        // ---- 3. Gauss-Jordan in sorted column order, one block barrier per column:
        // each wave publishes its first candidate row before the barrier, so the
        // winner's row is already in LDS when the pivot is known.  A wave with a
        // candidate takes the atomic maximum of its key (j + 1) << 16 | (0xFFFF -
        // row) into slot j & 1, which every wave reads after the barrier; a key of
        // an earlier step (smaller) left there means no candidate.  Step j + 2
        // writes the slot again only after every wave passed barrier j + 1, so
        // after its read of step j's key (n < 2^16: slot positions are u16).
        int rank = 0;
        int buf = 0;  // row buffers and key slots alternate over 2
        uint64_t tab = n > 0 ? ptab[0] : 0ull;
        for (int j = 0; j < n && rank < m; ++j) {
            const uint64_t tu = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(tab >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)tab);
            tab = ptab[j + 1];  // the next column's checks (past the list at j = n - 1: unused, inside the block's LDS)
            uint32_t x[R];
            reduced_bits<NW, R>(g, tu, x);
            uint64_t xm[R];
#pragma unroll
            for (int k = 0; k < R; ++k) xm[k] = __ballot(x[k]);
            // every slot k publishes its lowest free row with a 1 in row buffer k * 8 + wave
            // (R = 1: the wave), and the publishing lane takes the atomic maximum of the key
            // tag | (1024 - row) << 4 | buffer: the block's lowest candidate row wins
            const uint32_t tag = (uint32_t)(j + 1) << 16;
#pragma unroll
            for (int k = R - 1; k >= 0; --k) {
                const uint64_t cm = xm[k] & freem[k];
                if (cm) {
                    // waves on the step's critical path (a candidate to publish, rows to
                    // update) issue ahead of the others until the next barrier
                    __builtin_amdgcn_s_setprio(2);
                    const int first = __ffsll((unsigned long long)cm) - 1;
                    if (lane == first) {
                        const int slot = k * 8 + wid;
                        vrow<NW> *cr = &crow[buf * 16 + slot];
                        *cr = g[k];
                        if constexpr (SP_IN_ROW)
                            ((uint32_t *)cr)[NW] = sp[k];
                        else
                            csp[buf * 16 + slot] = sp[k];
                        const uint32_t kk = tag | (uint32_t)(1024 - row[k]) << 4 | (uint32_t)slot;
                        __hip_atomic_fetch_max(&wkey[j & 1], kk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            }
            __syncthreads();
            __builtin_amdgcn_s_setprio(0);
            // this step's winning key less the tag is (1024 - row) << 4 | buffer, in
            // [1, 0xFFFF]; an earlier step's key (tag t' < t, or the initial 0) leaves
            // 2^32 - (t - t') 2^16 + low >= 2^16 modulo 2^32
            const uint32_t kd = (uint32_t)__builtin_amdgcn_readfirstlane(wkey[j & 1]) - tag;
            const int pb = buf;
            buf ^= 1;
            if (kd - 1u >= 0xFFFFu) continue;  // no row of this column is free
            const int rv = (int)kd;
            const int slot = rv & 15;
            const int pk = R == 2 ? slot >> 3 : 0;
            const int pw = R == 2 ? slot & 7 : slot;  // the pivot row's wave
            uint64_t um[R];  // rows to update: every row with a 1 but the pivot row
#pragma unroll
            for (int k = 0; k < R; ++k) um[k] = xm[k];
            if (wid == pw) {
                const int pl = (1024 - (rv >> 4)) & 63;  // the pivot row's lane
                const uint64_t bit = 1ull << pl;
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (k == pk) {
                        freem[k] &= ~bit;
                        um[k] &= ~bit;
                    }
                if (lane == pl) {  // the sorted position; its column is looked up after the elimination
                    if (pk == 0)
                        pcol[0] = j;
                    else
                        pcol[R - 1] = j;
                    isb[j] = 1;
                }
            }
            // reduced columns are sparse early on: waves with no row to update skip the row read
            if (um[0] | um[R - 1]) {
                __builtin_amdgcn_s_setprio(2);
                // one load of the whole padded row (its s' bit in the padding word, if any)
                using vpad = vrow<sizeof(vrow<NW>) / 4>;
                const vpad full = *(const vpad *)&crow[pb * 16 + slot];
                vrow<NW> pr;
#pragma unroll
                for (int w = 0; w < NW; ++w) pr[w] = full[w];
                uint32_t ps;
                if constexpr (SP_IN_ROW)
                    ps = full[NW];
                else
                    ps = csp[pb * 16 + slot];
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (__builtin_amdgcn_inverse_ballot_w64(um[k])) {  // lane's row k has a 1
                        g[k] ^= pr;
                        sp[k] ^= ps;
                    }
            }
            ++rank;
        }
        __builtin_amdgcn_s_setprio(0);
        bool piv[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            piv[k] = valid[k] && !((freem[k] >> lane) & 1ull);
            if (piv[k]) pcol[k] = perm[pcol[k]];
        }

        // ---- consistency: a row with no pivot reduced to 0 = s'_r
        bool bad = false;
#pragma unroll
        for (int k = 0; k < R; ++k) bad = bad || (valid[k] && !piv[k] && sp[k]);
        if (__syncthreads_or(bad)) {
            if (tid == 0) a.flags[shot] = (uint8_t)(FLAG_OSD | FLAG_OSD_INCONSISTENT);
            __syncthreads();
            continue;
        }

        // ---- 4. OSD-CS candidate sweep on 64-row column ballots of G (G is dead afterwards)
        int t0 = -1, t1 = -1;
        uint32_t e[R];
#pragma unroll
        for (int k = 0; k < R; ++k) e[k] = sp[k];
        if (a.mode == OSD_CS) {
            const int nt = list_nonbasis(isb, perm, n, tl, scr);
            // lane i takes the ballot of column c0 + i from a bit transpose of words
            // c0 / 32 and c0 / 32 + 1 of the rows (rows of invalid lanes are zero); one
            // store per 64 columns and slot
            static_assert(NW % 2 == 0, "rows are read as word pairs");
            for (int c0 = 0; c0 < m; c0 += 64) {
                const int w = c0 >> 5;
                // the transpose's per-lane masks are rebuilt here rather than hoisted and
                // held across the shot loop, where they crowd the elimination's registers
                int ln = lane;
                asm volatile("" : "+v"(ln));
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const uint64_t bl = column_ballots(g[k][w], g[k][w + 1], ln);
                    if (c0 + lane < m) B[(size_t)(c0 + lane) * 16 + k * nwv + wid] = bl;
                }
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const uint64_t yb = __ballot(valid[k] && sp[k]);
                if (lane == 0) Y[k * nwv + wid] = yb;
            }
            if (tid == 0) *best64 = ~0ull;
            __syncthreads();
            uint32_t cost0 = 0;
            for (int w = 0; w < ngr; ++w) cost0 += __popcll(Y[w]);
            unsigned long long best = (unsigned long long)cost0 << 32;
            // candidates 0 .. nt - 1 flip one non-basis column, nt + pi the pair pi of the
            // first w; the enumeration index 1 + ci breaks cost ties.  One index space keeps
            // every thread at ceil((nt + npairs) / nth) candidates, and a thread issues the
            // column-table loads of QS candidates before it scores the first.
            const int w = a.order < nt ? a.order : nt;
            const int npairs = w * (w - 1) / 2;
            const int ncand = nt + npairs;
            constexpr int QS = 4;
            for (int cb = tid; cb < ncand; cb += QS * nth) {
                uint64_t ta[QS], tb[QS];
#pragma unroll
                for (int q = 0; q < QS; ++q) {
                    const int ci = cb + q * nth;
                    ta[q] = ~0ull;
                    tb[q] = ~0ull;
                    if (ci < nt) {
                        ta[q] = a.vn_tab[tl[ci]];
                    } else if (ci < ncand) {
                        int aa, bb;
                        pair_of(ci - nt, w, aa, bb);
                        ta[q] = a.vn_tab[tl[aa]];
                        tb[q] = a.vn_tab[tl[bb]];
                    }
                }
#pragma unroll
                for (int q = 0; q < QS; ++q) {
                    const int ci = cb + q * nth;
                    if (ci < ncand) {
                        const unsigned long long cost =
                            (ci < nt ? 1u : 2u) + ballot_cost((const uint4 *)B, (const uint4 *)Y, ngr, ta[q], tb[q]);
                        const unsigned long long key = (cost << 32) | (unsigned long long)(1 + ci);
                        best = key < best ? key : best;
                    }
                }
            }
            best = wave_min_u64(best);
            if (lane == 0) atomicMin(best64, best);
            __syncthreads();
            const unsigned idx = (unsigned)(*best64 & 0xFFFFFFFFull);
            if (idx >= 1 && idx <= (unsigned)nt) {
                t0 = tl[idx - 1];
            } else if (idx > (unsigned)nt) {
                int aa, bb;
                pair_of((int)idx - 1 - nt, w, aa, bb);
                t0 = tl[aa];
                t1 = tl[bb];
            }
            // each row's bit of the chosen candidate's reduced columns, from the ballots
            const uint64_t tab0 = t0 >= 0 ? a.vn_tab[t0] : ~0ull, tab1 = t1 >= 0 ? a.vn_tab[t1] : ~0ull;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const uint64_t xb = ballot_cost_mask(B, k * nwv + wid, tab0, tab1);
                e[k] ^= (uint32_t)(xb >> lane) & 1u;
            }
        }

        // ---- 5. e_S = s' + G H_T t on the basis, t on the rest; scatter to columns
        for (int ww = tid; ww < a.nw; ww += nth) cw[ww] = 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (valid[k] && piv[k] && e[k]) atomicOr(&cw[pcol[k] >> 5], 1u << (pcol[k] & 31));
        if (tid == 0) {
            if (t0 >= 0) atomicOr(&cw[t0 >> 5], 1u << (t0 & 31));
            if (t1 >= 0) atomicOr(&cw[t1 >> 5], 1u << (t1 & 31));
        }
        __syncthreads();
        for (int ww = tid; ww < a.nw; ww += nth) a.corr[shot * a.nw + ww] = cw[ww];
        if (tid == 0) a.flags[shot] = (uint8_t)FLAG_OSD;  // clears a serving ring's pending bit
        __syncthreads();
    }
}

}  // namespace

int osd_block_bytes(int m, int n, int lds_limit, int rows_per_lane, int i16, int *variant, int *mws, int *sort_p,
                    int *threads) {
    int P = 1;
    while (P < n) P <<= 1;
    int mw = (m + 31) / 32;
    int s = mw | 1;
    auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
    *sort_p = P;
    size_t common = al((size_t)n * 4) + al((size_t)n * 2) * 2 + al((size_t)n) + al((size_t)((n + 31) / 32) * 4) +
                    16 * 4 + 32 * 4 + 16;
    if (m < 1024) {  // m < 32 NW: bit m of every row is a zero bit
        int nw = m < 256 ? 8 : (m < 512 ? 16 : (m < 896 ? 28 : 32));
        const int r = rows_per_lane == 1 ? 1 : 2;
        *variant = 100 * r + nw;
        *mws = mw;
        *threads = 64 * ((m + 64 * r - 1) / (64 * r));
        int vb = 4;  // a vector of nw words occupies the next power of two bytes
        while (vb < nw * 4) vb <<= 1;
        return (int)reg_lds_layout(n, P, (n + 31) / 32, vb, i16).total;
    }
    *threads = OSD_THREADS;
    // pivot row words, s' ballots, and for G in global memory at large m its occupancy mask
    const size_t plist = 2 * al((size_t)mw * 4) + al((size_t)((m + 63) / 64) * 8);
    const size_t occb = m >= OSD_OCC_MIN_M ? al((size_t)osd_occ_words(m) * 4) : 0;
    size_t rows = al((size_t)m * 2) + al((size_t)m) * 2 + plist + occb + al((size_t)((n + 31) / 32) * 4) + 16 * 4 +
                  32 * 4 + 16;
    size_t rest = common + al((size_t)m * 2) + al((size_t)m) * 2 + plist;
    size_t gb = (size_t)m * s * 4;
    size_t with_g = al(gb > (size_t)P * 8 ? gb : (size_t)P * 8) + rest;
    if ((int64_t)with_g <= lds_limit) {
        *variant = 0;  // G in LDS
        *mws = s;
        return (int)with_g;
    }
    *mws = mw;
    if ((int64_t)(al((size_t)P * 8) + rest + occb) <= lds_limit) {
        *variant = -1;  // G in global memory
        return (int)(al((size_t)P * 8) + rest + occb);
    }
    *variant = -2;      // G and the per-column arrays in global memory
    // latency-bound steps: half-size blocks put more shots in flight per CU (LDS permitting)
    if (m <= 8 * OSD_THREADS) *threads = OSD_THREADS / 2;
    return (int)rows;
}

size_t osd_scratch_layout(int variant, int m, int n, int mws, int sort_p, int cs, size_t *cs_off) {
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
    *cs_off = 0;
    if (variant > 0) return (size_t)16 * m * 8;       // per-wave column ballots
    size_t b = 0;
    if (variant == -1) b = a256((size_t)m * mws * 4);  // G
    if (variant == -2)                                 // G, sort keys, sort columns, order, non-basis list, flags
        b = a256(a256((size_t)m * mws * 4) + a256((size_t)sort_p * 8) + al((size_t)n * 4) + 2 * al((size_t)n * 2) +
                 al((size_t)n));
    *cs_off = b;
    if (cs) b += a256((size_t)((m + 63) / 64) * m * 8);  // OSD-CS: 64-row ballots of G's columns
    return b;
}

size_t osd_scratch_bytes(int variant, int m, int n, int mws, int sort_p, int cs) {
    size_t c;
    return osd_scratch_layout(variant, m, n, mws, sort_p, cs, &c);
}

template <class K>
static hipError_t launch_k(K kern, const OsdArgs &a, int blocks, int threads, int lds, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), (size_t)lds, s, a);
    return hipGetLastError();
}

hipError_t launch_osd(const OsdArgs &a, int variant, int blocks, int threads, int lds, hipStream_t s) {
    switch (variant) {
    case 108: return launch_k(osd_reg_kernel<8, 1>, a, blocks, threads, lds, s);
    case 116: return launch_k(osd_reg_kernel<16, 1>, a, blocks, threads, lds, s);
    case 128: return launch_k(osd_reg_kernel<28, 1>, a, blocks, threads, lds, s);
    case 132: return launch_k(osd_reg_kernel<32, 1>, a, blocks, threads, lds, s);
    case 208: return launch_k(osd_reg_kernel<8, 2>, a, blocks, threads, lds, s);
    case 216: return launch_k(osd_reg_kernel<16, 2>, a, blocks, threads, lds, s);
    case 228: return launch_k(osd_reg_kernel<28, 2>, a, blocks, threads, lds, s);
    case 232: return launch_k(osd_reg_kernel<32, 2>, a, blocks, threads, lds, s);
    case 0: case -1: case -2: return launch_k(osd_lds_kernel, a, blocks, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

template <class K>
static hipError_t occ_k(K kern, int threads, int lds, int *out) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, kern, threads, (size_t)lds);
}

hipError_t osd_max_blocks_per_cu(int variant, int threads, int lds, int *out) {
    switch (variant) {
    case 108: return occ_k(osd_reg_kernel<8, 1>, threads, lds, out);
    case 116: return occ_k(osd_reg_kernel<16, 1>, threads, lds, out);
    case 128: return occ_k(osd_reg_kernel<28, 1>, threads, lds, out);
    case 132: return occ_k(osd_reg_kernel<32, 1>, threads, lds, out);
    case 208: return occ_k(osd_reg_kernel<8, 2>, threads, lds, out);
    case 216: return occ_k(osd_reg_kernel<16, 2>, threads, lds, out);
    case 228: return occ_k(osd_reg_kernel<28, 2>, threads, lds, out);
    case 232: return occ_k(osd_reg_kernel<32, 2>, threads, lds, out);
    case 0: case -1: case -2: return occ_k(osd_lds_kernel, threads, lds, out);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbp
