// zs_train.hip - dictionary generation on gfx950: Algorithm 1 (Sec. IV-C) with
// the rank of Eq. (1).
//
//   (pre-process  the corpus's ring IDs, Sec. IV-A: zs_preprocess, when asked)
//   count     every substring s of every line with Lmin <= |s| <= Lmax,
//             overlapping occurrences included: one thread per byte position
//             inserts the substrings that start there into an open-addressing
//             table in device memory (keys of up to 16 bytes as two 64-bit
//             words, inserted with a compare-and-swap on the first word);
//   compact   the occupied slots into candidate arrays;
//   select    T steps, each two launches: every candidate's overlap is raised
//             to its longest common substring with the pattern chosen in the
//             step before, its rank occ * (len - overlap) is computed, and a
//             block-wise then a single-block reduction picks the candidate of
//             highest rank (ties: longer, then bytewise smaller); it is
//             written out and removed from the candidates.  The steps stop
//             early when no candidate has a positive rank.
//
// The update_rank of Algorithm 1 and the overlap of Eq. (1) are read as: the
// overlap of a pattern at step t is the longest common substring it shares
// with any pattern selected before t.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/zsmiles.h"
#include "zs_common.hpp"

using namespace zs;

namespace {

constexpr uint64_t kLoMark = 1ull << 63;  // set in a slot's second word once it is written (bytes are < 0x80)
constexpr uint8_t kTaken = 0xFF;          // overlap value of a candidate already chosen
constexpr int kSelBlocks = 1024;          // workgroups of a selection step (partial results)
constexpr uint32_t kMaxSpin = 1u << 26;   // bound of an insertion's probe-and-wait loop

struct TrainState {
    WsHeader h;         // errors of the corpus (first bad line), through note_error
    uint32_t ncand;     // candidates after compaction
    uint32_t done;      // the selection has stopped (or never starts: an error)
    uint32_t full;      // an insertion found no free slot
    uint32_t pick_len;  // the pattern chosen in the last step
    uint64_t pick_hi, pick_lo;
    uint64_t pad[4];
};
static_assert(sizeof(TrainState) == 128, "state is 128 bytes");

struct Best {
    uint64_t rank, hi, lo;
    uint32_t len, idx;
    uint32_t valid, pad;
};

struct TrainArgs {
    const uint8_t* buf;     // the corpus to count (pre-processed copy, or the input)
    const uint64_t* off;    // its line offsets, n + 1
    uint64_t n;
    uint64_t in_mem;        // bytes of buf in memory (the last line may end one past it)
    uint32_t lmin, lmax;
    uint64_t* khi;          // table: first key word (0 = free)
    uint64_t* klo;          // second key word | kLoMark (0 = not yet written)
    uint32_t* cnt;          // occurrences
    uint64_t mask;          // table slots - 1
    uint64_t* c_hi;         // candidates
    uint64_t* c_lo;
    uint32_t* c_occ;
    uint8_t* c_len;
    uint8_t* c_ov;          // overlap so far, or kTaken
    uint64_t ccap;          // candidate capacity
    Best* part;
    TrainState* st;
};

__device__ inline uint64_t hash2(uint64_t a, uint64_t b) {
    // a 64-bit mix of the two key words (it only places keys in the table)
    uint64_t x = a * 0x9E3779B97F4A7C15ull ^ (b + 0x632BE59BD9B4E019ull + (a << 6) + (a >> 2));
    x ^= x >> 31;
    x *= 0xD6E8FEB86659FD93ull;
    x ^= x >> 32;
    return x;
}

__device__ inline uint64_t ld_relaxed(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One occurrence of the substring (hi, lo).  Returns false if the table has no
// free slot for it.  The slot's owner (the thread whose compare-and-swap put
// hi there) writes lo right after; a thread that finds hi already there but lo
// not yet written reads the slot again (it never waits inside this loop on a
// lane of its own wavefront: the owner's write comes first in program order).
__device__ inline bool insert(const TrainArgs& a, uint64_t hi, uint64_t lo) {
    uint64_t slot = hash2(hi, lo) & a.mask;
    uint64_t probes = 0;
    const uint64_t want = lo | kLoMark;
    for (uint32_t it = 0; it < kMaxSpin; it++) {
        uint64_t cur = ld_relaxed(&a.khi[slot]);
        bool won = false;
        if (cur == 0) {
            cur = atomicCAS((unsigned long long*)&a.khi[slot], 0ull, (unsigned long long)hi);
            won = cur == 0;
        }
        if (won) {
            __hip_atomic_store(&a.klo[slot], want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicAdd(&a.cnt[slot], 1u);
            return true;
        }
        if (cur == hi) {
            const uint64_t lv = ld_relaxed(&a.klo[slot]);
            if (lv == 0) continue;  // its owner has not written the second word yet
            if (lv == want) {
                atomicAdd(&a.cnt[slot], 1u);
                return true;
            }
        }
        slot = (slot + 1) & a.mask;
        if (++probes > a.mask) return false;
    }
    return false;
}

// Framing and bytes of every input line (the uncompressed corpus is used as it
// is): the same rules as compression (Sec. I; bytes 0x20..0x7E, at most
// ZS_MAX_LINE bytes, ended by a newline or the virtual one).
__global__ void __launch_bounds__(kWG) validate_kernel(const uint8_t* in, uint64_t in_bytes, const uint64_t* off,
                                                       uint64_t n, TrainState* st) {
    for (uint64_t k = (uint64_t)blockIdx.x * kWG + threadIdx.x; k < n; k += (uint64_t)gridDim.x * kWG) {
        const uint64_t a = off[k], b = off[k + 1];
        uint32_t kind = 0;
        if (b <= a || b > in_bytes + 1 || (b == in_bytes + 1 && k + 1 != n) || b - a - 1 > ZS_MAX_LINE) {
            kind = kErrInval;
        } else if (b <= in_bytes && in[b - 1] != '\n') {
            kind = kErrInval;
        } else {
            for (uint64_t p = a; p + 1 < b; p++) {
                const uint32_t c = in[p];
                if (c < 0x20 || c > 0x7E) {
                    kind = kErrCorrupt;
                    break;
                }
            }
        }
        if (kind) note_error(&st->h, k, kind);
    }
}

__global__ void train_init_kernel(TrainState* st, uint64_t* khi, uint64_t* klo, uint32_t* cnt, uint64_t slots,
                                  uint32_t* n_chosen) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        st->h.ticket = st->h.done = st->h.enospc = 0;
        st->h.errkey = ~0ull;
        st->h.total = 0;
        st->ncand = st->done = st->full = st->pick_len = 0;
        st->pick_hi = st->pick_lo = 0;
        *n_chosen = 0;
    }
    for (uint64_t k = i; k < slots; k += (uint64_t)gridDim.x * blockDim.x) {
        khi[k] = 0;
        klo[k] = 0;
        cnt[k] = 0;
    }
}

// The result word of the pre-processing launch becomes the corpus's error.
__global__ void take_preprocess_result(const ResultOut* pre, TrainState* st) {
    if (threadIdx.x == 0 && pre->code != 0)
        note_error(&st->h, (uint64_t)pre->first_bad, pre->code == ZS_EINVAL ? kErrInval : kErrCorrupt);
}

// One thread per byte position of the corpus: every substring starting there,
// of Lmin..Lmax bytes, that stays inside its line.
__global__ void __launch_bounds__(kWG) count_kernel(TrainArgs a) {
    if (a.st->h.errkey != ~0ull || a.n == 0) return;
    const uint64_t lo = a.off[0];
    const uint64_t hi = min(a.off[a.n], a.in_mem);
    bool full = false;
    for (uint64_t p = lo + (uint64_t)blockIdx.x * kWG + threadIdx.x; p < hi; p += (uint64_t)gridDim.x * kWG) {
        uint64_t w0 = 0, w1 = 0;
        for (uint32_t L = 1; L <= a.lmax; L++) {
            const uint64_t q = p + L - 1;
            if (q >= hi) break;
            const uint64_t c = a.buf[q];
            if (c == '\n') break;
            if (L <= 8) w0 |= c << (64 - 8 * L);
            else w1 |= c << (64 - 8 * (L - 8));
            if (L >= a.lmin && !insert(a, w0, w1)) full = true;
        }
    }
    if (full) atomicOr(&a.st->full, 1u);
}

__device__ inline uint32_t key_len(uint64_t hi, uint64_t lo) {
    // bytes are nonzero and packed from the top: the length is the number of nonzero bytes
    uint32_t n = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) n += ((hi >> (56 - 8 * j)) & 0xFF) != 0;
#pragma unroll
    for (int j = 0; j < 8; j++) n += ((lo >> (56 - 8 * j)) & 0xFF) != 0;
    return n;
}

__global__ void __launch_bounds__(kWG) compact_kernel(TrainArgs a) {
    for (uint64_t k = (uint64_t)blockIdx.x * kWG + threadIdx.x; k <= a.mask; k += (uint64_t)gridDim.x * kWG) {
        const uint64_t h = a.khi[k];
        if (!h) continue;
        const uint64_t l = a.klo[k] & ~kLoMark;
        const uint32_t i = atomicAdd(&a.st->ncand, 1u);
        if (i >= a.ccap) continue;  // cannot happen: the capacity bounds the occurrences
        a.c_hi[i] = h;
        a.c_lo[i] = l;
        a.c_occ[i] = a.cnt[k];
        a.c_len[i] = (uint8_t)key_len(h, l);
        a.c_ov[i] = 0;
    }
}

// ---- 128-bit helpers on (hi, lo) pairs: byte i of a pattern sits at bits
//      127-8i .. 120-8i (byte 0 at the top of hi)
struct U128 {
    uint64_t h, l;
};
__device__ inline U128 shr(U128 x, uint32_t s) {  // s < 128
    if (s == 0) return x;
    if (s >= 64) return {0, x.h >> (s - 64)};
    return {x.h >> s, (x.l >> s) | (x.h << (64 - s))};
}
__device__ inline U128 shl(U128 x, uint32_t s) {
    if (s == 0) return x;
    if (s >= 64) return {x.l << (s - 64), 0};
    return {(x.h << s) | (x.l >> (64 - s)), x.l << s};
}
// bytes [0, n) set to 0xFF
__device__ inline U128 top_bytes(uint32_t n) {
    if (n == 0) return {0, 0};
    return shl({~0ull, ~0ull}, 128 - 8 * n);
}
__device__ inline uint64_t zero_flags(uint64_t x) {
    return ~(((x & 0x7F7F7F7F7F7F7F7Full) + 0x7F7F7F7F7F7F7F7Full) | x) & 0x8080808080808080ull;
}

// Longest common substring of a (la bytes) and b (lb bytes), both at most 16:
// for every alignment d of b against a (a[i] against b[i - d]) the positions
// where the bytes agree are flagged, and the longest run of flags is found by
// repeated AND with the flags shifted by one byte.  `floor`: the caller only
// needs the result when it exceeds floor.
__device__ inline uint32_t lcs16(U128 a, uint32_t la, U128 b, uint32_t lb, uint32_t floor) {
    uint32_t best = floor;
    const U128 ma = top_bytes(la);
    for (int d = -(int)lb + 1; d <= (int)la - 1; d++) {
        const U128 w = d >= 0 ? shr(b, 8u * (uint32_t)d) : shl(b, 8u * (uint32_t)(-d));
        const uint32_t s = (uint32_t)max(d, 0), e = (uint32_t)min((int)la, (int)lb + d);
        if (e <= s + best) continue;  // this alignment overlaps in too few bytes
        const U128 vm = top_bytes(e), vs = top_bytes(s);
        U128 f = {zero_flags(a.h ^ w.h) & vm.h & ~vs.h & ma.h, zero_flags(a.l ^ w.l) & vm.l & ~vs.l & ma.l};
        uint32_t r = 0;
        while (f.h | f.l) {
            const U128 g = shl(f, 8);
            f = {f.h & g.h, f.l & g.l};
            r++;
        }
        best = max(best, r);
    }
    return best;
}

__device__ inline bool ahead(const Best& x, const Best& y) {
    if (!y.valid) return x.valid != 0;
    if (!x.valid) return false;
    if (x.rank != y.rank) return x.rank > y.rank;
    if (x.len != y.len) return x.len > y.len;
    if (x.hi != y.hi) return x.hi < y.hi;
    return x.lo < y.lo;
}

__device__ inline Best shfl_best(const Best& b, int lane) {
    Best o;
    o.rank = __shfl(b.rank, lane, 64);
    o.hi = __shfl(b.hi, lane, 64);
    o.lo = __shfl(b.lo, lane, 64);
    o.len = __shfl(b.len, lane, 64);
    o.idx = __shfl(b.idx, lane, 64);
    o.valid = __shfl(b.valid, lane, 64);
    o.pad = 0;
    return o;
}

// The best of the workgroup's values (all threads call; result in thread 0).
__device__ inline Best block_best(Best b) {
    __shared__ Best wbest[kWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const Best o = shfl_best(b, lane ^ d);
        if (ahead(o, b)) b = o;
    }
    if (lane == 0) wbest[w] = b;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < kWaves; k++)
            if (ahead(wbest[k], b)) b = wbest[k];
    __syncthreads();
    return b;
}

// Step t: the overlaps against the pattern chosen at step t-1 (Eq. (1)), then
// the best rank of this workgroup's candidates.
__global__ void __launch_bounds__(kWG) select_kernel(TrainArgs a, uint32_t t) {
    if (a.st->done) return;
    const uint32_t nc = min((uint64_t)a.st->ncand, a.ccap);
    const U128 pk = {a.st->pick_hi, a.st->pick_lo};
    const uint32_t pl = a.st->pick_len;
    Best b;
    b.valid = 0;
    b.rank = b.hi = b.lo = 0;
    b.len = b.idx = b.pad = 0;
    for (uint32_t i = blockIdx.x * kWG + threadIdx.x; i < nc; i += gridDim.x * kWG) {
        uint32_t ov = a.c_ov[i];
        if (ov == kTaken) continue;
        const uint32_t len = a.c_len[i];
        const U128 c = {a.c_hi[i], a.c_lo[i]};
        if (t > 0 && ov < len) {
            const uint32_t l = lcs16(c, len, pk, pl, ov);
            if (l > ov) {
                ov = l;
                a.c_ov[i] = (uint8_t)ov;
            }
        }
        Best x;
        x.rank = (uint64_t)a.c_occ[i] * (uint64_t)(len - ov);
        x.hi = c.h;
        x.lo = c.l;
        x.len = len;
        x.idx = i;
        x.valid = 1;
        x.pad = 0;
        if (ahead(x, b)) b = x;
    }
    b = block_best(b);
    if (threadIdx.x == 0) a.part[blockIdx.x] = b;
}

// The step's choice: the best of the partial results, written out as pattern t.
__global__ void __launch_bounds__(kWG) pick_kernel(TrainArgs a, uint32_t t, uint32_t nparts, uint8_t* pat,
                                                   uint8_t* pat_len, uint32_t* n_chosen) {
    if (a.st->done) return;
    Best b;
    b.valid = 0;
    b.rank = b.hi = b.lo = 0;
    b.len = b.idx = b.pad = 0;
    for (uint32_t k = threadIdx.x; k < nparts; k += kWG)
        if (ahead(a.part[k], b)) b = a.part[k];
    b = block_best(b);
    if (threadIdx.x == 0) {
        if (!b.valid || b.rank == 0) {
            a.st->done = 1;  // no candidate left with a positive rank
        } else {
            a.c_ov[b.idx] = kTaken;
            a.st->pick_hi = b.hi;
            a.st->pick_lo = b.lo;
            a.st->pick_len = b.len;
            for (int j = 0; j < 8; j++) {
                pat[(uint64_t)t * 16 + j] = (uint8_t)(b.hi >> (56 - 8 * j));
                pat[(uint64_t)t * 16 + 8 + j] = (uint8_t)(b.lo >> (56 - 8 * j));
            }
            pat_len[t] = (uint8_t)b.len;
            *n_chosen = t + 1;
        }
    }
}

// Stop before the first step when the corpus had an error or the table filled.
__global__ void select_gate_kernel(TrainState* st) {
    if (threadIdx.x == 0 && (st->h.errkey != ~0ull || st->full)) st->done = 1;
}

__global__ void train_result_kernel(TrainState* st, ResultOut* res, uint32_t* n_chosen) {
    if (threadIdx.x != 0) return;
    int32_t code = 0;
    int64_t fb = -1;
    const uint64_t ek = st->h.errkey;
    if (ek != ~0ull) {
        fb = (int64_t)(ek >> 3);
        code = (ek & 7) == kErrInval ? ZS_EINVAL : ZS_ECORRUPT;
        *n_chosen = 0;
    } else if (st->full) {
        code = ZS_ENOSPC;
        *n_chosen = 0;
    }
    res->code = code;
    res->reserved = 0;
    res->first_bad = fb;
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of a training call, carved in this order.
struct TrainWs {
    TrainState* st;
    ResultOut* pre_res;
    void* pre_ws;
    size_t pre_ws_bytes;
    uint8_t* pre;
    uint64_t pre_cap;
    uint64_t* pre_off;
    uint64_t* khi;
    uint64_t* klo;
    uint32_t* cnt;
    uint64_t slots;
    uint64_t* c_hi;
    uint64_t* c_lo;
    uint32_t* c_occ;
    uint8_t* c_len;
    uint8_t* c_ov;
    uint64_t ccap;
    Best* part;
    size_t bytes;
};

TrainWs train_ws(void* ws, uint64_t in_bytes, uint64_t n, uint32_t lmin, uint32_t lmax, bool prep) {
    TrainWs w;
    uint8_t* base = (uint8_t*)ws;
    size_t o = 0;
    auto take = [&](size_t b) {
        uint8_t* p = base ? base + o : nullptr;
        o += al256(b);
        return p;
    };
    // corpus bytes counted: a pre-processed line is at most three times its raw length
    const uint64_t corpus = prep ? 3 * in_bytes + n + 16 : in_bytes;
    // every occurrence may be a new substring: the table holds twice that many slots
    const uint64_t occ = std::max<uint64_t>(1, corpus * (uint64_t)(lmax - lmin + 1));
    w.slots = next_pow2(std::max<uint64_t>(2 * occ, 1024));
    w.ccap = std::min<uint64_t>(occ, w.slots);
    w.st = (TrainState*)take(sizeof(TrainState));
    w.pre_res = (ResultOut*)take(sizeof(ResultOut));
    w.pre_ws_bytes = prep ? zs_workspace_bytes(ZS_OP_COMPRESS, n) : 0;
    w.pre_ws = take(w.pre_ws_bytes);
    w.pre_cap = prep ? corpus : 0;
    w.pre = take(w.pre_cap);
    w.pre_off = (uint64_t*)take(prep ? (n + 1) * 8 : 0);
    w.khi = (uint64_t*)take(w.slots * 8);
    w.klo = (uint64_t*)take(w.slots * 8);
    w.cnt = (uint32_t*)take(w.slots * 4);
    w.c_hi = (uint64_t*)take(w.ccap * 8);
    w.c_lo = (uint64_t*)take(w.ccap * 8);
    w.c_occ = (uint32_t*)take(w.ccap * 4);
    w.c_len = take(w.ccap);
    w.c_ov = take(w.ccap);
    w.part = (Best*)take(sizeof(Best) * kSelBlocks);
    w.bytes = o;
    return w;
}

bool bad_params(uint32_t lmin, uint32_t lmax, uint32_t T) {
    return lmin < 1 || lmin > lmax || lmax > ZS_LMAX_CAP || T > ZS_TRAIN_MAX_T;
}

}  // namespace

extern "C" {

size_t zs_train_workspace_bytes(uint64_t in_bytes, uint64_t n_lines, uint32_t lmin, uint32_t lmax, uint32_t flags) {
    if (bad_params(lmin, lmax, 0)) return 0;
    return train_ws(nullptr, in_bytes, n_lines, lmin, lmax, (flags & ZS_F_PREPROCESS) != 0).bytes;
}

zs_status zs_train_patterns(const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off, uint64_t n_lines,
                            uint32_t flags, uint32_t lmin, uint32_t lmax, uint32_t T, uint8_t* pat,
                            uint8_t* pat_len, uint32_t* n_chosen, void* ws, size_t ws_bytes, zs_result* res,
                            void* stream) {
    if (!in_off || !ws || !res || !n_chosen || (!in && in_bytes) || ((!pat || !pat_len) && T)) return ZS_EINVAL;
    if (flags & ~ZS_F_PREPROCESS) return ZS_EINVAL;
    if (bad_params(lmin, lmax, T)) return ZS_EINVAL;
    const bool prep = (flags & ZS_F_PREPROCESS) != 0;
    TrainWs w = train_ws(ws, in_bytes, n_lines, lmin, lmax, prep);
    if (ws_bytes < w.bytes) return ZS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    const uint32_t fill_grid = (uint32_t)std::min<uint64_t>((w.slots + 255) / 256, (uint64_t)cus * 16);
    hipLaunchKernelGGL(train_init_kernel, dim3(fill_grid), dim3(256), 0, s, w.st, w.khi, w.klo, w.cnt, w.slots,
                       n_chosen);
    TrainArgs a;
    a.lmin = lmin;
    a.lmax = lmax;
    a.khi = w.khi;
    a.klo = w.klo;
    a.cnt = w.cnt;
    a.mask = w.slots - 1;
    a.c_hi = w.c_hi;
    a.c_lo = w.c_lo;
    a.c_occ = w.c_occ;
    a.c_len = w.c_len;
    a.c_ov = w.c_ov;
    a.ccap = w.ccap;
    a.part = w.part;
    a.st = w.st;
    a.n = n_lines;
    if (prep) {
        // the corpus's pre-processed copy, framed like the input (bad lines come out empty
        // and are reported)
        zs_status rc = zs_preprocess(in, in_bytes, in_off, n_lines, w.pre, w.pre_cap, w.pre_off, w.pre_ws,
                                     w.pre_ws_bytes, (zs_result*)w.pre_res, stream);
        if (rc != ZS_OK) return rc;
        hipLaunchKernelGGL(take_preprocess_result, dim3(1), dim3(64), 0, s, w.pre_res, w.st);
        a.buf = w.pre;
        a.off = w.pre_off;
        a.in_mem = w.pre_cap;
    } else {
        const uint32_t vg = (uint32_t)std::min<uint64_t>((n_lines + kWG - 1) / kWG + 1, (uint64_t)cus * 8);
        hipLaunchKernelGGL(validate_kernel, dim3(vg), dim3(kWG), 0, s, in, in_bytes, in_off, n_lines, w.st);
        a.buf = in;
        a.off = in_off;
        a.in_mem = in_bytes;
    }
    hipLaunchKernelGGL(count_kernel, dim3((uint32_t)cus * 8), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(compact_kernel, dim3(fill_grid), dim3(kWG), 0, s, a);
    hipLaunchKernelGGL(select_gate_kernel, dim3(1), dim3(64), 0, s, w.st);
    for (uint32_t t = 0; t < T; t++) {
        hipLaunchKernelGGL(select_kernel, dim3(kSelBlocks), dim3(kWG), 0, s, a, t);
        hipLaunchKernelGGL(pick_kernel, dim3(1), dim3(kWG), 0, s, a, t, (uint32_t)kSelBlocks, pat, pat_len, n_chosen);
    }
    hipLaunchKernelGGL(train_result_kernel, dim3(1), dim3(64), 0, s, w.st, (ResultOut*)res, n_chosen);
    return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
}

}  // extern "C"
