// zs_kernels.hip - gfx950 kernels and C ABI of the ZSMILES codec.
//
// Compression (Sec. IV-A, IV-D-1), one workgroup of 256 threads per tile of
// 256 lines, one lane per line:
//   load     the tile's bytes HBM -> LDS with 16-byte loads;
//   ring IDs forward scan per lane: brackets, ring labels, pairing, the ID of
//            each ring from the labels that closed inside it (Sec. IV-A), the
//            new label text marked in place;
//   expand   markers -> the pre-processed line, packed by a block scan;
//   parse    backward scan per lane: one automaton step gives the patterns
//            that start at the position, one (min,+) step over a window of
//            the next LK costs gives cost[i] and the longest optimal edge;
//            the chosen code is written over the consumed byte;
//   offsets  block scan of line lengths, decoupled look-back across tiles;
//   emit     forward walk of the chosen edges into an LDS stage, flushed with
//            16-byte stores.
// Decompression (Sec. IV-D-2) is byte-parallel: whole lines in LDS, escape
// parity from a scan of space runs, expansion lengths from the LEN table, a
// block scan for positions, expansions written to an LDS stage.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/zsmiles.h"
#include "zs_common.hpp"
#include "zs_tables.hpp"

using namespace zs;

extern "C" int zsi_compile_dict(const uint8_t* len, const uint8_t* exp, std::vector<uint8_t>* blob_out);

namespace {

// ============================================================================
// Compression
// ============================================================================

constexpr int kCL = 256;              // lines per tile (one per thread)
constexpr int kRawCap = 14336;        // LDS bytes for the raw lines of a batch
constexpr int kPreCap = 14336;        // LDS bytes for their pre-processed form
constexpr int kTabLane = 96;          // per-lane ring tables: 16 open slots u32 + 16 last-close u16
constexpr int kOpenSlots = 16;
constexpr int kIdFast = 16;
constexpr int kGenLane = 400;         // per-lane ring tables in global memory (any line):
                                      // 100 open positions u16 + 100 last-close u16
static_assert(kPreCap >= 3 * (int)ZS_MAX_LINE, "a pre-processed line must fit");
static_assert(kRawCap >= (int)ZS_MAX_LINE + 1 + 16, "a raw line must fit");

constexpr int kStageCap = kRawCap + kCL * kTabLane;  // RAW + TABS, reused for output
constexpr uint8_t kSkip = 0x7F;                      // marker: byte dropped by pre-processing
constexpr uint8_t kIdMark = 0x80;                    // marker: ring-label with ID (low 7 bits)

struct CompressLds {
    uint32_t tab_bytes;  // dictionary part staged
    uint32_t raw, tabs, pre, esc, cost, eoff, off, misc;
    uint32_t total;
};

__host__ __device__ inline CompressLds compress_lds(uint32_t tab_bytes) {
    CompressLds L;
    L.tab_bytes = align16(tab_bytes);
    uint32_t o = L.tab_bytes;
    L.raw = o;  o += kRawCap;
    L.tabs = o; o += kCL * kTabLane;
    L.pre = o;  o += kPreCap;
    L.esc = o;  o += kPreCap / 8;
    L.cost = o; o += kCL * 4;
    L.eoff = o; o += kCL * 4;
    L.off = o;  o += (kCL + 1) * 8;
    L.misc = o; o += 256;
    L.total = align16(o);
    return L;
}

struct CompressArgs {
    const uint8_t* tables;  // device image
    uint32_t tab_bytes;     // bytes of the image staged (prefix up to EXP)
    const uint8_t* in;
    uint64_t in_bytes;
    const uint64_t* in_off;
    uint64_t n;
    uint8_t* out;
    uint64_t out_cap;
    uint64_t* out_off;
    uint32_t flags;
    uint32_t ntiles;
    WsHeader* ws;
    uint64_t* status;
    uint8_t* gen;           // general ring tables, kGenLane bytes per (workgroup, lane)
    ResultOut* res;
};

struct Dict {
    const TableHeader* h;
    const uint8_t* len;
    const uint8_t* col;
    const uint8_t* code1;
    const uint16_t* trans;
    const uint32_t* outk;
    const uint8_t* code;
};

__device__ inline bool is_digit(uint32_t c) { return c - '0' < 10u; }

// Per-lane state of one line inside a batch.
struct LineState {
    uint32_t R;     // raw offset in RAW
    uint32_t len;   // raw length (newline excluded)
    uint32_t m;     // pre-processed length (0 for a bad line)
    uint32_t P;     // offset in PRE
    bool in;        // this lane holds a line of the batch
    bool bad;       // framing or byte error: the output line is empty
};

// Ring-ID pass over one raw line held in RAW[R .. R+len), writing markers in
// place.  Tables live wherever `open`/`last` point (LDS for the fast path,
// global memory for the general one).  Returns false when the line is
// malformed (then the caller restores it); *delta receives m - len.
// open: nslots u32 entries, slot = value % nslots, entry ((pos+1) << 8 | value);
// last: nid u16 entries, (position of the latest closing label with that ID) + 1.
// *overflow is set when the tables are too small for the line.
template <typename OpenT, typename LastT>
__device__ inline bool ring_pass(uint8_t* raw, uint32_t R, const uint16_t* labels, uint32_t nlab, OpenT* open,
                                 uint32_t nslots, LastT* last, uint32_t nid, int* delta, bool* overflow) {
    int opens = 0, dl = 0;
    for (uint32_t q = 0; q < nlab; q++) {
        uint32_t p = labels[q];
        uint32_t c0 = raw[R + p];
        uint32_t v, tl;
        if (c0 == '%') {
            v = (raw[R + p + 1] - '0') * 10u + (raw[R + p + 2] - '0');
            tl = 3;
        } else {
            v = c0 - '0';
            tl = 1;
        }
        uint32_t slot = v % nslots;
        uint32_t e = open[slot];
        if (e == 0) {
            open[slot] = ((p + 1) << 8) | v;
            opens++;
        } else if ((e & 0xFF) == v) {
            uint32_t o = (e >> 8) - 1;
            open[slot] = 0;
            opens--;
            uint32_t id = 0;
            while (id < nid && (uint32_t)last[id] > o + 1) id++;
            if (id >= nid) {
                *overflow = true;
                return false;
            }
            last[id] = (LastT)(p + 1);
            uint32_t to = (raw[R + o] == '%') ? 3u : 1u;
            raw[R + o] = (uint8_t)(kIdMark | id);
            if (to == 3) raw[R + o + 1] = raw[R + o + 2] = kSkip;
            raw[R + p] = (uint8_t)(kIdMark | id);
            if (tl == 3) raw[R + p + 1] = raw[R + p + 2] = kSkip;
            int nlen = id < 10 ? 1 : 3;
            dl += (nlen - (int)to) + (nlen - (int)tl);
        } else {
            *overflow = true;
            return false;
        }
    }
    *delta = dl;
    return opens == 0;
}

__device__ inline void restore_line(uint8_t* raw, uint32_t R, const uint8_t* src, uint32_t len) {
    for (uint32_t i = 0; i < len; i++) raw[R + i] = src[i];
}

template <int LK>
struct Compressor {
    const CompressArgs& A;
    uint8_t* smem;
    CompressLds L;
    Dict D;
    uint32_t C;  // automaton columns

    __device__ Compressor(const CompressArgs& a, uint8_t* s) : A(a), smem(s) {
        L = compress_lds(a.tab_bytes);
        D.h = (const TableHeader*)smem;
        D.len = smem + D.h->off_len;
        D.col = smem + D.h->off_col;
        D.code1 = smem + D.h->off_code1;
        D.trans = (const uint16_t*)(smem + D.h->off_trans);
        D.outk = (const uint32_t*)(smem + D.h->off_outk);
        D.code = smem + D.h->off_code;
        C = D.h->ncols;
    }

    __device__ uint64_t* OFF() { return (uint64_t*)(smem + L.off); }
    __device__ uint32_t* COST() { return (uint32_t*)(smem + L.cost); }
    __device__ uint32_t* EOFF() { return (uint32_t*)(smem + L.eoff); }
    __device__ uint32_t* MISC() { return (uint32_t*)(smem + L.misc); }
    __device__ uint8_t* RAW() { return smem + L.raw; }
    __device__ uint8_t* PRE() { return smem + L.pre; }
    __device__ uint32_t* ESC() { return (uint32_t*)(smem + L.esc); }

    // Framing of line j of the tile (OFF staged).  0 = ok, else error kind.
    __device__ uint32_t frame_error(uint64_t k0, uint32_t j) {
        uint64_t a = OFF()[j], b = OFF()[j + 1];
        if (b <= a || b > A.in_bytes + 1) return kErrInval;
        if (b - a - 1 > ZS_MAX_LINE) return kErrInval;
        if (b == A.in_bytes + 1 && k0 + j + 1 != A.n) return kErrInval;
        return 0;
    }

    // Process lines [b0, ...) of the tile as one batch: load, ring IDs, expand,
    // parse.  Fills COST for the batch lines and returns b1.  The per-lane
    // state needed for emission is left in `st`.
    __device__ uint32_t batch(uint64_t k0, uint32_t nl, uint32_t b0, bool regular, LineState& st) {
        uint32_t* misc = MISC();
        uint64_t* off = OFF();
        const uint32_t tid = threadIdx.x;
        // ---- extent of the batch
        if (tid == 0) misc[0] = nl;
        __syncthreads();
        {
            uint32_t j = b0 + tid;
            if (j < nl) {
                bool stop;
                if (!regular) {
                    stop = j > b0;  // irregular tile: one line per batch
                } else {
                    uint64_t lo = off[b0];
                    stop = (off[j + 1] - lo) + 16 > (uint64_t)kRawCap;
                    if (j == b0) stop = false;
                }
                if (stop) atomicMin(&misc[0], j);
            }
        }
        __syncthreads();
        uint32_t b1 = misc[0];
        __syncthreads();
        // ---- load
        const uint32_t fe0 = frame_error(k0, b0);
        uint64_t lo = off[b0];
        uint64_t hi = off[b1];
        if (hi > A.in_bytes) hi = A.in_bytes;
        uintptr_t a0 = ((uintptr_t)(A.in + lo)) & ~(uintptr_t)15;
        uint32_t base_off = (uint32_t)((uintptr_t)(A.in + lo) - a0);
        uint8_t* raw = RAW();
        if (fe0 == 0) load_range(A.in, A.in_bytes, lo, hi, a0, raw);
        __syncthreads();
        if (tid == 0 && fe0 == 0 && off[b1] == A.in_bytes + 1) raw[(uint32_t)(off[b1] - 1 - lo) + base_off] = '\n';
        // clear this lane's fast ring tables
        {
            uint4* t4 = (uint4*)(smem + L.tabs + tid * kTabLane);
#pragma unroll
            for (int k = 0; k < kTabLane / 16; k++) t4[k] = make_uint4(0, 0, 0, 0);
        }
        __syncthreads();
        // ---- per line: framing, bytes, ring IDs
        const uint32_t j = b0 + tid;
        st.in = j < b1;
        st.bad = false;
        st.len = 0;
        st.m = 0;
        st.R = 0;
        bool overflow = false, malformed = false;
        int delta = 0;
        uint16_t* pre16 = (uint16_t*)PRE();
        uint32_t listbase = 0, nlab = 0;
        const bool prep = (A.flags & ZS_F_PREPROCESS) != 0;
        if (st.in) {
            uint32_t fe = frame_error(k0, j);
            if (fe == 0) {
                st.len = (uint32_t)(off[j + 1] - off[j] - 1);
                st.R = (uint32_t)(off[j] - lo) + base_off;
                if (raw[st.R + st.len] != '\n') fe = kErrInval;
            }
            if (fe) {
                st.bad = true;
                note_error(A.ws, k0 + j, fe);
            }
        }
        if (st.in && !st.bad) {
            // forward scan: validate bytes, brackets, collect ring labels
            uint32_t inbr = 0, corrupt = 0;
            listbase = (st.R + 1) >> 1;  // u16 index into PRE
            const uint32_t cap = st.len >> 1;
            bool list_over = false;
            for (uint32_t i = 0; i < st.len; i++) {
                uint32_t c = raw[st.R + i];
                corrupt |= (c < 0x20u) | (c > 0x7Eu);
                if (c == '[') {
                    malformed |= inbr != 0;
                    inbr = 1;
                } else if (c == ']') {
                    malformed |= inbr == 0;
                    inbr = 0;
                } else if (!inbr) {
                    bool lab = false;
                    uint32_t adv = 0;
                    if (is_digit(c)) {
                        lab = true;
                    } else if (c == '%') {
                        if (i + 2 < st.len && is_digit(raw[st.R + i + 1]) && is_digit(raw[st.R + i + 2])) {
                            lab = true;
                            adv = 2;
                        } else {
                            malformed = true;
                        }
                    }
                    if (lab) {
                        if (nlab < cap) pre16[listbase + nlab] = (uint16_t)i;
                        else list_over = true;
                        nlab++;
                    }
                    i += adv;
                }
            }
            malformed |= inbr != 0;
            if (corrupt) {
                st.bad = true;
                note_error(A.ws, k0 + j, kErrCorrupt);
            } else if (prep && !malformed) {
                if (list_over) {
                    overflow = true;
                } else {
                    uint32_t* open = (uint32_t*)(smem + L.tabs + tid * kTabLane);
                    uint16_t* last = (uint16_t*)(open + kOpenSlots);
                    bool ok = ring_pass(raw, st.R, pre16 + listbase, nlab, open, kOpenSlots, last, kIdFast, &delta,
                                        &overflow);
                    if (!ok && !overflow) {
                        malformed = true;
                        restore_line(raw, st.R, A.in + off[j], st.len);
                    }
                }
            }
        }
        // ---- general path: lines whose rings do not fit the fast tables
        if (overflow) {
            restore_line(raw, st.R, A.in + off[j], st.len);
            uint16_t* open = (uint16_t*)(A.gen + ((uint64_t)blockIdx.x * kWG + tid) * kGenLane);
            uint16_t* last = open + 100;
            for (int k = 0; k < 100; k++) { open[k] = 0; last[k] = 0; }
            // labels again, straight from the raw bytes (the list may be incomplete)
            int dl = 0, opens = 0;
            bool bad_ring = false;
            uint32_t inbr = 0;
            for (uint32_t i = 0; i < st.len && !bad_ring; i++) {
                uint32_t c = raw[st.R + i];
                if (c == '[') { inbr = 1; continue; }
                if (c == ']') { inbr = 0; continue; }
                if (inbr) continue;
                uint32_t v, tl;
                if (is_digit(c)) { v = c - '0'; tl = 1; }
                else if (c == '%') { v = (raw[st.R + i + 1] - '0') * 10u + (raw[st.R + i + 2] - '0'); tl = 3; }
                else continue;
                uint32_t e = open[v];
                if (e == 0) {
                    open[v] = (uint16_t)(i + 1);
                    opens++;
                } else {
                    uint32_t o = e - 1;
                    open[v] = 0;
                    opens--;
                    uint32_t id = 0;
                    while (id < 100 && (uint32_t)last[id] > o + 1) id++;
                    if (id >= 100) { bad_ring = true; break; }
                    last[id] = (uint16_t)(i + 1);
                    uint32_t to = (raw[st.R + o] == '%') ? 3u : 1u;
                    raw[st.R + o] = (uint8_t)(kIdMark | id);
                    if (to == 3) raw[st.R + o + 1] = raw[st.R + o + 2] = kSkip;
                    raw[st.R + i] = (uint8_t)(kIdMark | id);
                    if (tl == 3) raw[st.R + i + 1] = raw[st.R + i + 2] = kSkip;
                    int nlen = id < 10 ? 1 : 3;
                    dl += (nlen - (int)to) + (nlen - (int)tl);
                }
                i += tl - 1;
            }
            if (bad_ring || opens != 0) {
                malformed = true;
                restore_line(raw, st.R, A.in + off[j], st.len);
            } else {
                delta = dl;
            }
        }
        if (st.in && !st.bad) st.m = (prep && !malformed) ? (uint32_t)((int)st.len + delta) : st.len;
        // ---- pack the pre-processed lines; cut the batch where PRE is full
        uint32_t total;
        uint32_t P = block_excl_scan(st.in ? st.m : 0u, misc + 4, &total);
        st.P = P;
        if (tid == 0) misc[0] = b1;
        __syncthreads();
        if (st.in && P + st.m > (uint32_t)kPreCap) atomicMin(&misc[0], j);
        __syncthreads();
        uint32_t b1c = misc[0];
        __syncthreads();
        st.in = st.in && j < b1c;
        b1 = b1c;
        // ---- expand markers into PRE
        uint8_t* pre = PRE();
        if (st.in && !st.bad) {
            uint32_t w = st.P;
            for (uint32_t i = 0; i < st.len; i++) {
                uint32_t c = raw[st.R + i];
                if (c < kSkip) {
                    pre[w++] = (uint8_t)c;
                } else if (c >= kIdMark) {
                    uint32_t id = c & 0x7F;
                    if (id < 10) {
                        pre[w++] = (uint8_t)('0' + id);
                    } else {
                        pre[w++] = '%';
                        pre[w++] = (uint8_t)('0' + id / 10);
                        pre[w++] = (uint8_t)('0' + id % 10);
                    }
                }
            }
        }
        // clear the escape bits of the batch
        {
            uint32_t words = (kPreCap + 31) / 32;
            uint32_t* esc = ESC();
            for (uint32_t k = tid; k < words; k += kWG) esc[k] = 0;
        }
        __syncthreads();
        // ---- parse (backward): automaton + (min,+) window
        uint32_t cost = 0;
        {
            const uint32_t m = (st.in && !st.bad) ? st.m : 0u;
            uint32_t mx = m;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, 64));
            uint32_t V[LK];
            V[0] = 32u;
#pragma unroll
            for (int k = 1; k < LK; k++) V[k] = 0xFFFFFFFFu;
            uint32_t s = 0;
            uint32_t* esc = ESC();
            for (uint32_t it = 0; it < mx; it++) {
                if (it < m) {
                    const uint32_t pos = st.P + (m - 1 - it);
                    const uint32_t c = pre[pos];
                    s = D.trans[s * C + D.col[c]];
                    const uint32_t* ok = D.outk + s * LK;
                    uint32_t K = V[0] + 63u;
#pragma unroll
                    for (int k = 0; k < LK; k++) K = min(K, V[k] | ok[k]);
                    const uint32_t ch = 31u - (K & 31u);
                    uint32_t tok;
                    if (ch == 0) {
                        tok = c;
                        atomicOr(&esc[pos >> 5], 1u << (pos & 31));
                    } else if (ch == 1) {
                        tok = D.code1[c];
                    } else {
                        tok = D.code[s * LK + ch - 1];
                    }
                    pre[pos] = (uint8_t)tok;
#pragma unroll
                    for (int k = LK - 1; k > 0; k--) V[k] = V[k - 1];
                    V[0] = (K | 31u) + 1u;
                }
            }
            cost = (V[0] >> 5) - 1u;
        }
        if (st.in) COST()[j] = st.bad ? 0u : cost;
        __syncthreads();
        return b1;
    }

    // Emit the lines of the batch held in LDS into the output, windows of the
    // stage at a time.  gbase: global output offset of the tile.
    __device__ void emit(uint32_t b0, uint32_t b1, const LineState& st, uint64_t gbase) {
        const uint32_t tid = threadIdx.x;
        const uint32_t j = b0 + tid;
        uint8_t* stage = RAW();  // RAW + TABS, both dead now
        const uint8_t* pre = PRE();
        const uint32_t* esc = ESC();
        const uint64_t gb0 = gbase + EOFF()[b0];
        const uint64_t gb1 = gbase + EOFF()[b1 - 1] + COST()[b1 - 1] + 1;
        const uint32_t m = (st.in && !st.bad) ? st.m : 0u;
        uint32_t ic = 0;
        bool nl_done = !st.in;
        uint64_t oc = st.in ? gbase + EOFF()[j] : 0;
        uint64_t wlo = gb0;
        while (wlo < gb1) {
            uint64_t whi = wlo + (uint64_t)(kStageCap - 16);
            if (whi > gb1) whi = gb1;
            const uintptr_t a0 = ((uintptr_t)(A.out + wlo)) & ~(uintptr_t)15;
            const uintptr_t sbase = (uintptr_t)A.out - a0;  // stage index of global offset g = sbase + g
            while (!nl_done && oc < whi) {
                uint32_t b[2];
                uint32_t tl, adv;
                if (ic < m) {
                    const uint32_t pos = st.P + ic;
                    const uint32_t t = pre[pos];
                    if ((esc[pos >> 5] >> (pos & 31)) & 1u) {
                        b[0] = ' ';
                        b[1] = t;
                        tl = 2;
                        adv = 1;
                    } else {
                        b[0] = t;
                        tl = 1;
                        adv = D.len[t];
                    }
                } else {
                    b[0] = '\n';
                    tl = 1;
                    adv = 0;
                }
                for (uint32_t k = 0; k < tl; k++) {
                    uint64_t g = oc + k;
                    if (g >= wlo && g < whi) stage[sbase + g] = (uint8_t)b[k];
                }
                if (oc + tl > whi) break;
                oc += tl;
                if (ic < m) ic += adv;
                else nl_done = true;
            }
            __syncthreads();
            flush_stage(A.out, wlo, whi, a0, stage);
            __syncthreads();
            wlo = whi;
        }
    }

    __device__ void run() {
        uint32_t* misc = MISC();
        uint64_t* off = OFF();
        const uint32_t tid = threadIdx.x;
        while (true) {
            const uint32_t t = claim_tile(A.ws, &misc[2]);
            if (t >= A.ntiles) break;
            const uint64_t k0 = (uint64_t)t * kCL;
            const uint32_t nl = (uint32_t)min((uint64_t)kCL, A.n - k0);
            for (uint32_t j = tid; j <= nl; j += kWG) off[j] = A.in_off[k0 + j];
            if (tid < kCL) COST()[tid] = 0;
            __syncthreads();
            const bool regular = __syncthreads_and(tid >= nl || frame_error(k0, tid) == 0) != 0;
            // sweep 1: parse every batch, sizes into COST
            LineState st;
            uint32_t nb = 0, b0 = 0;
            while (b0 < nl) {
                b0 = batch(k0, nl, b0, regular, st);
                nb++;
            }
            // offsets inside the tile, then across tiles
            uint32_t total;
            uint32_t mylen = tid < nl ? COST()[tid] + 1 : 0u;
            uint32_t e = block_excl_scan(mylen, misc + 4, &total);
            if (tid < nl) EOFF()[tid] = e;
            if (tid == 0) {
                uint64_t ex = lookback(A.status, t, total);
                ((uint64_t*)misc)[6] = ex;
            }
            __syncthreads();
            const uint64_t gbase = ((uint64_t*)misc)[6];
            if (tid < nl) A.out_off[k0 + tid + 1] = gbase + e + mylen;
            if (t == 0 && tid == 0) A.out_off[0] = 0;
            const bool fits = gbase + total <= A.out_cap;
            if (A.out && !fits && tid == 0) atomicOr(&A.ws->enospc, 1u);
            if (A.out && fits) {
                if (nb == 1) {
                    emit(0, nl, st, gbase);
                } else {
                    b0 = 0;
                    while (b0 < nl) {
                        uint32_t b1 = batch(k0, nl, b0, regular, st);
                        emit(b0, b1, st, gbase);
                        b0 = b1;
                    }
                }
            }
            __syncthreads();
        }
        finish_workgroup(A.ws, A.res, gridDim.x);
    }
};

template <int LK>
__global__ void __launch_bounds__(kWG) compress_kernel(CompressArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    // stage the dictionary image (up to EXP) in LDS
    {
        const uint4* src = (const uint4*)a.tables;
        uint4* dst = (uint4*)smem;
        for (uint32_t k = threadIdx.x; k < a.tab_bytes / 16; k += kWG) dst[k] = src[k];
    }
    __syncthreads();
    Compressor<LK> c(a, smem);
    c.run();
}

// ============================================================================
// Decompression (bulk and random access)
// ============================================================================

constexpr int kDL = 256;            // lines (or requests) per tile
constexpr int kCbCap = 8192 + 16;   // LDS bytes of compressed lines per batch
constexpr int kDStage = 24576;      // LDS output stage
constexpr uint32_t kMaxCLine = 8191;  // longest compressed line accepted (newline excluded)
constexpr int kSeg = kWG * 16;      // bytes per decode segment

struct DecompressLds {
    uint32_t tabs, cb, stage, qoff, llen, lstart, bad, off, misc, total;
};

__host__ __device__ inline DecompressLds decompress_lds() {
    DecompressLds L;
    uint32_t o = 0;
    L.tabs = o;   o += 64 + 256 + 256 * kExpStride;  // header, LEN, EXP
    o = align16(o);
    L.cb = o;     o += align16(kCbCap);
    L.stage = o;  o += kDStage;
    L.qoff = o;   o += (kDL + 1) * 4;
    L.llen = o;   o += kDL * 4;
    L.lstart = o; o += kDL * 4;
    L.bad = o;    o += kDL;
    o = align16(o);
    L.off = o;    o += (kDL + 1) * 16;  // a and b per line (gather) or offsets (bulk)
    L.misc = o;   o += 256;
    L.total = align16(o);
    return L;
}

struct DecompressArgs {
    const uint8_t* tables;
    const uint8_t* in;
    uint64_t in_bytes;
    const uint64_t* in_off;
    uint64_t n;           // lines of the compressed buffer
    const uint64_t* ids;  // null for bulk
    uint64_t nreq;        // requests (= n for bulk)
    uint8_t* out;
    uint64_t out_cap;
    uint64_t* out_off;
    uint32_t ntiles;
    WsHeader* ws;
    uint64_t* status;
    ResultOut* res;
};

// misc words of the decoder (uint32 indices)
constexpr int kDmB1 = 0, kDmSlot = 2, kDmCarry = 4, kDmRun = 8, kDmScanA = 16, kDmScanB = 24, kDmBase64 = 20;

struct Decoder {
    const DecompressArgs& A;
    uint64_t r0 = 0;  // first request of the current tile
    uint8_t* smem;
    DecompressLds L;
    const uint8_t* LEN;
    const uint8_t* EXP;

    __device__ Decoder(const DecompressArgs& a, uint8_t* s) : A(a), smem(s) {
        L = decompress_lds();
        LEN = smem + 64;
        EXP = smem + 64 + 256;
    }
    __device__ uint32_t* QOFF() { return (uint32_t*)(smem + L.qoff); }
    __device__ uint32_t* LLEN() { return (uint32_t*)(smem + L.llen); }
    __device__ uint32_t* LSTART() { return (uint32_t*)(smem + L.lstart); }
    __device__ uint8_t* BAD() { return smem + L.bad; }
    __device__ uint64_t* LA() { return (uint64_t*)(smem + L.off); }  // [kDL+1] line start (abs)
    __device__ uint64_t* LB() { return (uint64_t*)(smem + L.off) + (kDL + 1); }
    __device__ uint32_t* MISC() { return (uint32_t*)(smem + L.misc); }

    // Scan state for escape parity: number of trailing spaces and whether the
    // whole piece is spaces.
    struct Run {
        uint32_t run;
        uint32_t all;
    };

    // Exclusive scan of Run over the workgroup (segment carry folded in by the caller).
    __device__ Run run_scan(Run v, Run* sc) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        Run inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            uint32_t ur = __shfl_up(inc.run, d, 64);
            uint32_t ua = __shfl_up(inc.all, d, 64);
            if (lane >= d && inc.all) {
                inc.run += ur;
                inc.all = ua;
            }
        }
        if (lane == 63) sc[w] = inc;
        __syncthreads();
        Run pre = {0, 1};
        for (int k = 0; k < w; k++) {
            Run s = sc[k];
            if (s.all) pre.run += s.run;
            else pre = s;
        }
        __syncthreads();
        // exclusive = combine(pre, inclusive-of-previous-lane)
        uint32_t pr = __shfl_up(inc.run, 1, 64), pa = __shfl_up(inc.all, 1, 64);
        Run ex;
        if (lane == 0) {
            ex = pre;
        } else {
            ex.run = pa ? pre.run + pr : pr;
            ex.all = pa ? pre.all : 0;
        }
        return ex;
    }

    // One pass over the batch bytes [cb_lo, cb_hi) of lines [b0, b1).
    // mode 0: sizes -> LLEN (raw, before bad-line adjustment) and BAD.
    // mode 1: emit the bytes whose batch-relative output position lies in
    //         [wlo, whi) into stage[sbase + pos].
    __device__ void pass(uint32_t b0, uint32_t b1, uint32_t cb_lo, uint32_t cb_hi, int mode, uint64_t wlo,
                         uint64_t whi, uint8_t* stage, intptr_t sbase, uint64_t gidx0) {
        const uint32_t tid = threadIdx.x;
        const uint8_t* cb = smem + L.cb;
        const uint32_t* qoff = QOFF();
        uint8_t* bad = BAD();
        uint32_t* misc = MISC();
        Run* rsc = (Run*)(misc + kDmRun);
        uint32_t* psc = misc + kDmScanA;
        uint32_t carry_run = 0;
        uint64_t carry_pos = 0;
        const uint32_t c0 = cb_lo & ~15u;
        for (uint32_t seg = c0; seg < cb_hi; seg += kSeg) {
            const uint32_t x0 = seg + tid * 16;
            uint8_t bytes[16];
            if (x0 < cb_hi) *(uint4*)bytes = *(const uint4*)(cb + x0);
            else *(uint4*)bytes = make_uint4(0, 0, 0, 0);
            uint32_t lo = max(x0, cb_lo), hi = min(x0 + 16, cb_hi);
            if (hi < lo) hi = lo;
            // run info of the piece
            Run me = {0, 1};
            for (uint32_t x = lo; x < hi; x++) {
                if (bytes[x - x0] == ' ') me.run++;
                else { me.run = 0; me.all = 0; }
            }
            if (lo == hi) { me.run = 0; me.all = 1; }
            Run ex = run_scan(me, rsc);
            uint32_t run = ex.all ? carry_run + ex.run : ex.run;
            // line of the first byte: last q with qoff[q] <= lo
            uint32_t q = b0;
            if (lo < hi) {
                uint32_t l = b0, r = b1;  // qoff[l] <= lo < qoff[r]
                while (r - l > 1) {
                    uint32_t mid = (l + r) >> 1;
                    if (qoff[mid] <= lo) l = mid;
                    else r = mid;
                }
                q = l;
            }
            // lengths
            uint32_t sum = 0;
            {
                uint32_t rr = run, qq = q;
                for (uint32_t x = lo; x < hi; x++) {
                    while (x >= qoff[qq + 1]) qq++;
                    const uint32_t c = bytes[x - x0];
                    const bool term = x + 1 == qoff[qq + 1];
                    const bool lit = rr & 1;
                    uint32_t len;
                    bool err = false;
                    if (term) {
                        len = 1;
                        err = lit;  // dangling escape
                    } else if (lit) {
                        len = 1;
                        err = c < 0x20 || c > 0x7E;
                    } else if (c == ' ') {
                        len = 0;
                    } else {
                        len = LEN[c];
                        err = len == 0;
                    }
                    rr = (c == ' ' && !term) ? rr + 1 : 0;
                    if (mode == 0) {
                        if (err && !bad[qq]) bad[qq] = kErrCorrupt;
                    } else if (bad[qq] && !term) {
                        len = 0;
                    }
                    sum += len;
                }
            }
            uint32_t segtot;
            uint32_t pos32 = block_excl_scan(sum, psc, &segtot);
            uint64_t pos = carry_pos + pos32;
            {
                uint32_t rr = run, qq = q;
                for (uint32_t x = lo; x < hi; x++) {
                    while (x >= qoff[qq + 1]) qq++;
                    const uint32_t c = bytes[x - x0];
                    const bool term = x + 1 == qoff[qq + 1];
                    const bool lit = rr & 1;
                    rr = (c == ' ' && !term) ? rr + 1 : 0;
                    if (mode == 0) {
                        uint32_t len;
                        if (term || lit) len = 1;
                        else if (c == ' ') len = 0;
                        else len = LEN[c];
                        pos += len;
                        if (term) LLEN()[qq] = (uint32_t)pos;  // end of line qq (batch-relative), fixed below
                    } else {
                        if (bad[qq] && !term) continue;
                        if (term) {
                            if (pos >= wlo && pos < whi) stage[sbase + (intptr_t)pos] = '\n';
                            pos += 1;
                        } else if (lit) {
                            if (pos >= wlo && pos < whi) stage[sbase + (intptr_t)pos] = (uint8_t)c;
                            pos += 1;
                        } else if (c != ' ') {
                            const uint32_t len = LEN[c];
                            const uint8_t* e = EXP + c * kExpStride;
                            for (uint32_t k = 0; k < len; k++) {
                                uint64_t p = pos + k;
                                if (p >= wlo && p < whi) stage[sbase + (intptr_t)p] = e[k];
                            }
                            pos += len;
                        }
                    }
                }
            }
            // carries for the next segment: the last thread's inclusive state
            if (tid == kWG - 1) {
                uint32_t rr = me.all ? (ex.all ? carry_run + ex.run : ex.run) + me.run : me.run;
                misc[kDmCarry] = rr;
            }
            __syncthreads();
            carry_run = misc[kDmCarry];
            carry_pos += segtot;
            __syncthreads();
        }
        (void)gidx0;
    }

    __device__ void run() {
        uint32_t* misc = MISC();
        const uint32_t tid = threadIdx.x;
        const bool gather = A.ids != nullptr;
        uint8_t* bad = BAD();
        uint32_t* qoff = QOFF();
        uint32_t* llen = LLEN();
        uint32_t* lstart = LSTART();
        uint64_t* la = LA();
        uint64_t* lb = LB();
        uint8_t* cb = smem + L.cb;
        while (true) {
            const uint32_t t = claim_tile(A.ws, &misc[kDmSlot]);
            if (t >= A.ntiles) break;
            r0 = (uint64_t)t * kDL;
            const uint32_t nl = (uint32_t)min((uint64_t)kDL, A.nreq - r0);
            // ---- framing of every line of the tile
            if (tid < nl) {
                const uint64_t r = r0 + tid;
                uint32_t fe = 0;
                uint64_t id = gather ? A.ids[r] : r;
                uint64_t a = 0, b = 0;
                if (id >= A.n) {
                    fe = kErrInval;
                } else {
                    a = A.in_off[id];
                    b = A.in_off[id + 1];
                    if (b <= a || b > A.in_bytes + 1 || b - a - 1 > kMaxCLine) fe = kErrInval;
                    else if (b == A.in_bytes + 1 && id + 1 != A.n) fe = kErrInval;
                }
                la[tid] = a;
                lb[tid] = b;
                bad[tid] = (uint8_t)fe;
                if (fe) note_error(A.ws, r, fe);
                llen[tid] = 0;
            }
            __syncthreads();
            const bool regular = __syncthreads_and(tid >= nl || bad[tid] == 0) != 0;
            // ---- sweep 1: sizes
            uint32_t nb = 0;
            uint32_t b0 = 0;
            uint32_t last_b1 = 0, last_lo = 0, last_hi = 0;
            while (b0 < nl) {
                uint32_t b1, cb_lo, cb_hi;
                load_batch(b0, nl, regular, gather, &b1, &cb_lo, &cb_hi);
                pass(b0, b1, cb_lo, cb_hi, 0, 0, 0, nullptr, 0, 0);
                __syncthreads();
                // LLEN holds line ends; turn them into lengths (bad lines: just the newline)
                {
                    uint32_t q = b0 + tid;
                    uint32_t v = 0;
                    if (q < b1) {
                        uint32_t end = llen[q];
                        uint32_t prev = (q > b0) ? llen[q - 1] : 0u;
                        v = bad[q] ? 1u : end - prev;
                        if (bad[q] == kErrCorrupt) note_error(A.ws, r0 + q, kErrCorrupt);
                    }
                    __syncthreads();
                    if (q < b1) llen[q] = v;
                }
                __syncthreads();
                nb++;
                last_b1 = b1;
                last_lo = cb_lo;
                last_hi = cb_hi;
                b0 = b1;
            }
            // ---- offsets
            uint32_t total;
            const uint32_t mylen = tid < nl ? llen[tid] : 0u;
            const uint32_t e = block_excl_scan(mylen, misc + kDmScanB, &total);
            if (tid < nl) lstart[tid] = e;
            if (tid == 0) ((uint64_t*)misc)[kDmBase64 / 2] = lookback(A.status, t, total);
            __syncthreads();
            const uint64_t gbase = ((uint64_t*)misc)[kDmBase64 / 2];
            if (tid < nl) A.out_off[r0 + tid + 1] = gbase + e + mylen;
            if (t == 0 && tid == 0) A.out_off[0] = 0;
            const bool fits = gbase + total <= A.out_cap;
            if (A.out && !fits && tid == 0) atomicOr(&A.ws->enospc, 1u);
            if (A.out && fits) {
                b0 = 0;
                while (b0 < nl) {
                    uint32_t b1, cb_lo, cb_hi;
                    if (nb == 1) {
                        b1 = last_b1;
                        cb_lo = last_lo;
                        cb_hi = last_hi;
                    } else {
                        load_batch(b0, nl, regular, gather, &b1, &cb_lo, &cb_hi);
                    }
                    // batch output range, tile-relative
                    const uint64_t o0 = lstart[b0];
                    const uint64_t o1 = (uint64_t)lstart[b1 - 1] + llen[b1 - 1];
                    uint64_t wlo = o0;
                    while (wlo < o1) {
                        uint64_t whi = min(o1, wlo + (uint64_t)(kDStage - 16));
                        const uintptr_t a0 = ((uintptr_t)(A.out + gbase + wlo)) & ~(uintptr_t)15;
                        // stage index of batch-relative position p: (out + gbase + o0 + p) - a0
                        const intptr_t sbase = (intptr_t)((uintptr_t)(A.out + gbase + o0) - a0);
                        pass(b0, b1, cb_lo, cb_hi, 1, wlo - o0, whi - o0, smem + L.stage, sbase, 0);
                        __syncthreads();
                        flush_stage(A.out, gbase + wlo, gbase + whi, a0, smem + L.stage);
                        __syncthreads();
                        wlo = whi;
                    }
                    b0 = b1;
                }
            }
            __syncthreads();
        }
        finish_workgroup(A.ws, A.res, gridDim.x);
        (void)cb;
    }

    // Choose the batch [b0, b1) that fits the CB buffer and load it.  Lines are
    // packed at qoff[q]; every line ends with its newline in CB.
    __device__ void load_batch(uint32_t b0, uint32_t nl, bool regular, bool gather, uint32_t* b1_out,
                               uint32_t* cb_lo, uint32_t* cb_hi) {
        const uint32_t tid = threadIdx.x;
        uint32_t* misc = MISC();
        uint8_t* bad = BAD();
        uint32_t* qoff = QOFF();
        uint64_t* la = LA();
        uint64_t* lb = LB();
        uint8_t* cb = smem + L.cb;
        // packed sizes: bad lines get a lone newline so that line framing stays intact
        const uint32_t q = b0 + tid;
        uint32_t sz = 0;
        if (q < nl) sz = bad[q] ? 1u : (uint32_t)(lb[q] - la[q]);
        uint32_t tot;
        // the bulk path keeps the bytes where they are: its first line starts at (in+a) & 15
        uint32_t lead = 0;
        if (!gather && regular) lead = (uint32_t)(((uintptr_t)(A.in + la[b0])) & 15);
        const uint32_t pos = block_excl_scan(q < nl ? sz : 0u, misc + kDmScanB, &tot) + lead;
        if (tid == 0) misc[kDmB1] = nl;
        __syncthreads();
        if (q < nl && q > b0) {
            // an irregular bulk tile goes one line per batch; otherwise fill CB
            const bool stop = (!gather && !regular) ? true : (pos + sz > (uint32_t)kCbCap);
            if (stop) atomicMin(&misc[kDmB1], q);
        }
        __syncthreads();
        const uint32_t b1 = misc[kDmB1];
        __syncthreads();
        if (q >= b0 && q < b1) qoff[q] = pos;
        if (q + 1 == b1) qoff[b1] = pos + sz;
        __syncthreads();
        if (!gather && regular) {
            const uint64_t lo = la[b0];
            uint64_t hi = lb[b1 - 1];
            if (hi > A.in_bytes) hi = A.in_bytes;
            const uintptr_t a0 = ((uintptr_t)(A.in + lo)) & ~(uintptr_t)15;
            load_range(A.in, A.in_bytes, lo, hi, a0, cb);
            __syncthreads();
            if (tid == 0 && lb[b1 - 1] == A.in_bytes + 1) cb[qoff[b1] - 1] = '\n';
        } else {
            // one lane per line copies its bytes
            if (q < b1) {
                uint32_t p = qoff[q];
                if (bad[q]) {
                    cb[p] = '\n';
                } else {
                    const uint8_t* s = A.in + la[q];
                    uint32_t n = (uint32_t)(lb[q] - la[q]);
                    bool virt = lb[q] == A.in_bytes + 1;
                    uint32_t nc = virt ? n - 1 : n;
                    for (uint32_t k = 0; k < nc; k++) cb[p + k] = s[k];
                    if (virt) cb[p + n - 1] = '\n';
                }
            }
            __syncthreads();
        }
        // the newline must be where the index says
        if (q < b1 && !bad[q]) {
            if (cb[qoff[q + 1] - 1] != '\n') {
                bad[q] = kErrInval;
                note_error(A.ws, r0 + q, kErrInval);
            }
        }
        __syncthreads();
        *b1_out = b1;
        *cb_lo = qoff[b0];
        *cb_hi = qoff[b1];
    }
};

__global__ void __launch_bounds__(kWG) decompress_kernel(DecompressArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    {
        // header + LEN at [0, 320), EXP at [320, 320 + 4096)
        const TableHeader* h = (const TableHeader*)a.tables;
        const uint32_t off_len = h->off_len, off_exp = h->off_exp;
        for (uint32_t k = threadIdx.x; k < 64 + 256 + 256 * kExpStride; k += kWG) {
            uint8_t v;
            if (k < 64) v = a.tables[k];
            else if (k < 320) v = a.tables[off_len + (k - 64)];
            else v = a.tables[off_exp + (k - 320)];
            smem[k] = v;
        }
    }
    __syncthreads();
    Decoder d(a, smem);
    d.run();
}

// ============================================================================
// Line index
// ============================================================================

constexpr int kIdxTile = kWG * 64;  // bytes per tile

struct IndexArgs {
    const uint8_t* buf;
    uint64_t len;
    uint64_t* off;
    uint64_t off_cap;
    uint64_t* n_lines_out;
    uint32_t ntiles;
    WsHeader* ws;
    uint64_t* status;
    ResultOut* res;
};

__global__ void __launch_bounds__(kWG) index_kernel(IndexArgs a) {
    __shared__ uint64_t sc[8];
    __shared__ uint32_t slot[4];
    __shared__ uint64_t sbase;
    const uint32_t tid = threadIdx.x;
    while (true) {
        const uint32_t t = claim_tile(a.ws, &slot[0]);
        if (t >= a.ntiles) break;
        const uint64_t x0 = (uint64_t)t * kIdxTile + (uint64_t)tid * 64;
        uint64_t cnt = 0;
        for (uint32_t k = 0; k < 64; k++) {
            uint64_t x = x0 + k;
            if (x < a.len && a.buf[x] == '\n') cnt++;
        }
        uint64_t tot;
        uint64_t ex = block_excl_scan64(cnt, sc, &tot);
        if (tid == 0) sbase = lookback(a.status, t, tot);
        __syncthreads();
        uint64_t k1 = sbase + ex;  // newlines before this thread's piece
        for (uint32_t k = 0; k < 64; k++) {
            uint64_t x = x0 + k;
            if (x < a.len && a.buf[x] == '\n') {
                k1++;
                if (k1 < a.off_cap) a.off[k1] = x + 1;
            }
        }
        if (t + 1 == a.ntiles && tid == 0) {
            uint64_t lines = sbase + tot;
            if (a.len > 0 && a.buf[a.len - 1] != '\n') {
                lines++;
                if (lines < a.off_cap) a.off[lines] = a.len + 1;
            }
            if (a.off_cap > 0) a.off[0] = 0;
            *a.n_lines_out = lines;
            if (lines + 1 > a.off_cap) atomicOr(&a.ws->enospc, 1u);
        }
        __syncthreads();
    }
    finish_workgroup(a.ws, a.res, gridDim.x);
}

// zero the workspace header and the tile status words; set errkey to "none"
__global__ void init_kernel(WsHeader* h, uint64_t* status, uint32_t ntiles, ResultOut* res) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        h->ticket = 0;
        h->done = 0;
        h->enospc = 0;
        h->errkey = ~0ull;
        h->total = 0;
        if (res) {
            res->code = 0;
            res->reserved = 0;
            res->first_bad = -1;
        }
    }
    for (uint32_t k = i; k < ntiles; k += gridDim.x * blockDim.x) status[k] = 0;
}

// index-only path with zero tiles: write off[0], count and result
__global__ void index_empty_kernel(uint64_t* off, uint64_t off_cap, uint64_t* n_lines_out, ResultOut* res) {
    if (off_cap > 0) off[0] = 0;
    *n_lines_out = 0;
    if (res) {
        res->code = off_cap > 0 ? 0 : -2;
        res->reserved = 0;
        res->first_bad = -1;
    }
}

__global__ void empty_result_kernel(uint64_t* out_off, ResultOut* res) {
    if (out_off) out_off[0] = 0;
    if (res) {
        res->code = 0;
        res->reserved = 0;
        res->first_bad = -1;
    }
}

// ============================================================================
// Host side
// ============================================================================

struct DeviceInfo {
    int cus = 0;
    bool ok = false;
};

DeviceInfo device_info() {
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DeviceInfo{};
    std::lock_guard<std::mutex> g(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1);
    if (!cache[dev].ok) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return DeviceInfo{};
        cache[dev].cus = p.multiProcessorCount;
        cache[dev].ok = true;
    }
    return cache[dev];
}

constexpr int kCompressWgPerCu = 2;
constexpr int kDecompressWgPerCu = 4;
constexpr int kIndexWgPerCu = 8;

uint32_t tiles_for(uint64_t n, uint64_t per) { return (uint32_t)((n + per - 1) / per); }

size_t ws_bytes_for(int op, uint64_t n) {
    DeviceInfo di = device_info();
    int cus = di.ok ? di.cus : 256;
    size_t h = sizeof(WsHeader);
    switch (op) {
        case ZS_OP_COMPRESS: {
            uint32_t nt = tiles_for(n, kCL);
            size_t st = ((size_t)nt * 8 + 255) & ~(size_t)255;
            size_t grid = (size_t)cus * kCompressWgPerCu;
            return h + st + grid * kWG * kGenLane;
        }
        case ZS_OP_DECOMPRESS:
        case ZS_OP_DECOMPRESS_LINES:
            return h + (size_t)tiles_for(n, kDL) * 8 + 64;
        case ZS_OP_INDEX:
            return h + (size_t)tiles_for(n, kIdxTile) * 8 + 64;
        default:
            return 0;
    }
}

}  // namespace

struct zs_dict {
    uint8_t* d_tables = nullptr;
    uint32_t blob_bytes = 0;
    uint32_t comp_bytes = 0;  // prefix staged by the compressor
    uint32_t lmax = 0;
    uint32_t lk = 8;
    int device = 0;
};

extern "C" {

const char* zs_status_str(int code) {
    switch (code) {
        case ZS_OK: return "ok";
        case ZS_EINVAL: return "invalid argument or framing";
        case ZS_ENOSPC: return "output does not fit";
        case ZS_ECORRUPT: return "corrupt data";
        case ZS_EDEVICE: return "device error";
        case ZS_ENOMEM: return "out of memory";
        default: return "unknown status";
    }
}

zs_status zs_dict_create(const uint8_t* len, const uint8_t* exp, zs_dict** out) {
    if (!len || !exp || !out) return ZS_EINVAL;
    std::vector<uint8_t> blob;
    int rc = zsi_compile_dict(len, exp, &blob);
    if (rc != ZS_OK) return (zs_status)rc;
    const TableHeader* h = (const TableHeader*)blob.data();
    zs_dict* d = new (std::nothrow) zs_dict;
    if (!d) return ZS_ENOMEM;
    d->blob_bytes = h->blob_bytes;
    d->comp_bytes = h->off_exp;
    d->lmax = h->lmax;
    d->lk = h->lk;
    if (hipGetDevice(&d->device) != hipSuccess) {
        delete d;
        return ZS_EDEVICE;
    }
    if (hipMalloc(&d->d_tables, blob.size()) != hipSuccess) {
        delete d;
        return ZS_ENOMEM;
    }
    if (hipMemcpy(d->d_tables, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d->d_tables);
        delete d;
        return ZS_EDEVICE;
    }
    CompressLds cl = compress_lds(d->comp_bytes);
    if (hipFuncSetAttribute((const void*)compress_kernel<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)cl.total) != hipSuccess ||
        hipFuncSetAttribute((const void*)compress_kernel<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)cl.total) != hipSuccess ||
        hipFuncSetAttribute((const void*)decompress_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)decompress_lds().total) != hipSuccess) {
        (void)hipFree(d->d_tables);
        delete d;
        return ZS_EDEVICE;
    }
    *out = d;
    return ZS_OK;
}

void zs_dict_destroy(zs_dict* d) {
    if (!d) return;
    if (d->d_tables) (void)hipFree(d->d_tables);
    delete d;
}

int zs_dict_lmax(const zs_dict* d) { return d ? (int)d->lmax : 0; }

uint64_t zs_compress_bound(uint64_t in_bytes, uint64_t n_lines) {
    (void)n_lines;
    return 6 * in_bytes + 1;
}

uint64_t zs_decompress_bound(const zs_dict* d, uint64_t in_bytes, uint64_t n_lines) {
    (void)n_lines;
    uint64_t l = (d && d->lmax) ? d->lmax : 1;
    return l * in_bytes + 1;
}

size_t zs_workspace_bytes(int op, uint64_t n) { return ws_bytes_for(op, n); }

static zs_status launch_init(WsHeader* h, uint64_t* status, uint32_t ntiles, ResultOut* res, hipStream_t s) {
    uint32_t blocks = ntiles / 256 + 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, s, h, status, ntiles, res);
    return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
}

zs_status zs_compress(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                      uint64_t n_lines, uint8_t* out, uint64_t out_cap, uint64_t* out_off, uint32_t flags,
                      void* ws, size_t ws_bytes, zs_result* res, void* stream) {
    if (!d || !in_off || !out_off || !ws || (!in && in_bytes)) return ZS_EINVAL;
    if (ws_bytes < zs_workspace_bytes(ZS_OP_COMPRESS, n_lines)) return ZS_EINVAL;
    if (flags & ~ZS_F_PREPROCESS) return ZS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (n_lines == 0) {
        hipLaunchKernelGGL(empty_result_kernel, dim3(1), dim3(1), 0, s, out_off, (ResultOut*)res);
        return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
    }
    DeviceInfo di = device_info();
    if (!di.ok) return ZS_EDEVICE;
    const uint32_t ntiles = tiles_for(n_lines, kCL);
    WsHeader* h = (WsHeader*)ws;
    uint64_t* status = (uint64_t*)(h + 1);
    size_t st_bytes = ((size_t)ntiles * 8 + 255) & ~(size_t)255;
    uint8_t* gen = (uint8_t*)status + st_bytes;
    if (launch_init(h, status, ntiles, (ResultOut*)res, s) != ZS_OK) return ZS_EDEVICE;
    CompressArgs a;
    a.tables = d->d_tables;
    a.tab_bytes = d->comp_bytes;
    a.in = in;
    a.in_bytes = in_bytes;
    a.in_off = in_off;
    a.n = n_lines;
    a.out = out;
    a.out_cap = out ? out_cap : ~0ull;
    a.out_off = out_off;
    a.flags = flags;
    a.ntiles = ntiles;
    a.ws = h;
    a.status = status;
    a.gen = gen;
    a.res = (ResultOut*)res;
    uint32_t grid = (uint32_t)di.cus * kCompressWgPerCu;
    if (grid > ntiles) grid = ntiles;
    CompressLds cl = compress_lds(d->comp_bytes);
    if (d->lk == 8)
        hipLaunchKernelGGL(compress_kernel<8>, dim3(grid), dim3(kWG), cl.total, s, a);
    else
        hipLaunchKernelGGL(compress_kernel<16>, dim3(grid), dim3(kWG), cl.total, s, a);
    return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
}

static zs_status decompress_common(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                                   uint64_t n_lines, const uint64_t* ids, uint64_t nreq, uint8_t* out,
                                   uint64_t out_cap, uint64_t* out_off, void* ws, size_t ws_bytes, zs_result* res,
                                   void* stream, int op) {
    if (!d || !in_off || !out_off || !ws || (!in && in_bytes)) return ZS_EINVAL;
    if (ws_bytes < zs_workspace_bytes(op, nreq)) return ZS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (nreq == 0) {
        hipLaunchKernelGGL(empty_result_kernel, dim3(1), dim3(1), 0, s, out_off, (ResultOut*)res);
        return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
    }
    DeviceInfo di = device_info();
    if (!di.ok) return ZS_EDEVICE;
    const uint32_t ntiles = tiles_for(nreq, kDL);
    WsHeader* h = (WsHeader*)ws;
    uint64_t* status = (uint64_t*)(h + 1);
    if (launch_init(h, status, ntiles, (ResultOut*)res, s) != ZS_OK) return ZS_EDEVICE;
    DecompressArgs a;
    a.tables = d->d_tables;
    a.in = in;
    a.in_bytes = in_bytes;
    a.in_off = in_off;
    a.n = n_lines;
    a.ids = ids;
    a.nreq = nreq;
    a.out = out;
    a.out_cap = out ? out_cap : ~0ull;
    a.out_off = out_off;
    a.ntiles = ntiles;
    a.ws = h;
    a.status = status;
    a.res = (ResultOut*)res;
    uint32_t grid = (uint32_t)di.cus * kDecompressWgPerCu;
    if (grid > ntiles) grid = ntiles;
    hipLaunchKernelGGL(decompress_kernel, dim3(grid), dim3(kWG), decompress_lds().total, s, a);
    return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
}

zs_status zs_decompress(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                        uint64_t n_lines, uint8_t* out, uint64_t out_cap, uint64_t* out_off, void* ws,
                        size_t ws_bytes, zs_result* res, void* stream) {
    return decompress_common(d, in, in_bytes, in_off, n_lines, nullptr, n_lines, out, out_cap, out_off, ws,
                             ws_bytes, res, stream, ZS_OP_DECOMPRESS);
}

zs_status zs_decompress_lines(const zs_dict* d, const uint8_t* in, uint64_t in_bytes, const uint64_t* in_off,
                              uint64_t n_lines, const uint64_t* ids, uint64_t n_ids, uint8_t* out,
                              uint64_t out_cap, uint64_t* out_off, void* ws, size_t ws_bytes, zs_result* res,
                              void* stream) {
    if (n_ids && !ids) return ZS_EINVAL;
    return decompress_common(d, in, in_bytes, in_off, n_lines, ids, n_ids, out, out_cap, out_off, ws, ws_bytes,
                             res, stream, ZS_OP_DECOMPRESS_LINES);
}

zs_status zs_index_lines(const uint8_t* buf, uint64_t len, uint64_t* off, uint64_t off_cap, uint64_t* n_lines_out,
                         void* ws, size_t ws_bytes, zs_result* res, void* stream) {
    if ((!buf && len) || !n_lines_out || !ws || (!off && off_cap)) return ZS_EINVAL;
    if (ws_bytes < zs_workspace_bytes(ZS_OP_INDEX, len)) return ZS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (len == 0) {
        hipLaunchKernelGGL(index_empty_kernel, dim3(1), dim3(1), 0, s, off, off_cap, n_lines_out, (ResultOut*)res);
        return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
    }
    DeviceInfo di = device_info();
    if (!di.ok) return ZS_EDEVICE;
    const uint32_t ntiles = tiles_for(len, kIdxTile);
    WsHeader* h = (WsHeader*)ws;
    uint64_t* status = (uint64_t*)(h + 1);
    if (launch_init(h, status, ntiles, (ResultOut*)res, s) != ZS_OK) return ZS_EDEVICE;
    IndexArgs a;
    a.buf = buf;
    a.len = len;
    a.off = off;
    a.off_cap = off_cap;
    a.n_lines_out = n_lines_out;
    a.ntiles = ntiles;
    a.ws = h;
    a.status = status;
    a.res = (ResultOut*)res;
    uint32_t grid = (uint32_t)di.cus * kIndexWgPerCu;
    if (grid > ntiles) grid = ntiles;
    hipLaunchKernelGGL(index_kernel, dim3(grid), dim3(kWG), 0, s, a);
    return hipGetLastError() == hipSuccess ? ZS_OK : ZS_EDEVICE;
}

}  // extern "C"
